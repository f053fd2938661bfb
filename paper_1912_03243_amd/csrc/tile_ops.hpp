// On-chip gate ops on an LDS-resident tile of 2^b amplitudes (generic,
// runtime tile size).  Shared by the tile-pass and batch kernels.
#pragma once

#include "juqcs_internal.hpp"

namespace juqcs {
namespace tileops {

constexpr int kThreads = 256;

// d[b_a + 2 b_c] with selects only (a table lookup would go through scratch).
template <typename T>
__device__ inline cplx<T> diag_pick(int e, int a, int c, cplx<T> d0, cplx<T> d1, cplx<T> d2,
                                    cplx<T> d3) {
  const bool x = (e >> a) & 1;
  const bool y = c >= 0 && ((e >> c) & 1);
  cplx<T> lo, hi;
  lo.re = x ? d1.re : d0.re;
  lo.im = x ? d1.im : d0.im;
  hi.re = x ? d3.re : d2.re;
  hi.im = x ? d3.im : d2.im;
  cplx<T> r;
  r.re = y ? hi.re : lo.re;
  r.im = y ? hi.im : lo.im;
  return r;
}

template <typename T>
__device__ inline void op_dense1(cplx<T>* sh, int b, int a, const cplx<T>* __restrict__ m) {
  const cplx<T> u0 = m[0], u1 = m[1], u2 = m[2], u3 = m[3];
  const int npairs = 1 << (b - 1);
  const int abit = 1 << a;
  for (int p = threadIdx.x; p < npairs; p += kThreads) {
    const int i0 = (int)insert_zero((uint64_t)p, a);
    const cplx<T> x = sh[i0], y = sh[i0 | abit];
    sh[i0] = cmad(u1, y, cmul(u0, x));
    sh[i0 | abit] = cmad(u3, y, cmul(u2, x));
  }
}

template <typename T>
__device__ inline void op_dense2(cplx<T>* sh, int b, int a, int c, const cplx<T>* __restrict__ m) {
  cplx<T> u[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) u[i] = m[i];
  const int lo = a < c ? a : c, hi = a < c ? c : a;
  const int ba = 1 << a, bc = 1 << c;
  const int nq = 1 << (b - 2);
  for (int p = threadIdx.x; p < nq; p += kThreads) {
    const int i = (int)insert_zero(insert_zero((uint64_t)p, lo), hi);
    const int idx[4] = {i, i | ba, i | bc, i | ba | bc};
    cplx<T> v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = sh[idx[r]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cplx<T> acc = cmul(u[4 * r], v[0]);
#pragma unroll
      for (int s = 1; s < 4; ++s) acc = cmad(u[4 * r + s], v[s], acc);
      sh[idx[r]] = acc;
    }
  }
}

template <typename T>
__device__ inline void op_diag2(cplx<T>* sh, int b, int a, int c, const cplx<T>* __restrict__ m) {
  const cplx<T> d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
  const int n = 1 << b;
  for (int e = threadIdx.x; e < n; e += kThreads) {
    sh[e] = cmul(diag_pick(e, a, c, d0, d1, d2, d3), sh[e]);
  }
}


// Dense 2^K x 2^K on K local bits (K = 3 or 4); bits[] in matrix order.
// All 2^K inputs of a group are read into registers first; each output row
// is then formed from uniform matrix loads and written straight back (row
// offsets are computed, not tabulated, so nothing is indexed dynamically).
template <typename T, int K>
__device__ inline void op_densek(cplx<T>* sh, int b, const int32_t* bits,
                                 const cplx<T>* __restrict__ m) {
  constexpr int D = 1 << K;
  int bt[K], sorted[K];
#pragma unroll
  for (int j = 0; j < K; ++j) bt[j] = sorted[j] = bits[j];
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j + 1 < K - i; ++j) {
      const int x = sorted[j], y = sorted[j + 1];
      sorted[j] = x < y ? x : y;
      sorted[j + 1] = x < y ? y : x;
    }
  const int ng = 1 << (b - K);
  for (int p = threadIdx.x; p < ng; p += kThreads) {
    int i = p;
#pragma unroll
    for (int j = 0; j < K; ++j) i = (int)insert_zero((uint64_t)i, sorted[j]);
    cplx<T> v[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      int o = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) o |= ((r >> j) & 1) << bt[j];
      v[r] = sh[i | o];
    }
#pragma unroll 1
    for (int r = 0; r < D; ++r) {
      cplx<T> acc = cmul(m[r * D], v[0]);
#pragma unroll
      for (int s = 1; s < D; ++s) acc = cmad(m[r * D + s], v[s], acc);
      int o = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) o |= ((r >> j) & 1) << bt[j];
      sh[i | o] = acc;
    }
  }
}

template <typename T>
__device__ inline void run_ops(cplx<T>* sh, int b, const TileOp* __restrict__ ops, int nops,
                               const cplx<T>* __restrict__ mats) {
  for (int o = 0; o < nops; ++o) {
    const TileOp op = ops[o];
    const cplx<T>* m = mats + op.moff;
    switch (op.kind) {
      case TOP_DENSE1: op_dense1<T>(sh, b, op.a, m); break;
      case TOP_DENSE2: op_dense2<T>(sh, b, op.a, op.b, m); break;
      case TOP_DIAG2: op_diag2<T>(sh, b, op.a, op.b, m); break;
      case TOP_DENSE3: op_densek<T, 3>(sh, b, op.bits, m); break;
      case TOP_DENSE4: op_densek<T, 4>(sh, b, op.bits, m); break;
      default: break;
    }
    __syncthreads();
  }
}

}  // namespace tileops
}  // namespace juqcs
