// On-chip gate ops on an LDS-resident tile of 2^b amplitudes.  Shared by the
// tile-pass kernels (single state, two-byte state) and the batch kernel.
//
// Two forms:
//  * Var<T, NT>   runtime tile size b (any b >= op width), NT threads;
//  * Fixed<T, TB, NT> compile-time tile size: every loop has a constant trip
//    count and is unrolled, and each op reads all of its operands before it
//    writes, so the LDS reads of a thread are issued back to back.
// Op kinds: dense 2x2 / 4x4 / 8x8 / 16x16 and two-bit diagonals (TileOp).
#pragma once

#include "juqcs_internal.hpp"

namespace juqcs {
namespace tileops {

// LDS slot of tile element e: e XOR a fold of its higher bits into the bits
// that pick the bank inside a 256-byte row (16 FP64 or 32 FP32 complex
// amplitudes).  Ops whose lanes step by large powers of two then spread over
// the banks instead of piling onto a few.  A bijection: the folded bits
// themselves are left unchanged.
template <typename T>
__device__ __forceinline__ int lds(int e) {
  constexpr int S = sizeof(T) == 8 ? 4 : 5;
  constexpr int M = (1 << S) - 1;
  return e ^ (((e >> S) ^ (e >> (2 * S))) & M);
}

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

template <int K>
__device__ inline void sort_bits(const int32_t* bits, int* bt, int* sorted) {
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
}

template <int K>
__device__ inline int group_base(int p, const int* sorted) {
  int i = p;
#pragma unroll
  for (int j = 0; j < K; ++j) i = (int)insert_zero((uint64_t)i, sorted[j]);
  return i;
}

template <int K>
__device__ inline int row_offset(int r, const int* bt) {
  int o = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) o |= ((r >> j) & 1) << bt[j];
  return o;
}

// ---------------------------------------------------------- runtime size ---
template <typename T, int NT>
struct Var {
  __device__ static void dense1(cplx<T>* sh, int b, int a, const cplx<T>* __restrict__ m) {
    const cplx<T> u0 = m[0], u1 = m[1], u2 = m[2], u3 = m[3];
    const int npairs = 1 << (b - 1), abit = 1 << a;
    for (int p = threadIdx.x; p < npairs; p += NT) {
      const int i0 = (int)insert_zero((uint64_t)p, a);
      const cplx<T> x = sh[lds<T>(i0)], y = sh[lds<T>(i0 | abit)];
      sh[lds<T>(i0)] = cmad(u1, y, cmul(u0, x));
      sh[lds<T>(i0 | abit)] = cmad(u3, y, cmul(u2, x));
    }
  }

  __device__ static void dense2(cplx<T>* sh, int b, int a, int c, const cplx<T>* __restrict__ m) {
    const int lo = a < c ? a : c, hi = a < c ? c : a;
    const int ba = 1 << a, bc = 1 << c, nq = 1 << (b - 2);
    for (int p = threadIdx.x; p < nq; p += NT) {
      const int i = (int)insert_zero(insert_zero((uint64_t)p, lo), hi);
      const cplx<T> v0 = sh[lds<T>(i)], v1 = sh[lds<T>(i | ba)], v2 = sh[lds<T>(i | bc)], v3 = sh[lds<T>(i | ba | bc)];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cplx<T> acc = cmul(m[4 * r], v0);
        acc = cmad(m[4 * r + 1], v1, acc);
        acc = cmad(m[4 * r + 2], v2, acc);
        acc = cmad(m[4 * r + 3], v3, acc);
        sh[lds<T>(i | ((r & 1) ? ba : 0) | ((r & 2) ? bc : 0))] = acc;
      }
    }
  }

  __device__ static void diag2(cplx<T>* sh, int b, int a, int c, const cplx<T>* __restrict__ m) {
    const cplx<T> d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
    for (int e = threadIdx.x; e < (1 << b); e += NT) sh[lds<T>(e)] = cmul(diag_pick(e, a, c, d0, d1, d2, d3), sh[lds<T>(e)]);
  }

  template <int K>
  __device__ static void densek(cplx<T>* sh, int b, const int32_t* bits,
                                const cplx<T>* __restrict__ m) {
    constexpr int D = 1 << K;
    int bt[K], sorted[K];
    sort_bits<K>(bits, bt, sorted);
    for (int p = threadIdx.x; p < (1 << (b - K)); p += NT) {
      const int i = group_base<K>(p, sorted);
      cplx<T> v[D];
#pragma unroll
      for (int r = 0; r < D; ++r) v[r] = sh[lds<T>(i | row_offset<K>(r, bt))];
#pragma unroll 1
      for (int r = 0; r < D; ++r) {
        cplx<T> acc = cmul(m[r * D], v[0]);
#pragma unroll
        for (int s = 1; s < D; ++s) acc = cmad(m[r * D + s], v[s], acc);
        sh[lds<T>(i | row_offset<K>(r, bt))] = acc;
      }
    }
  }

  __device__ static void run(cplx<T>* sh, int b, const TileOp* __restrict__ ops, int nops,
                             const cplx<T>* __restrict__ mats) {
    for (int o = 0; o < nops; ++o) {
      const TileOp op = ops[o];
      const cplx<T>* m = mats + op.moff;
      switch (op.kind) {
        case TOP_DENSE1: dense1(sh, b, op.a, m); break;
        case TOP_DENSE2: dense2(sh, b, op.a, op.b, m); break;
        case TOP_DIAG2: diag2(sh, b, op.a, op.b, m); break;
        case TOP_DENSE3: densek<3>(sh, b, op.bits, m); break;
        case TOP_DENSE4: densek<4>(sh, b, op.bits, m); break;
        default: break;
      }
      __syncthreads();
    }
  }
};

// ------------------------------------------------------- fixed tile size ---
// Groups of an op are processed in register blocks of KB: all reads of a
// block are issued before its writes (groups are disjoint, so blocks need no
// ordering among themselves), which bounds the live registers.  Ops of up to
// three qubits; a pass with a 4-qubit op must use Var.
template <typename T, int TB, int NT>
struct Fixed {
  static constexpr int NA = 1 << TB;

  __device__ static void dense1(cplx<T>* sh, int a, const cplx<T>* __restrict__ m, int tid) {
    constexpr int ITEMS = NA / 2, CNT = (ITEMS + NT - 1) / NT, KB = CNT < 4 ? CNT : 4;
    const cplx<T> u0 = m[0], u1 = m[1], u2 = m[2], u3 = m[3];
    const int abit = 1 << a;
#pragma unroll
    for (int k0 = 0; k0 < CNT; k0 += KB) {
      cplx<T> x[KB], y[KB];
      int i0[KB];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int p = (k0 + kk) * NT + tid;
        const int pc = (ITEMS % NT == 0 || p < ITEMS) ? p : 0;
        i0[kk] = (int)insert_zero((uint64_t)pc, a);
        x[kk] = sh[lds<T>(i0[kk])];
        y[kk] = sh[lds<T>(i0[kk] | abit)];
      }
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (ITEMS % NT == 0 || (k0 + kk) * NT + tid < ITEMS) {
          sh[lds<T>(i0[kk])] = cmad(u1, y[kk], cmul(u0, x[kk]));
          sh[lds<T>(i0[kk] | abit)] = cmad(u3, y[kk], cmul(u2, x[kk]));
        }
      }
    }
  }

  __device__ static void dense2(cplx<T>* sh, int a, int c, const cplx<T>* __restrict__ m, int tid) {
    constexpr int ITEMS = NA / 4, CNT = (ITEMS + NT - 1) / NT, KB = CNT < 2 ? CNT : 2;
    const int lo = a < c ? a : c, hi = a < c ? c : a;
    const int ba = 1 << a, bc = 1 << c;
#pragma unroll
    for (int k0 = 0; k0 < CNT; k0 += KB) {
      cplx<T> v[KB][4];
      int ix[KB];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int p = (k0 + kk) * NT + tid;
        const int pc = (ITEMS % NT == 0 || p < ITEMS) ? p : 0;
        ix[kk] = (int)insert_zero(insert_zero((uint64_t)pc, lo), hi);
        v[kk][0] = sh[lds<T>(ix[kk])];
        v[kk][1] = sh[lds<T>(ix[kk] | ba)];
        v[kk][2] = sh[lds<T>(ix[kk] | bc)];
        v[kk][3] = sh[lds<T>(ix[kk] | ba | bc)];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cplx<T> m0 = m[4 * r], m1 = m[4 * r + 1], m2 = m[4 * r + 2], m3 = m[4 * r + 3];
        const int off = ((r & 1) ? ba : 0) | ((r & 2) ? bc : 0);
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          cplx<T> acc = cmul(m0, v[kk][0]);
          acc = cmad(m1, v[kk][1], acc);
          acc = cmad(m2, v[kk][2], acc);
          acc = cmad(m3, v[kk][3], acc);
          if (ITEMS % NT == 0 || (k0 + kk) * NT + tid < ITEMS) sh[lds<T>(ix[kk] | off)] = acc;
        }
      }
    }
  }

  __device__ static void diag2(cplx<T>* sh, int a, int c, const cplx<T>* __restrict__ m, int tid) {
    constexpr int CNT = (NA + NT - 1) / NT;
    const cplx<T> d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const int e = k * NT + tid;
      if (NA % NT == 0 || e < NA) sh[lds<T>(e)] = cmul(diag_pick(e, a, c, d0, d1, d2, d3), sh[lds<T>(e)]);
    }
  }

  // 8x8 on three local bits; one group of 8 amplitudes in registers at a time
  __device__ static void dense3(cplx<T>* sh, const int32_t* bits, const cplx<T>* __restrict__ m,
                                int tid) {
    constexpr int ITEMS = NA / 8, CNT = (ITEMS + NT - 1) / NT;
    int bt[3], sorted[3];
    sort_bits<3>(bits, bt, sorted);
    int off[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) off[r] = row_offset<3>(r, bt);
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const int p = k * NT + tid;
      const bool ok = ITEMS % NT == 0 || p < ITEMS;
      const int ix = group_base<3>(ok ? p : 0, sorted);
      cplx<T> v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = sh[lds<T>(ix | off[r])];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        cplx<T> acc = cmul(m[8 * r], v[0]);
#pragma unroll
        for (int s = 1; s < 8; ++s) acc = cmad(m[8 * r + s], v[s], acc);
        if (ok) sh[lds<T>(ix | off[r])] = acc;
      }
    }
  }

  __device__ static void run(cplx<T>* sh, const TileOp* __restrict__ ops, int nops,
                             const cplx<T>* __restrict__ mats) {
    for (int o = 0; o < nops; ++o) {
      const TileOp op = ops[o];
      const cplx<T>* m = mats + op.moff;
      const int tid = (int)threadIdx.x;
      if (op.kind == TOP_DENSE2) dense2(sh, op.a, op.b, m, tid);
      else if (op.kind == TOP_DENSE1) dense1(sh, op.a, m, tid);
      else if (op.kind == TOP_DIAG2) diag2(sh, op.a, op.b, m, tid);
      else dense3(sh, op.bits, m, tid);  // callers route passes with 4-qubit ops elsewhere
      __syncthreads();
    }
  }
};

}  // namespace tileops
}  // namespace juqcs
