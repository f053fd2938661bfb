// On-chip gate ops on an LDS-resident tile of 2^b amplitudes.  Shared by the
// tile-pass kernels (single state, two-byte state) and the batch kernel.
//
// Two forms:
//  * Var<T, NT>   runtime tile size b (any b >= op width), NT threads;
//  * Fixed<T, TB, NT> compile-time tile size: every loop has a constant trip
//    count and is unrolled, and each op reads all of its operands before it
//    writes, so the LDS reads of a thread are issued back to back.
// Op kinds: dense 2x2 / 4x4 / 8x8 / 16x16, two-bit diagonals and monomial
// (permutation times phases) ops on up to three bits (TileOp).
// In the fixed form the FP32 8x8 ops run on the matrix cores (16x16x4 MFMA).
#pragma once

#include "juqcs_internal.hpp"

namespace juqcs {
namespace tileops {

// LDS slot of tile element e: e XOR a fold of its higher bits into the bits
// that pick the bank inside a 256-byte row (16 FP64 or 32 FP32 complex
// amplitudes).  Ops whose lanes step by large powers of two then spread over
// the banks instead of piling onto a few.  A bijection (the folded bits
// themselves are left unchanged), and linear over XOR:
// lds(a ^ b) = lds(a) ^ lds(b).
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

// 32-bit group_base for tile-local indices.  Spreading is a bit
// permutation, so spread(x | y) = spread(x) | spread(y) for disjoint x, y;
// together with the XOR-linear LDS swizzle this splits every element
// address into a wave-uniform part and a per-lane part fixed for the op.
template <int K>
__device__ inline int spread(int x, const int* sorted) {
#pragma unroll
  for (int j = 0; j < K; ++j) x = ((x >> sorted[j]) << (sorted[j] + 1)) | (x & ((1 << sorted[j]) - 1));
  return x;
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

  // monomial: out[r] = c[r] in[sigma(r)] on the group of 2^K amplitudes
  template <int K>
  __device__ static void perm(cplx<T>* sh, int b, const int32_t* bits, int sigma,
                              const cplx<T>* __restrict__ m) {
    constexpr int D = 1 << K;
    int bt[K], sorted[K];
    sort_bits<K>(bits, bt, sorted);
    for (int p = threadIdx.x; p < (1 << (b - K)); p += NT) {
      const int i = group_base<K>(p, sorted);
      cplx<T> v[D];
#pragma unroll
      for (int r = 0; r < D; ++r) v[r] = sh[lds<T>(i | row_offset<K>((sigma >> (3 * r)) & 7, bt))];
#pragma unroll
      for (int r = 0; r < D; ++r) sh[lds<T>(i | row_offset<K>(r, bt))] = cmul(m[r], v[r]);
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
        case TOP_PERM:
          if (op.k == 1) perm<1>(sh, b, op.bits, op.a, m);
          else if (op.k == 2) perm<2>(sh, b, op.bits, op.a, m);
          else perm<3>(sh, b, op.bits, op.a, m);
          break;
        default: break;
      }
      __syncthreads();
    }
  }
};

// Per-lane tables of one FP32 matrix-core 8x8 op on a tile of 16 NBLK groups:
// what the op's lanes would otherwise recompute from the op's bits for every
// tile (sorting, bit spreading, lane swaps, swizzling, operand selection).
// Built once per pass; all offsets are tile-local and fit 16 bits (tiles of
// at most 2^14 amplitudes).
template <int NBLK>
struct alignas(16) MmaTab {
  float a[64][4];       // A operand of lane l for the steps j = 0..3
  uint16_t off[64][2];  // lds slots of the lane's two amplitudes (block part excluded)
  uint16_t ub[NBLK];    // block part of the slots of each block of 16 groups
};

// Uniform parameters of one in-tile op of a pass, built once per launch (the
// fixed-size kernels would otherwise recompute them for every tile).  Byte
// offsets within the tile; the group of item k NT + tid sits at
// grp[k] ^ lds(spread(tid)) * sizeof(amplitude).
struct alignas(16) OpPre {
  int32_t row[8];   // offsets of the op's rows within a group (the rows written)
  int32_t src[8];   // monomial ops: offsets of the rows read for each written row
  int32_t grp[16];  // uniform part of the group offset of items k NT + tid
  int32_t pos;      // group-bit positions, ascending, 4 bits each
  int32_t lsw;      // lane swaps (lane_swap): count in bits 0-2, then pairs of
                    // thread-index bits (2 + 4 bits each) to exchange
  int32_t pad[2];
};

// Thread index with the op's lane swaps applied.  An op's groups are handed
// to threads through spread(lane_swap(tid)): the swaps move thread-index
// bits so that the lanes of one LDS access phase (8 lanes for 16-byte, 16
// for 8-byte amplitudes: 128 bytes) fall into distinct bank slots, which the
// plain order misses when the op's targets sit among the low tile bits.
__device__ __forceinline__ int lane_swap(int t, int lsw) {
  const int n = lsw & 7;
  for (int i = n - 1; i >= 0; --i) {  // last recorded swap first
    const int a = (lsw >> (3 + 6 * i)) & 3, b = (lsw >> (5 + 6 * i)) & 15;
    const int x = ((t >> a) ^ (t >> b)) & 1;
    t ^= (x << a) | (x << b);
  }
  return t;
}

// ------------------------------------------------------- fixed tile size ---
// Groups of an op are processed in register blocks of KB: all reads of a
// block are issued before its writes (groups are disjoint, so blocks need no
// ordering among themselves), which bounds the live registers.  Ops of up to
// three qubits; a pass with a 4-qubit op must use Var.
template <typename T, int TB, int NT>
struct Fixed {
  static constexpr int NA = 1 << TB;

  static constexpr int CB = (int)sizeof(cplx<T>);

  // Target positions of an op (ascending) packed 4 bits each.
  template <int K>
  __device__ static void unpack(int packed, int* pos) {
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = (packed >> (4 * j)) & 15;
  }

  // Fills pre[0..nops) (one op per thread, written straight to LDS; the
  // caller synchronises).
  __device__ static void build_pre(OpPre* pre, const TileOp* __restrict__ ops, int nops) {
    for (int o = threadIdx.x; o < nops; o += NT) {
      const TileOp op = ops[o];
      OpPre& p = pre[o];
      int b0 = 0, b1 = 0, b2 = 0, np = 0;  // target bits in matrix order
      if (op.kind == TOP_DENSE1) {
        b0 = op.a;
        np = 1;
      } else if (op.kind == TOP_DENSE2) {
        b0 = op.a;
        b1 = op.b;
        np = 2;
      } else if (op.kind == TOP_PERM || op.kind == TOP_DENSE3 || op.kind == TOP_DENSE3G) {
        np = op.kind == TOP_PERM ? op.k : 3;
        b0 = op.bits[0];
        b1 = np > 1 ? op.bits[1] : 0;
        b2 = np > 2 ? op.bits[2] : 0;
      }  // TOP_DIAG2: items are single elements (np = 0)
      for (int r = 0; r < 8; ++r) {
        const int sr = op.kind == TOP_PERM ? (op.a >> (3 * r)) & 7 : r;
        const int ro = (np > 0 ? (r & 1) << b0 : 0) | (np > 1 ? ((r >> 1) & 1) << b1 : 0) |
                       (np > 2 ? ((r >> 2) & 1) << b2 : 0);
        const int rs = (np > 0 ? (sr & 1) << b0 : 0) | (np > 1 ? ((sr >> 1) & 1) << b1 : 0) |
                       (np > 2 ? ((sr >> 2) & 1) << b2 : 0);
        p.row[r] = r < (1 << np) ? lds<T>(ro) * CB : 0;
        p.src[r] = r < (1 << np) ? lds<T>(rs) * CB : 0;
      }
      // ascending positions
      int s0 = b0, s1 = b1, s2 = b2;
      if (np > 1 && s0 > s1) { const int t = s0; s0 = s1; s1 = t; }
      if (np > 2 && s1 > s2) { const int t = s1; s1 = s2; s2 = t; }
      if (np > 1 && s0 > s1) { const int t = s0; s0 = s1; s1 = t; }
      const int items = NA >> np;
      for (int k = 0; k < 16; ++k) {
        int g = k * NT < items ? k * NT : 0;
        if (np > 0) g = ((g >> s0) << (s0 + 1)) | (g & ((1 << s0) - 1));
        if (np > 1) g = ((g >> s1) << (s1 + 1)) | (g & ((1 << s1) - 1));
        if (np > 2) g = ((g >> s2) << (s2 + 1)) | (g & ((1 << s2) - 1));
        p.grp[k] = lds<T>(g) * CB;
      }
      p.pos = (np > 0 ? s0 : 0) | ((np > 1 ? s1 : 0) << 4) | ((np > 2 ? s2 : 0) << 8);
      p.lsw = np > 0 ? lane_swaps(np, s0, s1, s2) : 0;
    }
  }

  // Lane swaps of an op with np targets at ascending positions s0 < s1 < s2:
  // thread-index bit j goes to the j-th non-target tile position; for the W
  // lane bits of an access phase, a bit whose bank slot (low W bits of its
  // LDS slot) is spanned by the previous ones trades places with the first
  // higher thread-index bit that adds a new slot direction.
  __device__ static int lane_swaps(int np, int s0, int s1, int s2) {
    constexpr int W = sizeof(T) == 8 ? 3 : 4;
    constexpr int SLOTS = 1 << W;
    int lt = 0;  // thread-index bits that index items
    for (int items = (NA >> np) < NT ? (NA >> np) : NT; (1 << lt) < items;) ++lt;
    // P: the non-target positions in order, 4 bits each (packed: no local
    // array, which would go to scratch)
    uint64_t P = 0;
    int cnt = 0;
    for (int b = 0; b < TB; ++b)
      if (!(np > 0 && b == s0) && !(np > 1 && b == s1) && !(np > 2 && b == s2)) P |= (uint64_t)b << (4 * cnt++);
    auto at = [&](int i) { return (int)((P >> (4 * i)) & 15); };
    int span = 1;  // bit v set: slot direction v is in the span of the accepted lanes
    int lsw = 0, n = 0;
    for (int j = 0; j < W && j < lt; ++j) {
      int pick = -1;
      for (int jj = j; jj < lt && pick < 0; ++jj) {
        const int v = lds<T>(1 << at(jj)) & (SLOTS - 1);
        if (!((span >> v) & 1)) pick = jj;
      }
      if (pick < 0) continue;  // no independent direction left: a conflict stays
      if (pick != j) {
        const uint64_t x = (uint64_t)(at(j) ^ at(pick));
        P ^= (x << (4 * j)) | (x << (4 * pick));
        lsw |= (j | (pick << 2)) << (3 + 6 * n);
        ++n;
      }
      const int v = lds<T>(1 << at(j)) & (SLOTS - 1);
      int grown = span;
      for (int u = 0; u < SLOTS; ++u)
        if ((span >> u) & 1) grown |= 1 << (u ^ v);
      span = grown;
    }
    return lsw | n;
  }

  __device__ static void dense1(cplx<T>* sh, const OpPre& q, const cplx<T>* __restrict__ m, int tid) {
    constexpr int ITEMS = NA / 2, CNT = (ITEMS + NT - 1) / NT, KB = CNT < 4 ? CNT : 4;
    const cplx<T> u0 = m[0], u1 = m[1], u2 = m[2], u3 = m[3];
    int pos[1];
    unpack<1>(q.pos, pos);
    const int ob = q.row[1];
    const int lt = lds<T>(spread<1>(lane_swap(tid, q.lsw), pos)) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k0 = 0; k0 < CNT; k0 += KB) {
      cplx<T> x[KB], y[KB];
      int o[KB];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int k = k0 + kk;
        const bool ok = ITEMS % NT == 0 || k * NT + tid < ITEMS;
        o[kk] = ok ? q.grp[k] ^ lt : 0;
        x[kk] = *reinterpret_cast<const cplx<T>*>(base + o[kk]);
        y[kk] = *reinterpret_cast<const cplx<T>*>(base + (o[kk] ^ ob));
      }
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (ITEMS % NT == 0 || (k0 + kk) * NT + tid < ITEMS) {
          *reinterpret_cast<cplx<T>*>(base + o[kk]) = cmad(u1, y[kk], cmul(u0, x[kk]));
          *reinterpret_cast<cplx<T>*>(base + (o[kk] ^ ob)) = cmad(u3, y[kk], cmul(u2, x[kk]));
        }
      }
    }
  }

  __device__ static void dense2(cplx<T>* sh, const OpPre& q, const cplx<T>* __restrict__ m, int tid) {
    constexpr int ITEMS = NA / 4, CNT = (ITEMS + NT - 1) / NT, KB = CNT < 2 ? CNT : 2;
    int pos[2];
    unpack<2>(q.pos, pos);
    int off[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) off[r] = q.row[r];
    const int lt = lds<T>(spread<2>(lane_swap(tid, q.lsw), pos)) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k0 = 0; k0 < CNT; k0 += KB) {
      cplx<T> v[KB][4];
      int o[KB];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int k = k0 + kk;
        const bool ok = ITEMS % NT == 0 || k * NT + tid < ITEMS;
        o[kk] = ok ? q.grp[k] ^ lt : 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[kk][r] = *reinterpret_cast<const cplx<T>*>(base + (o[kk] ^ off[r]));
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cplx<T> m0 = m[4 * r], m1 = m[4 * r + 1], m2 = m[4 * r + 2], m3 = m[4 * r + 3];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          cplx<T> acc = cmul(m0, v[kk][0]);
          acc = cmad(m1, v[kk][1], acc);
          acc = cmad(m2, v[kk][2], acc);
          acc = cmad(m3, v[kk][3], acc);
          if (ITEMS % NT == 0 || (k0 + kk) * NT + tid < ITEMS)
            *reinterpret_cast<cplx<T>*>(base + (o[kk] ^ off[r])) = acc;
        }
      }
    }
  }

  __device__ static void diag2(cplx<T>* sh, const OpPre& q, int a, int c, const cplx<T>* __restrict__ m,
                               int tid) {
    constexpr int CNT = (NA + NT - 1) / NT;
    const cplx<T> d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
    const int lt = lds<T>(tid) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const int e = k * NT + tid;
      if (NA % NT == 0 || e < NA) {
        cplx<T>* z = reinterpret_cast<cplx<T>*>(base + (q.grp[k] ^ lt));
        *z = cmul(diag_pick(e, a, c, d0, d1, d2, d3), *z);
      }
    }
  }

  // monomial on K <= 3 local bits: out[r] = c[r] in[sigma(r)]; the reads go
  // straight to the permuted rows, so no selects
  template <int K>
  __device__ static void perm(cplx<T>* sh, const OpPre& q, const cplx<T>* __restrict__ m, int tid) {
    constexpr int D = 1 << K, ITEMS = NA >> K, CNT = (ITEMS + NT - 1) / NT;
    constexpr int KB = CNT < 2 || K == 3 ? 1 : 2;  // at most 8 amplitudes in flight
    int pos[K];
    unpack<K>(q.pos, pos);
    const int lt = lds<T>(spread<K>(lane_swap(tid, q.lsw), pos)) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k0 = 0; k0 < CNT; k0 += KB) {
      cplx<T> v[KB][D];
      int o[KB];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int k = k0 + kk;
        const bool ok = ITEMS % NT == 0 || k * NT + tid < ITEMS;
        o[kk] = ok ? q.grp[k] ^ lt : 0;
#pragma unroll
        for (int r = 0; r < D; ++r) v[kk][r] = *reinterpret_cast<const cplx<T>*>(base + (o[kk] ^ q.src[r]));
      }
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        if (ITEMS % NT == 0 || (k0 + kk) * NT + tid < ITEMS) {
#pragma unroll
          for (int r = 0; r < D; ++r)
            *reinterpret_cast<cplx<T>*>(base + (o[kk] ^ q.row[r])) = cmul(m[r], v[kk][r]);
        }
      }
    }
  }

  // 8x8 on three local bits on the vector units (FP64: the matrix cores run
  // FP64 at the vector rate, and the uniform coefficients come through the
  // scalar cache); one group of 8 amplitudes in registers at a time.
  __device__ static void dense3_valu(cplx<T>* sh, const OpPre& q, const cplx<T>* __restrict__ m, int tid) {
    constexpr int ITEMS = NA / 8, CNT = (ITEMS + NT - 1) / NT;
    int pos[3];
    unpack<3>(q.pos, pos);
    int off[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) off[r] = q.row[r];
    const int lt = lds<T>(spread<3>(lane_swap(tid, q.lsw), pos)) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const bool ok = ITEMS % NT == 0 || k * NT + tid < ITEMS;
      const int gb = ok ? q.grp[k] ^ lt : 0;
      cplx<T> v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = *reinterpret_cast<const cplx<T>*>(base + (gb ^ off[r]));
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        cplx<T> acc = cmul(m[8 * r], v[0]);
#pragma unroll
        for (int s = 1; s < 8; ++s) acc = cmad(m[8 * r + s], v[s], acc);
        if (ok) *reinterpret_cast<cplx<T>*>(base + (gb ^ off[r])) = acc;
      }
    }
  }

  // 8x8 in three-product form (Gauss): with s = Re x + Im x per input,
  // Re y_r = sum_s Re m_rs s_s - (Re + Im) m_rs Im x_s and
  // Im y_r = sum_s Re m_rs s_s + (Im - Re) m_rs Re x_s: 26 instead of 32
  // FP64 operations per output (g: 24 reals per row, uniform).
  __device__ static void dense3_gauss(cplx<T>* sh, const OpPre& q, const T* __restrict__ g, int tid) {
    constexpr int ITEMS = NA / 8, CNT = (ITEMS + NT - 1) / NT;
    int pos[3];
    unpack<3>(q.pos, pos);
    int off[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) off[r] = q.row[r];
    const int lt = lds<T>(spread<3>(lane_swap(tid, q.lsw), pos)) * CB;
    char* base = reinterpret_cast<char*>(sh);
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
      const bool ok = ITEMS % NT == 0 || k * NT + tid < ITEMS;
      const int gb = ok ? q.grp[k] ^ lt : 0;
      T xr[8], xi[8], xs[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const cplx<T> v = *reinterpret_cast<const cplx<T>*>(base + (gb ^ off[r]));
        xr[r] = v.re;
        xi[r] = v.im;
        xs[r] = v.re + v.im;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const T* w = g + 24 * r;
        T t = w[0] * xs[0], a = w[8] * xi[0], c = w[16] * xr[0];
#pragma unroll
        for (int s = 1; s < 8; ++s) {
          t = fma(w[s], xs[s], t);
          a = fma(w[8 + s], xi[s], a);
          c = fma(w[16 + s], xr[s], c);
        }
        if (ok) *reinterpret_cast<cplx<T>*>(base + (gb ^ off[r])) = cplx<T>{t - a, t + c};
      }
    }
  }

  // 8x8 on three local bits, on the matrix cores (FP32).  The complex product
  // is a real 16x16 product over the 16 components (Re, Im of the 8
  // amplitudes) of a group; a wave takes 16 groups at a time as the 16
  // columns.  Lane 16 q + c (c: column) reads amplitudes q and q + 4 of its
  // group (8 bytes each) and feeds, in the four 16x16x4 steps j, Re a_q,
  // Im a_q, Re a_(q+4), Im a_(q+4) as K slot q.  The output rows are ordered
  // so that the lane receives exactly what it read: rows 4 q .. 4 q + 3 hold
  // Re a_q, Im a_q, Re a_(q+4), Im a_(q+4), written back in place (groups
  // are disjoint across waves and a wave reads a block before it writes it:
  // no barrier inside the op).  A (row rho, K slot q of step j) is the
  // real-embedding entry of output component (amplitude rho/4 + 4 (rho%4 >= 2),
  // part rho%2) and input component (amplitude q + 4 (j >= 2), part j%2).
  // The 16 columns of block b are the groups lane_swap(16 b + c): the op's
  // lane swaps put the 16 lanes of an 8-byte LDS access phase on distinct
  // bank slots.
  __device__ static T mma_a(const cplx<T>* m, int lane, int j) {
    const int c = lane & 15, q = lane >> 4;
    const int r = (c >> 2) + 4 * ((c & 3) >> 1), p = c & 1;
    const int sc = q + 4 * (j >> 1), pp = j & 1;
    const cplx<T> z = m[8 * r + sc];
    return p == pp ? z.re : (p ? z.im : -z.im);
  }

  __device__ static void dense3_mma(cplx<T>* sh, const OpPre& q, const cplx<T>* m, int tid) {
    static_assert(sizeof(T) == 4, "FP32 matrix-core op");
    constexpr int ITEMS = NA / 8, NBLK = ITEMS / 16, W = NT / 64, CB = (int)sizeof(cplx<T>);
    static_assert(ITEMS % 16 == 0 && NBLK % W == 0, "whole 16-group blocks per wave");
    int pos[3];
    unpack<3>(q.pos, pos);
    const int lane = tid & 63, c = lane & 15, qq = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    T a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = mma_a(m, lane, j);
    const int lc = lds<T>(spread<3>(lane_swap(c, q.lsw), pos)) * CB;
    const int o0 = lc ^ q.row[qq], o1 = lc ^ q.row[qq + 4];
    char* base = reinterpret_cast<char*>(sh);
    constexpr int NB = NBLK / W >= 2 ? 2 : 1;
#pragma unroll
    for (int i0 = 0; i0 < NBLK / W; i0 += NB) {
      int ub[NB];  // block parts (wave-uniform)
      cplx<T> x0[NB], x1[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        ub[u] = lds<T>(spread<3>(lane_swap(((i0 + u) * W + wave) * 16, q.lsw), pos)) * CB;
        x0[u] = *reinterpret_cast<const cplx<T>*>(base + (ub[u] ^ o0));
        x1[u] = *reinterpret_cast<const cplx<T>*>(base + (ub[u] ^ o1));
      }
      mma_block<NB>(a, x0, x1, base, ub, o0, o1);
    }
  }

  // Four 16x16x4 steps for NB blocks, then the write-back in place.
  template <int NB>
  __device__ static void mma_block(const T* a, const cplx<T>* x0, const cplx<T>* x1, char* base,
                                   const int* ub, int o0, int o1) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f acc[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], x0[u].re, v4f{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], x0[u].im, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], x1[u].re, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], x1[u].im, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      *reinterpret_cast<cplx<T>*>(base + (ub[u] ^ o0)) = cplx<T>{acc[u][0], acc[u][1]};
      *reinterpret_cast<cplx<T>*>(base + (ub[u] ^ o1)) = cplx<T>{acc[u][2], acc[u][3]};
    }
  }

  static constexpr int kBlocks = NA / 8 / 16;
  using Tab = MmaTab<kBlocks>;

  // Fills tabs[0..) with the tables of the pass's 8x8 ops in order (the
  // caller guarantees room and synchronises afterwards).
  __device__ static void build_tabs(Tab* tabs, const TileOp* __restrict__ ops, int nops,
                                    const cplx<T>* __restrict__ mats) {
    int k = 0;
    for (int o = 0; o < nops; ++o) {
      const TileOp op = ops[o];
      if (op.kind != TOP_DENSE3) continue;
      Tab& t = tabs[k++];
      int bt[3], sorted[3];
      sort_bits<3>(op.bits, bt, sorted);
      const int lsw = lane_swaps(3, sorted[0], sorted[1], sorted[2]);
      const cplx<T>* m = mats + op.moff;
      for (int i = threadIdx.x; i < 64 + kBlocks; i += NT) {
        if (i < 64) {
          const int c = i & 15, q = i >> 4;
          const int lc = lds<T>(spread<3>(lane_swap(c, lsw), sorted));
#pragma unroll
          for (int j = 0; j < 4; ++j) t.a[i][j] = mma_a(m, i, j);
          t.off[i][0] = (uint16_t)(lc ^ lds<T>(row_offset<3>(q, bt)));
          t.off[i][1] = (uint16_t)(lc ^ lds<T>(row_offset<3>(q + 4, bt)));
        } else {
          t.ub[i - 64] = (uint16_t)lds<T>(spread<3>(lane_swap((i - 64) * 16, lsw), sorted));
        }
      }
    }
  }

  // The 8x8 matrix-core op from its tables (same data layout as dense3_mma).
  __device__ static void dense3_tab(cplx<T>* sh, const Tab& t, int tid) {
    static_assert(sizeof(T) == 4, "FP32 matrix-core op");
    constexpr int W = NT / 64, PER_W = kBlocks / W, CB = (int)sizeof(cplx<T>);
    static_assert(kBlocks % W == 0, "whole 16-group blocks per wave");
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f av = *reinterpret_cast<const v4f*>(t.a[lane]);
    const T a[4] = {av[0], av[1], av[2], av[3]};
    const int o0 = t.off[lane][0] * CB, o1 = t.off[lane][1] * CB;
    char* base = reinterpret_cast<char*>(sh);
    constexpr int NB = PER_W >= 2 ? 2 : 1;
#pragma unroll
    for (int i0 = 0; i0 < PER_W; i0 += NB) {
      int ub[NB];
      cplx<T> x0[NB], x1[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        ub[u] = t.ub[(i0 + u) * W + wave] * CB;
        x0[u] = *reinterpret_cast<const cplx<T>*>(base + (ub[u] ^ o0));
        x1[u] = *reinterpret_cast<const cplx<T>*>(base + (ub[u] ^ o1));
      }
      mma_block<NB>(a, x0, x1, base, ub, o0, o1);
    }
  }

  // The matrix cores pay off for FP32 (twice the vector rate), not for FP64.
  static constexpr bool kMma = sizeof(T) == 4;

  // How a kernel applies 8x8 ops: on the vector units (FP64), on the matrix
  // cores from per-pass tables (FP32), or on the matrix cores from
  // coefficients staged in LDS (FP32 kernels without room for the tables).
  enum { D3_VALU = 0, D3_TAB = 1, D3_STAGED = 2 };

  // Applies the pass's ops to the tile in sh.  pre: the ops' uniform
  // parameters (build_pre); aux: the 8x8 tables (D3_TAB) or the staged
  // coefficients from ops[0].moff on (D3_STAGED).
  template <int MODE>
  __device__ static void run(cplx<T>* sh, const TileOp* __restrict__ ops, int nops,
                             const cplx<T>* __restrict__ mats, const OpPre* pre, const void* aux) {
    const int64_t mbase = nops > 0 ? ops[0].moff : 0;
    int k3 = 0;
    for (int o = 0; o < nops; ++o) {
      const TileOp op = ops[o];
      const OpPre& q = pre[o];
      const int tid = (int)threadIdx.x;
      const cplx<T>* m = mats + op.moff;
      if (op.kind == TOP_DENSE2) dense2(sh, q, m, tid);
      else if (op.kind == TOP_DENSE1) dense1(sh, q, m, tid);
      else if (op.kind == TOP_DIAG2) diag2(sh, q, op.a, op.b, m, tid);
      else if (op.kind == TOP_PERM) {
        if (op.k == 1) perm<1>(sh, q, m, tid);
        else if (op.k == 2) perm<2>(sh, q, m, tid);
        else perm<3>(sh, q, m, tid);
      } else if (op.kind == TOP_DENSE3G) {
        dense3_gauss(sh, q, reinterpret_cast<const T*>(m), tid);
      } else {  // 8x8 (callers route passes with 4-qubit ops elsewhere)
        if constexpr (MODE == D3_VALU) dense3_valu(sh, q, m, tid);
        else if constexpr (MODE == D3_TAB) dense3_tab(sh, reinterpret_cast<const Tab*>(aux)[k3++], tid);
        else dense3_mma(sh, q, reinterpret_cast<const cplx<T>*>(aux) + (op.moff - mbase), tid);
      }
      __syncthreads();
    }
  }
};

// Copies the n coefficients of a pass into LDS (the caller synchronises).
template <typename T, int NT>
__device__ inline void stage_mats(cplx<T>* dst, const cplx<T>* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

// LDS coefficient slots of a fixed-size kernel: what remains of the LDS
// budget of one workgroup (wgs workgroups per CU) after the tile and the
// geometry tables, at most 8192, in whole 8x8 matrices.
constexpr int mat_slots(int tile_bytes, int other_bytes, int coef_bytes, int wgs) {
  const int left = 163840 / wgs - tile_bytes - other_bytes;
  const int n = left / coef_bytes;
  return (n > 8192 ? 8192 : n) & ~63;
}

}  // namespace tileops
}  // namespace juqcs
