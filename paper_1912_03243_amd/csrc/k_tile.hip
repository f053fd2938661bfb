// On-chip tile passes.  A workgroup gathers 2^b amplitudes -- 2^H chunks of
// 2^L contiguous amplitudes, the chunk bits being chosen physical qubits --
// into LDS, applies a program of gate ops whose qubits all lie in those b
// bits, and writes the tile back: one HBM read + write per pass however many
// gates the pass holds.  This is the single-GPU counterpart of the paper's
// reduction of data movement for gates on qubits that are not local
// (Section 2), with LDS in the role of node memory.
//
// Storage forms: C128 and C64 amplitudes, and the two-byte form (ENC2),
// which is decoded into FP32 on load and re-encoded with fresh per-block
// scales on store (Section 1, adaptive two-byte coding).
//
// The fixed-size kernels (tile size known at compile time, 512 or 1024 threads) run
// on a persistent grid and prefetch the next tile into registers while the
// current one is processed on chip; they stage the pass's coefficients in LDS
// (the 8x8 ops run on the matrix cores).  The generic kernels cover small
// states and passes with 4-qubit ops.
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "tile_ops.hpp"

namespace juqcs {

namespace {

using tileops::Fixed;
using tileops::lds;
using tileops::OpPre;
using tileops::mat_slots;
using tileops::stage_mats;
using tileops::Var;

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;       // generic kernels
constexpr int kFixedThreads = 512;  // pipelined kernels
constexpr float kTiny = 7.888609052210118e-31f;  // 2^-100: smaller block maxima code as zero

template <typename T>
struct TileCfg;
template <>
struct TileCfg<double> {
  static constexpr int kMaxBits = 13;  // 128 KiB of C128 amplitudes
};
template <>
struct TileCfg<float> {
  static constexpr int kMaxBits = 14;  // 128 KiB of C64 amplitudes
};

// Tile geometry copied to LDS once per workgroup (dynamic indexing of the
// kernel-argument struct would go through scratch); room for 2^HMAX chunks.
template <int HMAX>
struct GeomLdsT {
  int hb[kHbitsCap];
  uint64_t choff[1 << HMAX];
};
using GeomLds = GeomLdsT<kMaxGather>;

// The pipelined kernels keep every op's uniform parameters in LDS; passes
// with more ops go to the generic kernels (the planner splits them).
constexpr int kFixedOps = kPassOps;
constexpr int kEnc2Gather = 6;  // two-byte tiles: chunks of at least 2^7 amplitudes

// LDS room of the pipelined FP32 kernels for the tables of their 8x8 ops
// (512-thread kernels run two workgroups per CU).
template <typename T, int TB, int NT>
struct FixedTabs {
  using Tab = typename Fixed<T, TB, NT>::Tab;
  static constexpr int kCap =
      Fixed<T, TB, NT>::kMma
          ? (163840 / (NT == 512 ? 2 : 1) - ((int)sizeof(cplx<T>) << TB) - (int)sizeof(GeomLds) -
             kFixedOps * (int)sizeof(OpPre)) /
                (int)sizeof(Tab)
          : 0;
};
template <int TB>
struct Enc2Mats {
  static constexpr int kSlots = mat_slots((int)sizeof(cplx<float>) << TB,
                                          (int)sizeof(GeomLdsT<kEnc2Gather>) + (4 << TB) / 8 +
                                              kFixedOps * (int)sizeof(OpPre),
                                          (int)sizeof(cplx<float>), 2);
};

template <int NT, int HMAX>
__device__ inline void load_geom(const TileGeom& g, GeomLdsT<HMAX>& s) {
  if (threadIdx.x < kHbitsCap) s.hb[threadIdx.x] = (int)threadIdx.x < g.H ? g.hbits[threadIdx.x] : 0;
  __syncthreads();
  for (int c = threadIdx.x; c < (1 << g.H); c += NT) {
    uint64_t o = 0;
    for (int j = 0; j < g.H; ++j) o |= (uint64_t)((c >> j) & 1) << s.hb[j];
    s.choff[c] = o;
  }
  __syncthreads();
}

// Tiles [lo, hi) of this workgroup in a persistent grid of at most ntiles
// workgroups: a contiguous run, so that consecutive tiles of a CU touch the
// same memory pages and the CU keeps reusing its address translations.
__device__ inline void tile_run(uint64_t ntiles, uint64_t* lo, uint64_t* hi) {
  const uint64_t per = ntiles / gridDim.x, extra = ntiles % gridDim.x, b = blockIdx.x;
  *lo = b * per + (b < extra ? b : extra);
  *hi = *lo + per + (b < extra ? 1 : 0);
}

// Base index of tile tau: tau's bits fill the non-tile positions in order.
__device__ inline uint64_t tile_base(uint64_t tau, int L, int H, const int* hb) {
  uint64_t base = tau << L;
  for (int j = 0; j < H; ++j) base = insert_zero(base, hb[j]);
  return base;
}

// ------------------------------------------------- generic C128 / C64 -----
template <typename T, int MAXB>
__global__ __launch_bounds__(kThreads) void k_tile(cplx<T>* __restrict__ psi, TileGeom g,
                                                   const TileOp* __restrict__ ops, int nops,
                                                   const cplx<T>* __restrict__ mats) {
  __shared__ cplx<T> sh[1 << MAXB];
  __shared__ GeomLds gs;
  load_geom<kThreads>(g, gs);
  const int b = g.b, L = g.L, lmask = (1 << L) - 1;
  const int tile_amps = 1 << b;
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2* gp = reinterpret_cast<v2*>(psi);
  v2* sp = reinterpret_cast<v2*>(sh);
  for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
    const uint64_t base = tile_base(tau, L, g.H, gs.hb);
    for (int e0 = 0; e0 < tile_amps; e0 += kThreads * 8) {
      v2 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + k * kThreads + threadIdx.x;
        const int ec = e < tile_amps ? e : 0;
        v[k] = ld_stream(&gp[base + gs.choff[ec >> L] + (ec & lmask)]);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + k * kThreads + threadIdx.x;
        if (e < tile_amps) sp[lds<T>(e)] = v[k];
      }
    }
    __syncthreads();
    Var<T, kThreads>::run(sh, b, ops, nops, mats);
    // written back through the relabel swaps (see k_tile_fixed)
    const int lt = lds<T>(swap_local((int)threadIdx.x, g));
    for (int e = threadIdx.x; e < tile_amps; e += kThreads)
      st_stream(&gp[base + gs.choff[e >> L] + (e & lmask)],
                sp[lt ^ lds<T>(swap_local(e - (int)threadIdx.x, g))]);
    __syncthreads();
  }
}

// ----------------------------------------------- pipelined C128 / C64 -----
// 512-thread variants are bounded to 128 VGPRs so that two workgroups share
// a CU (one computes while the other's memory traffic is in flight).
template <typename T, int TB, int NT>
__global__ __launch_bounds__(NT, NT == 512 ? 4 : 1) void k_tile_fixed(cplx<T>* __restrict__ psi, TileGeom g,
                                                   const TileOp* __restrict__ ops, int nops,
                                                   const cplx<T>* __restrict__ mats) {
  constexpr int NA = 1 << TB, PER = NA / NT;
  __shared__ cplx<T> sh[NA];
  __shared__ GeomLds gs;
  __shared__ OpPre pre[kFixedOps];
  using F = Fixed<T, TB, NT>;
  constexpr int kCap = FixedTabs<T, TB, NT>::kCap;
  __shared__ typename F::Tab tabs[kCap > 0 ? kCap : 1];
  // relabel swaps for the write-back: the pairs (a | c << 8) and, per k,
  // the uniform part lds(swap(k NT)) of the LDS offsets
  __shared__ int swp[kSwapCap];
  __shared__ int swk[PER];
  if (threadIdx.x < PER) swk[threadIdx.x] = lds<T>(swap_local((int)threadIdx.x * NT, g));
  if (threadIdx.x < kSwapCap) {
    const int i = threadIdx.x;
    swp[i] = i < g.nswap ? (int)g.swap_a[i] | ((int)g.swap_b[i] << 8) : 0;
  }
  F::build_pre(pre, ops, nops);
  if constexpr (kCap > 0) F::build_tabs(tabs, ops, nops, mats);
  load_geom<NT>(g, gs);  // synchronises
  const int H = g.H, L = g.L, lmask = (1 << L) - 1, nswap = g.nswap;
  const uint64_t ntiles = uint64_t(1) << (g.n - TB);
  // a native 2-vector keeps the prefetch buffer in registers (an array of
  // the cplx struct is demoted to scratch for FP64)
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2* gp = reinterpret_cast<v2*>(psi);
  v2* sp = reinterpret_cast<v2*>(sh);
  v2 v[PER];
  uint64_t tau, tau_end;
  tile_run(ntiles, &tau, &tau_end);
  // Loads of tile tau + 1 go out before the ops on tile tau and land in v;
  // v is copied into LDS right after tile tau's stores have been issued, so
  // those stores drain while the next tile is worked on.  (Copying at the
  // top of the loop instead makes the compiler merge the first iteration's
  // counters with the later ones and wait for every store in flight.)
  // The thread's addresses are recomputed every tile from an opaque tid:
  // hoisted out of the loop they would stay live across the ops and spill,
  // and a spill reload also waits for every store in flight.
  auto load = [&](uint64_t t, int tid) {
    const uint64_t nb = tile_base(t, L, H, gs.hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * NT + tid;
      v[k] = ld_stream(&gp[nb + gs.choff[e >> L] + (e & lmask)]);
    }
  };
  auto fill = [&](int tid) {
#pragma unroll
    for (int k = 0; k < PER; ++k) sp[lds<T>(k * NT + tid)] = v[k];
  };
  if (tau < tau_end) {
    int tid = threadIdx.x;
    load(tau, tid);
    fill(tid);
    __syncthreads();
    // after the last tile the current one is read again (in bounds, unused)
    load(tau + 1 < tau_end ? tau + 1 : tau, tid);
  }
  for (; tau < tau_end; ++tau) {
    if constexpr (kCap > 0) F::template run<F::D3_TAB>(sh, ops, nops, mats, pre, tabs);
    else F::template run<F::D3_VALU>(sh, ops, nops, mats, pre, nullptr);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint64_t base = tile_base(tau, L, H, gs.hb);
    // The tile goes back to HBM through the pass's relabel swaps: destination
    // local index e takes LDS element swap(e).  swap and lds are both linear
    // over bit-XOR, so swap(k NT + t) splits into a per-thread part and the
    // uniform per-k part swk[k], joined by one XOR (no swaps: the identity).
    int t = tid;
    for (int i = 0; i < nswap; ++i) {
      const int pr = swp[i], a = pr & 255, c = pr >> 8;
      const int x = ((t >> a) ^ (t >> c)) & 1;
      t ^= (x << a) | (x << c);
    }
    const int lt = lds<T>(t);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * NT + tid;
      st_stream(&gp[base + gs.choff[e >> L] + (e & lmask)], sp[lt ^ swk[k]]);
    }
    __syncthreads();
    if (tau + 1 < tau_end) {
      fill(tid);
      __syncthreads();
      load(tau + 2 < tau_end ? tau + 2 : tau + 1, tid);
    }
  }
}

// --------------------------------------------------------------- ENC2 -----
// Codes are int8 (re, im) pairs; a thread moves 8 amplitudes (16 bytes of
// codes) at a time, which always lie in one scale block (block_bits >= 3).
__device__ inline void decode8(int4 raw, float d, cplx<float>* sh, int e) {
  const int w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int8_t c0 = (int8_t)(w[j] & 0xff), c1 = (int8_t)((w[j] >> 8) & 0xff);
    const int8_t c2 = (int8_t)((w[j] >> 16) & 0xff), c3 = (int8_t)((w[j] >> 24) & 0xff);
    sh[lds<float>(e + 2 * j)] = {(float)c0 * d, (float)c1 * d};
    sh[lds<float>(e + 2 * j + 1)] = {(float)c2 * d, (float)c3 * d};
  }
}

// Relabel swaps staged in LDS as pairs a | c << 8 (see k_tile_fixed).
__device__ inline int swap_staged(int e, const int* swp, int nswap) {
  for (int i = 0; i < nswap; ++i) {
    const int pr = swp[i], a = pr & 255, c = pr >> 8;
    const int x = ((e >> a) ^ (e >> c)) & 1;
    e ^= (x << a) | (x << c);
  }
  return e;
}

// The 8 amplitudes of destination group e (e % 8 == 0) sit at LDS slots
// lds(e + j) without relabeling, at ls ^ lsj[j] with it (ls = lds(swap(e)),
// lsj[j] = lds(swap(j)): swap and lds are linear over bit-XOR).
template <bool SW>
__device__ inline int enc_slot(int e, int ls, const int* lsj, int j) {
  return SW ? ls ^ lsj[j] : lds<float>(e + j);
}

template <bool SW>
__device__ inline int4 encode8(const cplx<float>* sh, int e, int ls, const int* lsj, float r) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cplx<float> v = sh[enc_slot<SW>(e, ls, lsj, j)];
    const float qr = fminf(fmaxf(rintf(v.re * r), -127.0f), 127.0f);
    const float qi = fminf(fmaxf(rintf(v.im * r), -127.0f), 127.0f);
    const uint32_t pr = ((uint32_t)(int)qr) & 0xffu, pi = ((uint32_t)(int)qi) & 0xffu;
    w[j >> 1] |= (pr | (pi << 8)) << (16 * (j & 1));
  }
  return make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
}

template <bool SW>
__device__ inline float max8(const cplx<float>* sh, int e, int ls, const int* lsj) {
  float mx = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cplx<float> v = sh[enc_slot<SW>(e, ls, lsj, j)];
    mx = fmaxf(mx, fmaxf(fabsf(v.re), fabsf(v.im)));
  }
  return mx;
}

// Re-encode the tile: per-block maxima through LDS atomics (non-negative
// floats order like their bit patterns), then codes and scales.  With
// relabel swaps (SW), destination amplitude d is LDS element swap(d), and
// the blocks are those of the destination order.
template <int NT, bool SW>
__device__ inline void store_enc2_t(const cplx<float>* sh, uint32_t* bmax, int tile_amps, int B,
                                    int L, int lmask, uint64_t base, const uint64_t* choff,
                                    int8_t* codes, float* scales, const int* swp, int nswap,
                                    const int* lsj) {
  const int ngroups = tile_amps >> 3;
  // Consecutive lanes hold consecutive groups of 8 amplitudes: when whole
  // waves take part, the lanes of a block reduce its maximum by shuffles
  // first, and one lane per block and wave does the LDS atomic (instead of
  // every lane hitting the block's one address).
  const int G = 1 << (B - 3);                    // groups per block
  const int span = G < 64 ? G : 64;              // lanes that reduce together
  const bool whole = (ngroups & 63) == 0;        // every wave fully active
  for (int gq = threadIdx.x; gq < ngroups; gq += NT) {
    const int e = gq << 3;
    const int ls = SW ? lds<float>(swap_staged(e, swp, nswap)) : 0;
    uint32_t mx = __float_as_uint(max8<SW>(sh, e, ls, lsj));
    if (whole) {
      for (int d = 1; d < span; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)mx, d, 64);
        mx = o > mx ? o : mx;
      }
      if ((threadIdx.x & (span - 1)) == 0) atomicMax(&bmax[e >> B], mx);
    } else {
      atomicMax(&bmax[e >> B], mx);
    }
  }
  __syncthreads();
  for (int gq = threadIdx.x; gq < ngroups; gq += NT) {
    const int e = gq << 3;
    const int ls = SW ? lds<float>(swap_staged(e, swp, nswap)) : 0;
    const uint64_t gi = base + choff[e >> L] + (e & lmask);
    const float s = __uint_as_float(bmax[e >> B]);
    const bool zero = !(s >= kTiny);
    const int4 w = zero ? make_int4(0, 0, 0, 0) : encode8<SW>(sh, e, ls, lsj, 127.0f / s);
    st_stream(reinterpret_cast<v4i*>(codes + 2 * gi), v4i{w.x, w.y, w.z, w.w});
    if ((e & ((1 << B) - 1)) == 0) st_stream(&scales[gi >> B], zero ? 0.0f : s);
  }
}

template <int NT>
__device__ inline void store_enc2(const cplx<float>* sh, uint32_t* bmax, int tile_amps, int B,
                                  int L, int lmask, uint64_t base, const uint64_t* choff,
                                  int8_t* codes, float* scales, const int* swp, int nswap,
                                  const int* lsj) {
  if (nswap > 0)
    store_enc2_t<NT, true>(sh, bmax, tile_amps, B, L, lmask, base, choff, codes, scales, swp, nswap, lsj);
  else
    store_enc2_t<NT, false>(sh, bmax, tile_amps, B, L, lmask, base, choff, codes, scales, swp, nswap, lsj);
}

// Stages a pass's relabel swaps in LDS for the two-byte store: the pairs,
// and lds(swap(j)) for the 8 amplitudes j of a group (the caller
// synchronises).
template <int NT>
__device__ inline void stage_swaps(const TileGeom& g, int* swp, int* lsj) {
  if (threadIdx.x < kSwapCap) {
    const int i = threadIdx.x;
    swp[i] = i < g.nswap ? (int)g.swap_a[i] | ((int)g.swap_b[i] << 8) : 0;
  }
  if (threadIdx.x >= 32 && threadIdx.x < 40) {
    const int j = threadIdx.x - 32;
    lsj[j] = lds<float>(swap_local(j, g));
  }
}

__global__ __launch_bounds__(kThreads) void k_tile_enc2(int8_t* __restrict__ codes,
                                                        float* __restrict__ scales, TileGeom g,
                                                        const TileOp* __restrict__ ops, int nops,
                                                        const cplx<float>* __restrict__ mats) {
  constexpr int MAXB = TileCfg<float>::kMaxBits;
  __shared__ cplx<float> sh[1 << MAXB];
  __shared__ GeomLds gs;
  __shared__ uint32_t bmax[1 << (MAXB - 3)];
  __shared__ int swp[kSwapCap], lsj[8];
  stage_swaps<kThreads>(g, swp, lsj);
  load_geom<kThreads>(g, gs);  // synchronises
  const int b = g.b, B = g.block_bits, L = g.L, lmask = (1 << L) - 1;
  const int tile_amps = 1 << b, ngroups = tile_amps >> 3, nblk = tile_amps >> B;
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
    const uint64_t base = tile_base(tau, L, g.H, gs.hb);
    for (int q = threadIdx.x; q < nblk; q += kThreads) bmax[q] = 0u;
    for (int gq = threadIdx.x; gq < ngroups; gq += kThreads) {
      const int e = gq << 3;
      const uint64_t gi = base + gs.choff[e >> L] + (e & lmask);
      const v4i w = ld_stream(reinterpret_cast<const v4i*>(codes + 2 * gi));
      decode8(make_int4(w.x, w.y, w.z, w.w), ld_stream(&scales[gi >> B]) / 127.0f, sh, e);
    }
    __syncthreads();
    Var<float, kThreads>::run(sh, b, ops, nops, mats);
    store_enc2<kThreads>(sh, bmax, tile_amps, B, L, lmask, base, gs.choff, codes, scales, swp, g.nswap, lsj);
    __syncthreads();
  }
}

// Pipelined two-byte kernel: codes and scales of the next tile are prefetched
// into registers (16 bytes of codes + one scale per 8 amplitudes).
template <int TB>
__global__ __launch_bounds__(kFixedThreads, 4) void k_tile_enc2_fixed(
    int8_t* __restrict__ codes, float* __restrict__ scales, TileGeom g,
    const TileOp* __restrict__ ops, int nops, const cplx<float>* __restrict__ mats) {
  constexpr int NA = 1 << TB, NG = NA / 8, PER = (NG + kFixedThreads - 1) / kFixedThreads;
  __shared__ cplx<float> sh[NA];
  __shared__ GeomLdsT<kEnc2Gather> gs;
  __shared__ uint32_t bmax[NA / 8];
  __shared__ OpPre pre[kFixedOps];
  __shared__ cplx<float> smat[Enc2Mats<TB>::kSlots];
  __shared__ int swp[kSwapCap], lsj[8];
  using F = Fixed<float, TB, kFixedThreads>;
  stage_swaps<kFixedThreads>(g, swp, lsj);
  stage_mats<float, kFixedThreads>(smat, mats + (nops > 0 ? ops[0].moff : 0), g.mat_count);
  F::build_pre(pre, ops, nops);
  load_geom<kFixedThreads>(g, gs);  // synchronises
  const int H = g.H, L = g.L, B = g.block_bits, lmask = (1 << L) - 1, nswap = g.nswap;
  const int nblk = NA >> B;
  const uint64_t ntiles = uint64_t(1) << (g.n - TB);
  int4 raw[PER];
  float sc[PER];
  auto fetch = [&](uint64_t t) {
    const uint64_t base = tile_base(t, L, H, gs.hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int gq = k * kFixedThreads + threadIdx.x;
      const int e = (NG % kFixedThreads == 0 || gq < NG) ? gq << 3 : 0;
      const uint64_t gi = base + gs.choff[e >> L] + (e & lmask);
      const v4i w = ld_stream(reinterpret_cast<const v4i*>(codes + 2 * gi));
      raw[k] = make_int4(w.x, w.y, w.z, w.w);
      sc[k] = ld_stream(&scales[gi >> B]);
    }
  };
  uint64_t tau, tau_end;
  tile_run(ntiles, &tau, &tau_end);
  fetch(tau);
  for (; tau < tau_end; ++tau) {
    for (int q = threadIdx.x; q < nblk; q += kFixedThreads) bmax[q] = 0u;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int gq = k * kFixedThreads + threadIdx.x;
      if (NG % kFixedThreads == 0 || gq < NG) decode8(raw[k], sc[k] / 127.0f, sh, gq << 3);
    }
    __syncthreads();
    fetch(tau + 1 < tau_end ? tau + 1 : tau);
    F::template run<F::D3_STAGED>(sh, ops, nops, mats, pre, smat);
    store_enc2<kFixedThreads>(sh, bmax, NA, B, L, lmask, tile_base(tau, L, H, gs.hb), gs.choff,
                              codes, scales, swp, nswap, lsj);
    __syncthreads();
  }
}

// ------------------------------------------------- expectation values ----
// <sigma^x_j>, <sigma^y_j>, <sigma^z_j> for the tile bits jlo..b-1 of one
// tile geometry: sums over the amplitude pairs that differ in bit j, of
// (2 Re conj(a0) a1, 2 Im conj(a0) a1, |a0|^2 - |a1|^2), in FP64.  Both
// members of every such pair lie in one tile, so one read pass covers b bits
// (Section 3: the expectation values of all qubits).  The nb = b - jlo bits
// form ng = ceil(nb / 3) groups of up to three consecutive bits; a wave
// reads items of 2^gk amplitudes that span its group's gk bits (one LDS
// read serves all pairs of the group: 12 pairs for three bits) and reduces
// a share of the items (16 / ng shares, rounded down).
// Wave w takes group w % ng, share w / ng; every sum runs over a fixed set
// of pairs in a fixed order.  The next tile is prefetched into registers
// while one is reduced.
constexpr int kExpectThreads = 1024;
constexpr int kExpectBits = 13;
constexpr int kExpectWaves = kExpectThreads / 64;
constexpr int kExpectGroup = 3;  // bits per wave group

__device__ __host__ inline int expect_groups(int nb) { return (nb + kExpectGroup - 1) / kExpectGroup; }
__device__ __host__ inline int expect_shares(int ng) { return kExpectWaves / ng; }

// Pair sums of one item (2^GK amplitudes at LDS byte offsets u ^ row[r]).
template <typename T, int GK>
__device__ inline void expect_item(const char* base, int u, const int* row, double* sx, double* sy,
                                   double* sz) {
  cplx<T> a[1 << GK];
#pragma unroll
  for (int r = 0; r < (1 << GK); ++r) a[r] = *reinterpret_cast<const cplx<T>*>(base + (u ^ row[r]));
#pragma unroll
  for (int jj = 0; jj < GK; ++jj)
#pragma unroll
    for (int r = 0; r < (1 << GK); ++r) {
      if ((r >> jj) & 1) continue;
      const double ar = a[r].re, ai = a[r].im, br = a[r | (1 << jj)].re, bi = a[r | (1 << jj)].im;
      sx[jj] = fma(ar, br, fma(ai, bi, sx[jj]));
      sy[jj] = fma(ar, bi, fma(-ai, br, sy[jj]));
      sz[jj] += fma(ar, ar, ai * ai) - fma(br, br, bi * bi);
    }
}

template <typename S>  // storage: double (C128), float (C64), int8_t (ENC2)
__global__ __launch_bounds__(kExpectThreads) void k_expect(const void* __restrict__ amps,
                                                           const float* __restrict__ scales,
                                                           TileGeom g, int jlo,
                                                           double* __restrict__ partials) {
  using T = typename std::conditional<sizeof(S) == 8, double, float>::type;
  constexpr int NA = 1 << kExpectBits;
  constexpr int CB = (int)sizeof(cplx<T>);
  __shared__ cplx<T> sh[NA];
  __shared__ GeomLds gs;
  load_geom<kExpectThreads>(g, gs);
  const int b = g.b, L = g.L, lmask = (1 << L) - 1, tile_amps = 1 << b;
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = b - jlo, ng = expect_groups(nb), shares = expect_shares(ng);
  const int grp = wave % ng, share = wave / ng;
  const bool active = share < shares;
  const int j0 = jlo + kExpectGroup * grp;
  const int gk = j0 + kExpectGroup <= b ? kExpectGroup : b - j0;  // bits of this wave's group
  // item i = (it * shares + share) * 64 + lane: its base element spreads i
  // over the positions around the group's bits j0..j0+gk-1 (a contiguous
  // run, so the spread is one shift); byte offsets in LDS
  const int nitems = tile_amps >> gk;
  int row[1 << kExpectGroup];
#pragma unroll
  for (int r = 0; r < (1 << kExpectGroup); ++r) row[r] = tileops::lds<T>((r & ((1 << gk) - 1)) << j0) * CB;
  auto item_off = [&](int i) {
    const int e = ((i >> j0) << (j0 + gk)) | (i & ((1 << j0) - 1));
    return tileops::lds<T>(e) * CB;
  };
  const char* base = reinterpret_cast<const char*>(sh);
  // register prefetch: whole amplitudes (C128/C64) or 16-byte code groups
  constexpr int PER = sizeof(S) == 1 ? NA / 8 / kExpectThreads : NA / kExpectThreads;
  typedef T v2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<sizeof(S) == 1, v4i, v2>::type Item;
  Item v[PER];
  float sc[PER];
  // the thread's addresses are recomputed every tile from an opaque tid:
  // hoisted out of the loop they would stay live and spill, and a spill
  // reload waits for the prefetch loads in flight
  auto fetch = [&](uint64_t tau, int tid) {
    const uint64_t tb = tile_base(tau, L, g.H, gs.hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int q = k * kExpectThreads + tid;
      if constexpr (sizeof(S) == 1) {
        const int e = (q << 3) < tile_amps ? q << 3 : 0;
        const uint64_t gi = tb + gs.choff[e >> L] + (e & lmask);
        v[k] = ld_stream(reinterpret_cast<const v4i*>((const int8_t*)amps + 2 * gi));
        sc[k] = ld_stream(&scales[gi >> g.block_bits]);
      } else {
        const int e = q < tile_amps ? q : 0;
        v[k] = ld_stream(&reinterpret_cast<const v2*>(amps)[tb + gs.choff[e >> L] + (e & lmask)]);
      }
    }
  };
  double sx[kExpectGroup] = {0.0, 0.0, 0.0}, sy[kExpectGroup] = {0.0, 0.0, 0.0},
         sz[kExpectGroup] = {0.0, 0.0, 0.0};
  uint64_t tau, tau_end;
  tile_run(ntiles, &tau, &tau_end);
  fetch(tau, (int)threadIdx.x);
  for (; tau < tau_end; ++tau) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int q = k * kExpectThreads + tid;
      if constexpr (sizeof(S) == 1) {
        if ((q << 3) < tile_amps) decode8(make_int4(v[k].x, v[k].y, v[k].z, v[k].w), sc[k] / 127.0f, sh, q << 3);
      } else {
        if (q < tile_amps) reinterpret_cast<v2*>(sh)[lds<T>(q)] = v[k];
      }
    }
    __syncthreads();
    fetch(tau + 1 < tau_end ? tau + 1 : tau, tid);
    if (active) {
      for (int p0 = share * 64; p0 < nitems; p0 += 64 * shares) {
        const int i = p0 + lane;
        if (i < nitems) {
          const int u = item_off(i);
          if (gk == 3) expect_item<T, 3>(base, u, row, sx, sy, sz);
          else if (gk == 2) expect_item<T, 2>(base, u, row, sx, sy, sz);
          else expect_item<T, 1>(base, u, row, sx, sy, sz);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int jj = 0; jj < kExpectGroup; ++jj)
    for (int off = 32; off > 0; off >>= 1) {
      sx[jj] += __shfl_xor(sx[jj], off, 64);
      sy[jj] += __shfl_xor(sy[jj], off, 64);
      sz[jj] += __shfl_xor(sz[jj], off, 64);
    }
  if (lane == 0) {
#pragma unroll
    for (int jj = 0; jj < kExpectGroup; ++jj) {
      const bool used = active && jj < gk;
      double* o = partials + 3 * (((size_t)wave * kExpectGroup + jj) * gridDim.x + blockIdx.x);
      o[0] = used ? 2.0 * sx[jj] : 0.0;
      o[1] = used ? 2.0 * sy[jj] : 0.0;
      o[2] = used ? sz[jj] : 0.0;
    }
  }
}

// out3[3 k + c]: bit jlo + k, summed over the waves of its group (in wave
// order) and over blocks, in that order.
__global__ __launch_bounds__(64) void k_expect_final(const double* __restrict__ partials, int nblk,
                                                     int nbits, double* __restrict__ out3) {
  const int k = threadIdx.x / 3, c = threadIdx.x % 3;
  if (k >= nbits) return;
  const int ng = expect_groups(nbits), shares = expect_shares(ng);
  const int grp = k / kExpectGroup, jj = k % kExpectGroup;
  double s = 0.0;
  for (int w = grp; w < shares * ng; w += ng)
    for (int i = 0; i < nblk; ++i) s += partials[3 * (((size_t)w * kExpectGroup + jj) * nblk + i) + c];
  out3[3 * k + c] = s;
}

// Workgroups of a kernel that fit on the device at once (cached per kernel).
uint64_t resident_blocks(const void* kern, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, uint64_t> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kern);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0) != hipSuccess || per < 1)
    per = 1;
  const uint64_t r = (uint64_t)cus * (uint64_t)per;
  cache[kern] = r;
  return r;
}

inline unsigned tile_grid(uint64_t ntiles) {
  return (unsigned)(ntiles < (1u << 20) ? ntiles : (1u << 20));
}

}  // namespace

int tile_max_bits(juqcs_dtype dt) {
  return dt == JUQCS_C128 ? TileCfg<double>::kMaxBits : TileCfg<float>::kMaxBits;
}

bool tile_pipelined(juqcs_dtype dt, const TileGeom& g, int nops) {
  const int cap = tile_mat_cap(dt, g.b), mcap = tile_mma_cap(dt, g.b);  // 0: no limit
  const bool sized = dt == JUQCS_C128   ? (g.b >= 11 && g.b <= 13)
                     : dt == JUQCS_C64 ? (g.b >= 11 && g.b <= 14)
                                       : (g.b == 12 || g.b == 13);
  return sized && g.maxk <= 3 && nops <= kFixedOps && (cap == 0 || g.mat_count <= cap) &&
         (mcap == 0 || g.mma_count <= mcap) && (dt != JUQCS_ENC2 || g.H <= kEnc2Gather);
}

int tile_mma_cap(juqcs_dtype dt, int b) {
  if (dt == JUQCS_C64) {
    if (b == 14) return FixedTabs<float, 14, 1024>::kCap;
    if (b == 13) return FixedTabs<float, 13, 1024>::kCap;
    if (b == 12) return FixedTabs<float, 12, 512>::kCap;
    if (b == 11) return FixedTabs<float, 11, 512>::kCap;
  }
  return 0;
}

int tile_mat_cap(juqcs_dtype dt, int b) {
  if (dt == JUQCS_ENC2) {
    if (b == 13) return Enc2Mats<13>::kSlots;
    if (b == 12) return Enc2Mats<12>::kSlots;
  }
  return 0;
}

hipError_t launch_tile(juqcs_dtype dt, void* amps, void* scales, const TileGeom& g,
                       const TileOp* d_ops, int nops, const void* d_mats, hipStream_t s) {
  const uint64_t ntiles = uint64_t(1) << (g.n - g.b);
  const dim3 grid(tile_grid(ntiles)), block(kThreads), fblock(kFixedThreads);
  // persistent grid for the pipelined kernels: every resident workgroup slot
  auto pgrid = [&](const void* kern, int threads) {
    const uint64_t slots = resident_blocks(kern, threads);
    return dim3((unsigned)(ntiles < slots ? ntiles : slots));
  };
#define JUQCS_FIXED(T, TB, NT)                                                             \
  hipLaunchKernelGGL((k_tile_fixed<T, TB, NT>), pgrid((const void*)k_tile_fixed<T, TB, NT>, NT), \
                     dim3(NT), 0, s, (cplx<T>*)amps, g, d_ops, nops, (const cplx<T>*)d_mats)
  // the pipelined kernels run ops of up to 3 qubits, with the coefficients in LDS
  const bool fixed_ok = tile_pipelined(dt, g, nops);
  if (g.nswap < 0 || g.nswap > kSwapCap) return hipErrorInvalidValue;
  for (int i = 0; i < g.nswap; ++i)
    if (g.swap_a[i] < 0 || g.swap_a[i] >= g.b || g.swap_b[i] < 0 || g.swap_b[i] >= g.b) return hipErrorInvalidValue;
  if (dt == JUQCS_C128) {
    auto* p = (cplx<double>*)amps;
    auto* m = (const cplx<double>*)d_mats;
    if (fixed_ok && g.b == 13) JUQCS_FIXED(double, 13, 1024);
    else if (fixed_ok && g.b == 12) JUQCS_FIXED(double, 12, 512);
    else if (fixed_ok && g.b == 11) JUQCS_FIXED(double, 11, 512);
    else if (g.b <= 12) hipLaunchKernelGGL((k_tile<double, 12>), grid, block, 0, s, p, g, d_ops, nops, m);
    else hipLaunchKernelGGL((k_tile<double, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
  } else if (dt == JUQCS_C64) {
    auto* p = (cplx<float>*)amps;
    auto* m = (const cplx<float>*)d_mats;
    if (fixed_ok && g.b == 14) JUQCS_FIXED(float, 14, 1024);
    else if (fixed_ok && g.b == 13) JUQCS_FIXED(float, 13, 1024);
    else if (fixed_ok && g.b == 12) JUQCS_FIXED(float, 12, 512);
    else if (fixed_ok && g.b == 11) JUQCS_FIXED(float, 11, 512);
    else if (g.b <= 13) hipLaunchKernelGGL((k_tile<float, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
    else hipLaunchKernelGGL((k_tile<float, 14>), grid, block, 0, s, p, g, d_ops, nops, m);
  } else {
    auto* c = (int8_t*)amps;
    auto* sc = (float*)scales;
    auto* m = (const cplx<float>*)d_mats;
    if (fixed_ok && g.b == 13)
      hipLaunchKernelGGL((k_tile_enc2_fixed<13>), pgrid((const void*)k_tile_enc2_fixed<13>, kFixedThreads), fblock,
                         0, s, c, sc, g, d_ops, nops, m);
    else if (fixed_ok && g.b == 12)
      hipLaunchKernelGGL((k_tile_enc2_fixed<12>), pgrid((const void*)k_tile_enc2_fixed<12>, kFixedThreads), fblock,
                         0, s, c, sc, g, d_ops, nops, m);
    else
      hipLaunchKernelGGL(k_tile_enc2, grid, block, 0, s, c, sc, g, d_ops, nops, m);
  }
#undef JUQCS_FIXED
  return hipGetLastError();
}

int expect_max_bits() { return kExpectBits; }

size_t expect_partials_bytes() {
  return sizeof(double) * 3 * kExpectWaves * kExpectGroup *
         (size_t)resident_blocks((const void*)k_expect<double>, kExpectThreads);
}

hipError_t launch_expect(juqcs_dtype dt, const void* amps, const void* scales, const TileGeom& g,
                         int jlo, double* partials, double* out3, hipStream_t s) {
  const int nbits = g.b - jlo;
  if (g.b > kExpectBits || nbits < 1 || nbits > kExpectWaves) return hipErrorInvalidValue;
  const uint64_t ntiles = uint64_t(1) << (g.n - g.b);
  const uint64_t slots = resident_blocks((const void*)k_expect<double>, kExpectThreads);
  const unsigned grid = (unsigned)(ntiles < slots ? ntiles : slots);
  const dim3 block(kExpectThreads);
  if (dt == JUQCS_C128)
    hipLaunchKernelGGL(k_expect<double>, dim3(grid), block, 0, s, amps, (const float*)scales, g, jlo, partials);
  else if (dt == JUQCS_C64)
    hipLaunchKernelGGL(k_expect<float>, dim3(grid), block, 0, s, amps, (const float*)scales, g, jlo, partials);
  else
    hipLaunchKernelGGL(k_expect<int8_t>, dim3(grid), block, 0, s, amps, (const float*)scales, g, jlo, partials);
  hipLaunchKernelGGL(k_expect_final, dim3(1), dim3(64), 0, s, partials, (int)grid, nbits, out3);
  return hipGetLastError();
}

}  // namespace juqcs
