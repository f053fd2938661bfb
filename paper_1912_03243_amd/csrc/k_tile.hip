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
// current one is processed on chip; the generic kernels cover small states.
#include <mutex>
#include <unordered_map>

#include "tile_ops.hpp"

namespace juqcs {

namespace {

using tileops::Fixed;
using tileops::lds;
using tileops::Var;

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
// kernel-argument struct would go through scratch).
struct GeomLds {
  int hb[kHbitsCap];
  uint64_t choff[1 << kMaxGather];
};

template <int NT>
__device__ inline void load_geom(const TileGeom& g, GeomLds& s) {
  if (threadIdx.x < kHbitsCap) s.hb[threadIdx.x] = (int)threadIdx.x < g.H ? g.hbits[threadIdx.x] : 0;
  __syncthreads();
  for (int c = threadIdx.x; c < (1 << g.H); c += NT) {
    uint64_t o = 0;
    for (int j = 0; j < g.H; ++j) o |= (uint64_t)((c >> j) & 1) << s.hb[j];
    s.choff[c] = o;
  }
  __syncthreads();
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
        v[k] = gp[base + gs.choff[ec >> L] + (ec & lmask)];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + k * kThreads + threadIdx.x;
        if (e < tile_amps) sp[lds<T>(e)] = v[k];
      }
    }
    __syncthreads();
    Var<T, kThreads>::run(sh, b, ops, nops, mats);
    for (int e = threadIdx.x; e < tile_amps; e += kThreads)
      gp[base + gs.choff[e >> L] + (e & lmask)] = sp[lds<T>(e)];
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
  load_geom<NT>(g, gs);
  const int H = g.H, L = g.L, lmask = (1 << L) - 1;
  const uint64_t ntiles = uint64_t(1) << (g.n - TB);
  // a native 2-vector keeps the prefetch buffer in registers (an array of
  // the cplx struct is demoted to scratch for FP64)
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2* gp = reinterpret_cast<v2*>(psi);
  v2* sp = reinterpret_cast<v2*>(sh);
  v2 v[PER];
  uint64_t tau = blockIdx.x;  // the grid never exceeds ntiles
  {
    const uint64_t base = tile_base(tau, L, H, gs.hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * NT + threadIdx.x;
      v[k] = gp[base + gs.choff[e >> L] + (e & lmask)];
    }
  }
  for (; tau < ntiles; tau += gridDim.x) {
#pragma unroll
    for (int k = 0; k < PER; ++k) sp[lds<T>(k * NT + threadIdx.x)] = v[k];
    __syncthreads();
    // prefetch the next tile while this one is on chip; after the last tile
    // the current one is read again (in bounds, values unused)
    const uint64_t nxt = tau + gridDim.x;
    const uint64_t pf = nxt < ntiles ? nxt : tau;
    {
      const uint64_t nb = tile_base(pf, L, H, gs.hb);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = k * NT + threadIdx.x;
        v[k] = gp[nb + gs.choff[e >> L] + (e & lmask)];
      }
    }
    Fixed<T, TB, NT>::run(sh, ops, nops, mats);
    const uint64_t base = tile_base(tau, L, H, gs.hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * NT + threadIdx.x;
      gp[base + gs.choff[e >> L] + (e & lmask)] = sp[lds<T>(e)];
    }
    __syncthreads();
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

__device__ inline int4 encode8(const cplx<float>* sh, int e, float r) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cplx<float> v = sh[lds<float>(e + j)];
    const float qr = fminf(fmaxf(rintf(v.re * r), -127.0f), 127.0f);
    const float qi = fminf(fmaxf(rintf(v.im * r), -127.0f), 127.0f);
    const uint32_t pr = ((uint32_t)(int)qr) & 0xffu, pi = ((uint32_t)(int)qi) & 0xffu;
    w[j >> 1] |= (pr | (pi << 8)) << (16 * (j & 1));
  }
  return make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
}

__device__ inline float max8(const cplx<float>* sh, int e) {
  float mx = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cplx<float> v = sh[lds<float>(e + j)];
    mx = fmaxf(mx, fmaxf(fabsf(v.re), fabsf(v.im)));
  }
  return mx;
}

// Re-encode the tile: per-block maxima through LDS atomics (non-negative
// floats order like their bit patterns), then codes and scales.
template <int NT>
__device__ inline void store_enc2(const cplx<float>* sh, uint32_t* bmax, int tile_amps, int B,
                                  int L, int lmask, uint64_t base, const uint64_t* choff,
                                  int8_t* codes, float* scales) {
  const int ngroups = tile_amps >> 3;
  for (int gq = threadIdx.x; gq < ngroups; gq += NT) {
    const int e = gq << 3;
    atomicMax(&bmax[e >> B], __float_as_uint(max8(sh, e)));
  }
  __syncthreads();
  for (int gq = threadIdx.x; gq < ngroups; gq += NT) {
    const int e = gq << 3;
    const uint64_t gi = base + choff[e >> L] + (e & lmask);
    const float s = __uint_as_float(bmax[e >> B]);
    const bool zero = !(s >= kTiny);
    *reinterpret_cast<int4*>(codes + 2 * gi) = zero ? make_int4(0, 0, 0, 0) : encode8(sh, e, 127.0f / s);
    if ((e & ((1 << B) - 1)) == 0) scales[gi >> B] = zero ? 0.0f : s;
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
  load_geom<kThreads>(g, gs);
  const int b = g.b, B = g.block_bits, L = g.L, lmask = (1 << L) - 1;
  const int tile_amps = 1 << b, ngroups = tile_amps >> 3, nblk = tile_amps >> B;
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
    const uint64_t base = tile_base(tau, L, g.H, gs.hb);
    for (int q = threadIdx.x; q < nblk; q += kThreads) bmax[q] = 0u;
    for (int gq = threadIdx.x; gq < ngroups; gq += kThreads) {
      const int e = gq << 3;
      const uint64_t gi = base + gs.choff[e >> L] + (e & lmask);
      decode8(*reinterpret_cast<const int4*>(codes + 2 * gi), scales[gi >> B] / 127.0f, sh, e);
    }
    __syncthreads();
    Var<float, kThreads>::run(sh, b, ops, nops, mats);
    store_enc2<kThreads>(sh, bmax, tile_amps, B, L, lmask, base, gs.choff, codes, scales);
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
  __shared__ GeomLds gs;
  __shared__ uint32_t bmax[NA / 8];
  load_geom<kFixedThreads>(g, gs);
  const int H = g.H, L = g.L, B = g.block_bits, lmask = (1 << L) - 1;
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
      raw[k] = *reinterpret_cast<const int4*>(codes + 2 * gi);
      sc[k] = scales[gi >> B];
    }
  };
  uint64_t tau = blockIdx.x;  // the grid never exceeds ntiles
  fetch(tau);
  for (; tau < ntiles; tau += gridDim.x) {
    for (int q = threadIdx.x; q < nblk; q += kFixedThreads) bmax[q] = 0u;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int gq = k * kFixedThreads + threadIdx.x;
      if (NG % kFixedThreads == 0 || gq < NG) decode8(raw[k], sc[k] / 127.0f, sh, gq << 3);
    }
    __syncthreads();
    const uint64_t nxt = tau + gridDim.x;
    fetch(nxt < ntiles ? nxt : tau);
    Fixed<float, TB, kFixedThreads>::run(sh, ops, nops, mats);
    store_enc2<kFixedThreads>(sh, bmax, NA, B, L, lmask, tile_base(tau, L, H, gs.hb), gs.choff,
                              codes, scales);
    __syncthreads();
  }
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
  const bool fixed_ok = g.maxk <= 3;  // the pipelined kernels run ops of up to 3 qubits
  if (dt == JUQCS_C128) {
    auto* p = (cplx<double>*)amps;
    auto* m = (const cplx<double>*)d_mats;
    if (!fixed_ok) hipLaunchKernelGGL((k_tile<double, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
    else if (g.b == 13) JUQCS_FIXED(double, 13, 1024);
    else if (g.b == 12) JUQCS_FIXED(double, 12, 512);
    else if (g.b == 11) JUQCS_FIXED(double, 11, 512);
    else if (g.b <= 12) hipLaunchKernelGGL((k_tile<double, 12>), grid, block, 0, s, p, g, d_ops, nops, m);
    else hipLaunchKernelGGL((k_tile<double, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
  } else if (dt == JUQCS_C64) {
    auto* p = (cplx<float>*)amps;
    auto* m = (const cplx<float>*)d_mats;
    if (!fixed_ok) hipLaunchKernelGGL((k_tile<float, 14>), grid, block, 0, s, p, g, d_ops, nops, m);
    else if (g.b == 13) JUQCS_FIXED(float, 13, 1024);
    else if (g.b == 12) JUQCS_FIXED(float, 12, 512);
    else if (g.b == 11) JUQCS_FIXED(float, 11, 512);
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

}  // namespace juqcs
