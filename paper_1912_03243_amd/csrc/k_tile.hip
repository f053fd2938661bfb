// On-chip tile passes.  A workgroup gathers 2^b amplitudes -- 2^H chunks of
// 2^L contiguous amplitudes, the chunk bits being chosen physical qubits --
// into LDS, applies a program of gate ops whose qubits all lie in those b
// bits, and writes the tile back: one HBM read + write per pass however many
// gates the pass holds.  This is the single-GPU counterpart of the paper's
// "minimise the data that must move" for gates on qubits that are not local
// (Section 2), with LDS playing the role of node memory.
//
// Storage forms: C128 and C64 amplitudes, and the two-byte form (ENC2),
// which is decoded into FP32 on load and re-encoded with fresh per-block
// scales on store (Section 1, adaptive two-byte coding).
#include <mutex>
#include <unordered_map>

#include "tile_ops.hpp"

namespace juqcs {

namespace {

using tileops::kThreads;
using tileops::run_ops;
using tileops::diag_pick;

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

__device__ inline uint64_t tile_base(uint64_t tau, const TileGeom& g) {
  uint64_t base = tau << g.L;
  for (int j = 0; j < g.H; ++j) base = insert_zero(base, g.hbits[j]);
  return base;
}

// ------------------------------------------------------- C128 / C64 -------
template <typename T, int MAXB>
__global__ __launch_bounds__(kThreads) void k_tile(cplx<T>* __restrict__ psi, TileGeom g,
                                                   const TileOp* __restrict__ ops, int nops,
                                                   const cplx<T>* __restrict__ mats) {
  __shared__ cplx<T> sh[1 << MAXB];
  __shared__ uint64_t choff[1 << kMaxGather];
  const int b = g.b;
  const int tile_amps = 1 << b;
  const int nch = 1 << g.H;
  for (int c = threadIdx.x; c < nch; c += kThreads) {
    uint64_t o = 0;
    for (int j = 0; j < g.H; ++j) o |= (uint64_t)((c >> j) & 1) << g.hbits[j];
    choff[c] = o;
  }
  __syncthreads();
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  const int lmask = (1 << g.L) - 1;
  for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
    const uint64_t base = tile_base(tau, g);
    // load: 8 independent loads in flight per thread per round (a native
    // 2-vector buffer stays in registers)
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2* gp = reinterpret_cast<const v2*>(psi);
    v2* sp = reinterpret_cast<v2*>(sh);
    for (int e0 = 0; e0 < tile_amps; e0 += kThreads * 8) {
      v2 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + k * kThreads + threadIdx.x;
        const int ec = e < tile_amps ? e : 0;
        v[k] = gp[base + choff[ec >> g.L] + (ec & lmask)];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + k * kThreads + threadIdx.x;
        if (e < tile_amps) sp[e] = v[k];
      }
    }
    __syncthreads();
    run_ops<T>(sh, b, ops, nops, mats);
    for (int e = threadIdx.x; e < tile_amps; e += kThreads)
      psi[base + choff[e >> g.L] + (e & lmask)] = sh[e];
    __syncthreads();
  }
}

// ------------------------------------------- pipelined fixed-size tiles ---
// Tile size fixed at compile time (TB bits) and 512 threads per workgroup:
// every loop below has a constant trip count and is unrolled, each op reads
// all of its LDS operands before it writes, and a persistent grid prefetches
// the next tile into registers while the current one is processed on chip,
// so HBM traffic overlaps the ops.
constexpr int kFixedThreads = 512;

template <typename T, int TB>
__device__ inline void fop_dense1(cplx<T>* sh, int a, const cplx<T>* __restrict__ m) {
  constexpr int NP = (1 << (TB - 1)) / kFixedThreads;
  const cplx<T> u0 = m[0], u1 = m[1], u2 = m[2], u3 = m[3];
  const int abit = 1 << a;
  cplx<T> x[NP], y[NP];
  int i0[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    i0[k] = (int)insert_zero((uint64_t)(k * kFixedThreads + threadIdx.x), a);
    x[k] = sh[i0[k]];
    y[k] = sh[i0[k] | abit];
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    sh[i0[k]] = cmad(u1, y[k], cmul(u0, x[k]));
    sh[i0[k] | abit] = cmad(u3, y[k], cmul(u2, x[k]));
  }
}

template <typename T, int TB>
__device__ inline void fop_dense2(cplx<T>* sh, int a, int c, const cplx<T>* __restrict__ m) {
  constexpr int NQ = (1 << (TB - 2)) / kFixedThreads;
  const int lo = a < c ? a : c, hi = a < c ? c : a;
  const int ba = 1 << a, bc = 1 << c;
  cplx<T> v[NQ][4];
  int ix[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    ix[k] = (int)insert_zero(insert_zero((uint64_t)(k * kFixedThreads + threadIdx.x), lo), hi);
    v[k][0] = sh[ix[k]];
    v[k][1] = sh[ix[k] | ba];
    v[k][2] = sh[ix[k] | bc];
    v[k][3] = sh[ix[k] | ba | bc];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const cplx<T> m0 = m[4 * r], m1 = m[4 * r + 1], m2 = m[4 * r + 2], m3 = m[4 * r + 3];
    const int off = ((r & 1) ? ba : 0) | ((r & 2) ? bc : 0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      cplx<T> acc = cmul(m0, v[k][0]);
      acc = cmad(m1, v[k][1], acc);
      acc = cmad(m2, v[k][2], acc);
      acc = cmad(m3, v[k][3], acc);
      sh[ix[k] | off] = acc;
    }
  }
}

template <typename T, int TB>
__device__ inline void fop_diag2(cplx<T>* sh, int a, int c, const cplx<T>* __restrict__ m) {
  constexpr int NE = (1 << TB) / kFixedThreads;
  const cplx<T> d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = k * kFixedThreads + threadIdx.x;
    sh[e] = cmul(diag_pick(e, a, c, d0, d1, d2, d3), sh[e]);
  }
}

// Base index of tile tau: tau's bits fill the non-tile positions in order.
__device__ inline uint64_t tile_base_lds(uint64_t tau, int L, int H, const int* hb) {
  uint64_t base = tau << L;
  for (int j = 0; j < H; ++j) base = insert_zero(base, hb[j]);
  return base;
}

template <typename T, int TB>
__global__ __launch_bounds__(kFixedThreads) void k_tile_fixed(cplx<T>* __restrict__ psi, TileGeom g,
                                                              const TileOp* __restrict__ ops,
                                                              int nops,
                                                              const cplx<T>* __restrict__ mats) {
  constexpr int NA = 1 << TB, PER = NA / kFixedThreads;
  __shared__ cplx<T> sh[NA];
  __shared__ uint64_t choff[1 << kMaxGather];
  __shared__ int hb[kHbitsCap];
  const int H = g.H, L = g.L, lmask = (1 << L) - 1;
  if (threadIdx.x < kHbitsCap) hb[threadIdx.x] = threadIdx.x < H ? g.hbits[threadIdx.x] : 0;
  __syncthreads();
  for (int c = threadIdx.x; c < (1 << H); c += kFixedThreads) {
    uint64_t o = 0;
    for (int j = 0; j < H; ++j) o |= (uint64_t)((c >> j) & 1) << hb[j];
    choff[c] = o;
  }
  __syncthreads();
  const uint64_t ntiles = uint64_t(1) << (g.n - TB);
  // the grid never exceeds ntiles, so blockIdx.x is a valid first tile.
  // (a native 2-vector keeps the buffer in registers; an array of the cplx
  // struct is demoted to scratch for FP64)
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2* gp = reinterpret_cast<v2*>(psi);
  v2* sp = reinterpret_cast<v2*>(sh);
  v2 v[PER];
  uint64_t tau = blockIdx.x;
  {
    const uint64_t base = tile_base_lds(tau, L, H, hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * kFixedThreads + threadIdx.x;
      v[k] = gp[base + choff[e >> L] + (e & lmask)];
    }
  }
  for (; tau < ntiles; tau += gridDim.x) {
#pragma unroll
    for (int k = 0; k < PER; ++k) sp[k * kFixedThreads + threadIdx.x] = v[k];
    __syncthreads();
    // prefetch the next tile while this one is on chip; after the last tile
    // the current one is read again (in bounds, values unused), which keeps
    // the buffer in registers
    const uint64_t nxt = tau + gridDim.x;
    const uint64_t pf = nxt < ntiles ? nxt : tau;
    {
      const uint64_t nb = tile_base_lds(pf, L, H, hb);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = k * kFixedThreads + threadIdx.x;
        v[k] = gp[nb + choff[e >> L] + (e & lmask)];
      }
    }
    for (int o = 0; o < nops; ++o) {
      const TileOp op = ops[o];
      const cplx<T>* m = mats + op.moff;
      if (op.kind == TOP_DENSE2) fop_dense2<T, TB>(sh, op.a, op.b, m);
      else if (op.kind == TOP_DENSE1) fop_dense1<T, TB>(sh, op.a, m);
      else fop_diag2<T, TB>(sh, op.a, op.b, m);
      __syncthreads();
    }
    const uint64_t base = tile_base_lds(tau, L, H, hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * kFixedThreads + threadIdx.x;
      gp[base + choff[e >> L] + (e & lmask)] = sp[e];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------- ENC2 -----
// Codes are int8 (re, im) pairs; a thread moves 8 amplitudes (16 bytes of
// codes) at a time, which always lie in one scale block (block_bits >= 3).
constexpr float kTiny = 7.888609052210118e-31f;  // 2^-100

__global__ __launch_bounds__(kThreads) void k_tile_enc2(int8_t* __restrict__ codes,
                                                        float* __restrict__ scales, TileGeom g,
                                                        const TileOp* __restrict__ ops, int nops,
                                                        const cplx<float>* __restrict__ mats) {
  constexpr int MAXB = TileCfg<float>::kMaxBits;
  __shared__ cplx<float> sh[1 << MAXB];
  __shared__ uint64_t choff[1 << kMaxGather];
  __shared__ uint32_t bmax[1 << (MAXB - 3)];
  const int b = g.b;
  const int B = g.block_bits;
  const int tile_amps = 1 << b;
  const int ngroups = tile_amps >> 3;
  const int nblk = tile_amps >> B;
  const int nch = 1 << g.H;
  for (int c = threadIdx.x; c < nch; c += kThreads) {
    uint64_t o = 0;
    for (int j = 0; j < g.H; ++j) o |= (uint64_t)((c >> j) & 1) << g.hbits[j];
    choff[c] = o;
  }
  __syncthreads();
  const uint64_t ntiles = uint64_t(1) << (g.n - b);
  const int lmask = (1 << g.L) - 1;
  for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
    const uint64_t base = tile_base(tau, g);
    for (int q = threadIdx.x; q < nblk; q += kThreads) bmax[q] = 0u;
    // load + decode
    for (int gq = threadIdx.x; gq < ngroups; gq += kThreads) {
      const int e = gq << 3;
      const uint64_t gi = base + choff[e >> g.L] + (e & lmask);
      const int4 raw = *reinterpret_cast<const int4*>(codes + 2 * gi);
      const float d = scales[gi >> B] / 127.0f;
      const int w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int8_t c0 = (int8_t)(w[j] & 0xff), c1 = (int8_t)((w[j] >> 8) & 0xff);
        const int8_t c2 = (int8_t)((w[j] >> 16) & 0xff), c3 = (int8_t)((w[j] >> 24) & 0xff);
        sh[e + 2 * j] = {(float)c0 * d, (float)c1 * d};
        sh[e + 2 * j + 1] = {(float)c2 * d, (float)c3 * d};
      }
    }
    __syncthreads();
    run_ops<float>(sh, b, ops, nops, mats);
    // per-block max of |component| (non-negative floats order like their bits)
    for (int gq = threadIdx.x; gq < ngroups; gq += kThreads) {
      const int e = gq << 3;
      float mx = 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const cplx<float> v = sh[e + j];
        mx = fmaxf(mx, fmaxf(fabsf(v.re), fabsf(v.im)));
      }
      atomicMax(&bmax[e >> B], __float_as_uint(mx));
    }
    __syncthreads();
    // encode + store
    for (int gq = threadIdx.x; gq < ngroups; gq += kThreads) {
      const int e = gq << 3;
      const uint64_t gi = base + choff[e >> g.L] + (e & lmask);
      const float s = __uint_as_float(bmax[e >> B]);
      int w[4] = {0, 0, 0, 0};
      if (s >= kTiny) {
        const float r = 127.0f / s;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const cplx<float> v = sh[e + j];
          const float qr = fminf(fmaxf(rintf(v.re * r), -127.0f), 127.0f);
          const float qi = fminf(fmaxf(rintf(v.im * r), -127.0f), 127.0f);
          const int pr = ((int)qr) & 0xff, pi = ((int)qi) & 0xff;
          w[j >> 1] |= (pr | (pi << 8)) << (16 * (j & 1));
        }
      }
      *reinterpret_cast<int4*>(codes + 2 * gi) = make_int4(w[0], w[1], w[2], w[3]);
      if (((e & ((1 << B) - 1)) == 0)) scales[gi >> B] = (s >= kTiny) ? s : 0.0f;
    }
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
  auto pgrid_for = [&](const void* kern) {
    const uint64_t slots = resident_blocks(kern, kFixedThreads);
    return dim3((unsigned)(ntiles < slots ? ntiles : slots));
  };
  const bool fixed_ok = g.maxk <= 2;  // the pipelined kernels run 1- and 2-qubit ops
  if (dt == JUQCS_C128) {
    auto* p = (cplx<double>*)amps;
    auto* m = (const cplx<double>*)d_mats;
    if (fixed_ok && g.b == 12)
      hipLaunchKernelGGL((k_tile_fixed<double, 12>), pgrid_for((const void*)k_tile_fixed<double, 12>), fblock, 0, s, p, g, d_ops, nops, m);
    else if (fixed_ok && g.b == 11)
      hipLaunchKernelGGL((k_tile_fixed<double, 11>), pgrid_for((const void*)k_tile_fixed<double, 11>), fblock, 0, s, p, g, d_ops, nops, m);
    else if (g.b <= 12)
      hipLaunchKernelGGL((k_tile<double, 12>), grid, block, 0, s, p, g, d_ops, nops, m);
    else
      hipLaunchKernelGGL((k_tile<double, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
  } else if (dt == JUQCS_C64) {
    auto* p = (cplx<float>*)amps;
    auto* m = (const cplx<float>*)d_mats;
    if (fixed_ok && g.b == 13)
      hipLaunchKernelGGL((k_tile_fixed<float, 13>), pgrid_for((const void*)k_tile_fixed<float, 13>), fblock, 0, s, p, g, d_ops, nops, m);
    else if (fixed_ok && g.b == 12)
      hipLaunchKernelGGL((k_tile_fixed<float, 12>), pgrid_for((const void*)k_tile_fixed<float, 12>), fblock, 0, s, p, g, d_ops, nops, m);
    else if (fixed_ok && g.b == 11)
      hipLaunchKernelGGL((k_tile_fixed<float, 11>), pgrid_for((const void*)k_tile_fixed<float, 11>), fblock, 0, s, p, g, d_ops, nops, m);
    else if (g.b <= 13)
      hipLaunchKernelGGL((k_tile<float, 13>), grid, block, 0, s, p, g, d_ops, nops, m);
    else
      hipLaunchKernelGGL((k_tile<float, 14>), grid, block, 0, s, p, g, d_ops, nops, m);
  } else {
    hipLaunchKernelGGL(k_tile_enc2, grid, block, 0, s, (int8_t*)amps, (float*)scales, g, d_ops,
                       nops, (const cplx<float>*)d_mats);
  }
  return hipGetLastError();
}

}  // namespace juqcs
