// Fused k-qubit blocks on the matrix cores.
//
// A product of gates on k qubits is one dense 2^k x 2^k complex matrix M.
// Viewing the state as a 2^k x 2^(n-k) matrix (rows: the k target bits,
// columns: all other bits), the block is the contraction  Psi <- M Psi.  With
// the real embedding  [Re;Im] <- [[Re M, -Im M],[Im M, Re M]] [Re;Im]  stored
// with interleaved rows (row 2r+p holds part p of amplitude r), it is a real
// GEMM  (2K x 2K) x (2K x C),  K = 2^k, which runs on MFMA:
//   FP64   v_mfma_f64_16x16x4f64        (C128 states)
//   FP32   v_mfma_f32_16x16x4f32        (C64 states)
//   BF16   v_mfma_f32_16x16x16bf16_1k   (C64 states, FP32 accumulation)
//   BF16X3 three BF16 products hi*hi + hi*lo + lo*hi (operands carried to
//          about 17 significant bits; lo*lo is dropped)
//
// A workgroup (4 waves) owns 64 consecutive columns: it stages the 2K x 64
// panel in LDS with coalesced loads, each wave multiplies its 16 columns, the
// results go back through LDS and are stored coalesced to the same places
// (in place: every column belongs to exactly one workgroup).
#include <map>
#include <mutex>

#include "juqcs_internal.hpp"

namespace juqcs {

namespace {

constexpr int kThreads = 256;
constexpr int kCols = 64;  // columns per workgroup, 16 per wave

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round to nearest even (finite inputs).
__device__ inline short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf16_to_f32(short h) {
  return __uint_as_float(((uint32_t)(unsigned short)h) << 16);
}

template <int P>
struct PrecTraits;
template <>
struct PrecTraits<P_F64> {
  using T = double;
};
template <>
struct PrecTraits<P_F32> {
  using T = float;
};
template <>
struct PrecTraits<P_BF16> {
  using T = float;
};
template <>
struct PrecTraits<P_BF16X3> {
  using T = float;
};

// KD: K = 2^k amplitudes per column; R = padded real rows (multiple of 16).
// Persistent: every workgroup loads the matrix once and then walks column
// panels (gridDim.x apart), prefetching the next panel into registers while
// the current one is multiplied.
template <int P, int KD>
__global__ __launch_bounds__(kThreads) void k_fused(
    cplx<typename PrecTraits<P>::T>* __restrict__ psi, uint64_t ncols, TileGeom tg,
    const typename PrecTraits<P>::T* __restrict__ At /* R x R, transposed: At[col*R+row] */) {
  using T = typename PrecTraits<P>::T;
  constexpr int R0 = 2 * KD;
  constexpr int R = R0 < 16 ? 16 : R0;
  constexpr bool kALds = (R * R * sizeof(T)) <= 64 * 1024;
  constexpr int PER = (KD * kCols + kThreads - 1) / kThreads;  // panel amplitudes per thread
  // register prefetch only where it fits beside the accumulators
  constexpr bool kPrefetch = PER * sizeof(cplx<T>) <= 8 * sizeof(cplx<double>);
  constexpr int PV = kPrefetch ? PER : 1;
  __shared__ T sB[R * kCols];
  __shared__ T sA[kALds ? R * R : 1];
  __shared__ uint64_t off[KD];
  __shared__ int hs[6];

  // tg.hbits[0..k) hold the targets in matrix order; tg.hbits[k..2k) sorted.
  const int k = tg.H;
  if (threadIdx.x < KD) {
    uint64_t o = 0;
    for (int j = 0; j < k; ++j) o |= (uint64_t)((threadIdx.x >> j) & 1) << tg.hbits[j];
    off[threadIdx.x] = o;
  }
  if (threadIdx.x < 6) hs[threadIdx.x] = (int)threadIdx.x < k ? tg.hbits[k + threadIdx.x] : 0;
  if (kALds) {
    for (int i = threadIdx.x; i < R * R; i += kThreads) sA[i] = At[i];
  }
  // padded rows of B stay zero
  if (R > R0) {
    for (int i = R0 * kCols + threadIdx.x; i < R * kCols; i += kThreads) sB[i] = T(0);
  }
  __syncthreads();
  const T* A = kALds ? sA : At;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lhi = lane >> 4;

  // element e = r * kCols + col of a panel: amplitude r of column col
  auto col_base = [&](uint64_t c) {
    uint64_t base = c;
    for (int j = 0; j < k; ++j) base = insert_zero(base, hs[j]);
    return base;
  };
  cplx<T> v[PV];
  auto fetch = [&](uint64_t cb) {
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int e = q * kThreads + threadIdx.x;
      const int col = e % kCols, r = e / kCols;
      const uint64_t c = cb + col;
      v[q] = cplx<T>{T(0), T(0)};
      if (e < KD * kCols && c < ncols) v[q] = ld_amp(&psi[col_base(c) | off[r]]);
    }
  };
  uint64_t cb = (uint64_t)blockIdx.x * kCols;
  const uint64_t stride = (uint64_t)gridDim.x * kCols;
  if (kPrefetch && cb < ncols) fetch(cb);
  for (; cb < ncols; cb += stride) {
    // ---- the 2K x 64 panel into LDS (prefetched, or loaded here)
    if constexpr (kPrefetch) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = q * kThreads + threadIdx.x;
        if (e < KD * kCols) {
          const int col = e % kCols, r = e / kCols;
          sB[(2 * r) * kCols + col] = v[q].re;
          sB[(2 * r + 1) * kCols + col] = v[q].im;
        }
      }
    } else {
      for (int e = threadIdx.x; e < KD * kCols; e += kThreads) {
        const int col = e % kCols, r = e / kCols;
        const uint64_t c = cb + col;
        cplx<T> w = {T(0), T(0)};
        if (c < ncols) w = ld_amp(&psi[col_base(c) | off[r]]);
        sB[(2 * r) * kCols + col] = w.re;
        sB[(2 * r + 1) * kCols + col] = w.im;
      }
    }
    __syncthreads();
    if (kPrefetch && cb + stride < ncols) fetch(cb + stride);

    // ---- per wave: out(R x 16) = A(R x R) * B(R x 16)
    const int cw = wave * 16;
    if constexpr (P == P_F64) {
      v4d acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4d{0, 0, 0, 0};
      for (int kk = 0; kk < R; kk += 4) {
        const double bv = sB[(kk + lhi) * kCols + cw + l16];
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          const double av = A[(kk + lhi) * R + t * 16 + l16];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
      // wave-private columns: safe to overwrite once this wave's reads are done
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g) sB[(t * 16 + 4 * g + lhi) * kCols + cw + l16] = acc[t][g];
    } else if constexpr (P == P_F32) {
      v4f acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4f{0, 0, 0, 0};
      for (int kk = 0; kk < R; kk += 4) {
        const float bv = sB[(kk + lhi) * kCols + cw + l16];
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          const float av = A[(kk + lhi) * R + t * 16 + l16];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[(t * 16 + 4 * lhi + i) * kCols + cw + l16] = acc[t][i];
    } else {
      v4f acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4f{0, 0, 0, 0};
      for (int kk = 0; kk < R; kk += 16) {
        v4s bh, bl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float x = sB[(kk + 4 * lhi + i) * kCols + cw + l16];
          const short h = bf16_rne(x);
          bh[i] = h;
          bl[i] = bf16_rne(x - bf16_to_f32(h));
        }
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          v4s ah, al;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float x = A[(kk + 4 * lhi + i) * R + t * 16 + l16];
            const short h = bf16_rne(x);
            ah[i] = h;
            al[i] = bf16_rne(x - bf16_to_f32(h));
          }
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[t], 0, 0, 0);
          if constexpr (P == P_BF16X3) {
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[(t * 16 + 4 * lhi + i) * kCols + cw + l16] = acc[t][i];
    }
    __syncthreads();

    // ---- store (coalesced over columns)
    for (int e = threadIdx.x; e < KD * kCols; e += kThreads) {
      const int col = e % kCols, r = e / kCols;
      const uint64_t c = cb + col;
      if (c < ncols) {
        cplx<T> w;
        w.re = sB[(2 * r) * kCols + col];
        w.im = sB[(2 * r + 1) * kCols + col];
        st_amp(&psi[col_base(c) | off[r]], w);
      }
    }
    __syncthreads();
  }
}

template <int P>
hipError_t dispatch_k(void* amps, int n, int k, const TileGeom& tg, const void* d_mat,
                      hipStream_t s) {
  using T = typename PrecTraits<P>::T;
  const uint64_t ncols = uint64_t(1) << (n - k);
  uint64_t g = (ncols + kCols - 1) / kCols;
  // persistent grid: the resident workgroups of the kernel
  static std::mutex mu;
  static std::map<const void*, uint64_t> slots;
  const void* kern = nullptr;
  switch (k) {
    case 1: kern = (const void*)k_fused<P, 2>; break;
    case 2: kern = (const void*)k_fused<P, 4>; break;
    case 3: kern = (const void*)k_fused<P, 8>; break;
    case 4: kern = (const void*)k_fused<P, 16>; break;
    case 5: kern = (const void*)k_fused<P, 32>; break;
    case 6: kern = (const void*)k_fused<P, 64>; break;
    default: return hipErrorInvalidValue;
  }
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = slots.find(kern);
    if (it == slots.end()) {
      int dev = 0, cus = 256, per = 1;
      if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kThreads, 0) != hipSuccess || per < 1)
        per = 1;
      it = slots.emplace(kern, (uint64_t)cus * per).first;
    }
    if (g > it->second) g = it->second;
  }
  const dim3 grid((unsigned)g), block(kThreads);
  auto* p = (cplx<T>*)amps;
  const T* A = (const T*)d_mat;
  switch (k) {
    case 1: hipLaunchKernelGGL((k_fused<P, 2>), grid, block, 0, s, p, ncols, tg, A); break;
    case 2: hipLaunchKernelGGL((k_fused<P, 4>), grid, block, 0, s, p, ncols, tg, A); break;
    case 3: hipLaunchKernelGGL((k_fused<P, 8>), grid, block, 0, s, p, ncols, tg, A); break;
    case 4: hipLaunchKernelGGL((k_fused<P, 16>), grid, block, 0, s, p, ncols, tg, A); break;
    case 5: hipLaunchKernelGGL((k_fused<P, 32>), grid, block, 0, s, p, ncols, tg, A); break;
    case 6: hipLaunchKernelGGL((k_fused<P, 64>), grid, block, 0, s, p, ncols, tg, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// d_mat: the real embedded matrix, transposed, padded to R = max(16, 2^(k+1)),
// in the precision of the mode (double for FP64, float otherwise).
hipError_t launch_fused(juqcs_dtype dt, void* amps, int n, int k, const int* targets,
                        const void* d_mat, juqcs_mma mode, hipStream_t s) {
  TileGeom tg{};
  tg.n = n;
  tg.H = k;
  int sorted[6];
  for (int j = 0; j < k; ++j) {
    tg.hbits[j] = targets[j];
    sorted[j] = targets[j];
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j + 1 < k - i; ++j)
      if (sorted[j] > sorted[j + 1]) {
        const int t = sorted[j];
        sorted[j] = sorted[j + 1];
        sorted[j + 1] = t;
      }
  if (2 * k > kHbitsCap) return hipErrorInvalidValue;
  for (int j = 0; j < k; ++j) tg.hbits[k + j] = sorted[j];
  if (dt == JUQCS_C128) {
    if (mode != JUQCS_MMA_FP64) return hipErrorInvalidValue;
    return dispatch_k<P_F64>(amps, n, k, tg, d_mat, s);
  }
  if (dt == JUQCS_C64) {
    if (mode == JUQCS_MMA_FP32) return dispatch_k<P_F32>(amps, n, k, tg, d_mat, s);
    if (mode == JUQCS_MMA_BF16) return dispatch_k<P_BF16>(amps, n, k, tg, d_mat, s);
    if (mode == JUQCS_MMA_BF16X3) return dispatch_k<P_BF16X3>(amps, n, k, tg, d_mat, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace juqcs
