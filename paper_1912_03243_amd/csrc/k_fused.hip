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
constexpr int kLdw = kCols + 1;  // LDS row stride of a panel: rows fall in different banks

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline v8bf as_bf(v8s x) { return __builtin_bit_cast(v8bf, x); }

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

// Panel geometry of a fused block.  A panel is the KD x NC sub-matrix of
// amplitudes (rows: the k target bits, columns: the NC = 2^cb lowest
// non-target bits) for one setting of every other bit.  In address order it
// is 2^khi contiguous chunks of 2^S amplitudes (S: the lowest S bits hold
// the low targets and the cb column bits; the khi high targets select the
// chunk), so loads and stores walk whole chunks of at least NC amplitudes.
struct FusedGeom {
  int32_t k, S, khi, cb;
  int32_t tbits[6];   // targets in matrix order (physical bits)
  int32_t hts[6];     // high targets (>= S), ascending: inserted into the panel index
};

// KD: K = 2^k amplitudes per column; R = padded real rows (multiple of 16).
// Persistent: every workgroup loads the matrix once, builds the panel map
// (element -> row, column) in LDS, and then walks panels (gridDim.x apart),
// prefetching the next panel into registers while the current one is
// multiplied.
template <int P, int KD>
__global__ __launch_bounds__(kThreads) void k_fused(
    cplx<typename PrecTraits<P>::T>* __restrict__ psi, uint64_t npanels, FusedGeom fg,
    const typename PrecTraits<P>::T* __restrict__ At /* R x R, transposed: At[col*R+row] */) {
  using T = typename PrecTraits<P>::T;
  constexpr int R0 = 2 * KD;
  constexpr int R = R0 < 16 ? 16 : R0;
  // FP64 / FP32 blocks of up to 4 qubits keep their matrix operands in
  // registers (R/16 x R/4 values per lane): no LDS copy of the matrix, so
  // more workgroups fit a CU
  constexpr bool kAReg = (P == P_F64 || P == P_F32) && R <= 32;
  constexpr int NAR = kAReg ? (R / 16) * (R / 4) : 1;
  constexpr bool kALds = !kAReg && (R * R * sizeof(T)) <= 64 * 1024;
  constexpr int E = KD * kCols;                           // panel elements (at most)
  constexpr int PER = (E + kThreads - 1) / kThreads;      // panel amplitudes per thread
  // register prefetch only where it fits beside the accumulators
  constexpr bool kPrefetch = PER * sizeof(cplx<T>) <= 8 * sizeof(cplx<double>);
  constexpr int PV = kPrefetch ? PER : 1;
  __shared__ T sB[R * kLdw];
  __shared__ T sA[kALds ? R * R : 1];
  __shared__ uint16_t map[E];        // row << 6 | column of panel element e
  __shared__ uint64_t offhi[KD];     // address offset of chunk h
  const int k = fg.k, S = fg.S, khi = fg.khi;
  const int ncols = 1 << fg.cb, ne = KD << fg.cb;
  const uint64_t omask = (uint64_t(1) << S) - 1;
  for (int e = threadIdx.x; e < ne; e += kThreads) {
    const int h = e >> S;
    const uint64_t o = (uint64_t)e & omask;
    int r = 0, c = 0, nc = 0, nh = 0;
    for (int j = 0; j < k; ++j) {
      const int t = fg.tbits[j];
      if (t < S) r |= (int)((o >> t) & 1) << j;
    }
    for (int b = 0; b < S; ++b) {
      bool tgt = false;
      for (int j = 0; j < k; ++j) tgt |= fg.tbits[j] == b;
      if (!tgt) c |= (int)((o >> b) & 1) << nc++;
    }
    // high target j is bit i of h, i = its rank among the high targets
    for (int j = 0; j < k; ++j) {
      if (fg.tbits[j] < S) continue;
      int i = 0;
      for (int jj = 0; jj < khi; ++jj) i += fg.hts[jj] < fg.tbits[j] ? 1 : 0;
      r |= ((h >> i) & 1) << j;
    }
    (void)nh;
    map[e] = (uint16_t)((r << 6) | c);
  }
  if (threadIdx.x < (1 << khi)) {
    uint64_t o = 0;
    for (int i = 0; i < khi; ++i) o |= (uint64_t)((threadIdx.x >> i) & 1) << fg.hts[i];
    offhi[threadIdx.x] = o;
  }
  if (kALds) {
    for (int i = threadIdx.x; i < R * R; i += kThreads) sA[i] = At[i];
  }
  // padded rows of B stay zero
  if (R > R0) {
    for (int i = R0 * kLdw + threadIdx.x; i < R * kLdw; i += kThreads) sB[i] = T(0);
  }
  __syncthreads();
  const T* A = kALds ? sA : At;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lhi = lane >> 4;
  T areg[NAR];
  if constexpr (kAReg) {
#pragma unroll
    for (int t = 0; t < R / 16; ++t)
#pragma unroll
      for (int kq = 0; kq < R / 4; ++kq) areg[t * (R / 4) + kq] = At[(4 * kq + lhi) * R + t * 16 + l16];
  }

  auto panel_base = [&](uint64_t pi) {
    uint64_t base = pi << S;
    for (int i = 0; i < khi; ++i) base = insert_zero(base, fg.hts[i]);
    return base;
  };
  auto addr = [&](uint64_t base, int e) { return base + offhi[e >> S] + ((uint64_t)e & omask); };
  auto to_lds = [&](int e, cplx<T> w) {
    const int m = map[e], r = m >> 6, c = m & 63;
    sB[(2 * r) * kLdw + c] = w.re;
    sB[(2 * r + 1) * kLdw + c] = w.im;
  };
  cplx<T> v[PV];
  auto fetch = [&](uint64_t pi) {
    const uint64_t base = panel_base(pi);
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int e = q * kThreads + threadIdx.x;
      v[q] = cplx<T>{T(0), T(0)};
      if (e < ne) v[q] = ld_amp(&psi[addr(base, e)]);
    }
  };
  uint64_t pi = blockIdx.x;
  const uint64_t stride = gridDim.x;
  if (kPrefetch && pi < npanels) fetch(pi);
  for (; pi < npanels; pi += stride) {
    const uint64_t base = panel_base(pi);
    // ---- the panel into LDS as 2K rows x NC columns (prefetched, or loaded here)
    if constexpr (kPrefetch) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = q * kThreads + threadIdx.x;
        if (e < ne) to_lds(e, v[q]);
      }
    } else {
      for (int e = threadIdx.x; e < ne; e += kThreads) to_lds(e, ld_amp(&psi[addr(base, e)]));
    }
    __syncthreads();
    if (kPrefetch && pi + stride < npanels) fetch(pi + stride);

    // ---- per wave: out(R x 16) = A(R x R) * B(R x 16)
    const int cw = wave * 16;
    if constexpr (P == P_F64) {
      v4d acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4d{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < R; kk += 4) {
        const double bv = sB[(kk + lhi) * kLdw + cw + l16];
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          const double av = kAReg ? areg[t * (R / 4) + kk / 4] : A[(kk + lhi) * R + t * 16 + l16];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
      // wave-private columns: safe to overwrite once this wave's reads are done
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g) sB[(t * 16 + 4 * g + lhi) * kLdw + cw + l16] = acc[t][g];
    } else if constexpr (P == P_F32) {
      v4f acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4f{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < R; kk += 4) {
        const float bv = sB[(kk + lhi) * kLdw + cw + l16];
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          const float av = kAReg ? areg[t * (R / 4) + kk / 4] : A[(kk + lhi) * R + t * 16 + l16];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[(t * 16 + 4 * lhi + i) * kLdw + cw + l16] = acc[t][i];
    } else {
      // BF16 operands on the gfx950 double-rate shape 16x16x32: lane
      // 16 q + c holds K slots 8 q .. 8 q + 7 (K padded to 32 with zeros)
      v4f acc[R / 16];
#pragma unroll
      for (int t = 0; t < R / 16; ++t) acc[t] = v4f{0, 0, 0, 0};
      for (int kk = 0; kk < R; kk += 32) {
        v8s bh, bl;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int kr = kk + 8 * lhi + i;
          const float x = kr < R ? sB[kr * kLdw + cw + l16] : 0.0f;
          const short h = bf16_rne(x);
          bh[i] = h;
          bl[i] = bf16_rne(x - bf16_to_f32(h));
        }
#pragma unroll
        for (int t = 0; t < R / 16; ++t) {
          v8s ah, al;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int kr = kk + 8 * lhi + i;
            const float x = kr < R ? A[kr * R + t * 16 + l16] : 0.0f;
            const short h = bf16_rne(x);
            ah[i] = h;
            al[i] = bf16_rne(x - bf16_to_f32(h));
          }
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bh), acc[t], 0, 0, 0);
          if constexpr (P == P_BF16X3) {
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bl), acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(bh), acc[t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < R / 16; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[(t * 16 + 4 * lhi + i) * kLdw + cw + l16] = acc[t][i];
    }
    __syncthreads();

    // ---- store in address order (whole chunks)
    for (int e = threadIdx.x; e < ne; e += kThreads) {
      const int m = map[e], r = m >> 6, c = m & 63;
      cplx<T> w;
      w.re = sB[(2 * r) * kLdw + c];
      w.im = sB[(2 * r + 1) * kLdw + c];
      st_amp(&psi[addr(base, e)], w);
    }
    (void)ncols;
    __syncthreads();
  }
}

template <int P>
hipError_t dispatch_k(void* amps, int n, int k, const FusedGeom& tg, const void* d_mat,
                      hipStream_t s) {
  using T = typename PrecTraits<P>::T;
  const uint64_t npanels = uint64_t(1) << (n - k - tg.cb);
  uint64_t g = npanels;
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
    case 1: hipLaunchKernelGGL((k_fused<P, 2>), grid, block, 0, s, p, npanels, tg, A); break;
    case 2: hipLaunchKernelGGL((k_fused<P, 4>), grid, block, 0, s, p, npanels, tg, A); break;
    case 3: hipLaunchKernelGGL((k_fused<P, 8>), grid, block, 0, s, p, npanels, tg, A); break;
    case 4: hipLaunchKernelGGL((k_fused<P, 16>), grid, block, 0, s, p, npanels, tg, A); break;
    case 5: hipLaunchKernelGGL((k_fused<P, 32>), grid, block, 0, s, p, npanels, tg, A); break;
    case 6: hipLaunchKernelGGL((k_fused<P, 64>), grid, block, 0, s, p, npanels, tg, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// d_mat: the real embedded matrix, transposed, padded to R = max(16, 2^(k+1)),
// in the precision of the mode (double for FP64, float otherwise).
hipError_t launch_fused(juqcs_dtype dt, void* amps, int n, int k, const int* targets,
                        const void* d_mat, juqcs_mma mode, hipStream_t s) {
  if (k < 1 || k > 6 || k > n) return hipErrorInvalidValue;
  FusedGeom tg{};
  tg.k = k;
  uint64_t tmask = 0;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 0 || targets[j] >= n) return hipErrorInvalidValue;
    tg.tbits[j] = targets[j];
    tmask |= uint64_t(1) << targets[j];
  }
  // column bits: the lowest min(6, n - k) non-target bits; S: the span that
  // holds them and the targets below them
  tg.cb = n - k < 6 ? n - k : 6;
  int S = 0, nc = 0;
  while (nc < tg.cb) {
    if (!((tmask >> S) & 1)) ++nc;
    ++S;
  }
  tg.S = S;
  tg.khi = 0;
  for (int b = S; b < n; ++b)
    if ((tmask >> b) & 1) tg.hts[tg.khi++] = b;
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
