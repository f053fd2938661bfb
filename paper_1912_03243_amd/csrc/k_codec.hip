// Two-byte amplitude codec (Section 1: adaptive two-byte coding, 8x less
// memory than FP64 complex) and the single-qubit Pauli sums behind the
// expectation values of Section 3.
//
// Format (defined by this library; the paper does not print one): blocks of
// 2^B consecutive amplitudes; s = max |component| over the block in FP32;
// s < 2^-100 -> scale 0 and zero codes; else r = fl32(127/s) and
// q = clamp(rint(fl32(x*r)), -127, 127) per component (int8); decoding is
// fl32(q * fl32(s/127)).  Divisions are the correctly rounded IEEE ones.
#include "juqcs_internal.hpp"

namespace juqcs {

namespace {

constexpr int kThreads = 256;
constexpr float kTiny = 7.888609052210118e-31f;  // 2^-100

__device__ inline float block_max(float v, float* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  float r = sh[0];
  for (int i = 1; i < kThreads / 64; ++i) r = fmaxf(r, sh[i]);
  __syncthreads();
  return r;
}

// One workgroup per scale block (grid-stride over blocks).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_encode2(const cplx<T>* __restrict__ src,
                                                      uint64_t count, int B,
                                                      char2* __restrict__ codes,
                                                      float* __restrict__ scales) {
  __shared__ float sh[kThreads / 64];
  const uint64_t bs = uint64_t(1) << B;
  const uint64_t nblocks = (count + bs - 1) >> B;
  for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const uint64_t lo = blk << B;
    const uint64_t hi = lo + bs < count ? lo + bs : count;
    float mx = 0.0f;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      const cplx<T> v = src[i];
      mx = fmaxf(mx, fmaxf(fabsf((float)v.re), fabsf((float)v.im)));
    }
    const float s = block_max(mx, sh);
    const bool zero = !(s >= kTiny);
    const float r = zero ? 0.0f : 127.0f / s;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      char2 c = {0, 0};
      if (!zero) {
        const cplx<T> v = src[i];
        const float xr = (float)v.re, xi = (float)v.im;
        c.x = (signed char)fminf(fmaxf(rintf(xr * r), -127.0f), 127.0f);
        c.y = (signed char)fminf(fmaxf(rintf(xi * r), -127.0f), 127.0f);
      }
      codes[i] = c;
    }
    if (threadIdx.x == 0) scales[blk] = zero ? 0.0f : s;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_decode2(const char2* __restrict__ codes,
                                                      const float* __restrict__ scales,
                                                      uint64_t count, int B,
                                                      cplx<T>* __restrict__ dst) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
    const char2 q = codes[i];
    const float d = scales[i >> B] / 127.0f;
    cplx<T> v;
    v.re = (T)((float)q.x * d);
    v.im = (T)((float)q.y * d);
    dst[i] = v;
  }
}

// ------------------------------------------------------- Pauli sums ----
constexpr int kPauliBlocks = 1024;

__device__ inline void block_sum3(double v[3], double* sh) {
  for (int c = 0; c < 3; ++c)
    for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int c = 0; c < 3; ++c) sh[3 * w + c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) {
      double r = 0.0;
      for (int i = 0; i < kThreads / 64; ++i) r += sh[3 * i + c];
      v[c] = r;
    }
  __syncthreads();
}

template <typename T>
__device__ inline cplx<double> load_amp(const void* amps, const float* scales, int B, uint64_t i) {
  const cplx<T> v = ((const cplx<T>*)amps)[i];
  return {(double)v.re, (double)v.im};
}
template <>
__device__ inline cplx<double> load_amp<char>(const void* amps, const float* scales, int B,
                                              uint64_t i) {
  const char2 q = ((const char2*)amps)[i];
  const float d = scales[i >> B] / 127.0f;
  return {(double)((float)q.x * d), (double)((float)q.y * d)};
}

// Pair p (target bit removed) -> (a0, a1); accumulate 2 conj(a0) a1 and
// |a0|^2 - |a1|^2 in FP64 over a fixed partition of the pairs.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pauli(const void* __restrict__ amps,
                                                    const float* __restrict__ scales, int B,
                                                    uint64_t npairs, int t, uint64_t chunk,
                                                    double* __restrict__ partials) {
  __shared__ double sh[3 * kThreads / 64];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < npairs ? lo + chunk : npairs;
  double v[3] = {0.0, 0.0, 0.0};
  for (uint64_t p = lo + threadIdx.x; p < hi; p += kThreads) {
    const uint64_t i0 = insert_zero(p, t), i1 = i0 | (uint64_t(1) << t);
    const cplx<double> a = load_amp<T>(amps, scales, B, i0);
    const cplx<double> b = load_amp<T>(amps, scales, B, i1);
    // conj(a) * b
    const double re = a.re * b.re + a.im * b.im;
    const double im = a.re * b.im - a.im * b.re;
    v[0] += 2.0 * re;
    v[1] += 2.0 * im;
    v[2] += (a.re * a.re + a.im * a.im) - (b.re * b.re + b.im * b.im);
  }
  block_sum3(v, sh);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) partials[3 * blockIdx.x + c] = v[c];
}

__global__ __launch_bounds__(kThreads) void k_pauli_final(const double* __restrict__ partials,
                                                          int nparts, double* __restrict__ out3) {
  __shared__ double sh[3 * kThreads / 64];
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += kThreads)
    for (int c = 0; c < 3; ++c) v[c] += partials[3 * i + c];
  block_sum3(v, sh);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out3[c] = v[c];
}

inline unsigned stride_grid(uint64_t count) {
  const uint64_t want = (count + kThreads - 1) / kThreads;
  return (unsigned)(want < 65536 ? (want ? want : 1) : 65536);
}

}  // namespace

hipError_t launch_encode2(const void* src, juqcs_dtype sdt, uint64_t count, int block_bits,
                          void* codes, void* scales, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint64_t nblocks = (count + (uint64_t(1) << block_bits) - 1) >> block_bits;
  const unsigned grid = (unsigned)(nblocks < (1u << 20) ? nblocks : (1u << 20));
  if (sdt == JUQCS_C128)
    hipLaunchKernelGGL(k_encode2<double>, dim3(grid), dim3(kThreads), 0, s,
                       (const cplx<double>*)src, count, block_bits, (char2*)codes,
                       (float*)scales);
  else
    hipLaunchKernelGGL(k_encode2<float>, dim3(grid), dim3(kThreads), 0, s,
                       (const cplx<float>*)src, count, block_bits, (char2*)codes,
                       (float*)scales);
  return hipGetLastError();
}

hipError_t launch_decode2(const void* codes, const void* scales, uint64_t count, int block_bits,
                          void* dst, juqcs_dtype ddt, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (ddt == JUQCS_C128)
    hipLaunchKernelGGL(k_decode2<double>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (const char2*)codes, (const float*)scales, count, block_bits,
                       (cplx<double>*)dst);
  else
    hipLaunchKernelGGL(k_decode2<float>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (const char2*)codes, (const float*)scales, count, block_bits,
                       (cplx<float>*)dst);
  return hipGetLastError();
}

hipError_t launch_pauli(juqcs_dtype dt, const void* amps, const void* scales, int n,
                        int block_bits, int t, double* partials, double* out3, hipStream_t s) {
  const uint64_t npairs = uint64_t(1) << (n - 1);
  uint64_t chunk = (npairs + kPauliBlocks - 1) / kPauliBlocks;
  chunk = (chunk + kThreads - 1) / kThreads * kThreads;
  const int nparts = (int)((npairs + chunk - 1) / chunk);
  if (dt == JUQCS_C128)
    hipLaunchKernelGGL(k_pauli<double>, dim3(nparts), dim3(kThreads), 0, s, amps,
                       (const float*)scales, block_bits, npairs, t, chunk, partials);
  else if (dt == JUQCS_C64)
    hipLaunchKernelGGL(k_pauli<float>, dim3(nparts), dim3(kThreads), 0, s, amps,
                       (const float*)scales, block_bits, npairs, t, chunk, partials);
  else
    hipLaunchKernelGGL(k_pauli<char>, dim3(nparts), dim3(kThreads), 0, s, amps,
                       (const float*)scales, block_bits, npairs, t, chunk, partials);
  hipLaunchKernelGGL(k_pauli_final, dim3(1), dim3(kThreads), 0, s, partials, nparts, out3);
  return hipGetLastError();
}

}  // namespace juqcs
