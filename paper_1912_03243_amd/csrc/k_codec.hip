// Two-byte amplitude codec (Section 1: adaptive two-byte coding, 8x less
// memory than FP64 complex).
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

}  // namespace juqcs
