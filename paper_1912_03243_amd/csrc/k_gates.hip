// Per-gate streaming kernels: one pass over the touched amplitudes per gate
// (Section 2: a gate changes every pair of coefficients that differ only in
// the target bit, Eq. (1); the work is a few flops per coefficient, so the
// pass is bound by memory bandwidth).  Also: state init, norm, amplitude
// read-out, scaling and the reference copy kernel.
#include "juqcs_internal.hpp"

namespace juqcs {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(uint64_t work, uint64_t per_block) {
  uint64_t g = (work + per_block - 1) / per_block;
  return (unsigned)(g ? g : 1);
}

// ---------------------------------------------------------------- init ----
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(cplx<T>* __restrict__ psi,
                                                   uint64_t count, uint64_t idx) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
    cplx<T> v;
    v.re = (i == idx) ? T(1) : T(0);
    v.im = T(0);
    st_amp(&psi[i], v);
  }
}

// ENC2 |idx>: all codes zero and all scales zero except idx's block, whose
// scale is 1 and whose code at idx is (127, 0).
__global__ __launch_bounds__(kThreads) void k_init_enc2(uint32_t* __restrict__ codes4,
                                                        uint64_t nwords,
                                                        float* __restrict__ scales,
                                                        uint64_t nblocks, uint64_t idx,
                                                        int block_bits) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t w = (uint64_t)blockIdx.x * kThreads + threadIdx.x; w < nwords; w += stride) {
    // one 32-bit word holds the codes of two amplitudes
    uint32_t v = 0;
    if ((idx >> 1) == w) v = (idx & 1) ? (127u << 16) : 127u;
    st_stream(&codes4[w], v);
  }
  for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < nblocks; b += stride)
    st_stream(&scales[b], (b == (idx >> block_bits)) ? 1.0f : 0.0f);
}

// ------------------------------------------------------------------ 1q ----
// Eq. (1) on target bit t, optionally restricted to indices whose control bit
// is set.  Pair index p enumerates the indices with the target (and control)
// bit removed; consecutive lanes take consecutive p, so for t >= 6 every load
// of a wave is one contiguous run of 64 amplitudes.
template <typename T, int U>
__global__ __launch_bounds__(kThreads) void k_1q(cplx<T>* __restrict__ psi, uint64_t npairs,
                                                 int z0, int z1, uint64_t tbit,
                                                 uint64_t cmask, Mat2<T> u) {
  const uint64_t base = (uint64_t)blockIdx.x * (kThreads * U) + threadIdx.x;
  cplx<T> a[U], b[U];
  uint64_t ix[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t p = base + (uint64_t)k * kThreads;
    uint64_t i = insert_zero(p, z0);
    if (z1 >= 0) i = insert_zero(i, z1);
    ix[k] = i | cmask;
    if (p < npairs) {
      a[k] = ld_amp(&psi[ix[k]]);
      b[k] = ld_amp(&psi[ix[k] | tbit]);
    }
  }
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t p = base + (uint64_t)k * kThreads;
    if (p < npairs) {
      cplx<T> r0 = cmul(u.m[0], a[k]);
      r0 = cmad(u.m[1], b[k], r0);
      cplx<T> r1 = cmul(u.m[2], a[k]);
      r1 = cmad(u.m[3], b[k], r1);
      st_amp(&psi[ix[k]], r0);
      st_amp(&psi[ix[k] | tbit], r1);
    }
  }
}

// ---------------------------------------------------------------- runs ----
// Per-gate passes in runs.  A run is 64 consecutive 16-byte words (one per
// lane of a wave): 64 C128 or 128 C64 amplitudes, so every load and store a
// wave issues covers 1 KiB of contiguous memory whatever the gate's qubits
// (Eq. (1) pairs indices that differ in the target bit only; when that bit
// is below the run width the partner sits in another lane of the same
// wave).  Bits below the run width RB (6 for C128, 7 for C64) are "low",
// the others "high":
//   * low target   (RUN_LOW): the partner amplitude comes from lane l ^ 2^t
//     (C64: l ^ 2^(t-1); t = 0 pairs the two amplitudes of one lane);
//   * high target  (RUN_HIGH): run r is paired with run r + 2^(t - RB);
//   * a high control or diagonal bit is set to 1 in the run index, so only
//     the runs it selects are read; a low one is a per-amplitude predicate
//     (amplitudes that fail it are written back unchanged).
enum RunMode { RUN_LOW = 0, RUN_HIGH = 1, RUN_DIAG = 2 };

template <typename T>
struct RunT;
template <>
struct RunT<double> {
  static constexpr int RB = 6;  // amplitudes per run: 64
  typedef double W __attribute__((ext_vector_type(2)));
};
template <>
struct RunT<float> {
  static constexpr int RB = 7;  // amplitudes per run: 128
  typedef float W __attribute__((ext_vector_type(4)));
};

struct RunArgs {
  uint64_t nruns;   // runs (RUN_HIGH: run pairs) to process
  int nins;         // run-index bits inserted (ascending positions ins[])
  int ins[3];
  uint64_t ones;    // inserted bits that are 1 (high controls and diagonal bits)
  uint64_t tstride; // RUN_HIGH: run-index distance of the partner run
  int t;            // RUN_LOW: the target bit
  uint32_t lmask;   // low control / diagonal bits that must all be 1
};

template <typename T>
__device__ __forceinline__ cplx<T> mat_row(cplx<T> m0, cplx<T> x, cplx<T> m1, cplx<T> y) {
  return cmad(m1, y, cmul(m0, x));
}

template <typename T, int MODE, int U>
__global__ __launch_bounds__(kThreads) void k_runs(cplx<T>* __restrict__ psi, RunArgs ra, Mat2<T> u,
                                                   cplx<T> ph) {
  using W = typename RunT<T>::W;
  constexpr int RB = RunT<T>::RB;
  constexpr int APL = sizeof(W) / sizeof(cplx<T>);  // amplitudes per lane: 1 or 2
  W* g = reinterpret_cast<W*>(psi);
  const int lane = threadIdx.x & 63;
  constexpr int NL = MODE == RUN_HIGH ? 2 * U : U;  // 16-byte words per lane
  const uint64_t nwaves = (ra.nruns + U - 1) / U;
  // grid-stride over waves: a launch stays below 2^32 work-items at any n
  for (uint64_t wave = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); wave < nwaves;
       wave += (uint64_t)gridDim.x * (kThreads / 64)) {
  W v[NL];
  uint64_t at[NL];
  bool ok[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t ri = wave * U + k;
    ok[k] = ri < ra.nruns;
    uint64_t r = ok[k] ? ri : 0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < ra.nins) r = insert_zero(r, ra.ins[j]);
    r |= ra.ones;
    at[k] = (r << (RB - (APL == 2 ? 1 : 0))) + lane;  // word index of this lane
    if (MODE == RUN_HIGH) at[U + k] = at[k] + (ra.tstride << (RB - (APL == 2 ? 1 : 0)));
  }
#pragma unroll
  for (int k = 0; k < NL; ++k)
    if (ok[k % U]) v[k] = ld_stream(&g[at[k]]);
  // amplitude index bits of this lane's amplitudes within their run
  const int a0 = APL == 2 ? 2 * lane : lane;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    if (MODE == RUN_LOW) {
      // partner values from the lane across the target bit
      const int xl = APL == 2 ? (ra.t > 0 ? 1 << (ra.t - 1) : 0) : 1 << ra.t;
      W w = v[k];
#pragma unroll
      for (int c = 0; c < (int)(sizeof(W) / sizeof(T)); ++c) w[c] = xl ? __shfl_xor(v[k][c], xl, 64) : v[k][c];
#pragma unroll
      for (int j = 0; j < APL; ++j) {
        const int a = a0 + j;
        const cplx<T> self = {v[k][2 * j], v[k][2 * j + 1]};
        // C64 t = 0: the partner is the other amplitude of this lane
        const int pj = (APL == 2 && ra.t == 0) ? 1 - j : j;
        const cplx<T> other = (APL == 2 && ra.t == 0) ? cplx<T>{v[k][2 * pj], v[k][2 * pj + 1]}
                                                       : cplx<T>{w[2 * j], w[2 * j + 1]};
        const bool hi = (a >> ra.t) & 1;
        cplx<T> r = hi ? mat_row(u.m[2], other, u.m[3], self) : mat_row(u.m[0], self, u.m[1], other);
        if (((uint32_t)a & ra.lmask) != ra.lmask) r = self;
        w[2 * j] = r.re;
        w[2 * j + 1] = r.im;
      }
      if (ok[k]) st_stream(&g[at[k]], w);
    } else if (MODE == RUN_HIGH) {
      W wa = v[k], wb = v[U + k];
#pragma unroll
      for (int j = 0; j < APL; ++j) {
        const int a = a0 + j;
        const cplx<T> x = {v[k][2 * j], v[k][2 * j + 1]}, y = {v[U + k][2 * j], v[U + k][2 * j + 1]};
        if (((uint32_t)a & ra.lmask) == ra.lmask) {
          const cplx<T> r0 = mat_row(u.m[0], x, u.m[1], y), r1 = mat_row(u.m[2], x, u.m[3], y);
          wa[2 * j] = r0.re;
          wa[2 * j + 1] = r0.im;
          wb[2 * j] = r1.re;
          wb[2 * j + 1] = r1.im;
        }
      }
      if (ok[k]) {
        st_stream(&g[at[k]], wa);
        st_stream(&g[at[U + k]], wb);
      }
    } else {
      W w = v[k];
#pragma unroll
      for (int j = 0; j < APL; ++j) {
        const int a = a0 + j;
        if (((uint32_t)a & ra.lmask) == ra.lmask) {
          const cplx<T> r = cmul(ph, cplx<T>{v[k][2 * j], v[k][2 * j + 1]});
          w[2 * j] = r.re;
          w[2 * j + 1] = r.im;
        }
      }
      if (ok[k]) st_stream(&g[at[k]], w);
    }
  }
  }
}

// --------------------------------------------------------------- diag ----
// Multiplies the amplitudes whose bits in mask are all 1 by phase (the
// nontrivial part of Z, S, T, CZ and controlled-phase); other amplitudes are
// not touched.  Up to two mask bits, z0 < z1.
template <typename T, int U>
__global__ __launch_bounds__(kThreads) void k_diag(cplx<T>* __restrict__ psi, uint64_t count,
                                                   int z0, int z1, uint64_t mask,
                                                   cplx<T> ph) {
  const uint64_t base = (uint64_t)blockIdx.x * (kThreads * U) + threadIdx.x;
  cplx<T> a[U];
  uint64_t ix[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t p = base + (uint64_t)k * kThreads;
    uint64_t i = insert_zero(p, z0);
    if (z1 >= 0) i = insert_zero(i, z1);
    ix[k] = i | mask;
    if (p < count) a[k] = ld_amp(&psi[ix[k]]);
  }
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t p = base + (uint64_t)k * kThreads;
    if (p < count) st_amp(&psi[ix[k]], cmul(ph, a[k]));
  }
}

// ------------------------------------------------------------------ 2q ----
template <typename T, int U>
__global__ __launch_bounds__(kThreads) void k_2q(cplx<T>* __restrict__ psi, uint64_t nquads,
                                                 int z0, int z1, uint64_t b0, uint64_t b1,
                                                 Mat4<T> m) {
  for (uint64_t base = (uint64_t)blockIdx.x * (kThreads * U) + threadIdx.x; base < nquads;
       base += (uint64_t)gridDim.x * (kThreads * U)) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t p = base + (uint64_t)k * kThreads;
      if (p >= nquads) continue;
      const uint64_t i = insert_zero(insert_zero(p, z0), z1);
      const uint64_t idx[4] = {i, i | b0, i | b1, i | b0 | b1};
      cplx<T> v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = ld_amp(&psi[idx[r]]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cplx<T> acc = cmul(m.m[4 * r], v[0]);
#pragma unroll
        for (int c = 1; c < 4; ++c) acc = cmad(m.m[4 * r + c], v[c], acc);
        st_amp(&psi[idx[r]], acc);
      }
    }
  }
}

// ---------------------------------------------------------------- norm ----
// Fixed partition: block g sums amplitudes [g*chunk, (g+1)*chunk) with a
// per-thread FP64 accumulator, then a fixed-shape tree inside the block.
// The final pass sums the partials in a fixed order, so results are
// reproducible bit for bit.
constexpr int kNormBlocks = 2048;

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_norm_partial(const cplx<T>* __restrict__ psi,
                                                           uint64_t count, uint64_t chunk,
                                                           double* __restrict__ partials) {
  __shared__ double sh[kThreads / 64];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const cplx<T> v = ld_amp(&psi[i]);
    acc += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void k_norm_partial_enc2(
    const char2* __restrict__ codes, const float* __restrict__ scales, uint64_t count,
    int block_bits, uint64_t chunk, double* __restrict__ partials) {
  __shared__ double sh[kThreads / 64];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const char2 q = codes[i];
    const float d = scales[i >> block_bits] / 127.0f;
    const float re = (float)q.x * d, im = (float)q.y * d;
    acc += (double)re * (double)re + (double)im * (double)im;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void k_sum_final(const double* __restrict__ partials,
                                                        int nparts, double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) acc += partials[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}

// -------------------------------------------------------------- gather ----
struct PhysMap {
  int8_t p[64];
  int32_t identity;
};

__device__ inline uint64_t to_phys(uint64_t z, int n, const PhysMap& m) {
  if (m.identity) return z;
  uint64_t out = 0;
  for (int q = 0; q < n; ++q) out |= ((z >> q) & 1ull) << m.p[q];
  return out;
}

// out[k] = g psi[phys(idx[k])] in FP64 (g: the state's global factor).
__device__ inline void put_amp(double* out, uint64_t k, double re, double im, cplx<double> g) {
  out[2 * k] = g.re * re - g.im * im;
  out[2 * k + 1] = g.re * im + g.im * re;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(const cplx<T>* __restrict__ psi, int n,
                                                     const uint64_t* __restrict__ idx,
                                                     uint64_t count, PhysMap pm, cplx<double> g,
                                                     double* __restrict__ out) {
  for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < count;
       k += (uint64_t)gridDim.x * kThreads) {
    const uint64_t z = idx[k];
    if ((z >> n) != 0) {  // index outside the state: NaN, no access
      out[2 * k] = out[2 * k + 1] = __builtin_nan("");
      continue;
    }
    const cplx<T> v = psi[to_phys(z, n, pm)];
    put_amp(out, k, (double)v.re, (double)v.im, g);
  }
}

__global__ __launch_bounds__(kThreads) void k_gather_enc2(const char2* __restrict__ codes,
                                                          const float* __restrict__ scales,
                                                          int n, int block_bits,
                                                          const uint64_t* __restrict__ idx,
                                                          uint64_t count, PhysMap pm,
                                                          cplx<double> g,
                                                          double* __restrict__ out) {
  for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < count;
       k += (uint64_t)gridDim.x * kThreads) {
    if ((idx[k] >> n) != 0) {
      out[2 * k] = out[2 * k + 1] = __builtin_nan("");
      continue;
    }
    const uint64_t i = to_phys(idx[k], n, pm);
    const char2 q = codes[i];
    const float d = scales[i >> block_bits] / 127.0f;
    put_amp(out, k, (double)((float)q.x * d), (double)((float)q.y * d), g);
  }
}

// --------------------------------------------------------------- scale ----
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale(cplx<T>* __restrict__ psi, uint64_t count,
                                                    T f) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) {
    cplx<T> v = ld_amp(&psi[i]);
    v.re *= f;
    v.im *= f;
    st_amp(&psi[i], v);
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_f32(float* __restrict__ x, uint64_t count,
                                                        float f) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride)
    x[i] *= f;
}

// ---------------------------------------------------------------- fill ----
// Zeroes count 32-bit words (used instead of a memset node where a caller
// may capture the work into a graph).
__global__ __launch_bounds__(kThreads) void k_zero(uint32_t* __restrict__ p, uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += stride) p[i] = 0u;
}

// ---------------------------------------------------------------- copy ----
// Reference streaming copy: each thread moves 4 x 16 bytes per iteration,
// with the same non-temporal accesses as the state passes.
__global__ __launch_bounds__(kThreads) void k_copy(uint4* __restrict__ dst,
                                                   const uint4* __restrict__ src,
                                                   uint64_t count) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  constexpr int U = 4;
  const v4u* s4 = reinterpret_cast<const v4u*>(src);
  v4u* d4 = reinterpret_cast<v4u*>(dst);
  for (uint64_t base = (uint64_t)blockIdx.x * (kThreads * U) + threadIdx.x; base < count;
       base += (uint64_t)gridDim.x * (kThreads * U)) {
    v4u v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t i = base + (uint64_t)k * kThreads;
      if (i < count) v[k] = ld_stream(&s4[i]);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t i = base + (uint64_t)k * kThreads;
      if (i < count) st_stream(&d4[i], v[k]);
    }
  }
}

// In-place stream: every 16-byte word read and written back, in the access
// pattern of the per-gate run kernels (each wave moves U consecutive runs of
// 64 words, loads before stores): the HBM ceiling of an in-place pass.
template <int U>
__global__ __launch_bounds__(kThreads) void k_stream(uint4* __restrict__ p, uint64_t count) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  v4u* q = reinterpret_cast<v4u*>(p);
  const int lane = threadIdx.x & 63;
  const uint64_t nwaves = (count + 64 * U - 1) / (64 * U);
  for (uint64_t wave = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); wave < nwaves;
       wave += (uint64_t)gridDim.x * (kThreads / 64)) {
    v4u v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t i = (wave * U + k) * 64 + lane;
      if (i < count) v[k] = ld_stream(&q[i]);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t i = (wave * U + k) * 64 + lane;
      if (i < count) st_stream(&q[i], v[k]);
    }
  }
}

inline unsigned stride_grid(uint64_t count) {
  // grid-stride kernels: enough blocks to fill 256 CUs many times over
  const uint64_t want = (count + kThreads - 1) / kThreads;
  return (unsigned)(want < 65536 ? (want ? want : 1) : 65536);
}

template <typename T>
Mat2<T> to_mat2(const cplx<double> u[4]) {
  Mat2<T> m;
  for (int i = 0; i < 4; ++i) m.m[i] = {(T)u[i].re, (T)u[i].im};
  return m;
}
template <typename T>
Mat4<T> to_mat4(const cplx<double> u[16]) {
  Mat4<T> m;
  for (int i = 0; i < 16; ++i) m.m[i] = {(T)u[i].re, (T)u[i].im};
  return m;
}

// Run geometry of a gate: high bits (>= RB) are inserted into the run index
// (ones: set to 1), low ones go to the lane predicate.  Returns false when
// the state is too small for runs.
template <typename T>
bool run_args(int n, int t_high, uint64_t set_mask, RunArgs* ra) {
  constexpr int RB = RunT<T>::RB;
  int hb[3], nh = 0;
  ra->lmask = 0;
  ra->ones = 0;
  for (int q = 0; q < 64; ++q) {
    if (!((set_mask >> q) & 1)) continue;
    if (q < RB) {
      ra->lmask |= 1u << q;
    } else {
      hb[nh++] = q - RB;
      ra->ones |= uint64_t(1) << (q - RB);
    }
  }
  if (t_high >= 0) hb[nh++] = t_high - RB;
  if (n < RB + nh + 1) return false;
  // ascending insertion positions
  for (int i = 0; i < nh; ++i)
    for (int j = i + 1; j < nh; ++j)
      if (hb[j] < hb[i]) {
        const int x = hb[i];
        hb[i] = hb[j];
        hb[j] = x;
      }
  ra->nins = nh;
  for (int i = 0; i < 3; ++i) ra->ins[i] = i < nh ? hb[i] : 0;
  ra->nruns = uint64_t(1) << (n - RB - nh);
  ra->tstride = t_high >= 0 ? uint64_t(1) << (t_high - RB) : 0;
  ra->t = 0;
  return true;
}

// Blocks of a grid-stride launch: every block of the work, at most
// kMaxBlocks (2^24 work-items, far beyond the resident blocks of 256 CUs).
constexpr uint64_t kMaxBlocks = uint64_t(1) << 16;
inline unsigned capped_grid(uint64_t work, uint64_t per_block) {
  const uint64_t g = grid_for(work, per_block);
  return (unsigned)(g < kMaxBlocks ? g : kMaxBlocks);
}

template <typename T, int MODE, int U>
hipError_t launch_runs(void* amps, const RunArgs& ra, const Mat2<T>& u, cplx<T> ph, hipStream_t s) {
  const uint64_t waves = (ra.nruns + U - 1) / U;
  hipLaunchKernelGGL((k_runs<T, MODE, U>), dim3(capped_grid(waves, kThreads / 64)), dim3(kThreads), 0, s,
                     (cplx<T>*)amps, ra, u, ph);
  return hipGetLastError();
}

template <typename T>
hipError_t do_1q(void* amps, int n, int t, int c, const cplx<double> u[4], hipStream_t s) {
  constexpr int RB = RunT<T>::RB;
  const uint64_t cm = c >= 0 ? uint64_t(1) << c : 0;
  RunArgs ra;
  if (run_args<T>(n, t >= RB ? t : -1, cm, &ra)) {
    if (t >= RB) return launch_runs<T, RUN_HIGH, 1>(amps, ra, to_mat2<T>(u), cplx<T>{}, s);
    ra.t = t;
    return launch_runs<T, RUN_LOW, 2>(amps, ra, to_mat2<T>(u), cplx<T>{}, s);
  }
  constexpr int U = 4;
  const uint64_t npairs = uint64_t(1) << (n - 1 - (c >= 0 ? 1 : 0));
  int z0 = t, z1 = -1;
  uint64_t cmask = 0;
  if (c >= 0) {
    z0 = t < c ? t : c;
    z1 = t < c ? c : t;
    cmask = uint64_t(1) << c;
  }
  hipLaunchKernelGGL((k_1q<T, U>), dim3(grid_for(npairs, kThreads * U)), dim3(kThreads), 0, s,
                     (cplx<T>*)amps, npairs, z0, z1, uint64_t(1) << t, cmask, to_mat2<T>(u));
  return hipGetLastError();
}

template <typename T>
hipError_t do_diag(void* amps, int n, uint64_t mask, cplx<double> ph, hipStream_t s) {
  RunArgs ra;
  if (run_args<T>(n, -1, mask, &ra))
    return launch_runs<T, RUN_DIAG, 2>(amps, ra, Mat2<T>{}, cplx<T>{(T)ph.re, (T)ph.im}, s);
  constexpr int U = 4;
  int z[2] = {-1, -1}, nb = 0;
  for (int q = 0; q < 64 && nb < 2; ++q)
    if ((mask >> q) & 1) z[nb++] = q;
  const uint64_t count = uint64_t(1) << (n - nb);
  cplx<T> p = {(T)ph.re, (T)ph.im};
  hipLaunchKernelGGL((k_diag<T, U>), dim3(grid_for(count, kThreads * U)), dim3(kThreads), 0, s,
                     (cplx<T>*)amps, count, z[0], z[1], mask, p);
  return hipGetLastError();
}

template <typename T>
hipError_t do_2q(void* amps, int n, int q0, int q1, const cplx<double> m[16], hipStream_t s) {
  constexpr int U = 2;
  const uint64_t nq = uint64_t(1) << (n - 2);
  const int z0 = q0 < q1 ? q0 : q1, z1 = q0 < q1 ? q1 : q0;
  hipLaunchKernelGGL((k_2q<T, U>), dim3(capped_grid(nq, kThreads * U)), dim3(kThreads), 0, s,
                     (cplx<T>*)amps, nq, z0, z1, uint64_t(1) << q0, uint64_t(1) << q1,
                     to_mat4<T>(m));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init(juqcs_dtype dt, void* amps, void* scales, int n, int block_bits,
                       uint64_t idx, hipStream_t s) {
  const uint64_t count = uint64_t(1) << n;
  if (dt == JUQCS_C128) {
    hipLaunchKernelGGL(k_init<double>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (cplx<double>*)amps, count, idx);
  } else if (dt == JUQCS_C64) {
    hipLaunchKernelGGL(k_init<float>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (cplx<float>*)amps, count, idx);
  } else {
    // n >= block_bits >= 3: the codes fill whole 32-bit words (two amplitudes each)
    const uint64_t nwords = count / 2;
    const uint64_t nblocks = count >> block_bits;
    hipLaunchKernelGGL(k_init_enc2, dim3(stride_grid(nwords)), dim3(kThreads), 0, s,
                       (uint32_t*)amps, nwords, (float*)scales, nblocks, idx, block_bits);
  }
  return hipGetLastError();
}

hipError_t launch_1q(juqcs_dtype dt, void* amps, int n, int t, int c, const cplx<double> u[4],
                     hipStream_t s) {
  if (dt == JUQCS_C128) return do_1q<double>(amps, n, t, c, u, s);
  if (dt == JUQCS_C64) return do_1q<float>(amps, n, t, c, u, s);
  return hipErrorInvalidValue;
}

hipError_t launch_diag(juqcs_dtype dt, void* amps, int n, uint64_t mask, cplx<double> ph,
                       hipStream_t s) {
  if (dt == JUQCS_C128) return do_diag<double>(amps, n, mask, ph, s);
  if (dt == JUQCS_C64) return do_diag<float>(amps, n, mask, ph, s);
  return hipErrorInvalidValue;
}

hipError_t launch_2q(juqcs_dtype dt, void* amps, int n, int q0, int q1, const cplx<double> m[16],
                     hipStream_t s) {
  if (dt == JUQCS_C128) return do_2q<double>(amps, n, q0, q1, m, s);
  if (dt == JUQCS_C64) return do_2q<float>(amps, n, q0, q1, m, s);
  return hipErrorInvalidValue;
}

hipError_t launch_norm(juqcs_dtype dt, const void* amps, const void* scales, int n,
                       int block_bits, double* partials, double* out, hipStream_t s) {
  const uint64_t count = uint64_t(1) << n;
  uint64_t chunk = (count + kNormBlocks - 1) / kNormBlocks;
  chunk = (chunk + kThreads - 1) / kThreads * kThreads;
  const int nparts = (int)((count + chunk - 1) / chunk);
  if (dt == JUQCS_C128)
    hipLaunchKernelGGL(k_norm_partial<double>, dim3(nparts), dim3(kThreads), 0, s,
                       (const cplx<double>*)amps, count, chunk, partials);
  else if (dt == JUQCS_C64)
    hipLaunchKernelGGL(k_norm_partial<float>, dim3(nparts), dim3(kThreads), 0, s,
                       (const cplx<float>*)amps, count, chunk, partials);
  else
    hipLaunchKernelGGL(k_norm_partial_enc2, dim3(nparts), dim3(kThreads), 0, s,
                       (const char2*)amps, (const float*)scales, count, block_bits, chunk,
                       partials);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kThreads), 0, s, partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_gather(juqcs_dtype dt, const void* amps, const void* scales, int n,
                         int block_bits, const uint64_t* idx, uint64_t count,
                         const int8_t* phys, cplx<double> g, double* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  PhysMap pm;
  pm.identity = 1;
  for (int q = 0; q < 64; ++q) pm.p[q] = (int8_t)(q < n ? phys[q] : q);
  for (int q = 0; q < n; ++q)
    if (phys[q] != q) pm.identity = 0;
  const dim3 grid(capped_grid(count, kThreads));
  if (dt == JUQCS_C128)
    hipLaunchKernelGGL(k_gather<double>, grid, dim3(kThreads), 0, s, (const cplx<double>*)amps, n,
                       idx, count, pm, g, out);
  else if (dt == JUQCS_C64)
    hipLaunchKernelGGL(k_gather<float>, grid, dim3(kThreads), 0, s, (const cplx<float>*)amps, n,
                       idx, count, pm, g, out);
  else
    hipLaunchKernelGGL(k_gather_enc2, grid, dim3(kThreads), 0, s, (const char2*)amps,
                       (const float*)scales, n, block_bits, idx, count, pm, g, out);
  return hipGetLastError();
}

hipError_t launch_scale(juqcs_dtype dt, void* amps, void* scales, int n, int block_bits,
                        double f, hipStream_t s) {
  const uint64_t count = uint64_t(1) << n;
  if (dt == JUQCS_C128)
    hipLaunchKernelGGL(k_scale<double>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (cplx<double>*)amps, count, f);
  else if (dt == JUQCS_C64)
    hipLaunchKernelGGL(k_scale<float>, dim3(stride_grid(count)), dim3(kThreads), 0, s,
                       (cplx<float>*)amps, count, (float)f);
  else {
    const uint64_t nb = (count + (uint64_t(1) << block_bits) - 1) >> block_bits;
    hipLaunchKernelGGL(k_scale_f32, dim3(stride_grid(nb)), dim3(kThreads), 0, s, (float*)scales,
                       nb, (float)f);
  }
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const uint64_t count = bytes / 4;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(stride_grid(count)), dim3(kThreads), 0, s, (uint32_t*)p, count);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t count = bytes / 16;
  if (dst == src) {
    constexpr int U = 2;
    const uint64_t waves = (count + 64 * U - 1) / (64 * U);
    hipLaunchKernelGGL((k_stream<U>), dim3(capped_grid(waves, kThreads / 64)), dim3(kThreads), 0, s,
                       (uint4*)dst, count);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_copy, dim3(capped_grid(count, kThreads * 4)), dim3(kThreads), 0, s,
                     (uint4*)dst, (const uint4*)src, count);
  return hipGetLastError();
}

}  // namespace juqcs
