// Many independent circuits in one graph launch (and the branch simulations
// of the entangling-gate decomposition, Section 4, whose terms are
// independent: the paper spreads them over MPI ranks and OpenMP threads,
// here they are work items of the same kernels).
//
// Work list: a "group" is one tile pass of one circuit (2^(n-b) tiles),
// cut into chunks of tiles.  Groups are ordered pass-major: round r holds
// pass r of every circuit that has one.  One persistent kernel per round
// claims the round's chunks through a ticket counter; the tiles of one pass
// are independent, and the kernel boundary between rounds orders pass r+1
// of a circuit after its pass r.  No workgroup ever waits for another, and
// no device-scope fence is needed inside a round (on this GPU such fences
// write back or invalidate a whole L2 slice).
#include "tile_ops.hpp"

namespace juqcs {

namespace {

using tileops::Fixed;
using tileops::lds;
using tileops::Var;

constexpr int kThreads = 256;       // helper kernels
// Two workgroups of 512 threads per CU on 2^12-amplitude tiles: their barriers
// are independent, so one's LDS and matrix-core phases overlap the other's
// (measured on MI355X: batch4096 -9%, the 42-qubit grid -8% against one
// workgroup of 1024 threads on 2^13 tiles).
constexpr int kBatchThreads = 512;   // the persistent batch kernel
constexpr int kBatchMaxBits = 12;   // 32 KiB of C64 amplitudes per tile
constexpr int kBatchTabs = 27;      // 8x8-op tables per pass (about 36 KiB of LDS)
constexpr int kBatchGather = 6;     // gathered chunk bits (tiles keep min(7, b) low bits)
using BatchTab = tileops::MmaTab<(1 << kBatchMaxBits) / 128>;  // the largest table

// Passes the fixed-size paths take: ops of up to 3 qubits, every 8x8 op's
// table and every op's parameters in LDS, chunk table in LDS.
__device__ inline bool fixed_pass(const BatchPass& ps) {
  return ps.g.maxk <= 3 && ps.g.mma_count <= kBatchTabs && ps.op_count <= kPassOps &&
         ps.g.H <= kBatchGather;
}

__device__ inline uint64_t tile_base_hb(uint64_t tau, int L, int H, const int* hb) {
  uint64_t base = tau << L;
  for (int j = 0; j < H; ++j) base = insert_zero(base, hb[j]);
  return base;
}

// Clears the rounds' ticket counters (a fill kernel, so that graph replays
// restart from zero).
__global__ __launch_bounds__(kThreads) void k_batch_reset(unsigned long long* __restrict__ tickets,
                                                          int nrounds) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < nrounds) tickets[i] = 0ull;
}

// One chunk of tiles of a pass with a compile-time tile size: the next tile
// of the chunk is prefetched into registers while the current one is on chip.
template <int TB>
__device__ inline void run_chunk_fixed(cplx<float>* sh, cplx<float>* psi, uint64_t tau0, int ntile,
                                       bool init, int L, int H, const int* hb,
                                       const uint64_t* choff, const TileOp* ops, int nops,
                                       const cplx<float>* mats, const tileops::OpPre* pre,
                                       const void* tabs, const int* swp, int nswap, const int* swk) {
  constexpr int NA = 1 << TB, PER = NA / kBatchThreads;
  const int lmask = (1 << L) - 1;
  typedef float v2 __attribute__((ext_vector_type(2)));
  v2* gp = reinterpret_cast<v2*>(psi);
  v2* sp = reinterpret_cast<v2*>(sh);
  v2 v[PER];
  if (!init) {
    const uint64_t base = tile_base_hb(tau0, L, H, hb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * kBatchThreads + threadIdx.x;
      v[k] = gp[base + choff[e >> L] + (e & lmask)];
    }
  }
  for (int j = 0; j < ntile; ++j) {
    const uint64_t tau = tau0 + j;
    const uint64_t base = tile_base_hb(tau, L, H, hb);
    if (init) {  // first pass: the state is |0...0>
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = k * kBatchThreads + threadIdx.x;
        sp[lds<float>(e)] = v2{(base == 0 && e == 0) ? 1.0f : 0.0f, 0.0f};
      }
    } else {
#pragma unroll
      for (int k = 0; k < PER; ++k) sp[lds<float>(k * kBatchThreads + threadIdx.x)] = v[k];
    }
    __syncthreads();
    if (!init) {  // prefetch the chunk's next tile (or this one again, unused)
      const uint64_t nb = tile_base_hb(j + 1 < ntile ? tau + 1 : tau, L, H, hb);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = k * kBatchThreads + threadIdx.x;
        v[k] = gp[nb + choff[e >> L] + (e & lmask)];
      }
    }
    using F = Fixed<float, TB, kBatchThreads>;
    F::template run<F::D3_TAB>(sh, ops, nops, mats, pre, tabs);
    // write-back through the pass's relabel swaps (see k_tile_fixed):
    // destination e takes LDS element lds(swap(t)) ^ swk[k]
    int t = threadIdx.x;
    for (int i = 0; i < nswap; ++i) {
      const int pr = swp[i], a = pr & 255, c = pr >> 8;
      const int x = ((t >> a) ^ (t >> c)) & 1;
      t ^= (x << a) | (x << c);
    }
    const int lt = lds<float>(t);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = k * kBatchThreads + threadIdx.x;
      gp[base + choff[e >> L] + (e & lmask)] = sp[lt ^ swk[k]];
    }
    __syncthreads();
  }
}

__device__ inline void run_chunk_var(cplx<float>* sh, cplx<float>* psi, uint64_t tau0, int ntile,
                                     bool init, int b, int L, int H, const int* hb,
                                     const uint64_t* choff, const TileOp* ops, int nops,
                                     const cplx<float>* mats, const int* swp, int nswap) {
  const int tile_amps = 1 << b, lmask = (1 << L) - 1;
  for (int j = 0; j < ntile; ++j) {
    const uint64_t base = tile_base_hb(tau0 + j, L, H, hb);
    if (init) {
      for (int e = threadIdx.x; e < tile_amps; e += kBatchThreads)
        sh[lds<float>(e)] = cplx<float>{(base == 0 && e == 0) ? 1.0f : 0.0f, 0.0f};
    } else {
      for (int e = threadIdx.x; e < tile_amps; e += kBatchThreads)
        sh[lds<float>(e)] = psi[base + choff[e >> L] + (e & lmask)];
    }
    __syncthreads();
    Var<float, kBatchThreads>::run(sh, b, ops, nops, mats);
    for (int e = threadIdx.x; e < tile_amps; e += kBatchThreads) {
      int t = e;  // relabel swaps of the write-back
      for (int i = 0; i < nswap; ++i) {
        const int pr = swp[i], a = pr & 255, c = pr >> 8;
        const int x = ((t >> a) ^ (t >> c)) & 1;
        t ^= (x << a) | (x << c);
      }
      psi[base + choff[e >> L] + (e & lmask)] = sh[lds<float>(t)];
    }
    __syncthreads();
  }
}

// One round: chunks [c0, c1) of groups [g0, g1).
__global__ __launch_bounds__(kBatchThreads) void k_batch(
    char* __restrict__ states, const BatchGroup* __restrict__ groups, int g0, int g1,
    const BatchPass* __restrict__ passes, const TileOp* __restrict__ ops,
    const cplx<float>* __restrict__ mats, unsigned long long* __restrict__ ticket, long long c0,
    long long c1) {
  __shared__ cplx<float> sh[1 << kBatchMaxBits];
  __shared__ uint64_t choff[1 << kBatchGather];
  __shared__ BatchTab tabs[kBatchTabs];  // the current pass's 8x8-op tables
  __shared__ tileops::OpPre pre[kPassOps];  // the current pass's op parameters
  __shared__ int hb[kHbitsCap];
  __shared__ int swp[kSwapCap];                // the current pass's relabel swaps
  __shared__ int swk[(1 << kBatchMaxBits) / kBatchThreads];  // lds(swap(k NT))
  __shared__ long long s_t;
  __shared__ int s_g;
  int cur_pass = -1;
  for (;;) {
    if (threadIdx.x == 0) {
      const long long t = c0 + (long long)atomicAdd(ticket, 1ull);
      int g = -1;
      if (t < c1) {  // last group of the round whose first chunk is <= t
        int lo = g0, hi = g1 - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (groups[mid].first_chunk <= t) lo = mid;
          else hi = mid - 1;
        }
        g = lo;
      }
      s_t = t;
      s_g = g;
    }
    __syncthreads();
    const long long t = s_t;
    const int gi = s_g;
    if (gi < 0) break;  // every workgroup leaves once the round's tickets run out
    const BatchGroup grp = groups[gi];
    const BatchPass ps = passes[grp.pass];
    const int b = ps.g.b, L = ps.g.L, H = ps.g.H;
    if (grp.pass != cur_pass) {
      // (straight from the pass table: indexing the local copy by thread
      // would put it in scratch)
      if (threadIdx.x < kHbitsCap)
        hb[threadIdx.x] = (int)threadIdx.x < H ? passes[grp.pass].g.hbits[threadIdx.x] : 0;
      if (threadIdx.x < kSwapCap) {
        const int i = threadIdx.x;
        const TileGeom& pg = passes[grp.pass].g;
        swp[i] = i < ps.g.nswap ? (int)pg.swap_a[i] | ((int)pg.swap_b[i] << 8) : 0;
      }
      __syncthreads();
      if (threadIdx.x < (1 << kBatchMaxBits) / kBatchThreads) {
        int t = threadIdx.x * kBatchThreads;
        for (int i = 0; i < ps.g.nswap; ++i) {
          const int pr = swp[i], a = pr & 255, c = pr >> 8;
          const int x = ((t >> a) ^ (t >> c)) & 1;
          t ^= (x << a) | (x << c);
        }
        swk[threadIdx.x] = lds<float>(t);
      }
      for (int c = threadIdx.x; c < (1 << H); c += kBatchThreads) {
        uint64_t o = 0;
        for (int j = 0; j < H; ++j) o |= (uint64_t)((c >> j) & 1) << hb[j];
        choff[c] = o;
      }
      if (fixed_pass(ps)) {
        const TileOp* pops = ops + ps.op_begin;
        if (b == 12) {
          using F = Fixed<float, 12, kBatchThreads>;
          F::build_tabs(reinterpret_cast<F::Tab*>(tabs), pops, ps.op_count, mats);
          F::build_pre(pre, pops, ps.op_count);
        } else if (b == 11) {
          using F = Fixed<float, 11, kBatchThreads>;
          F::build_tabs(reinterpret_cast<F::Tab*>(tabs), pops, ps.op_count, mats);
          F::build_pre(pre, pops, ps.op_count);
        }
      }
      __syncthreads();
      cur_pass = grp.pass;
    }
    cplx<float>* psi = reinterpret_cast<cplx<float>*>(states + grp.state_off);
    const uint64_t tau0 = (uint64_t)(t - grp.first_chunk) * grp.chunk_tiles;
    const TileOp* pops = ops + ps.op_begin;
    const bool init = grp.init != 0;
    // the fixed-size paths run ops of up to 3 qubits, 8x8 ops from their tables
    switch (fixed_pass(ps) ? b : 0) {
      case 12: run_chunk_fixed<12>(sh, psi, tau0, grp.chunk_tiles, init, L, H, hb, choff, pops, ps.op_count, mats, pre, tabs, swp, ps.g.nswap, swk); break;
      case 11: run_chunk_fixed<11>(sh, psi, tau0, grp.chunk_tiles, init, L, H, hb, choff, pops, ps.op_count, mats, pre, tabs, swp, ps.g.nswap, swk); break;
      default: run_chunk_var(sh, psi, tau0, grp.chunk_tiles, init, b, L, H, hb, choff, pops, ps.op_count, mats, swp, ps.g.nswap); break;
    }
    __syncthreads();
  }
}

// out[c * m + k] = amplitude idx[c * m + k] of circuit c (FP64 pairs);
// logical bit q of the index sits at physical bit pos[c * 32 + q].
__global__ __launch_bounds__(kThreads) void k_batch_gather(const char* __restrict__ states,
                                                           const uint64_t* __restrict__ state_off,
                                                           const int32_t* __restrict__ nq,
                                                           const int8_t* __restrict__ pos, int count,
                                                           int m, const uint64_t* __restrict__ idx,
                                                           double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= (long long)count * m) return;
  const int c = (int)(k / m);
  const uint64_t z = idx[k];
  const int n = nq[c];
  if ((z >> n) != 0) {
    out[2 * k] = out[2 * k + 1] = __builtin_nan("");
    return;
  }
  uint64_t p = 0;
  for (int q = 0; q < n; ++q) p |= ((z >> q) & 1) << pos[(size_t)c * 32 + q];
  const cplx<float> v = reinterpret_cast<const cplx<float>*>(states + state_off[c])[p];
  out[2 * k] = (double)v.re;
  out[2 * k + 1] = (double)v.im;
}

// One block per circuit: sum |psi|^2 in FP64 with a fixed order.
__global__ __launch_bounds__(kThreads) void k_batch_norms(const char* __restrict__ states,
                                                          const uint64_t* __restrict__ state_off,
                                                          const int32_t* __restrict__ nq,
                                                          double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  const int c = blockIdx.x;
  const cplx<float>* psi = reinterpret_cast<const cplx<float>*>(states + state_off[c]);
  const uint64_t count = uint64_t(1) << nq[c];
  double acc = 0.0;
  for (uint64_t i = threadIdx.x; i < count; i += kThreads) {
    const cplx<float> v = psi[i];
    acc += (double)v.re * v.re + (double)v.im * v.im;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
    out[c] = r;
  }
}

// Per-part bitstrings z_p of Eq. (3), each mapped through its part state's
// layout: zp[p count + k] (one thread per bitstring).
// A bitstring with a bit at or above n sets *bad.
__global__ __launch_bounds__(kThreads) void k_branch_split(const uint64_t* __restrict__ z, int words,
                                                           long long count, int P, int n,
                                                           const int32_t* __restrict__ tab,
                                                           uint32_t* __restrict__ zp, int* __restrict__ bad) {
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= count) return;
  const uint64_t* row = z + k * words;
  uint64_t w[kBranchMaxWords];
  uint64_t over = 0;
#pragma unroll
  for (int i = 0; i < kBranchMaxWords; ++i) {
    w[i] = i < words ? row[i] : 0;
    const int lo = n - 64 * i;  // bits of word i below n
    over |= lo >= 64 ? 0 : lo <= 0 ? w[i] : w[i] >> lo;
  }
  if (over) atomicOr(bad, 1);
  const int32_t* qs = tab + kBranchMaxParts + 1;
  const int32_t* phys = qs + kBranchMaxQubits;
  for (int p = 0; p < P; ++p) {
    uint32_t v = 0;
    for (int i = tab[p]; i < tab[p + 1]; ++i) {
      const int q = qs[i], wi = q >> 6;  // wave-uniform
      const uint64_t x = wi == 0 ? w[0] : wi == 1 ? w[1] : wi == 2 ? w[2] : w[3];
      v |= (uint32_t)((x >> (q & 63)) & 1) << phys[i];
    }
    zp[(size_t)p * count + k] = v;
  }
}

// Eq. (3) over one group of g branches, one thread per bitstring: the
// product over parts in FP64 (p = 0..P-1), added to acc for j = 0..g-1 in
// order, so the sum over all groups runs in one order whatever the group
// size.  tab[j P + p] is the state holding part p of branch j (wave-uniform
// loads).
__global__ __launch_bounds__(kThreads) void k_branch_gather_accum(
    const char* __restrict__ states, const uint64_t* __restrict__ state_off, int P, long long g,
    const int32_t* __restrict__ tab, const uint32_t* __restrict__ zp, long long count,
    double* __restrict__ acc, int last, double scale) {
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= count) return;
  uint32_t zi[kBranchMaxParts];
#pragma unroll
  for (int p = 0; p < kBranchMaxParts; ++p) zi[p] = p < P ? zp[(size_t)p * count + k] : 0u;
  double re = acc[2 * k], im = acc[2 * k + 1];
  // prefix products over the parts, recomputed from the first part whose
  // state differs from the previous branch's (as in k_branch_sum_lds)
  double pr[kBranchMaxParts], pi[kBranchMaxParts];
  for (long long j = 0; j < g; ++j) {
    const int32_t* t = tab + j * P;
    int p0 = 0;
    if (j > 0)
      while (p0 < P && t[p0] == t[p0 - P]) ++p0;  // wave-uniform
#pragma unroll
    for (int p = 0; p < kBranchMaxParts; ++p) {
      if (p < p0) continue;
      if (p < P) {
        const cplx<float> b = reinterpret_cast<const cplx<float>*>(states + state_off[t[p]])[zi[p]];
        if (p == 0) {
          pr[0] = b.re;
          pi[0] = b.im;
        } else {
          const double br = b.re, bi = b.im;
          pr[p] = pr[p - 1] * br - pi[p - 1] * bi;
          pi[p] = pr[p - 1] * bi + pi[p - 1] * br;
        }
      } else {
        pr[p] = pr[p - 1];
        pi[p] = pi[p - 1];
      }
    }
    re += pr[kBranchMaxParts - 1];
    im += pi[kBranchMaxParts - 1];
  }
  if (last) {
    re *= scale;
    im *= scale;
  }
  acc[2 * k] = re;
  acc[2 * k + 1] = im;
}

// The same sum from LDS: each thread first gathers its coefficient's
// amplitude of every state of the group (at most kBranchSumValues) into its
// own LDS column (conflict-free: value c of thread t at c * threads + t),
// then runs the branches from there.  Threads share nothing, so there is no
// barrier.  Same arithmetic, in the same order, as k_branch_gather_accum.
__global__ __launch_bounds__(kBranchSumThreads) void k_branch_sum_lds(
    const char* __restrict__ states, const uint64_t* __restrict__ state_off, int P, BranchParts bp,
    long long g, const uint64_t* __restrict__ tab8, const uint32_t* __restrict__ zp, long long count,
    double* __restrict__ acc, int last, double scale) {
  extern __shared__ cplx<float> vals[];
  const int tid = threadIdx.x;
  const long long k = (long long)blockIdx.x * kBranchSumThreads + tid;
  if (k >= count) return;
#pragma unroll
  for (int p = 0; p < kBranchMaxParts; ++p) {
    if (p < P) {
      const uint32_t zi = zp[(size_t)p * count + k];
      for (int c = bp.first[p]; c < bp.first[p + 1]; ++c)
        vals[c * kBranchSumThreads + tid] = reinterpret_cast<const cplx<float>*>(states + state_off[c])[zi];
    }
  }
  double re = acc[2 * k], im = acc[2 * k + 1];
  // Prefix products over the parts, kept from branch to branch: branch j
  // recomputes them only from the first part whose state differs from
  // branch j-1's (a wave-uniform test on the table words), so parts whose
  // crossings come early are multiplied once per run of branches.  The
  // products are the same values, in the same order, as in
  // k_branch_gather_accum.  Entries past the last part repeat the full
  // product, so it is always pr[kBranchMaxParts - 1].
  double pr[kBranchMaxParts], pi[kBranchMaxParts];
  uint64_t prev = 0;
  for (long long j = 0; j < g; ++j) {
    const uint64_t t = tab8[j];
    const uint64_t diff = t ^ prev;
    const int p0 = j == 0 ? 0 : diff ? __builtin_ctzll(diff) >> 3 : kBranchMaxParts;
    prev = t;
#pragma unroll
    for (int p = 0; p < kBranchMaxParts; ++p) {
      if (p < p0) continue;
      if (p < P) {
        const cplx<float> b = vals[(int)((t >> (8 * p)) & 0xff) * kBranchSumThreads + tid];
        if (p == 0) {
          pr[0] = b.re;
          pi[0] = b.im;
        } else {
          const double br = b.re, bi = b.im;
          pr[p] = pr[p - 1] * br - pi[p - 1] * bi;
          pi[p] = pr[p - 1] * bi + pi[p - 1] * br;
        }
      } else {
        pr[p] = pr[p - 1];
        pi[p] = pi[p - 1];
      }
    }
    re += pr[kBranchMaxParts - 1];
    im += pi[kBranchMaxParts - 1];
  }
  if (last) {
    re *= scale;
    im *= scale;
  }
  acc[2 * k] = re;
  acc[2 * k + 1] = im;
}

}  // namespace

int batch_max_bits() { return kBatchMaxBits; }
int batch_mma_cap() { return kBatchTabs; }
int batch_max_gather() { return kBatchGather; }

hipError_t launch_batch(char* states, const BatchDevice& d, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3((d.nrounds + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     (unsigned long long*)d.tickets, d.nrounds);
  static uint64_t slots = 0;
  if (slots == 0) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_batch, kBatchThreads, 0) !=
            hipSuccess ||
        per < 1)
      per = 1;
    slots = (uint64_t)cus * per;
  }
  for (int r = 0; r < d.nrounds; ++r) {
    const long long c0 = d.round_chunk[r], c1 = d.round_chunk[r + 1];
    if (c1 <= c0) continue;
    const uint64_t grid = (uint64_t)(c1 - c0) < slots ? (uint64_t)(c1 - c0) : slots;
    hipLaunchKernelGGL(k_batch, dim3((unsigned)grid), dim3(kBatchThreads), 0, s, states, d.groups,
                       d.round_group[r], d.round_group[r + 1], d.passes, d.ops, d.mats,
                       (unsigned long long*)d.tickets + r, c0, c1);
  }
  return hipGetLastError();
}

hipError_t launch_batch_gather(const char* states, const uint64_t* state_off, const int32_t* nq,
                               const int8_t* pos, int count, int m, const uint64_t* idx, double* out,
                               hipStream_t s) {
  const long long total = (long long)count * m;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_gather, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, states, state_off, nq, pos, count, m, idx, out);
  return hipGetLastError();
}

hipError_t launch_batch_norms(const char* states, const uint64_t* state_off, const int32_t* nq,
                              int count, double* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_norms, dim3(count), dim3(kThreads), 0, s, states, state_off, nq, out);
  return hipGetLastError();
}

hipError_t launch_branch_split(const uint64_t* z, int words, long long count, int P, int n,
                               const int32_t* tab, uint32_t* zp, int* bad, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (words < 1 || words > kBranchMaxWords || P < 1 || P > kBranchMaxParts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_branch_split, dim3((unsigned)((count + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, z, words, count, P, n, tab, zp, bad);
  return hipGetLastError();
}

hipError_t launch_branch_gather_accum(const char* states, const uint64_t* state_off, int P,
                                      long long g, const int32_t* tab, const uint32_t* zp,
                                      long long count, double* acc, bool last, double scale,
                                      hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (P < 1 || P > kBranchMaxParts || g < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_branch_gather_accum, dim3((unsigned)((count + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, states, state_off, P, g, tab, zp, count, acc, last ? 1 : 0,
                     scale);
  return hipGetLastError();
}

hipError_t launch_branch_sum_lds(const char* states, const uint64_t* state_off, int P,
                                 const BranchParts& parts, long long g, const uint64_t* tab8,
                                 const uint32_t* zp, long long count, double* acc, bool last,
                                 double scale, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (P < 1 || P > kBranchMaxParts || g < 1) return hipErrorInvalidValue;
  const int values = parts.first[P];
  if (values < 1 || values > kBranchSumValues || parts.first[0] != 0) return hipErrorInvalidValue;
  for (int p = 0; p < P; ++p)
    if (parts.first[p + 1] < parts.first[p]) return hipErrorInvalidValue;
  const size_t lds = (size_t)values * kBranchSumThreads * sizeof(cplx<float>);
  hipLaunchKernelGGL(k_branch_sum_lds, dim3((unsigned)((count + kBranchSumThreads - 1) / kBranchSumThreads)),
                     dim3(kBranchSumThreads), lds, s, states, state_off, P, parts, g, tab8, zp, count, acc,
                     last ? 1 : 0, scale);
  return hipGetLastError();
}

}  // namespace juqcs
