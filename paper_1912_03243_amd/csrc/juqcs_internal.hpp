// Internal declarations shared by the kernel translation units and the
// host-side engine of libjuqcs_gpu.  Not installed; the public interface is
// include/juqcs_gpu.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "juqcs_gpu.h"

namespace juqcs {

// ---------------------------------------------------------------------------
// Complex arithmetic on interleaved (re, im) storage.  The alignment makes a
// C128 amplitude one 16-byte load and a C64 amplitude one 8-byte load.
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a*b as four fused multiply-adds (one rounding each)
template <typename T>
__host__ __device__ inline cplx<T> cmad(cplx<T> a, cplx<T> b, cplx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}

template <typename T>
struct Mat2 {
  cplx<T> m[4];  // row-major
};
template <typename T>
struct Mat4 {
  cplx<T> m[16];  // row-major, index b_q0 + 2 b_q1
};

// Streaming accesses to state vectors: non-temporal, so data a pass touches
// once does not evict from L2 the coefficients and tables it keeps
// re-reading.  V is a scalar or a clang vector type.
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  return __builtin_nontemporal_load(p);
}
template <typename V>
__device__ __forceinline__ void st_stream(V* p, V v) {
  __builtin_nontemporal_store(v, p);
}

template <typename T>
__device__ __forceinline__ cplx<T> ld_amp(const cplx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return cplx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_amp(cplx<T>* p, cplx<T> a) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2{a.re, a.im}, reinterpret_cast<v2*>(p));
}

// Insert a zero bit at position pos of x (bits >= pos move up by one).
__host__ __device__ inline uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t low = x & ((uint64_t(1) << pos) - 1);
  return ((x >> pos) << (pos + 1)) | low;
}

// ---------------------------------------------------------------------------
// Tile passes: 2^b amplitudes per workgroup, made of 2^H chunks of 2^L
// contiguous amplitudes; local index bit j < L is physical bit j, local bit
// L + i is physical bit hbits[i].  Ops act on local bits.
// ---------------------------------------------------------------------------
constexpr int kMaxGather = 10;  // gathered chunk bits of a tile pass
constexpr int kPassOps = 48;    // most ops the planner puts in one pass
constexpr int kHbitsCap = 12;   // fused blocks reuse the struct: 2k <= 12
constexpr int kSwapCap = 8;     // relabel swaps at the end of one pass

struct TileGeom {
  int32_t n, L, H, b;
  int32_t hbits[kHbitsCap];      // ascending physical positions (>= L)
  int32_t block_bits;            // ENC2 only
  int32_t maxk;                  // widest op of the pass (1..4)
  int32_t mat_count;             // coefficients of the pass's ops, from ops[0].moff on
  int32_t mma_count;             // 8x8 (TOP_DENSE3) ops of the pass
  // Relabeling (C128 / C64 only): after its ops the pass writes the tile
  // back with local bits swap_a[i] and swap_b[i] exchanged (disjoint pairs),
  // i.e. the qubits at those two physical positions trade places.
  int32_t nswap;
  int8_t swap_a[kSwapCap], swap_b[kSwapCap];
};

// Local index after the pass's relabel swaps (an involution: the swaps are
// disjoint transpositions of bit positions).
// The loop has a fixed trip count so that a kernel reads the pairs from its
// argument block with constant offsets (no vector memory loads).
__host__ __device__ inline int swap_local(int e, const TileGeom& g) {
  for (int i = 0; i < kSwapCap; ++i) {
    if (i < g.nswap) {
      const int a = g.swap_a[i], c = g.swap_b[i];
      const int x = ((e >> a) ^ (e >> c)) & 1;
      e ^= (x << a) | (x << c);
    }
  }
  return e;
}

enum TileOpKind : int32_t {
  TOP_DENSE1 = 0,  // 2x2 on local bit a
  TOP_DENSE2 = 1,  // 4x4 on local bits (a, b), index b_a + 2 b_b
  TOP_DIAG2 = 2,   // phases d[b_a + 2 b_b] (b may equal -1: d[b_a])
  TOP_DENSE3 = 3,  // 8x8 on local bits bits[0..3) (matrix order)
  TOP_DENSE4 = 4,  // 16x16 on local bits bits[0..4)
  TOP_PERM = 5,    // monomial on local bits bits[0..k), k <= 3: out[r] =
                   // c[r] in[sigma(r)], sigma(r) in bits 3r..3r+2 of a
  TOP_DENSE3G = 6, // 8x8 on bits[0..3) in three-product form (FP64 pipelined
                   // kernels only): per row r, 24 reals Re m_r., (Re + Im) m_r.,
                   // (Im - Re) m_r.
};

struct TileOp {
  int32_t kind;
  int32_t a, b;
  int32_t k;
  int32_t bits[4];
  int64_t moff;  // offset of the matrix in the complex coefficient array
};

// A tile pass: geometry plus a range of ops.
struct TilePass {
  TileGeom g;
  int32_t op_begin, op_count;
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All asynchronous on stream.
// Return hipSuccess or the launch error.
// ---------------------------------------------------------------------------
hipError_t launch_init(juqcs_dtype dt, void* amps, void* scales, int n,
                       int block_bits, uint64_t idx, hipStream_t s);
hipError_t launch_1q(juqcs_dtype dt, void* amps, int n, int t, int c,
                     const cplx<double> u[4], hipStream_t s);
hipError_t launch_diag(juqcs_dtype dt, void* amps, int n, uint64_t mask,
                       cplx<double> phase, hipStream_t s);
hipError_t launch_2q(juqcs_dtype dt, void* amps, int n, int q0, int q1,
                     const cplx<double> m[16], hipStream_t s);
hipError_t launch_norm(juqcs_dtype dt, const void* amps, const void* scales,
                       int n, int block_bits, double* partials, double* out,
                       hipStream_t s);
hipError_t launch_gather(juqcs_dtype dt, const void* amps, const void* scales,
                         int n, int block_bits, const uint64_t* idx,
                         uint64_t count, const int8_t* phys, cplx<double> g, double* out,
                         hipStream_t s);
hipError_t launch_scale(juqcs_dtype dt, void* amps, void* scales, int n,
                        int block_bits, double f, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Zeroes bytes (a multiple of 4, 4-byte aligned) with a kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

hipError_t launch_tile(juqcs_dtype dt, void* amps, void* scales,
                       const TileGeom& g, const TileOp* d_ops, int nops,
                       const void* d_mats, hipStream_t s);
// Whether launch_tile runs a pass on a pipelined (fixed tile size) kernel.
bool tile_pipelined(juqcs_dtype dt, const TileGeom& g, int nops);
int tile_max_bits(juqcs_dtype dt);
// Expectation values of sigma^x,y,z for the tile bits jlo..b-1 of geometry
// g (b <= expect_max_bits(), at most 16 bits per launch):
// out3[3 (j - jlo) + c].  partials: expect_partials_bytes() of device memory.
int expect_max_bits();
size_t expect_partials_bytes();
hipError_t launch_expect(juqcs_dtype dt, const void* amps, const void* scales, const TileGeom& g,
                         int jlo, double* partials, double* out3, hipStream_t s);

// What a pass of 2^b-amplitude tiles may carry so that it runs on the
// pipelined kernel: coefficients (staged in LDS by the two-byte kernels) and
// 8x8 ops (whose tables the FP32 kernels build in LDS); 0 = no limit.
int tile_mat_cap(juqcs_dtype dt, int b);
int tile_mma_cap(juqcs_dtype dt, int b);

hipError_t launch_fused(juqcs_dtype dt, void* amps, int n, int k,
                        const int* targets, const void* d_mat, juqcs_mma mode,
                        hipStream_t s);

hipError_t launch_encode2(const void* src, juqcs_dtype sdt, uint64_t count,
                          int block_bits, void* codes, void* scales,
                          hipStream_t s);
hipError_t launch_decode2(const void* codes, const void* scales,
                          uint64_t count, int block_bits, void* dst,
                          juqcs_dtype ddt, hipStream_t s);
// ---------------------------------------------------------------------------
// Batches (k_batch.hip, batch.cpp)
// ---------------------------------------------------------------------------
struct BatchPass {  // one tile pass of one circuit
  TileGeom g;
  int32_t op_begin, op_count;
};

struct BatchGroup {  // every tile of one pass of one circuit
  uint64_t state_off;    // byte offset of the circuit's C64 state
  int64_t first_chunk;   // first ticket of this group
  int32_t circuit;
  int32_t pass;          // index into the BatchPass array
  int32_t chunk_tiles;   // tiles claimed per ticket
  int32_t init;          // 1: start from |0...0> instead of loading
};

struct BatchDevice {
  const BatchGroup* groups;
  int ngroups;
  const BatchPass* passes;
  const TileOp* ops;
  const cplx<float>* mats;
  uint64_t* tickets;               // one counter per round (device)
  int nrounds;                     // round r: pass r of every circuit that has one
  std::vector<int32_t> round_group;    // host: first group of each round (+ end)
  std::vector<int64_t> round_chunk;    // host: first chunk of each round (+ end)
  int count;
  long long nchunks;
};

int batch_max_bits();
int batch_mma_cap();  // 8x8 ops per pass whose tables the batch kernel holds in LDS
int batch_max_gather();  // most gathered chunk bits of a batch pass
hipError_t launch_batch(char* states, const BatchDevice& d, hipStream_t s);
hipError_t launch_batch_gather(const char* states, const uint64_t* state_off, const int32_t* nq,
                               const int8_t* pos, int count, int m, const uint64_t* idx, double* out,
                               hipStream_t s);
hipError_t launch_batch_norms(const char* states, const uint64_t* state_off, const int32_t* nq,
                              int count, double* out, hipStream_t s);

// Entangling-gate decomposition (Eq. (3)) on the device.
constexpr int kBranchMaxParts = 8;    // parts of a decomposition
constexpr int kBranchMaxQubits = 240; // kBranchMaxParts parts of at most 30 qubits
constexpr int kBranchMaxWords = 4;    // 64-bit words per bitstring
// Bitstring split table (int32 entries): [0, P] part starts into the qubit
// lists, then kBranchMaxQubits qubit numbers (part by part, ascending), then
// the physical bit of each in its part state.
constexpr int kBranchTabInts = kBranchMaxParts + 1 + 2 * kBranchMaxQubits;
// Sets *bad (device int) when a bitstring has a bit at or above n.
hipError_t launch_branch_split(const uint64_t* z, int words, long long count, int P, int n,
                               const int32_t* tab, uint32_t* zp, int* bad, hipStream_t s);
// acc[k] += sum over the group's g branches (in order) of prod_p
// psi_{tab[j P + p]}[zp[p count + k]] (FP64); the last group multiplies by
// scale.  States are read where they lie.
hipError_t launch_branch_gather_accum(const char* states, const uint64_t* state_off, int P,
                                      long long g, const int32_t* tab, const uint32_t* zp,
                                      long long count, double* acc, bool last, double scale,
                                      hipStream_t s);
// The same sum when the group has at most kBranchSumValues states, stored
// part by part (part p: circuits first[p] .. first[p + 1]): every thread
// gathers its coefficient's amplitude of each state into LDS once, then sums
// the branches from there; byte p of tab8[j] is branch j's circuit of part p.
constexpr int kBranchSumValues = 48;
constexpr int kBranchSumThreads = 128;
struct BranchParts {
  int32_t first[kBranchMaxParts + 1];
};
hipError_t launch_branch_sum_lds(const char* states, const uint64_t* state_off, int P,
                                 const BranchParts& parts, long long g, const uint64_t* tab8,
                                 const uint32_t* zp, long long count, double* acc, bool last,
                                 double scale, hipStream_t s);

// ---------------------------------------------------------------------------
// Host-side planning (planner.cpp)
// ---------------------------------------------------------------------------
struct Gate {  // decoded gate: matrix on 1 or 2 qubits (physical positions)
  int nq;
  int q[2];
  cplx<double> m[16];  // 2x2 (first 4) or 4x4, index b_q0 + 2 b_q1
  bool diag;
};

bool decode_gate(const juqcs_gate& g, int n, Gate* out, std::string* err);
// Algorithmic flops per state amplitude of a gate (planner.cpp).
double gate_flops(const Gate& g);

struct TilePlan {
  std::vector<TilePass> passes;
  std::vector<TileOp> ops;
  std::vector<cplx<double>> mats;
  // for every op: the gates folded into it, in merge order, so the matrices
  // can be rebuilt for gates with other values but the same structure
  std::vector<std::vector<int>> op_gates;
  int64_t gates = 0;
};

// Recomputes every op matrix of plan from gates (same qubits and zero
// pattern as the gates the plan was made for).
void rebuild_mats(const std::vector<Gate>& gates, TilePlan* plan);

// Tile selection alone: the passes (geometry) and the gates each absorbs.
struct TileSchedule {
  std::vector<TilePass> passes;
  std::vector<std::vector<int>> taken;
  int64_t gates = 0;
  // Relabeling schedules only: the absorbed gates on the physical bits of
  // their pass (taken indexes these), the index of each in the input gate
  // list, and final_pos[p] = where the qubit at physical bit p before the
  // schedule sits after it.
  std::vector<Gate> tgates;
  std::vector<int> tsrc;
  std::vector<int> final_pos;
};
// max_take > 0 caps the gates one pass absorbs (later gates wait for the
// next pass), which moves on-chip work from crowded passes to light ones.
void select_tiles(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                  TileSchedule* sched, int max_take = 0);
// Same with relabeling: between passes, qubits of the finished tile may take
// over the low L physical bits (swapped in by the finished pass's store), so
// that the next tile is any b qubits of which at least L were in the
// finished one.  Fills sched->tgates and sched->final_pos.
void select_tiles_relabel(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                          TileSchedule* sched, int max_take = 0);
// Fuses every pass's gates into ops of at most kin qubits.  A pass whose
// coefficients would exceed max_mats (> 0), or whose 8x8 ops would exceed
// max_mma (> 0), is split into consecutive passes of the same geometry (the
// relabel swaps go with the last of them).  taken indexes sched.tgates when
// that is non-empty, else gates; plan->op_gates index the same vector.
void emit_schedule(const TileSchedule& sched, const std::vector<Gate>& gates, int kin,
                   TilePlan* plan, int max_mats = 0, int max_mma = 0);

// Plans tile passes for gates (physical qubits).  L, b: low contiguous bits
// and total tile bits; the low L bits are always tile bits.
// relabel: plan with select_tiles_relabel; *final_pos (if given) receives
// the schedule's final_pos (identity without relabeling).
void plan_tiles(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                TilePlan* plan, int kin = 2, int max_mats = 0, int max_take = 0,
                int max_mma = 0, bool relabel = false, std::vector<int>* final_pos = nullptr);

struct FusedBlock {
  std::vector<int> targets;           // physical
  std::vector<cplx<double>> m;        // 2^k x 2^k
};
void plan_fused(int n, int kmax, const std::vector<Gate>& gates,
                std::vector<FusedBlock>* blocks);

void set_error(const std::string& msg);

}  // namespace juqcs
