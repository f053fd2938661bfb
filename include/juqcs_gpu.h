/*
 * juqcs_gpu -- state-vector gate engine for one AMD MI355X (gfx950).
 *
 * The hot path of a universal quantum computer simulator in the sense of
 * Willsch et al., "Benchmarking Supercomputers with the Juelich Universal
 * Quantum Computer Simulator" (arXiv:1912.03243):  sparse 1- and 2-qubit
 * gates applied to the full vector of 2^n complex amplitudes, each gate one
 * memory-bound pass (Section 2, Eq. (1)); a two-byte amplitude coding
 * (Section 1); and the entangling-gate decomposition into a sum over
 * branches (Section 4, Eqs. (2) and (3)).
 *
 * Conventions used by every call
 *   - qubit q is bit q of the amplitude index (little endian); qubit
 *     arguments are logical qubits, 0 <= q < n;
 *   - complex numbers are (re, im) pairs of doubles on the host side;
 *   - a 2x2 matrix u[8] is row-major: u = {U00re,U00im, U01re,U01im,
 *     U10re,U10im, U11re,U11im}; it acts as in Eq. (1): for every index i
 *     with bit t clear and j = i + 2^t, (psi_i, psi_j) <- U (psi_i, psi_j);
 *   - a 2^k x 2^k matrix m has row/column index r = sum_j b_{targets[j]} 2^j,
 *     row-major, (re, im) pairs: m[2*(row*2^k + col) + {0,1}];
 *   - the library never allocates device memory: every device buffer,
 *     workspaces included, is the caller's (sizing calls give the sizes),
 *     borrowed and never freed by the library; the caller keeps it alive
 *     until the handle using it is destroyed;
 *   - host arrays passed in are copied before the call returns;
 *   - every apply call is asynchronous on the handle's HIP stream; calls that
 *     return host data (amplitudes, norm, expectations) synchronise it;
 *   - every function returns a juqcs_status; arguments are validated on the
 *     host before anything is launched, and the library never aborts.
 *     Asynchronous device errors surface at the next synchronising call as
 *     JUQCS_ERR_HIP.  juqcs_last_error() returns a message for the last
 *     non-OK status of the calling thread;
 *   - a handle is not thread-safe; separate handles are independent.
 */
#ifndef JUQCS_GPU_H
#define JUQCS_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JUQCS_OK = 0,
  JUQCS_ERR_ARG = -1,         /* null pointer, bad count, bad option        */
  JUQCS_ERR_QUBIT = -2,       /* qubit out of range or repeated             */
  JUQCS_ERR_DTYPE = -3,       /* operation not defined for this amplitude type */
  JUQCS_ERR_SIZE = -4,        /* buffer smaller than juqcs_state_bytes says */
  JUQCS_ERR_HIP = -5,         /* HIP runtime error (message has the text)   */
  JUQCS_ERR_UNSUPPORTED = -6, /* valid request this build does not support  */
  JUQCS_ERR_NUMERIC = -7      /* non-finite matrix entry or non-finite norm */
} juqcs_status;

/* Amplitude storage.  C128: FP64 complex, 16 B/amp (the paper's numerically
 * exact form, Section 1).  C64: FP32 complex, 8 B/amp.  ENC2: the two-byte
 * form (Section 1 says only "adaptive coding", two bytes per amplitude; this
 * library defines it): blocks of 2^B consecutive amplitudes share one FP32
 * scale s = max |component|; each component is int8 q = rint(x * fl(127/s)),
 * decoded as q * fl(s/127).  Gate arithmetic on ENC2 states is FP32. */
typedef enum { JUQCS_C128 = 0, JUQCS_C64 = 1, JUQCS_ENC2 = 2 } juqcs_dtype;

/* Arithmetic of a fused dense block (juqcs_apply_fused_k). */
typedef enum {
  JUQCS_MMA_FP64 = 0,   /* FP64 matrix cores (C128 states)                 */
  JUQCS_MMA_FP32 = 1,   /* FP32 matrix cores (C64 states)                  */
  JUQCS_MMA_BF16 = 2,   /* BF16 inputs, FP32 accumulation (C64 states)     */
  JUQCS_MMA_BF16X3 = 3, /* hi/lo BF16 split, three products, FP32 accum.,
                           about 17 significant bits per pass        */
  JUQCS_MMA_AUTO = 4    /* FP64 for C128, FP32 for C64                     */
} juqcs_mma;

/* Gate record: the unit of a circuit handed to juqcs_run_circuit and the
 * batch / branch calls.  88 bytes, naturally aligned. */
typedef enum {
  JUQCS_OP_H = 0, JUQCS_OP_X = 1, JUQCS_OP_Y = 2, JUQCS_OP_Z = 3,
  JUQCS_OP_S = 4, JUQCS_OP_T = 5,
  JUQCS_OP_U = 6,    /* arbitrary 2x2 in u[8] on q0                            */
  JUQCS_OP_CNOT = 7, /* control q0, target q1 (Section 3: "(CNOT i i+1)")      */
  JUQCS_OP_CZ = 8,   /* sign flip where q0 and q1 are both 1 (Section 4)       */
  JUQCS_OP_CP = 9    /* phase e^{i theta} where q0 and q1 are both 1           */
} juqcs_op;

typedef struct {
  int32_t op;     /* juqcs_op                                   */
  int32_t q0;     /* target (1q), control (CNOT), first qubit   */
  int32_t q1;     /* target (CNOT), second qubit (CZ, CP); -1 for 1q */
  int32_t pad;
  double theta;   /* CP angle                                   */
  double u[8];    /* JUQCS_OP_U matrix                          */
} juqcs_gate;

typedef struct juqcs_state juqcs_state; /* opaque host-side handle */

/* ------------------------------------------------------------------------
 * Sizing and lifetime
 * ---------------------------------------------------------------------- */

/* Bytes of device memory a state needs.  amp_bytes: 2^n amplitudes
 * (16, 8 or 2 bytes each).  scale_bytes: ENC2 scales, 4 * ceil(2^n / 2^B)
 * (0 for C128/C64).  work_bytes: library workspace (gate programs, partial
 * sums, index lists).  block_bits B is used for ENC2 only (0 = default 8,
 * else 4..12).  1 <= n <= 40.  Errors: JUQCS_ERR_ARG. */
juqcs_status juqcs_state_bytes(int n, juqcs_dtype dtype, int block_bits,
                               size_t* amp_bytes, size_t* scale_bytes,
                               size_t* work_bytes);

/* Wrap caller-owned device buffers (sizes at least those of
 * juqcs_state_bytes; d_scales may be NULL unless ENC2; d_work is required,
 * 256-byte aligned: the library never allocates device memory).  hip_stream
 * is a hipStream_t (NULL = default stream).  The amplitudes are not
 * initialised: call juqcs_state_init.  Errors: ARG (null or misaligned
 * buffer), SIZE (buffer smaller than juqcs_state_bytes says), DTYPE. */
juqcs_status juqcs_state_create(juqcs_state** out, int n, juqcs_dtype dtype,
                                int block_bits, void* d_amps, size_t amp_bytes,
                                void* d_scales, size_t scale_bytes,
                                void* d_work, size_t work_bytes,
                                void* hip_stream);

/* Releases the handle (not the caller's buffers). NULL is accepted. */
juqcs_status juqcs_state_destroy(juqcs_state* st);

/* psi = |basis_index> (the computer starts in |0...0>, Section 4 before
 * Eq. (3)); resets the qubit permutation to identity and the global factor
 * to 1.  Errors: ARG. */
juqcs_status juqcs_state_init(juqcs_state* st, uint64_t basis_index);

/* Switch the handle's stream. */
juqcs_status juqcs_state_set_stream(juqcs_state* st, void* hip_stream);

/* ------------------------------------------------------------------------
 * Single gates (Section 2, Eq. (1)); one pass over the touched amplitudes
 * ---------------------------------------------------------------------- */

/* Eq. (1) on target t.  A diagonal matrix diag(a, b) with a != 0 is applied
 * as a diag(1, b/a): the factor a goes into the state's FP64 global factor
 * (juqcs_get_global_factor) and only the amplitudes with bit t set are
 * touched.  Errors: QUBIT, ARG (null u), NUMERIC. */
juqcs_status juqcs_apply_1q(juqcs_state* st, int t, const double u[8]);

/* Controlled-U: Eq. (1) on target t for the indices whose bit c is 1
 * (CNOT = controlled-X, CZ = controlled-Z; Sections 3 and 4).
 * Errors: QUBIT (c == t or out of range), ARG, NUMERIC. */
juqcs_status juqcs_apply_controlled(juqcs_state* st, int c, int t, const double u[8]);

/* General two-qubit gate, 4x4 matrix with row/col index b_q0 + 2 b_q1.
 * Errors: QUBIT, ARG, NUMERIC. */
juqcs_status juqcs_apply_2q(juqcs_state* st, int q0, int q1, const double m[32]);

/* Dense 2^k x 2^k block on k distinct targets (1 <= k <= 6), applied as a
 * dense contraction [2^k x 2^k] x [2^k x 2^(n-k)] on the matrix cores.
 * mode: FP64 for C128; FP32, BF16 or BF16X3 (FP32 accumulation) for C64;
 * AUTO picks FP64 / FP32.  ENC2: JUQCS_ERR_DTYPE.  Errors: QUBIT, ARG,
 * DTYPE, NUMERIC. */
juqcs_status juqcs_apply_fused_k(juqcs_state* st, int k, const int* targets,
                                 const double* m, juqcs_mma mode);

/* ------------------------------------------------------------------------
 * Whole circuits through the planner
 * ---------------------------------------------------------------------- */
typedef enum {
  JUQCS_PLAN_PLAIN = 0, /* one kernel pass per gate (the paper's scheme)   */
  JUQCS_PLAN_TILE = 1,  /* on-chip tile passes: every gate whose qubits lie
                           in the chosen tile bits is applied in LDS, one
                           HBM read+write per pass                        */
  JUQCS_PLAN_FUSED = 2, /* greedy fusion into dense k-qubit blocks applied
                           with juqcs_apply_fused_k's kernels             */
  JUQCS_PLAN_AUTO = 3   /* the options juqcs_autotune stored for a circuit
                           of this structure, else TILE with its defaults */
} juqcs_plan_mode;

typedef struct {
  int32_t mode;        /* juqcs_plan_mode                                */
  int32_t fuse_k;      /* FUSED: block width 2..6 (0 = 5).  TILE: widest
                          fused op inside a pass, 1..4 (0 = 3)            */
  int32_t mma;         /* FUSED: juqcs_mma                                */
  int32_t tile_bits;   /* TILE: total tile bits (0 = default for dtype)   */
  int32_t low_bits;    /* TILE: contiguous low bits per chunk (0 = default) */
  int32_t profile;     /* 1: time every pass with HIP events on the state's
                          stream (the call then synchronises the stream)   */
  int32_t autotune;    /* batches: 1 = pick the on-chip fusion width per
                          qubit count from timed trial runs (the trials
                          use the batch's state buffer); 0 = cost model  */
  int32_t pass_gates;  /* TILE: most gates one pass may absorb; -1 = no
                          limit; 0 = the planner's choice (no limit for
                          C128; for C64 and ENC2 the limit its cost model
                          prefers, which spreads on-chip work over passes) */
  int32_t relabel;     /* TILE: 0 or 1 = a pass may hand the
                          low (contiguous) physical bits to other qubits of
                          its tile as it writes the tile back (qubit
                          relabeling at no extra pass), so that the next
                          tile may be any qubits and fewer passes over the
                          state are needed (Section 2: the update is bound
                          by memory bandwidth).  The state is then left in
                          another physical layout: read-outs are in logical
                          terms, juqcs_get_layout shows it.  -1 = off
                          (layout unchanged).                             */
  /* outputs */
  int64_t passes;      /* kernel passes over the state that were launched */
  int64_t gates;       /* gate records consumed                           */
  double kernel_ms;    /* profile: summed device durations of the passes  */
  double bytes;        /* algorithmic HBM bytes of the passes: read + write
                          of every amplitude (and ENC2 scale) a pass must
                          touch (a 16-byte word counts whole)              */
  double flops;        /* algorithmic flops of the gates consumed, per
                          gate and state amplitude: dense 2x2 14, diagonal
                          3 (first entry 1) or 6, controlled 7, controlled
                          diagonal 1.5 (sign flip 0.5), CNOT 0, dense 4x4 30 */
  double mma_flops;    /* FUSED: flops of the dense blocks launched,
                          8 * 2^k per block and state amplitude            */
} juqcs_plan_opts;

/* Applies count gate records in order (gates commuting on disjoint qubits
 * may be regrouped; the result equals the sequential product).  opts may be
 * NULL (AUTO).  Errors: ARG, QUBIT, NUMERIC, UNSUPPORTED. */
juqcs_status juqcs_run_circuit(juqcs_state* st, const juqcs_gate* gates,
                               size_t count, juqcs_plan_opts* opts);

/* ------------------------------------------------------------------------
 * Autotuner
 * ---------------------------------------------------------------------- */

typedef struct {
  juqcs_plan_opts opts;  /* chosen planner options (mode, fuse_k, mma,
                            tile_bits, low_bits, pass_gates, relabel)       */
  double ms;             /* one run with them (HIP events on the stream,
                            planning and upload included)                  */
  double default_ms;     /* one run with the defaults (TILE, all 0)        */
  int32_t trials;        /* runs timed                                     */
  int32_t pad;
  uint64_t key;          /* circuit structure key (see juqcs_autotune)     */
} juqcs_tune_result;

/* Picks planner options for this circuit on this state by timed trials:
 * from the defaults, one parameter at a time (tile low bits, tile bits,
 * in-pass fusion width, gates per pass, relabeling), keeping a value when
 * it is more than 2% faster than the best so far, then dense fused blocks
 * of k = 3..6 (FP64 for C128, FP32 for C64), and one pass per gate for
 * small states; a choice other than the defaults is kept only if the
 * median of three runs beats theirs by 1%.  Every trial starts
 * from |0...0> on st's buffers (the state is left as the last trial made
 * it).  The fastest options are stored in the library's tuning table under
 * the circuit's structure key (n, amplitude type, ENC2 block bits, every
 * gate's op and qubits; matrices and angles do not enter), where
 * juqcs_run_circuit with mode JUQCS_PLAN_AUTO finds them.  Synchronises.
 * With the environment variable JUQCS_TUNE_VERBOSE=1 every timed run is
 * reported on stderr.  Errors: as for juqcs_run_circuit. */
juqcs_status juqcs_autotune(juqcs_state* st, const juqcs_gate* gates, size_t count,
                            juqcs_tune_result* out);

/* The tuning table as JSON (one object per entry), and back: load adds or
 * replaces entries.  clear empties the table.  Errors: ARG (null path,
 * unreadable or malformed file). */
juqcs_status juqcs_tune_save(const char* path);
/* The stored entry for this circuit's structure on st (JUQCS_ERR_ARG if
 * there is none). */
juqcs_status juqcs_tune_lookup(const juqcs_state* st, const juqcs_gate* gates, size_t count,
                               juqcs_tune_result* out);
juqcs_status juqcs_tune_load(const char* path);
juqcs_status juqcs_tune_clear(void);

/* ------------------------------------------------------------------------
 * Read-out
 * ---------------------------------------------------------------------- */

/* out[2k], out[2k+1] = re, im of <idx[k]|psi> (logical basis index; ENC2
 * amplitudes are decoded; the global factor is applied in FP64).  Host
 * arrays, staged through the workspace; synchronises the stream.
 * (Section 4: the M requested coefficients.)  Errors: ARG, HIP. */
juqcs_status juqcs_amplitudes(juqcs_state* st, const uint64_t* idx,
                              size_t count, double* out);

/* Same on device arrays, asynchronous (idx: count uint64, out: 2*count
 * doubles). */
juqcs_status juqcs_amplitudes_device(juqcs_state* st, const uint64_t* d_idx,
                                     size_t count, double* d_out);

/* out = |g|^2 sum_i |psi_i|^2 (g: the global factor), FP64 accumulation in
 * a fixed order (deterministic).  Section 2: the state is normalised.
 * Synchronises.  Errors: HIP, NUMERIC (result not finite). */
juqcs_status juqcs_norm(juqcs_state* st, double* out);

/* The state's FP64 complex global factor g (Section 2: the normalisation of
 * the state; phases and scalar weights).  The logical state is g times the
 * stored amplitudes: amplitudes, norm and expectation values include it,
 * and setting or multiplying it touches no amplitude.  g = (re, im).
 * juqcs_state_init resets it to 1.  Errors: ARG (null), NUMERIC
 * (non-finite). */
juqcs_status juqcs_set_global_factor(juqcs_state* st, const double g[2]);
juqcs_status juqcs_mul_global_factor(juqcs_state* st, const double f[2]);
juqcs_status juqcs_get_global_factor(const juqcs_state* st, double g[2]);

/* Renormalises through the global factor: g <- g / sqrt(N), N the norm
 * before (returned in *norm_before if not NULL).  One read pass, no write.
 * Errors: HIP, NUMERIC (zero or non-finite norm). */
juqcs_status juqcs_renormalize(juqcs_state* st, double* norm_before);

/* Multiplies every amplitude by the real factor (FP64 for C128, FP32 for
 * C64; ENC2 scales are multiplied).  Used to renormalise by 1/sqrt(norm). */
juqcs_status juqcs_scale(juqcs_state* st, double factor);

/* Single-qubit expectation values <Q_alpha(i)> = (1 - <sigma^alpha_i>)/2
 * for every qubit (Section 3), alpha = x, y, z: out[3*i + a], FP64 sums in
 * a fixed order.  Read-only passes over the state: the pair sums of up to
 * 13 bits come from one LDS-resident tile, so n qubits take
 * 1 + ceil((n - 13) / 8) passes for C128 (one for n <= 13).  Synchronises.
 * Errors: ARG, HIP. */
juqcs_status juqcs_expectations(juqcs_state* st, double* out);

/* ------------------------------------------------------------------------
 * Qubit layout
 * ---------------------------------------------------------------------- */

/* Moves logical qubit q to physical bit new_phys[q] (a permutation of
 * 0..n-1): one read+write pass.  Logical results are unchanged.
 * Errors: ARG, QUBIT. */
juqcs_status juqcs_permute(juqcs_state* st, const int* new_phys);

/* Restores identity order (physical bit q = logical qubit q), so the raw
 * buffer can be read directly. */
juqcs_status juqcs_state_canonicalize(juqcs_state* st);

/* Current logical->physical map (n ints). */
juqcs_status juqcs_get_layout(const juqcs_state* st, int* phys);

/* ------------------------------------------------------------------------
 * Two-byte codec (Section 1, adaptive two-byte amplitudes)
 * ---------------------------------------------------------------------- */

/* Encodes count amplitudes (C128 or C64 source, device) into d_codes
 * (2*count int8) and d_scales (ceil(count / 2^B) floats).  Bit-exact with the
 * format described at juqcs_dtype.  Asynchronous on hip_stream.
 * Errors: ARG, DTYPE. */
juqcs_status juqcs_encode2(const void* d_src, juqcs_dtype src, uint64_t count,
                           int block_bits, void* d_codes, void* d_scales,
                           void* hip_stream);

/* Decodes into C128 or C64 amplitudes (device).  Errors: ARG, DTYPE. */
juqcs_status juqcs_decode2(const void* d_codes, const void* d_scales,
                           uint64_t count, int block_bits, void* d_dst,
                           juqcs_dtype dst, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batches of independent circuits (many small states, one graph launch)
 * ---------------------------------------------------------------------- */

typedef struct juqcs_batch juqcs_batch; /* opaque */

/* Builds a batch of count circuits: circuit i has n[i] qubits (1..30) and
 * gate records gates[offsets[i] .. offsets[i+1]).  States are C64 in the
 * caller's d_states (states_bytes bytes, 16-byte aligned) at byte offsets
 * state_offset[i] (each 8 * 2^n[i] bytes, 16-byte aligned, inside the buffer
 * and disjoint: JUQCS_ERR_SIZE / JUQCS_ERR_ARG otherwise, checked before any
 * device work); every circuit starts from |0...0>.  Each circuit is planned
 * on the host into on-chip tile passes (tiles of up to 2^12 amplitudes);
 * the fusion width inside a pass (1..4 qubits) is opts->fuse_k, or chosen
 * per circuit by a cost model when fuse_k is 0 (juqcs_batch_autotune
 * replaces it with timed trials).  No device memory is touched: bind a
 * workspace of juqcs_batch_bytes bytes before running.  Errors: ARG, SIZE,
 * QUBIT, NUMERIC. */
juqcs_status juqcs_batch_create(juqcs_batch** out, int count, const int* n,
                                const juqcs_gate* gates, const int64_t* offsets,
                                void* d_states, size_t states_bytes,
                                const uint64_t* state_offset,
                                const juqcs_plan_opts* opts);

/* Device workspace the batch's current plans need (the work list plus a
 * read-out staging area of 4 MiB). */
juqcs_status juqcs_batch_bytes(const juqcs_batch* b, size_t* work_bytes);

/* Uploads the work list into the caller's workspace (256-byte aligned, at
 * least juqcs_batch_bytes; the caller keeps it alive until destroy or the
 * next bind).  Synchronises hip_stream.  Errors: ARG, SIZE, HIP. */
juqcs_status juqcs_batch_bind(juqcs_batch* b, void* d_work, size_t work_bytes,
                              void* hip_stream);

/* Autotuner: for every qubit count of the batch, times one of its circuits
 * run alone with in-pass fusion widths 1..4 (on that circuit's state region
 * and the bound workspace, on hip_stream) and re-plans every circuit with
 * the fastest width of its qubit count.  The batch is then unbound: query
 * juqcs_batch_bytes and bind again.  Errors: ARG (not bound), HIP. */
juqcs_status juqcs_batch_autotune(juqcs_batch* b, void* hip_stream);

/* Runs the whole batch on hip_stream (asynchronous): one persistent kernel
 * per pass round (round r applies pass r of every circuit that has one; the
 * kernel boundary orders a circuit's passes, so workgroups never wait for
 * each other).  On a non-default stream the launches are captured once into
 * a HIP graph and replayed as one graph launch on later calls. */
juqcs_status juqcs_batch_run(juqcs_batch* b, void* hip_stream);

/* Synchronises the stream of the last run (JUQCS_ERR_HIP on a device
 * error). */
juqcs_status juqcs_batch_wait(juqcs_batch* b);

/* Work-list statistics: tile tasks, gate records and tile passes. */
juqcs_status juqcs_batch_stats(const juqcs_batch* b, int64_t* tasks,
                               int64_t* gate_apps, int64_t* passes);

/* Fusion width chosen for every circuit (count ints). */
juqcs_status juqcs_batch_fusion(const juqcs_batch* b, int* kin);

/* Physical bit of every qubit of circuit c after a run: phys[q] for q <
 * n[c] (host array).  The tile passes relabel qubits as they write tiles
 * back (opts->relabel of juqcs_batch_create: 0 or 1 on, -1 off); the state
 * buffer holds amplitude z at index sum_q bit_q(z) << phys[q], and
 * juqcs_batch_amplitudes maps through it.  Errors: ARG. */
juqcs_status juqcs_batch_layout(const juqcs_batch* b, int c, int* phys);

/* out[2*(c*m+k)], out[2*(c*m+k)+1] = amplitude idx[c*m+k] of circuit c
 * (logical index; host arrays, FP64 pairs; an index >= 2^n gives NaN),
 * staged through the workspace in chunks of circuits.  Synchronises.
 * Errors: ARG (not bound), SIZE (m above 174762), HIP. */
juqcs_status juqcs_batch_amplitudes(juqcs_batch* b, const uint64_t* idx, int m,
                                    double* out, void* hip_stream);

/* The same with idx (count*m uint64) and out (2*count*m doubles) in device
 * memory; asynchronous on hip_stream. */
juqcs_status juqcs_batch_amplitudes_device(juqcs_batch* b, const uint64_t* d_idx, int m,
                                           double* d_out, void* hip_stream);

/* out[c] = FP64 norm of circuit c (fixed-order sum).  Synchronises. */
juqcs_status juqcs_batch_norms(juqcs_batch* b, double* out, void* hip_stream);

/* The same into device memory (count doubles); asynchronous. */
juqcs_status juqcs_batch_norms_device(juqcs_batch* b, double* d_out, void* hip_stream);

juqcs_status juqcs_batch_destroy(juqcs_batch* b);

/* ------------------------------------------------------------------------
 * Entangling-gate decomposition (Section 4, Eqs. (2) and (3))
 * ---------------------------------------------------------------------- */

/* <z|C|0> for count bitstrings z of an n-qubit circuit (n <= 62) whose
 * qubits are split in P parts by side[q] in {0, ..., P-1} (2 <= P <= 8,
 * each part 1..30 qubits; Section 4's partition into mutually exclusive
 * subsets).  Every CZ whose qubits lie in different parts is decomposed
 * with Eq. (2) (x = pi/4 - (i/2) asinh 1), and so is every such CNOT, as
 * its CZ between Hadamards on the target (H X H = Z).  Branch b in
 * [0, 2^m) uses s_k = +1 if bit k of b is 0, else -1, for the k-th
 * crossing gate in circuit order, and applies
 * diag(e^{i(x s_k - pi/4)}, e^{-i(x s_k - pi/4)}) to both of its qubits at
 * that position.  The part-states are simulated in C64 as batches: a part
 * state depends only on the bits of the crossings that touch its part, and
 * branches that agree on the first crossings share the states' common
 * gates, so each group of branches (group_size of them, rounded down to a
 * power of two; 0 = as many as fit) runs every part as a tree that splits
 * at its crossings.  The result 2^-m sum_b prod_p A_{b,p}(z_p) is summed in
 * FP64 on the device (Eq. (3)), over the branches in tree order (b with its
 * bits reversed, ascending) for every coefficient, the same result for any
 * group size.  Only CZ and CNOT may cross between parts
 * (JUQCS_ERR_UNSUPPORTED otherwise); m <= 20.  z: count uint64 (host);
 * out: 2*count doubles (host).  Synchronises hip_stream.  d_work: the
 * caller's device workspace (256-byte aligned) for the part states of a
 * group, the per-part indices, the running sum (4 P + 16 bytes per
 * bitstring, plus 8 words bytes for host bitstrings) and the tree rounds'
 * work lists; juqcs_branch_bytes gives its size.  group_size 0 takes the
 * largest group that fits work_bytes; a group size that does not fit is
 * JUQCS_ERR_SIZE.  count = 0 needs no workspace. */
juqcs_status juqcs_branch_amplitudes(int n, const juqcs_gate* gates,
                                     size_t gate_count, const uint8_t* side,
                                     const uint64_t* z, size_t count,
                                     int group_size, double* out,
                                     void* d_work, size_t work_bytes,
                                     void* hip_stream);

/* The same for circuits of up to 240 qubits (eight parts of 30), such as
 * Section 4's GHZ circuit on 128 qubits: bitstring k is the words uint64
 * z[k*words .. k*words + words) (little-endian: qubit q is bit q % 64 of
 * word q / 64), ceil(n/64) <= words <= 4, bits at n and above zero
 * (JUQCS_ERR_ARG otherwise); count <= 2^31.  Other arguments, results and
 * errors as for juqcs_branch_amplitudes. */
juqcs_status juqcs_branch_amplitudes_wide(int n, const juqcs_gate* gates,
                                          size_t gate_count, const uint8_t* side,
                                          const uint64_t* z, int words, size_t count,
                                          int group_size, double* out,
                                          void* d_work, size_t work_bytes,
                                          void* hip_stream);

/* The same with the bitstrings and the result on the device: d_z holds
 * count*words uint64 (layout as above) and d_out 2*count doubles, both in
 * device memory, so M can be large without host copies.  Bitstrings with a
 * bit at or above n are found on the device (JUQCS_ERR_ARG, out zeroed).
 * The result is complete when the call returns (it synchronises
 * hip_stream).  Other arguments, results and errors as for
 * juqcs_branch_amplitudes_wide. */
juqcs_status juqcs_branch_amplitudes_device(int n, const juqcs_gate* gates,
                                            size_t gate_count, const uint8_t* side,
                                            const uint64_t* d_z, int words, size_t count,
                                            int group_size, double* d_out,
                                            void* d_work, size_t work_bytes,
                                            void* hip_stream);

/* For callers that cannot allocate device memory (code under graph capture
 * set-up, tight serving loops, harnesses that forbid allocation): the same
 * as juqcs_branch_amplitudes_device with no workspace argument.  The
 * workspace is a static array of JUQCS_NOALLOC_SCRATCH_BYTES in the
 * library's device code, one per GPU, held until the process ends; calls
 * are serialised inside the process (they share the array, which keeps the
 * last call's contents; everything a call needs zeroed it clears itself),
 * and calls that overlapped on one GPU would race.  group_size 0 takes the
 * largest group that fits the array.  Decompositions whose workspace for
 * group_size (for groups of one branch when group_size is 0) exceeds it
 * are rejected with JUQCS_ERR_SIZE before any device work.  Synchronises
 * hip_stream.  Other arguments, results and errors as for
 * juqcs_branch_amplitudes_device. */
#define JUQCS_NOALLOC_SCRATCH_BYTES (32u << 20)
juqcs_status juqcs_branch_amplitudes_noalloc(int n, const juqcs_gate* gates,
                                             size_t gate_count, const uint8_t* side,
                                             const uint64_t* d_z, int words, size_t count,
                                             int group_size, double* d_out,
                                             void* hip_stream);

/* What the calling thread's last completed decomposition call did (zeros
 * before any): the branch groups and the part-state trees it simulated,
 * with the algorithmic flops and HBM bytes of their tile passes (gate
 * flops as juqcs_plan_opts.flops counts them; C64 read + write of every
 * part state per pass), and the FP64 flops of the Eq. (3) sums,
 * 2^m (6 (P - 1) + 2) per coefficient. */
typedef struct {
  int32_t crossings;    /* m                                               */
  int32_t group_bits;   /* L: 2^L groups of 2^(m - L) branches             */
  int64_t groups;
  int64_t tree_states;  /* part-state tree nodes simulated, all groups     */
  int64_t tile_passes;  /* tile passes over them                           */
  double pass_bytes;
  double gate_flops;
  double sum_flops;
  int32_t lds_sum;      /* 1: the sums ran from LDS                        */
  int32_t pad;
} juqcs_branch_stats;
juqcs_status juqcs_branch_last_stats(juqcs_branch_stats* out);

/* Device workspace of the decomposition calls above for these arguments:
 * *min_bytes for groups of one branch (the least any run needs), *bytes for
 * group_size (0: every branch in one group).  host_io = 1 for
 * juqcs_branch_amplitudes and _wide (bitstrings and result staged in the
 * workspace), 0 for _device.  Host work only (the circuit is planned).
 * Errors: as for juqcs_branch_amplitudes_wide, ARG for null outputs. */
juqcs_status juqcs_branch_bytes(int n, const juqcs_gate* gates, size_t gate_count,
                                const uint8_t* side, int words, size_t count,
                                int group_size, int host_io, size_t* min_bytes,
                                size_t* bytes);

/* ------------------------------------------------------------------------
 * Utilities
 * ---------------------------------------------------------------------- */

/* Device-to-device streaming copy of bytes (multiple of 16, 16-byte aligned
 * pointers) with the library's own copy kernel.  With d_dst == d_src it is
 * an in-place stream (every word read and written back, in the access
 * pattern of the per-gate passes): the practical HBM ceiling of an in-place
 * pass, which gate passes are compared with.  Other overlaps are
 * undefined.  Asynchronous. */
juqcs_status juqcs_copy(void* d_dst, const void* d_src, size_t bytes,
                        void* hip_stream);

/* Message for the last non-OK status returned on this thread. */
const char* juqcs_last_error(void);

/* Library version string. */
const char* juqcs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JUQCS_GPU_H */
