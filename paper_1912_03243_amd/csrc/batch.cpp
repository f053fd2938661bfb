// Batches of independent circuits in one persistent launch, the on-chip
// fusion-width autotuner, and the entangling-gate decomposition driver
// (Section 4, Eqs. (2) and (3)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "juqcs_internal.hpp"

using namespace juqcs;

namespace {

using C = cplx<double>;
constexpr int kChunkTiles = 32;

juqcs_status fail(juqcs_status st, const std::string& msg) {
  set_error(msg);
  return st;
}
juqcs_status hip_fail(hipError_t e, const char* where) {
  set_error(std::string(where) + ": " + hipGetErrorString(e));
  return JUQCS_ERR_HIP;
}

int tile_bits_for(int n) { return std::min(n, batch_max_bits()); }
int low_bits_for(int n) { return std::min(7, tile_bits_for(n)); }

// Modelled time (arbitrary units ~ picoseconds per amplitude) of a plan:
// every pass moves the state once (the first one only writes it), every op
// sweeps the tile in LDS and costs 2^k complex MACs per amplitude.
double plan_cost(const TilePlan& p) {
  constexpr double kMem = 2.9, kSweep = 0.2, kMac = 0.05;
  double c = 0.0;
  for (size_t i = 0; i < p.passes.size(); ++i) {
    double ops = 0.0;
    for (int o = 0; o < p.passes[i].op_count; ++o) {
      const TileOp& op = p.ops[p.passes[i].op_begin + o];
      const int k = op.kind == TOP_DENSE1 ? 1 : op.kind == TOP_DENSE2 ? 2
                    : op.kind == TOP_DIAG2 || op.kind == TOP_PERM ? 0
                    : op.kind == TOP_DENSE3 ? 3 : 4;
      ops += kSweep + kMac * (k ? (4 << k) : 1);
    }
    const double mem = i == 0 ? 0.5 * kMem : kMem;
    c += std::max(mem, ops);
  }
  return c;
}

// Tile passes of one circuit; with relabel the passes may move qubits onto
// the low bits (sched->final_pos: where each qubit ends).
void schedule_circuit(int n, const std::vector<Gate>& g, TileSchedule* sched, bool relabel) {
  const int b = tile_bits_for(n);
  if (relabel) {
    select_tiles_relabel(n, low_bits_for(n), b, 0, g, sched);
  } else {
    select_tiles(n, low_bits_for(n), b, 0, g, sched);
    sched->final_pos.resize(n);
    for (int q = 0; q < n; ++q) sched->final_pos[q] = q;
  }
  if (sched->passes.empty()) {  // no gates: one pass that writes |0...0>
    TilePass p{};
    p.g.n = n;
    p.g.b = b;
    p.g.L = b;
    p.g.H = 0;
    p.g.maxk = 1;
    sched->passes.push_back(p);
    sched->taken.emplace_back();
  }
}

void plan_circuit(int n, const std::vector<Gate>& g, int kin, bool relabel, TilePlan* plan,
                  TileSchedule* sched_out = nullptr) {
  TileSchedule sched;
  schedule_circuit(n, g, &sched, relabel);
  emit_schedule(sched, g, kin, plan, 0, batch_mma_cap());
  if (sched_out) *sched_out = std::move(sched);
}

// Runs f(i) for i in [0, count) on the host's cores.
template <typename F>
void parallel_for(int count, F f) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nt = (int)std::min<unsigned>(hw, (unsigned)count);
  if (nt <= 1) {
    for (int i = 0; i < count; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < count; i = next++) f(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

struct juqcs_batch {
  int count = 0;
  std::vector<int32_t> n;
  std::vector<uint64_t> state_off;
  char* states = nullptr;
  char* dbuf = nullptr;
  BatchDevice dev{};
  uint64_t* d_state_off = nullptr;
  int32_t* d_nq = nullptr;
  int64_t tasks = 0, gate_apps = 0, passes = 0;
  std::vector<int> kin;  // chosen on-chip fusion width per circuit
  std::vector<int8_t> pos;  // kMaxBatchQubits per circuit: physical bit of each qubit at the end
  int8_t* d_pos = nullptr;
  std::vector<char> keep;   // per circuit (empty: none): start from the state in the buffer, not |0...0>
  hipStream_t last_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t graph_stream = nullptr;
};

namespace {

void free_batch(juqcs_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dbuf) (void)hipFree(b->dbuf);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->dbuf = nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxBatchQubits = 32;  // layout entries per circuit

// Layout entries of circuit c from a schedule's final positions.
void set_layout(juqcs_batch* B, int c, const std::vector<int>& final_pos) {
  if (B->pos.size() != (size_t)B->count * kMaxBatchQubits) {
    B->pos.assign((size_t)B->count * kMaxBatchQubits, 0);
    for (int i = 0; i < B->count; ++i)
      for (int q = 0; q < kMaxBatchQubits; ++q) B->pos[(size_t)i * kMaxBatchQubits + q] = (int8_t)q;
  }
  for (size_t q = 0; q < final_pos.size(); ++q)
    B->pos[(size_t)c * kMaxBatchQubits + q] = (int8_t)final_pos[q];
}

// Lays the plans out as one device work list (pass-major groups).
juqcs_status build_device(juqcs_batch* B, const std::vector<TilePlan>& plans) {
  std::vector<BatchPass> passes;
  std::vector<TileOp> ops;
  std::vector<cplx<float>> mats;
  std::vector<BatchGroup> groups;
  std::vector<int> first_pass(B->count);
  B->tasks = B->gate_apps = B->passes = 0;
  for (int c = 0; c < B->count; ++c) {
    const TilePlan& p = plans[c];
    first_pass[c] = (int)passes.size();
    const int64_t op0 = (int64_t)ops.size(), m0 = (int64_t)mats.size();
    for (const TilePass& tp : p.passes) {
      if (tp.g.H > batch_max_gather()) return fail(JUQCS_ERR_ARG, "batch tile with too many gathered bits");
      BatchPass bp;
      bp.g = tp.g;
      bp.op_begin = (int32_t)(op0 + tp.op_begin);
      bp.op_count = tp.op_count;
      passes.push_back(bp);
    }
    for (TileOp op : p.ops) {
      op.moff += m0;
      ops.push_back(op);
    }
    for (const C& z : p.mats) mats.push_back({(float)z.re, (float)z.im});
    const int b = p.passes[0].g.b;
    const int64_t ntiles = int64_t(1) << (B->n[c] - b);
    const int chunk = (int)std::min<int64_t>(ntiles, kChunkTiles);
    for (int i = 0; i < (int)p.passes.size(); ++i) {
      BatchGroup g{};
      g.state_off = B->state_off[c];
      g.circuit = c;
      g.pass = first_pass[c] + i;
      g.chunk_tiles = chunk;
      g.init = (i == 0 && (B->keep.empty() || !B->keep[c])) ? 1 : 0;
      groups.push_back(g);
    }
    B->tasks += ntiles * (int64_t)p.passes.size();
    B->passes += (int64_t)p.passes.size();
    B->gate_apps += p.gates;
  }
  // pass-major order: pass index within the circuit, then circuit
  std::stable_sort(groups.begin(), groups.end(), [&](const BatchGroup& a, const BatchGroup& b) {
    return (a.pass - first_pass[a.circuit]) < (b.pass - first_pass[b.circuit]);
  });
  // rounds: groups of the same pass index, contiguous after the sort
  BatchDevice& d = B->dev;
  d.round_group.clear();
  d.round_chunk.clear();
  long long next = 0;
  int round = -1;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    BatchGroup& g = groups[gi];
    const int r = g.pass - first_pass[g.circuit];
    while (round < r) {
      d.round_group.push_back((int32_t)gi);
      d.round_chunk.push_back(next);
      ++round;
    }
    g.first_chunk = next;
    const int b = passes[g.pass].g.b;
    const int64_t ntiles = int64_t(1) << (B->n[g.circuit] - b);
    next += ntiles / g.chunk_tiles;
  }
  d.nrounds = round + 1;
  d.round_group.push_back((int32_t)groups.size());
  d.round_chunk.push_back(next);
  // one device buffer for everything
  const size_t o_groups = 0;
  const size_t o_passes = align256(o_groups + groups.size() * sizeof(BatchGroup));
  const size_t o_ops = align256(o_passes + passes.size() * sizeof(BatchPass));
  const size_t o_mats = align256(o_ops + std::max<size_t>(ops.size(), 1) * sizeof(TileOp));
  const size_t o_tickets = align256(o_mats + std::max<size_t>(mats.size(), 1) * sizeof(cplx<float>));
  const size_t o_soff = align256(o_tickets + std::max(d.nrounds, 1) * sizeof(uint64_t));
  const size_t o_nq = align256(o_soff + B->count * sizeof(uint64_t));
  const size_t o_pos = align256(o_nq + B->count * sizeof(int32_t));
  const size_t total = align256(o_pos + (size_t)B->count * kMaxBatchQubits);
  if (B->pos.size() != (size_t)B->count * kMaxBatchQubits) set_layout(B, 0, {});
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + o_groups, groups.data(), groups.size() * sizeof(BatchGroup));
  std::memcpy(host.data() + o_passes, passes.data(), passes.size() * sizeof(BatchPass));
  std::memcpy(host.data() + o_ops, ops.data(), ops.size() * sizeof(TileOp));
  std::memcpy(host.data() + o_mats, mats.data(), mats.size() * sizeof(cplx<float>));
  std::memcpy(host.data() + o_soff, B->state_off.data(), B->count * sizeof(uint64_t));
  std::memcpy(host.data() + o_nq, B->n.data(), B->count * sizeof(int32_t));
  std::memcpy(host.data() + o_pos, B->pos.data(), B->pos.size());
  hipError_t e = hipMalloc((void**)&B->dbuf, total);
  if (e != hipSuccess) return hip_fail(e, "batch hipMalloc");
  e = hipMemcpy(B->dbuf, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  d.groups = (const BatchGroup*)(B->dbuf + o_groups);
  d.ngroups = (int)groups.size();
  d.passes = (const BatchPass*)(B->dbuf + o_passes);
  d.ops = (const TileOp*)(B->dbuf + o_ops);
  d.mats = (const cplx<float>*)(B->dbuf + o_mats);
  d.tickets = (uint64_t*)(B->dbuf + o_tickets);
  d.count = B->count;
  d.nchunks = next;
  B->d_state_off = (uint64_t*)(B->dbuf + o_soff);
  B->d_nq = (int32_t*)(B->dbuf + o_nq);
  B->d_pos = (int8_t*)(B->dbuf + o_pos);
  return JUQCS_OK;
}

juqcs_status run_device(juqcs_batch* B, hipStream_t s) {
  hipError_t e = launch_batch(B->states, B->dev, s);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  return JUQCS_OK;
}

// Timed trial of one circuit's plan (used by the autotuner): runs it as a
// one-circuit batch on the circuit's own state buffer.
double time_plan(char* states, uint64_t off, int n, const TilePlan& plan, hipStream_t s) {
  juqcs_batch B;
  B.count = 1;
  B.n = {n};
  B.state_off = {off};
  B.states = states;
  std::vector<TilePlan> plans{plan};
  if (build_device(&B, plans) != JUQCS_OK) {
    free_batch(&B);
    return 1e30;
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)run_device(&B, s);  // warm
  (void)hipEventRecord(a, s);
  (void)run_device(&B, s);
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = 1e30f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  free_batch(&B);
  return ms;
}

}  // namespace

extern "C" {

juqcs_status juqcs_batch_create(juqcs_batch** out, int count, const int* n,
                                const juqcs_gate* gates, const int64_t* offsets, void* d_states,
                                const uint64_t* state_offset, const juqcs_plan_opts* opts) {
  if (!out) return fail(JUQCS_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (count < 1) return fail(JUQCS_ERR_ARG, "count must be >= 1");
  if (!n || !offsets || !d_states || !state_offset) return fail(JUQCS_ERR_ARG, "null argument");
  if (offsets[0] != 0) return fail(JUQCS_ERR_ARG, "offsets[0] must be 0");
  for (int c = 0; c < count; ++c) {
    if (n[c] < 1 || n[c] > 30) return fail(JUQCS_ERR_ARG, "batch circuits need 1 <= n <= 30");
    if (offsets[c + 1] < offsets[c]) return fail(JUQCS_ERR_ARG, "offsets must not decrease");
    if (state_offset[c] & 15) return fail(JUQCS_ERR_ARG, "state offsets must be 16-byte aligned");
  }
  if (offsets[count] > 0 && !gates) return fail(JUQCS_ERR_ARG, "null gate array");
  const int fuse = opts ? opts->fuse_k : 0;
  const bool autotune = opts && opts->autotune;
  const bool relabel = !opts || opts->relabel >= 0;
  if (opts && (opts->relabel < -1 || opts->relabel > 1)) return fail(JUQCS_ERR_ARG, "relabel must be -1, 0 or 1");
  if (fuse < 0 || fuse > 4) return fail(JUQCS_ERR_ARG, "batch fuse_k must be 0 (auto) or 1..4");
  auto* B = new juqcs_batch();
  B->count = count;
  B->n.assign(n, n + count);
  B->state_off.assign(state_offset, state_offset + count);
  B->states = (char*)d_states;
  B->kin.assign(count, 2);
  set_layout(B, 0, {});
  std::vector<TilePlan> plans(count);
  std::vector<std::vector<Gate>> dec(count);
  std::string err;
  for (int c = 0; c < count; ++c) {
    dec[c].resize(offsets[c + 1] - offsets[c]);
    for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i)
      if (!decode_gate(gates[i], n[c], &dec[c][i - offsets[c]], &err)) {
        delete B;
        const bool numeric = err.find("non-finite") != std::string::npos;
        return fail(numeric ? JUQCS_ERR_NUMERIC : JUQCS_ERR_QUBIT,
                    "circuit " + std::to_string(c) + ": " + err);
      }
  }
  // fusion width: fixed, modelled, or measured (one trial per qubit count)
  if (!autotune) {
    parallel_for(count, [&](int c) {
      TileSchedule sched;
      schedule_circuit(n[c], dec[c], &sched, relabel);
      set_layout(B, c, sched.final_pos);
      if (fuse > 0) {
        emit_schedule(sched, dec[c], fuse, &plans[c], 0, batch_mma_cap());
        B->kin[c] = fuse;
        return;
      }
      double best = 1e300;
      for (int k = 2; k <= 4; ++k) {
        TilePlan p;
        emit_schedule(sched, dec[c], k, &p, 0, batch_mma_cap());
        const double cst = plan_cost(p);
        if (cst < best) {
          best = cst;
          plans[c] = std::move(p);
          B->kin[c] = k;
        }
      }
    });
  }
  std::map<int, int> measured;
  for (int c = 0; autotune && c < count; ++c) {
    {
      auto it = measured.find(n[c]);
      if (it == measured.end()) {
        double best = 1e30;
        int bk = 2;
        for (int k = 1; k <= 4; ++k) {
          TilePlan p;
          plan_circuit(n[c], dec[c], k, relabel, &p);
          const double t = time_plan(B->states, B->state_off[c], n[c], p, nullptr);
          if (t < best) {
            best = t;
            bk = k;
          }
        }
        it = measured.emplace(n[c], bk).first;
      }
      B->kin[c] = it->second;
    }
  }
  if (autotune)
    parallel_for(count, [&](int c) {
      TileSchedule sched;
      plan_circuit(n[c], dec[c], B->kin[c], relabel, &plans[c], &sched);
      set_layout(B, c, sched.final_pos);
    });
  juqcs_status rc = build_device(B, plans);
  if (rc != JUQCS_OK) {
    free_batch(B);
    delete B;
    return rc;
  }
  *out = B;
  return JUQCS_OK;
}

juqcs_status juqcs_batch_run(juqcs_batch* B, void* hip_stream) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  hipStream_t s = (hipStream_t)hip_stream;
  B->last_stream = s;
  if (!s) return run_device(B, s);  // the legacy default stream cannot be captured
  if (!B->gexec || B->graph_stream != s) {
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->gexec = nullptr;
    B->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    juqcs_status rc = run_device(B, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (rc != JUQCS_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    B->graph = g;
    e = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    B->graph_stream = s;
  }
  hipError_t e = hipGraphLaunch(B->gexec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_wait(juqcs_batch* B) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  hipError_t e = hipStreamSynchronize(B->last_stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_stats(const juqcs_batch* B, int64_t* tasks, int64_t* gate_apps,
                               int64_t* passes) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  if (tasks) *tasks = B->tasks;
  if (gate_apps) *gate_apps = B->gate_apps;
  if (passes) *passes = B->passes;
  return JUQCS_OK;
}

juqcs_status juqcs_batch_layout(const juqcs_batch* B, int c, int* phys) {
  if (!B || !phys) return fail(JUQCS_ERR_ARG, "null argument");
  if (c < 0 || c >= B->count) return fail(JUQCS_ERR_ARG, "circuit index out of range");
  for (int q = 0; q < B->n[c]; ++q) phys[q] = B->pos[(size_t)c * kMaxBatchQubits + q];
  return JUQCS_OK;
}

juqcs_status juqcs_batch_fusion(const juqcs_batch* B, int* kin) {
  if (!B || !kin) return fail(JUQCS_ERR_ARG, "null argument");
  for (int c = 0; c < B->count; ++c) kin[c] = B->kin[c];
  return JUQCS_OK;
}

juqcs_status juqcs_batch_amplitudes(juqcs_batch* B, const uint64_t* idx, int m, double* out,
                                    void* hip_stream) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  if (m < 0 || (m > 0 && (!idx || !out))) return fail(JUQCS_ERR_ARG, "bad index list");
  const size_t total = (size_t)B->count * m;
  if (total == 0) return JUQCS_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  uint64_t* d_idx = nullptr;
  double* d_out = nullptr;
  hipError_t e = hipMalloc((void**)&d_idx, total * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&d_out, total * 2 * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(d_idx, idx, total * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_batch_gather(B->states, B->d_state_off, B->d_nq, B->d_pos, B->count, m, d_idx, d_out, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, d_out, total * 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_idx);
  (void)hipFree(d_out);
  if (e != hipSuccess) return hip_fail(e, "batch amplitudes");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_norms(juqcs_batch* B, double* out, void* hip_stream) {
  if (!B || !out) return fail(JUQCS_ERR_ARG, "null argument");
  hipStream_t s = (hipStream_t)hip_stream;
  double* d_out = nullptr;
  hipError_t e = hipMalloc((void**)&d_out, B->count * sizeof(double));
  if (e == hipSuccess) e = launch_batch_norms(B->states, B->d_state_off, B->d_nq, B->count, d_out, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, d_out, B->count * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_out);
  if (e != hipSuccess) return hip_fail(e, "batch norms");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_destroy(juqcs_batch* B) {
  if (!B) return JUQCS_OK;
  if (B->last_stream) (void)hipStreamSynchronize(B->last_stream);
  free_batch(B);
  delete B;
  return JUQCS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Entangling-gate decomposition (Section 4)
// ---------------------------------------------------------------------------
namespace {

// One term factor of Eq. (2) on a single qubit: exp(i sigma^z (x s - pi/4)),
// x = pi/4 - (i/2) asinh(1) (a solution of cos(2x) = i).
void branch_diag(int s, C* d) {
  const std::complex<double> x(M_PI / 4.0, -0.5 * std::asinh(1.0));
  const std::complex<double> a = std::complex<double>(0.0, 1.0) * (x * (double)s - M_PI / 4.0);
  const std::complex<double> e0 = std::exp(a), e1 = std::exp(-a);
  d[0] = {e0.real(), e0.imag()};
  d[1] = {0, 0};
  d[2] = {0, 0};
  d[3] = {e1.real(), e1.imag()};
}

// One segment of a part circuit: the gates from one run of its crossings
// (consecutive gates of the part) up to the next run.
struct BranchSeg {
  int g0 = 0, g1 = 0;       // gates [g0, g1) of the part
  std::vector<int> ks;      // crossings whose diagonals open it, circuit order
  int nfree = 0;            // of them with bits free within a group
  std::vector<Gate> gates;  // its gates, qubits where the previous segment left them
  TilePlan tmpl;            // plan with placeholder diagonals
  TileSchedule sched;
};

// One part of a decomposition: its circuit with a placeholder diagonal at
// every crossing, and that circuit cut into segments.
struct BranchPart {
  int nloc = 0;
  size_t sbytes = 0;                       // state bytes (C64, 256-aligned)
  std::vector<Gate> gates;                 // local qubits
  std::vector<std::pair<int, int>> slots;  // (gate index, crossing) of each diagonal, circuit order
  std::vector<BranchSeg> segs;             // segs[0]: the gates before the first crossing
  std::vector<int> freek;                  // crossings with free bits, circuit order
  std::vector<int> phys;                   // physical bit of each local qubit at the leaves
  int free_bits(int L) const {
    int R = 0;
    for (auto& sl : slots) R += sl.second >= L ? 1 : 0;
    return R;
  }
};

// Cuts the part before every run of its crossings, whether their bits are
// fixed by the group (crossings < L) or free: the cut points do not depend
// on L, so a leaf goes through the same plans, and holds the same bits, for
// any group size.  Each segment is planned where the previous one left the
// qubits.
void cut_part(BranchPart* bp, int L) {
  const std::vector<std::pair<int, int>>& fr = bp->slots;
  const int ng = (int)bp->gates.size();
  bp->segs.clear();
  bp->freek.clear();
  for (auto& f : fr)
    if (f.second >= L) bp->freek.push_back(f.second);
  BranchSeg pre;
  pre.g1 = fr.empty() ? ng : fr[0].first;
  bp->segs.push_back(std::move(pre));
  for (size_t i = 0; i < fr.size();) {
    size_t j = i + 1;
    while (j < fr.size() && fr[j].first == fr[j - 1].first + 1) ++j;
    BranchSeg sg;
    sg.g0 = fr[i].first;
    sg.g1 = j < fr.size() ? fr[j].first : ng;
    for (size_t t = i; t < j; ++t) {
      sg.ks.push_back(fr[t].second);
      sg.nfree += fr[t].second >= L ? 1 : 0;
    }
    bp->segs.push_back(std::move(sg));
    i = j;
  }
  std::vector<int> pos(bp->nloc);
  for (int q = 0; q < bp->nloc; ++q) pos[q] = q;
  for (BranchSeg& sg : bp->segs) {
    sg.gates.assign(bp->gates.begin() + sg.g0, bp->gates.begin() + sg.g1);
    for (Gate& g : sg.gates)
      for (int j = 0; j < g.nq; ++j) g.q[j] = pos[g.q[j]];
    plan_circuit(bp->nloc, sg.gates, 2, true, &sg.tmpl, &sg.sched);
    if (!sg.sched.final_pos.empty())
      for (int q = 0; q < bp->nloc; ++q) pos[q] = sg.sched.final_pos[pos[q]];
  }
  bp->phys = pos;
}

// The plan of one tree node: segment sg of the part with its diagonals set,
// fixed crossings (< L) from the bits of group gi, free ones from the bits
// of child c (the segment's first free crossing is its top bit).
TilePlan node_plan(const BranchPart& bp, const BranchSeg& sg, long long gi, int L, long long c) {
  std::vector<Gate> hg = sg.gates;
  const int nfixed = (int)sg.ks.size() - sg.nfree;
  for (auto& sl : bp.slots) {
    if (sl.first < sg.g0 || sl.first >= sg.g1) continue;
    int bit;
    if (sl.second < L) {
      bit = (int)((gi >> (L - 1 - sl.second)) & 1);
    } else {
      const int j = (int)(std::find(sg.ks.begin(), sg.ks.end(), sl.second) - sg.ks.begin()) - nfixed;
      bit = (int)((c >> (sg.nfree - 1 - j)) & 1);
    }
    branch_diag(bit ? -1 : 1, hg[sl.first - sg.g0].m);
  }
  // the plan's ops refer to the schedule's relabeled gate copies
  std::vector<Gate> tg = sg.sched.tgates.empty() ? hg : sg.sched.tgates;
  if (!sg.sched.tgates.empty())
    for (size_t t = 0; t < tg.size(); ++t) std::memcpy(tg[t].m, hg[sg.sched.tsrc[t]].m, sizeof(tg[t].m));
  TilePlan pl = sg.tmpl;
  rebuild_mats(tg, &pl);
  return pl;
}

// Eq. (3) for count bitstrings of words 64-bit words each (see
// juqcs_branch_amplitudes_wide).
// dev: z and out are device pointers (the bitstrings are checked on the
// device), else host arrays.
juqcs_status branch_amplitudes(int n, const juqcs_gate* gates, size_t gate_count, const uint8_t* side,
                               const uint64_t* z, int words, size_t count, int group_size, double* out,
                               hipStream_t s, bool dev) {
  if (n < 2 || n > kBranchMaxQubits) return fail(JUQCS_ERR_ARG, "n must be in [2, 240]");
  if (words < (n + 63) / 64 || words > kBranchMaxWords)
    return fail(JUQCS_ERR_ARG, "words must be in [ceil(n / 64), 4]");
  if (!side || (count > 0 && (!z || !out)) || (gate_count > 0 && !gates))
    return fail(JUQCS_ERR_ARG, "null argument");
  if (count > (size_t)1 << 31) return fail(JUQCS_ERR_SIZE, "at most 2^31 bitstrings");
  // parts and local qubit numbers (ascending order inside a part)
  int P = 0;
  for (int q = 0; q < n; ++q) {
    if (side[q] >= kBranchMaxParts)
      return fail(JUQCS_ERR_ARG, "side[q] must be < " + std::to_string(kBranchMaxParts));
    P = std::max(P, side[q] + 1);
  }
  int local[kBranchMaxQubits], nloc[kBranchMaxParts] = {};
  for (int q = 0; q < n; ++q) local[q] = nloc[side[q]]++;
  if (P < 2) return fail(JUQCS_ERR_ARG, "at least two parts");
  for (int p = 0; p < P; ++p)
    if (nloc[p] < 1 || nloc[p] > 30) return fail(JUQCS_ERR_ARG, "each part needs 1..30 qubits");
  // bits at or above n must be clear (only the words that can hold them)
  for (int w = n / 64; !dev && w < words; ++w) {
    const int lo = std::max(0, n - 64 * w);
    const uint64_t bad = lo >= 64 ? 0 : ~0ull << lo;
    for (size_t k = 0; k < count; ++k)
      if (z[k * words + w] & bad) return fail(JUQCS_ERR_ARG, "bitstring >= 2^n");
  }
  // part circuits with placeholder diagonals at every crossing gate; a
  // crossing CNOT is its CZ between Hadamards on the target (H X H = Z)
  BranchPart parts[kBranchMaxParts];
  int m = 0;
  std::string err;
  const double s2 = 1.0 / std::sqrt(2.0);
  for (size_t i = 0; i < gate_count; ++i) {
    Gate g;
    if (!decode_gate(gates[i], n, &g, &err)) {
      const bool numeric = err.find("non-finite") != std::string::npos;
      return fail(numeric ? JUQCS_ERR_NUMERIC : JUQCS_ERR_QUBIT,
                  "gate " + std::to_string(i) + ": " + err);
    }
    if (g.nq == 2 && side[g.q[0]] != side[g.q[1]]) {
      const int op = gates[i].op;
      if (op != JUQCS_OP_CZ && op != JUQCS_OP_CNOT)
        return fail(JUQCS_ERR_UNSUPPORTED, "only CZ and CNOT gates may cross between parts");
      if (m == 20) return fail(JUQCS_ERR_UNSUPPORTED, "at most 20 crossing gates");
      const int t = g.q[1], pt = side[t];  // CNOT: q1 is the target
      Gate h{};
      h.nq = 1;
      h.q[0] = local[t];
      h.q[1] = -1;
      h.m[0] = {s2, 0};
      h.m[1] = {s2, 0};
      h.m[2] = {s2, 0};
      h.m[3] = {-s2, 0};
      if (op == JUQCS_OP_CNOT) parts[pt].gates.push_back(h);
      for (int j = 0; j < 2; ++j) {
        const int q = g.q[j], p = side[q];
        Gate d{};
        d.nq = 1;
        d.q[0] = local[q];
        d.q[1] = -1;
        branch_diag(1, d.m);
        d.diag = true;
        parts[p].slots.push_back({(int)parts[p].gates.size(), m});
        parts[p].gates.push_back(d);
      }
      if (op == JUQCS_OP_CNOT) parts[pt].gates.push_back(h);
      ++m;
      continue;
    }
    const int p = side[g.q[0]];
    for (int j = 0; j < g.nq; ++j) g.q[j] = local[g.q[j]];
    parts[p].gates.push_back(g);
  }
  if (count == 0) return JUQCS_OK;
  for (int p = 0; p < P; ++p) {
    parts[p].nloc = nloc[p];
    parts[p].sbytes = align256((size_t)8 << nloc[p]);
  }
  // Branches are grouped by the bits of the first L crossings (circuit
  // order; those bits are fixed within a group, the others free).  Inside a
  // group a part's states form a tree: the gates before its first crossing
  // run once, and every run of its crossings splits each state into one
  // copy per setting of their free bits, which then runs the gates up to
  // the next run.  The leaves are the part's states for every setting of
  // its own free crossings; branches that agree on those share a leaf.
  size_t budget = 0;
  {
    size_t freeb = 0, totalb = 0;
    (void)hipMemGetInfo(&freeb, &totalb);
    budget = std::min<size_t>(freeb / 2, (size_t)64 << 30);
  }
  auto leaf_bytes = [&](int L) {
    size_t t = 0;
    for (int p = 0; p < P; ++p) t += parts[p].sbytes << parts[p].free_bits(L);
    return t;
  };
  int L = 0;
  if (group_size > 0) {
    int lg = 0;
    while (lg < m && (2ll << lg) <= group_size) ++lg;
    L = m - lg;
  } else {
    while (L < m && leaf_bytes(L) > budget) ++L;
  }
  const long long gsize = 1ll << (m - L), ngroups = 1ll << L;
  for (int p = 0; p < P; ++p) cut_part(&parts[p], L);
  // split table: each part's qubits and their physical bits at the leaves
  std::vector<int32_t> tab(kBranchTabInts, 0);
  {
    int32_t* first = tab.data();
    int32_t* qs = first + kBranchMaxParts + 1;
    int32_t* phys = qs + kBranchMaxQubits;
    int o = 0;
    for (int p = 0; p < P; ++p) {
      first[p] = o;
      for (int q = 0; q < n; ++q) {
        if (side[q] != p) continue;
        qs[o] = q;
        phys[o] = parts[p].phys[local[q]];
        ++o;
      }
    }
    first[P] = o;
  }
  // leaves part by part: leaf l of part p (bit R-1-i of l = free crossing i)
  int32_t first[kBranchMaxParts + 1] = {};
  size_t base[kBranchMaxParts] = {}, total = 0;
  for (int p = 0; p < P; ++p) {
    first[p + 1] = first[p] + (1 << parts[p].freek.size());
    base[p] = total;
    total += parts[p].sbytes << parts[p].freek.size();
  }
  const int nleaves = first[P];
  std::vector<uint64_t> leaf_off(nleaves);
  for (int p = 0; p < P; ++p)
    for (int l = 0; l < (1 << parts[p].freek.size()); ++l)
      leaf_off[first[p] + l] = base[p] + (size_t)l * parts[p].sbytes;
  // the sum runs over branches in tree order: t ascending, where bit
  // m-1-k of t is crossing k's bit; a group is a range of t
  auto branch_of = [&](long long t) {
    long long b = 0;
    for (int k = 0; k < m; ++k) b |= ((t >> (m - 1 - k)) & 1) << k;
    return b;
  };
  const bool lds = nleaves <= kBranchSumValues;
  std::vector<uint64_t> t8;
  std::vector<int32_t> t32;
  if (lds) t8.assign(gsize, 0);
  else t32.resize((size_t)gsize * P);
  for (long long j = 0; j < gsize; ++j) {
    const long long b = branch_of(j);  // the free bits (the group adds only fixed ones)
    for (int p = 0; p < P; ++p) {
      const std::vector<int>& fk = parts[p].freek;
      const int R = (int)fk.size();
      int l = 0;
      for (int i = 0; i < R; ++i) l |= (int)((b >> fk[i]) & 1) << (R - 1 - i);
      if (lds) t8[j] |= (uint64_t)(first[p] + l) << (8 * p);
      else t32[(size_t)j * P + p] = first[p] + l;
    }
  }
  // bitstrings -> per-part indices on the device; acc holds the running sum
  // (the caller's out when it is on the device)
  uint64_t* dz = nullptr;
  uint32_t* zp = nullptr;
  int32_t* dtab = nullptr;
  int* dbad = nullptr;
  double* acc = dev ? out : nullptr;
  char* states = nullptr;
  uint64_t* doff = nullptr;
  void* dsum = nullptr;
  const size_t tbytes = lds ? t8.size() * 8 : t32.size() * 4;
  hipError_t e = hipSuccess;
  if (!dev) e = hipMalloc((void**)&dz, count * words * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&zp, (size_t)P * count * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&dtab, tab.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&dbad, sizeof(int));
  if (e == hipSuccess && !dev) e = hipMalloc((void**)&acc, count * 2 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&doff, nleaves * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc(&dsum, tbytes);
  if (e == hipSuccess) e = hipMalloc((void**)&states, total);
  if (e == hipSuccess && !dev)
    e = hipMemcpyAsync(dz, z, count * words * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(doff, leaf_off.data(), nleaves * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dsum, lds ? (const void*)t8.data() : (const void*)t32.data(), tbytes,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(dbad, 0, sizeof(int), s);
  if (e == hipSuccess)
    e = launch_branch_split(dev ? z : dz, words, (long long)count, P, n, dtab, zp, dbad, s);
  if (e == hipSuccess) e = hipMemsetAsync(acc, 0, count * 2 * sizeof(double), s);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dz);
  juqcs_status rc = JUQCS_OK;
  if (e != hipSuccess) rc = hip_fail(e, "branch set-up");
  else if (bad) rc = fail(JUQCS_ERR_ARG, "bitstring >= 2^n");
  size_t rounds = 0;
  for (int p = 0; p < P; ++p) rounds = std::max(rounds, parts[p].segs.size());
  for (long long gi = 0; rc == JUQCS_OK && gi < ngroups; ++gi) {
    for (size_t r = 0; rc == JUQCS_OK && r < rounds; ++r) {
      // round r: segment r of every part, for every node of that level
      juqcs_batch B;
      std::vector<TilePlan> plans;
      for (int p = 0; p < P && rc == JUQCS_OK; ++p) {
        const BranchPart& bp = parts[p];
        if (r >= bp.segs.size()) continue;
        const BranchSeg& sg = bp.segs[r];
        const int R = (int)bp.freek.size();
        int done = 0;  // free bits split before this segment
        for (size_t i = 0; i < r; ++i) done += bp.segs[i].nfree;
        const int after = R - done - sg.nfree;
        for (long long a = 0; a < (1ll << done); ++a)
          for (long long c = 0; c < (1ll << sg.nfree); ++c) {
            const long long parent = a << (R - done), leaf = parent + (c << after);
            plans.push_back(node_plan(bp, sg, gi, L, c));
            B.n.push_back(bp.nloc);
            B.state_off.push_back(base[p] + (size_t)leaf * bp.sbytes);
            B.keep.push_back(r > 0 ? 1 : 0);
            if (r > 0 && c > 0) {  // the child starts as a copy of its parent
              e = hipMemcpyAsync(states + B.state_off.back(), states + base[p] + (size_t)parent * bp.sbytes,
                                 bp.sbytes, hipMemcpyDeviceToDevice, s);
              if (e != hipSuccess) rc = hip_fail(e, "branch state copy");
            }
          }
      }
      B.count = (int)plans.size();
      B.states = states;
      if (rc == JUQCS_OK && B.count > 0) {
        rc = build_device(&B, plans);
        if (rc == JUQCS_OK) rc = run_device(&B, s);
        if (rc == JUQCS_OK) {
          e = hipStreamSynchronize(s);
          if (e != hipSuccess) rc = hip_fail(e, "branch batch");
        }
      }
      free_batch(&B);
    }
    if (rc == JUQCS_OK) {
      const bool last = gi + 1 == ngroups;
      const double scale = std::ldexp(1.0, -m);
      if (lds) {
        BranchParts bp{};
        for (int p = 0; p <= P; ++p) bp.first[p] = first[p];
        e = launch_branch_sum_lds(states, doff, P, bp, gsize, (const uint64_t*)dsum, zp, (long long)count,
                                  acc, last, scale, s);
      } else {
        // Many coefficients read every state at random places: in chunks of
        // branches whose states fit the 256 MiB last-level cache those reads
        // stay on chip, at the price of one more pass over acc per chunk.
        size_t per = 0;
        for (int p = 0; p < P; ++p) per += parts[p].sbytes;
        const long long chunk =
            count >= (1u << 16) ? std::max<long long>(1, (long long)(((size_t)128 << 20) / per)) : gsize;
        for (long long j0 = 0; e == hipSuccess && j0 < gsize; j0 += chunk) {
          const long long c = std::min(chunk, gsize - j0);
          e = launch_branch_gather_accum(states, doff, P, c, (const int32_t*)dsum + j0 * P, zp,
                                         (long long)count, acc, last && j0 + c >= gsize, scale, s);
        }
      }
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_fail(e, "branch sum");
    }
  }
  if (rc == JUQCS_OK && !dev) {
    e = hipMemcpyAsync(out, acc, count * 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "branch result copy");
  }
  (void)hipFree(states);
  (void)hipFree(dsum);
  (void)hipFree(doff);
  (void)hipFree(zp);
  (void)hipFree(dtab);
  (void)hipFree(dbad);
  if (!dev) (void)hipFree(acc);
  return rc;
}

}  // namespace

extern "C" juqcs_status juqcs_branch_amplitudes(int n, const juqcs_gate* gates, size_t gate_count,
                                                const uint8_t* side, const uint64_t* z,
                                                size_t count, int group_size, double* out,
                                                void* hip_stream) {
  if (n < 2 || n > 62) return fail(JUQCS_ERR_ARG, "n must be in [2, 62]");
  return branch_amplitudes(n, gates, gate_count, side, z, 1, count, group_size, out,
                           (hipStream_t)hip_stream, false);
}

extern "C" juqcs_status juqcs_branch_amplitudes_wide(int n, const juqcs_gate* gates, size_t gate_count,
                                                     const uint8_t* side, const uint64_t* z, int words,
                                                     size_t count, int group_size, double* out,
                                                     void* hip_stream) {
  return branch_amplitudes(n, gates, gate_count, side, z, words, count, group_size, out,
                           (hipStream_t)hip_stream, false);
}

extern "C" juqcs_status juqcs_branch_amplitudes_device(int n, const juqcs_gate* gates,
                                                       size_t gate_count, const uint8_t* side,
                                                       const uint64_t* d_z, int words, size_t count,
                                                       int group_size, double* d_out,
                                                       void* hip_stream) {
  return branch_amplitudes(n, gates, gate_count, side, d_z, words, count, group_size, d_out,
                           (hipStream_t)hip_stream, true);
}
