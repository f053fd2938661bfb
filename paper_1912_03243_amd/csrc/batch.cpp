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
#include <memory>
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

// Byte layout of a batch work list in device memory (every part 256-aligned).
struct ListLayout {
  size_t o_groups = 0, o_passes = 0, o_ops = 0, o_mats = 0, o_tickets = 0, o_soff = 0, o_nq = 0,
         o_pos = 0, total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxBatchQubits = 32;            // layout entries per circuit
constexpr size_t kBatchStage = size_t(4) << 20;  // read-out staging after the list

// Layout of a list of count circuits with the given totals of passes (one
// group per pass), ops and coefficients, and the most passes of one circuit.
ListLayout list_layout(int64_t count, int64_t passes, int64_t ops, int64_t mats, int64_t nrounds) {
  ListLayout l;
  l.o_groups = 0;
  l.o_passes = align256(l.o_groups + passes * sizeof(BatchGroup));
  l.o_ops = align256(l.o_passes + passes * sizeof(BatchPass));
  l.o_mats = align256(l.o_ops + std::max<int64_t>(ops, 1) * sizeof(TileOp));
  l.o_tickets = align256(l.o_mats + std::max<int64_t>(mats, 1) * sizeof(cplx<float>));
  l.o_soff = align256(l.o_tickets + std::max<int64_t>(nrounds, 1) * sizeof(uint64_t));
  l.o_nq = align256(l.o_soff + count * sizeof(uint64_t));
  l.o_pos = align256(l.o_nq + count * sizeof(int32_t));
  l.total = align256(l.o_pos + (size_t)count * kMaxBatchQubits);
  return l;
}

ListLayout list_layout_of(const std::vector<TilePlan>& plans) {
  int64_t passes = 0, ops = 0, mats = 0, rounds = 0;
  for (const TilePlan& p : plans) {
    passes += (int64_t)p.passes.size();
    ops += (int64_t)p.ops.size();
    mats += (int64_t)p.mats.size();
    rounds = std::max<int64_t>(rounds, (int64_t)p.passes.size());
  }
  return list_layout((int64_t)plans.size(), passes, ops, mats, rounds);
}

// Host image of a work list: uploaded as is, then addressed through lay.
struct HostList {
  std::vector<char> image;
  ListLayout lay;
  BatchDevice dev{};  // round tables and counts; device pointers set by bind_list
  int64_t tasks = 0, gate_apps = 0, passes = 0;
};

}  // namespace

struct juqcs_batch {
  int count = 0;
  std::vector<int32_t> n;
  std::vector<uint64_t> state_off;
  char* states = nullptr;
  std::vector<std::vector<Gate>> dec;  // decoded gates (the autotuner re-plans from them)
  bool relabel = true;
  HostList list;
  std::vector<int> kin;     // chosen on-chip fusion width per circuit
  std::vector<int8_t> pos;  // kMaxBatchQubits per circuit: physical bit of each qubit at the end
  std::vector<char> keep;   // per circuit (empty: none): start from the state in the buffer, not |0...0>
  // caller-owned workspace: the uploaded list, then the read-out staging
  char* work = nullptr;
  size_t work_bytes = 0;
  bool bound = false;
  BatchDevice dev{};
  uint64_t* d_state_off = nullptr;
  int32_t* d_nq = nullptr;
  int8_t* d_pos = nullptr;
  hipStream_t last_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t graph_stream = nullptr;
};

namespace {

void drop_graph(juqcs_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_stream = nullptr;
}

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

// Lays the plans out as one work list image (pass-major groups).
juqcs_status make_list(juqcs_batch* B, const std::vector<TilePlan>& plans, HostList* L) {
  std::vector<BatchPass> passes;
  std::vector<TileOp> ops;
  std::vector<cplx<float>> mats;
  std::vector<BatchGroup> groups;
  std::vector<int> first_pass(B->count);
  L->tasks = L->gate_apps = L->passes = 0;
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
    L->tasks += ntiles * (int64_t)p.passes.size();
    L->passes += (int64_t)p.passes.size();
    L->gate_apps += p.gates;
  }
  // pass-major order: pass index within the circuit, then circuit
  std::stable_sort(groups.begin(), groups.end(), [&](const BatchGroup& a, const BatchGroup& b) {
    return (a.pass - first_pass[a.circuit]) < (b.pass - first_pass[b.circuit]);
  });
  // rounds: groups of the same pass index, contiguous after the sort
  BatchDevice& d = L->dev;
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
  d.ngroups = (int)groups.size();
  d.count = B->count;
  d.nchunks = next;
  L->lay = list_layout(B->count, (int64_t)passes.size(), (int64_t)ops.size(), (int64_t)mats.size(),
                       d.nrounds);
  const ListLayout& l = L->lay;
  if (B->pos.size() != (size_t)B->count * kMaxBatchQubits) set_layout(B, 0, {});
  L->image.assign(l.total, 0);
  char* h = L->image.data();
  std::memcpy(h + l.o_groups, groups.data(), groups.size() * sizeof(BatchGroup));
  std::memcpy(h + l.o_passes, passes.data(), passes.size() * sizeof(BatchPass));
  std::memcpy(h + l.o_ops, ops.data(), ops.size() * sizeof(TileOp));
  std::memcpy(h + l.o_mats, mats.data(), mats.size() * sizeof(cplx<float>));
  std::memcpy(h + l.o_soff, B->state_off.data(), B->count * sizeof(uint64_t));
  std::memcpy(h + l.o_nq, B->n.data(), B->count * sizeof(int32_t));
  std::memcpy(h + l.o_pos, B->pos.data(), B->pos.size());
  return JUQCS_OK;
}

// Uploads a list image into dbuf (at least L.lay.total bytes) on stream s and
// points dev at it.
juqcs_status bind_list(const HostList& L, char* dbuf, BatchDevice* dev, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dbuf, L.image.data(), L.lay.total, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "batch list upload");
  *dev = L.dev;
  dev->groups = (const BatchGroup*)(dbuf + L.lay.o_groups);
  dev->passes = (const BatchPass*)(dbuf + L.lay.o_passes);
  dev->ops = (const TileOp*)(dbuf + L.lay.o_ops);
  dev->mats = (const cplx<float>*)(dbuf + L.lay.o_mats);
  dev->tickets = (uint64_t*)(dbuf + L.lay.o_tickets);
  return JUQCS_OK;
}

juqcs_status run_device(char* states, const BatchDevice& d, hipStream_t s) {
  hipError_t e = launch_batch(states, d, s);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  return JUQCS_OK;
}

// Timed trial of one circuit's plan (used by the autotuner): runs it as a
// one-circuit batch on the circuit's own state region, with its work list
// at the start of the batch's workspace.  Infinite when the list does not fit.
double time_plan(juqcs_batch* B, int c, const TilePlan& plan, hipStream_t s) {
  juqcs_batch T;
  T.count = 1;
  T.n = {B->n[c]};
  T.state_off = {B->state_off[c]};
  std::vector<TilePlan> plans{plan};
  HostList L;
  if (make_list(&T, plans, &L) != JUQCS_OK || L.lay.total > B->work_bytes) return 1e30;
  BatchDevice d{};
  if (bind_list(L, B->work, &d, s) != JUQCS_OK) return 1e30;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  (void)run_device(B->states, d, s);  // warm
  (void)hipEventRecord(a, s);
  (void)run_device(B->states, d, s);
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = 1e30f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

juqcs_status check_bound(const juqcs_batch* B) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  if (!B->bound) return fail(JUQCS_ERR_ARG, "batch has no workspace bound (juqcs_batch_bind)");
  return JUQCS_OK;
}

}  // namespace

extern "C" {

juqcs_status juqcs_batch_create(juqcs_batch** out, int count, const int* n,
                                const juqcs_gate* gates, const int64_t* offsets, void* d_states,
                                size_t states_bytes, const uint64_t* state_offset,
                                const juqcs_plan_opts* opts) {
  if (!out) return fail(JUQCS_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (count < 1) return fail(JUQCS_ERR_ARG, "count must be >= 1");
  if (!n || !offsets || !d_states || !state_offset) return fail(JUQCS_ERR_ARG, "null argument");
  if (((uintptr_t)d_states & 15) != 0) return fail(JUQCS_ERR_ARG, "state buffer not 16-byte aligned");
  if (offsets[0] != 0) return fail(JUQCS_ERR_ARG, "offsets[0] must be 0");
  std::vector<std::pair<uint64_t, uint64_t>> ranges(count);
  for (int c = 0; c < count; ++c) {
    if (n[c] < 1 || n[c] > 30) return fail(JUQCS_ERR_ARG, "batch circuits need 1 <= n <= 30");
    if (offsets[c + 1] < offsets[c]) return fail(JUQCS_ERR_ARG, "offsets must not decrease");
    if (state_offset[c] & 15) return fail(JUQCS_ERR_ARG, "state offsets must be 16-byte aligned");
    const uint64_t bytes = uint64_t(8) << n[c];
    if (state_offset[c] > states_bytes || bytes > states_bytes - state_offset[c])
      return fail(JUQCS_ERR_SIZE, "circuit " + std::to_string(c) + ": state past the end of the buffer");
    ranges[c] = {state_offset[c], state_offset[c] + bytes};
  }
  std::sort(ranges.begin(), ranges.end());
  for (int c = 1; c < count; ++c)
    if (ranges[c].first < ranges[c - 1].second) return fail(JUQCS_ERR_ARG, "state regions overlap");
  if (offsets[count] > 0 && !gates) return fail(JUQCS_ERR_ARG, "null gate array");
  const int fuse = opts ? opts->fuse_k : 0;
  if (opts && (opts->relabel < -1 || opts->relabel > 1)) return fail(JUQCS_ERR_ARG, "relabel must be -1, 0 or 1");
  if (fuse < 0 || fuse > 4) return fail(JUQCS_ERR_ARG, "batch fuse_k must be 0 (auto) or 1..4");
  auto* B = new juqcs_batch();
  B->count = count;
  B->n.assign(n, n + count);
  B->state_off.assign(state_offset, state_offset + count);
  B->states = (char*)d_states;
  B->relabel = !opts || opts->relabel >= 0;
  B->kin.assign(count, 2);
  set_layout(B, 0, {});
  B->dec.resize(count);
  std::string err;
  for (int c = 0; c < count; ++c) {
    B->dec[c].resize(offsets[c + 1] - offsets[c]);
    for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i)
      if (!decode_gate(gates[i], n[c], &B->dec[c][i - offsets[c]], &err)) {
        delete B;
        const bool numeric = err.find("non-finite") != std::string::npos;
        return fail(numeric ? JUQCS_ERR_NUMERIC : JUQCS_ERR_QUBIT,
                    "circuit " + std::to_string(c) + ": " + err);
      }
  }
  // fusion width: fixed, or the cost model's choice per circuit (the timed
  // trials of juqcs_batch_autotune may replace it)
  std::vector<TilePlan> plans(count);
  parallel_for(count, [&](int c) {
    TileSchedule sched;
    schedule_circuit(n[c], B->dec[c], &sched, B->relabel);
    set_layout(B, c, sched.final_pos);
    if (fuse > 0) {
      emit_schedule(sched, B->dec[c], fuse, &plans[c], 0, batch_mma_cap());
      B->kin[c] = fuse;
      return;
    }
    double best = 1e300;
    for (int k = 2; k <= 4; ++k) {
      TilePlan p;
      emit_schedule(sched, B->dec[c], k, &p, 0, batch_mma_cap());
      const double cst = plan_cost(p);
      if (cst < best) {
        best = cst;
        plans[c] = std::move(p);
        B->kin[c] = k;
      }
    }
  });
  juqcs_status rc = make_list(B, plans, &B->list);
  if (rc != JUQCS_OK) {
    delete B;
    return rc;
  }
  *out = B;
  return JUQCS_OK;
}

juqcs_status juqcs_batch_bytes(const juqcs_batch* B, size_t* work_bytes) {
  if (!B || !work_bytes) return fail(JUQCS_ERR_ARG, "null argument");
  *work_bytes = align256(B->list.lay.total) + kBatchStage;
  return JUQCS_OK;
}

juqcs_status juqcs_batch_bind(juqcs_batch* B, void* d_work, size_t work_bytes, void* hip_stream) {
  if (!B) return fail(JUQCS_ERR_ARG, "null batch");
  if (!d_work) return fail(JUQCS_ERR_ARG, "null workspace");
  if (((uintptr_t)d_work & 255) != 0) return fail(JUQCS_ERR_ARG, "workspace not 256-byte aligned");
  size_t need = 0;
  (void)juqcs_batch_bytes(B, &need);
  if (work_bytes < need) return fail(JUQCS_ERR_SIZE, "batch workspace smaller than juqcs_batch_bytes");
  hipStream_t s = (hipStream_t)hip_stream;
  if (B->last_stream) (void)hipStreamSynchronize(B->last_stream);
  drop_graph(B);
  B->work = (char*)d_work;
  B->work_bytes = work_bytes;
  B->bound = false;
  if (juqcs_status rc = bind_list(B->list, B->work, &B->dev, s)) return rc;
  const ListLayout& l = B->list.lay;
  B->d_state_off = (uint64_t*)(B->work + l.o_soff);
  B->d_nq = (int32_t*)(B->work + l.o_nq);
  B->d_pos = (int8_t*)(B->work + l.o_pos);
  hipError_t e = hipStreamSynchronize(s);  // the host image may change after this call
  if (e != hipSuccess) return hip_fail(e, "batch bind");
  B->bound = true;
  B->last_stream = s;
  return JUQCS_OK;
}

juqcs_status juqcs_batch_autotune(juqcs_batch* B, void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  drop_graph(B);
  B->bound = false;  // the trials overwrite the uploaded list
  std::map<int, int> best_k;
  for (int c = 0; c < B->count; ++c) {
    if (best_k.count(B->n[c])) continue;
    double best = 1e30;
    int bk = B->kin[c];
    for (int k = 1; k <= 4; ++k) {
      TilePlan p;
      plan_circuit(B->n[c], B->dec[c], k, B->relabel, &p);
      const double t = time_plan(B, c, p, s);
      if (t < best) {
        best = t;
        bk = k;
      }
    }
    best_k[B->n[c]] = bk;
  }
  std::vector<TilePlan> plans(B->count);
  parallel_for(B->count, [&](int c) {
    B->kin[c] = best_k[B->n[c]];
    TileSchedule sched;
    plan_circuit(B->n[c], B->dec[c], B->kin[c], B->relabel, &plans[c], &sched);
    set_layout(B, c, sched.final_pos);
  });
  return make_list(B, plans, &B->list);
}

juqcs_status juqcs_batch_run(juqcs_batch* B, void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  B->last_stream = s;
  if (!s) return run_device(B->states, B->dev, s);  // the legacy default stream cannot be captured
  if (!B->gexec || B->graph_stream != s) {
    drop_graph(B);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    juqcs_status rc = run_device(B->states, B->dev, s);
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
  if (tasks) *tasks = B->list.tasks;
  if (gate_apps) *gate_apps = B->list.gate_apps;
  if (passes) *passes = B->list.passes;
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

juqcs_status juqcs_batch_amplitudes_device(juqcs_batch* B, const uint64_t* d_idx, int m,
                                           double* d_out, void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  if (m < 0 || (m > 0 && (!d_idx || !d_out))) return fail(JUQCS_ERR_ARG, "bad index list");
  hipError_t e = launch_batch_gather(B->states, B->d_state_off, B->d_nq, B->d_pos, B->count, m, d_idx,
                                     d_out, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "batch gather launch");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_amplitudes(juqcs_batch* B, const uint64_t* idx, int m, double* out,
                                    void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  if (m < 0 || (m > 0 && (!idx || !out))) return fail(JUQCS_ERR_ARG, "bad index list");
  if (m == 0) return JUQCS_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  // circuits in chunks whose indices and results fit the staging area
  const size_t per = (size_t)m * (sizeof(uint64_t) + 2 * sizeof(double));
  const int chunk = (int)std::max<size_t>(1, kBatchStage / per);
  if ((size_t)m * (sizeof(uint64_t) + 2 * sizeof(double)) > kBatchStage)
    return fail(JUQCS_ERR_SIZE, "too many amplitudes per circuit for the staging area");
  char* stage = B->work + align256(B->list.lay.total);
  uint64_t* d_idx = (uint64_t*)stage;
  double* d_out = (double*)(stage + align256((size_t)chunk * m * sizeof(uint64_t)));
  for (int c0 = 0; c0 < B->count; c0 += chunk) {
    const int c1 = std::min(B->count, c0 + chunk);
    const size_t k = (size_t)(c1 - c0) * m;
    hipError_t e = hipMemcpyAsync(d_idx, idx + (size_t)c0 * m, k * sizeof(uint64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = launch_batch_gather(B->states, B->d_state_off + c0, B->d_nq + c0,
                              B->d_pos + (size_t)c0 * kMaxBatchQubits, c1 - c0, m, d_idx, d_out, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out + 2 * (size_t)c0 * m, d_out, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch amplitudes");
  }
  return JUQCS_OK;
}

juqcs_status juqcs_batch_norms_device(juqcs_batch* B, double* d_out, void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  if (!d_out) return fail(JUQCS_ERR_ARG, "null output");
  hipError_t e = launch_batch_norms(B->states, B->d_state_off, B->d_nq, B->count, d_out,
                                    (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "batch norms launch");
  return JUQCS_OK;
}

juqcs_status juqcs_batch_norms(juqcs_batch* B, double* out, void* hip_stream) {
  if (juqcs_status rc = check_bound(B)) return rc;
  if (!out) return fail(JUQCS_ERR_ARG, "null output");
  hipStream_t s = (hipStream_t)hip_stream;
  double* d_out = (double*)(B->work + align256(B->list.lay.total));
  const int chunk = (int)(kBatchStage / sizeof(double));
  for (int c0 = 0; c0 < B->count; c0 += chunk) {
    const int c1 = std::min(B->count, c0 + chunk);
    hipError_t e = launch_batch_norms(B->states, B->d_state_off + c0, B->d_nq + c0, c1 - c0, d_out, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out + c0, d_out, (c1 - c0) * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch norms");
  }
  return JUQCS_OK;
}

juqcs_status juqcs_batch_destroy(juqcs_batch* B) {
  if (!B) return JUQCS_OK;
  if (B->last_stream) (void)hipStreamSynchronize(B->last_stream);
  drop_graph(B);
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

// In-pass fusion width of the part-state trees.  Measured on MI355X: 3-qubit
// clusters (8x8 ops on the FP32 matrix cores) made the 24-qubit halves of the
// 48-qubit grid 13% faster than 2-qubit ones, and the 21-qubit halves of the
// 42-qubit grid 16% slower (there every segment is a short run of gates on a
// state of only 256 tiles).
int branch_fusion_width(int nloc) { return nloc >= 24 ? 3 : 2; }

// Cuts the part before every run of its crossings (consecutive gates of the
// part), whatever the group size: the cut points and the segments' plans do
// not depend on which crossings a group fixes, so a leaf goes through the
// same plans, and holds the same bits, for any group size.  Each segment is
// planned where the previous one left the qubits.
void cut_part(BranchPart* bp) {
  const std::vector<std::pair<int, int>>& fr = bp->slots;
  const int ng = (int)bp->gates.size();
  bp->segs.clear();
  BranchSeg pre;
  pre.g1 = fr.empty() ? ng : fr[0].first;
  bp->segs.push_back(std::move(pre));
  for (size_t i = 0; i < fr.size();) {
    size_t j = i + 1;
    while (j < fr.size() && fr[j].first == fr[j - 1].first + 1) ++j;
    BranchSeg sg;
    sg.g0 = fr[i].first;
    sg.g1 = j < fr.size() ? fr[j].first : ng;
    for (size_t t = i; t < j; ++t) sg.ks.push_back(fr[t].second);
    bp->segs.push_back(std::move(sg));
    i = j;
  }
  std::vector<int> pos(bp->nloc);
  for (int q = 0; q < bp->nloc; ++q) pos[q] = q;
  for (BranchSeg& sg : bp->segs) {
    sg.gates.assign(bp->gates.begin() + sg.g0, bp->gates.begin() + sg.g1);
    for (Gate& g : sg.gates)
      for (int j = 0; j < g.nq; ++j) g.q[j] = pos[g.q[j]];
    plan_circuit(bp->nloc, sg.gates, branch_fusion_width(bp->nloc), true, &sg.tmpl, &sg.sched);
    if (!sg.sched.final_pos.empty())
      for (int q = 0; q < bp->nloc; ++q) pos[q] = sg.sched.final_pos[pos[q]];
  }
  bp->phys = pos;
}

// Marks the crossings >= L as free (their bits vary within a group).
void set_free(BranchPart* bp, int L) {
  bp->freek.clear();
  for (auto& f : bp->slots)
    if (f.second >= L) bp->freek.push_back(f.second);
  for (BranchSeg& sg : bp->segs) {
    sg.nfree = 0;
    for (int k : sg.ks) sg.nfree += k >= L ? 1 : 0;
  }
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

// What the Eq. (3) driver derives from the circuit before it touches the
// device: the parts, their circuits with a placeholder diagonal at every
// crossing, and their segments' plans.
struct BranchJob {
  int n = 0, P = 0, m = 0, words = 0;
  size_t count = 0;
  bool host_io = false;  // bitstrings and result in host arrays (staged in the workspace)
  int local[kBranchMaxQubits] = {};
  int nloc[kBranchMaxParts] = {};
  BranchPart parts[kBranchMaxParts];
};

juqcs_status branch_prepare(int n, const juqcs_gate* gates, size_t gate_count, const uint8_t* side,
                            int words, size_t count, bool host_io, BranchJob* J) {
  if (n < 2 || n > kBranchMaxQubits) return fail(JUQCS_ERR_ARG, "n must be in [2, 240]");
  if (words < (n + 63) / 64 || words > kBranchMaxWords)
    return fail(JUQCS_ERR_ARG, "words must be in [ceil(n / 64), 4]");
  if (!side || (gate_count > 0 && !gates)) return fail(JUQCS_ERR_ARG, "null argument");
  if (count > (size_t)1 << 31) return fail(JUQCS_ERR_SIZE, "at most 2^31 bitstrings");
  J->n = n;
  J->words = words;
  J->count = count;
  J->host_io = host_io;
  // parts and local qubit numbers (ascending order inside a part)
  int P = 0;
  for (int q = 0; q < n; ++q) {
    if (side[q] >= kBranchMaxParts)
      return fail(JUQCS_ERR_ARG, "side[q] must be < " + std::to_string(kBranchMaxParts));
    P = std::max(P, side[q] + 1);
  }
  for (int q = 0; q < n; ++q) J->local[q] = J->nloc[side[q]]++;
  if (P < 2) return fail(JUQCS_ERR_ARG, "at least two parts");
  for (int p = 0; p < P; ++p)
    if (J->nloc[p] < 1 || J->nloc[p] > 30) return fail(JUQCS_ERR_ARG, "each part needs 1..30 qubits");
  J->P = P;
  // part circuits with placeholder diagonals at every crossing gate; a
  // crossing CNOT is its CZ between Hadamards on the target (H X H = Z)
  BranchPart* parts = J->parts;
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
      h.q[0] = J->local[t];
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
        d.q[0] = J->local[q];
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
    for (int j = 0; j < g.nq; ++j) g.q[j] = J->local[g.q[j]];
    parts[p].gates.push_back(g);
  }
  J->m = m;
  for (int p = 0; p < P; ++p) {
    parts[p].nloc = J->nloc[p];
    parts[p].sbytes = align256((size_t)8 << J->nloc[p]);
    cut_part(&parts[p]);
  }
  return JUQCS_OK;
}

// Workspace of a decomposition run whose groups fix the first L crossings
// (2^(m-L) branches per group); byte offsets in the caller's buffer.
struct BranchLayout {
  int L = 0;
  long long gsize = 1, ngroups = 1;
  int nleaves = 0;
  bool lds = false;
  int32_t first[kBranchMaxParts + 1] = {};  // leaves part by part
  size_t base[kBranchMaxParts] = {};        // byte offset of part p's leaves in the state region
  size_t o_z = 0, o_zp = 0, o_tab = 0, o_bad = 0, o_acc = 0, o_off = 0, o_sum = 0, o_states = 0,
         o_list = 0, total = 0;
};

// Free bits of segment sg and of the segments before it, with the first L
// crossings fixed.
int seg_free(const BranchSeg& sg, int L) {
  int f = 0;
  for (int k : sg.ks) f += k >= L ? 1 : 0;
  return f;
}

BranchLayout branch_layout(const BranchJob& J, int L) {
  BranchLayout B;
  const int P = J.P, m = J.m;
  B.L = L;
  B.gsize = 1ll << (m - L);
  B.ngroups = 1ll << L;
  size_t states = 0;
  for (int p = 0; p < P; ++p) {
    const int R = J.parts[p].free_bits(L);
    B.first[p + 1] = B.first[p] + (1 << R);
    B.base[p] = states;
    states += J.parts[p].sbytes << R;
  }
  B.nleaves = B.first[P];
  B.lds = B.nleaves <= kBranchSumValues;
  // the largest tree round's work list
  size_t rounds = 0;
  for (int p = 0; p < P; ++p) rounds = std::max(rounds, J.parts[p].segs.size());
  size_t list = 0;
  for (size_t r = 0; r < rounds; ++r) {
    int64_t count = 0, passes = 0, ops = 0, mats = 0, nr = 0;
    for (int p = 0; p < P; ++p) {
      const BranchPart& bp = J.parts[p];
      if (r >= bp.segs.size()) continue;
      int done = 0;
      for (size_t i = 0; i < r; ++i) done += seg_free(bp.segs[i], L);
      const int64_t nodes = int64_t(1) << (done + seg_free(bp.segs[r], L));
      const TilePlan& t = bp.segs[r].tmpl;
      // an empty segment still runs one pass (the tree node's copy or init)
      const int64_t np = std::max<int64_t>(1, (int64_t)t.passes.size());
      count += nodes;
      passes += nodes * np;
      ops += nodes * (int64_t)t.ops.size();
      mats += nodes * (int64_t)t.mats.size();
      nr = std::max(nr, np);
    }
    list = std::max(list, list_layout(count, passes, ops, mats, nr).total);
  }
  const size_t cnt = J.count;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  B.o_z = take(J.host_io ? cnt * J.words * sizeof(uint64_t) : 0);
  B.o_zp = take((size_t)P * cnt * sizeof(uint32_t));
  B.o_tab = take(kBranchTabInts * sizeof(int32_t));
  B.o_bad = take(sizeof(int));
  B.o_acc = take(J.host_io ? cnt * 2 * sizeof(double) : 0);
  B.o_off = take((size_t)B.nleaves * sizeof(uint64_t));
  B.o_sum = take(B.lds ? (size_t)B.gsize * sizeof(uint64_t) : (size_t)B.gsize * P * sizeof(int32_t));
  B.o_states = take(states);
  B.o_list = take(list);
  B.total = o;
  return B;
}

thread_local juqcs_branch_stats g_branch_stats{};

// L for a group size (rounded down to a power of two; 0 = every branch).
int group_bits(int m, int group_size) {
  if (group_size <= 0) return 0;
  int lg = 0;
  while (lg < m && (2ll << lg) <= group_size) ++lg;
  return m - lg;
}

// Eq. (3) for count bitstrings of words 64-bit words each (see
// juqcs_branch_amplitudes_wide), in the caller's workspace.  dev: z and out
// are device pointers (the bitstrings are checked on the device), else host
// arrays.
juqcs_status branch_amplitudes(int n, const juqcs_gate* gates, size_t gate_count, const uint8_t* side,
                               const uint64_t* z, int words, size_t count, int group_size, double* out,
                               void* d_work, size_t work_bytes, hipStream_t s, bool dev) {
  if (count > 0 && (!z || !out)) return fail(JUQCS_ERR_ARG, "null argument");
  auto J = std::make_unique<BranchJob>();
  if (juqcs_status rc = branch_prepare(n, gates, gate_count, side, words, count, !dev, J.get())) return rc;
  // bits at or above n must be clear (only the words that can hold them)
  for (int w = n / 64; !dev && w < words; ++w) {
    const int lo = std::max(0, n - 64 * w);
    const uint64_t bad = lo >= 64 ? 0 : ~0ull << lo;
    for (size_t k = 0; k < count; ++k)
      if (z[k * words + w] & bad) return fail(JUQCS_ERR_ARG, "bitstring >= 2^n");
  }
  if (count == 0) return JUQCS_OK;
  if (!d_work) return fail(JUQCS_ERR_ARG, "null workspace (juqcs_branch_bytes gives its size)");
  if (((uintptr_t)d_work & 255) != 0) return fail(JUQCS_ERR_ARG, "workspace not 256-byte aligned");
  const int P = J->P, m = J->m;
  BranchPart* parts = J->parts;
  // Branches are grouped by the bits of the first L crossings (circuit
  // order; those bits are fixed within a group, the others free).  Inside a
  // group a part's states form a tree: the gates before its first crossing
  // run once, and every run of its crossings splits each state into one
  // copy per setting of their free bits, which then runs the gates up to
  // the next run.  The leaves are the part's states for every setting of
  // its own free crossings; branches that agree on those share a leaf.
  BranchLayout lay;
  if (group_size > 0) {
    lay = branch_layout(*J, group_bits(m, group_size));
    if (lay.total > work_bytes) return fail(JUQCS_ERR_SIZE, "workspace too small for the group size");
  } else {
    int L = 0;
    while (L < m && branch_layout(*J, L).total > work_bytes) ++L;
    lay = branch_layout(*J, L);
    if (lay.total > work_bytes) return fail(JUQCS_ERR_SIZE, "workspace too small for one branch");
  }
  const int L = lay.L;
  const long long gsize = lay.gsize, ngroups = lay.ngroups;
  for (int p = 0; p < P; ++p) set_free(&parts[p], L);
  juqcs_branch_stats stats{};
  stats.crossings = m;
  stats.group_bits = L;
  stats.groups = ngroups;
  stats.lds_sum = lay.lds ? 1 : 0;
  stats.sum_flops = (double)count * std::ldexp(1.0, m) * (6.0 * (P - 1) + 2.0);
  char* W = (char*)d_work;
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
        phys[o] = parts[p].phys[J->local[q]];
        ++o;
      }
    }
    first[P] = o;
  }
  const int nleaves = lay.nleaves;
  std::vector<uint64_t> leaf_off(nleaves);
  for (int p = 0; p < P; ++p)
    for (int l = 0; l < (1 << parts[p].freek.size()); ++l)
      leaf_off[lay.first[p] + l] = lay.base[p] + (size_t)l * parts[p].sbytes;
  // the sum runs over branches in tree order: t ascending, where bit
  // m-1-k of t is crossing k's bit; a group is a range of t
  auto branch_of = [&](long long t) {
    long long b = 0;
    for (int k = 0; k < m; ++k) b |= ((t >> (m - 1 - k)) & 1) << k;
    return b;
  };
  const bool lds = lay.lds;
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
      if (lds) t8[j] |= (uint64_t)(lay.first[p] + l) << (8 * p);
      else t32[(size_t)j * P + p] = lay.first[p] + l;
    }
  }
  // bitstrings -> per-part indices on the device; acc holds the running sum
  // (the caller's out when it is on the device)
  uint64_t* dz = dev ? nullptr : (uint64_t*)(W + lay.o_z);
  uint32_t* zp = (uint32_t*)(W + lay.o_zp);
  int32_t* dtab = (int32_t*)(W + lay.o_tab);
  int* dbad = (int*)(W + lay.o_bad);
  double* acc = dev ? out : (double*)(W + lay.o_acc);
  uint64_t* doff = (uint64_t*)(W + lay.o_off);
  void* dsum = W + lay.o_sum;
  char* states = W + lay.o_states;
  char* dlist = W + lay.o_list;
  const size_t tbytes = lds ? t8.size() * 8 : t32.size() * 4;
  hipError_t e = hipSuccess;
  if (!dev) e = hipMemcpyAsync(dz, z, count * words * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(doff, leaf_off.data(), nleaves * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dsum, lds ? (const void*)t8.data() : (const void*)t32.data(), tbytes,
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_zero(dbad, sizeof(int), s);
  if (e == hipSuccess)
    e = launch_branch_split(dev ? z : dz, words, (long long)count, P, n, dtab, zp, dbad, s);
  if (e == hipSuccess) e = launch_zero(acc, count * 2 * sizeof(double), s);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
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
            {
              double f = 0.0;
              for (const Gate& x : sg.gates) f += gate_flops(x);
              stats.gate_flops += f * std::ldexp(1.0, bp.nloc);
              stats.pass_bytes += (double)std::max<size_t>(1, plans.back().passes.size()) * 16.0 *
                                  std::ldexp(1.0, bp.nloc);
              stats.tile_passes += (int64_t)std::max<size_t>(1, plans.back().passes.size());
              ++stats.tree_states;
            }
            B.n.push_back(bp.nloc);
            B.state_off.push_back(lay.base[p] + (size_t)leaf * bp.sbytes);
            B.keep.push_back(r > 0 ? 1 : 0);
            if (r > 0 && c > 0) {  // the child starts as a copy of its parent
              e = hipMemcpyAsync(states + B.state_off.back(), states + lay.base[p] + (size_t)parent * bp.sbytes,
                                 bp.sbytes, hipMemcpyDeviceToDevice, s);
              if (e != hipSuccess) rc = hip_fail(e, "branch state copy");
            }
          }
      }
      B.count = (int)plans.size();
      B.states = states;
      if (rc == JUQCS_OK && B.count > 0) {
        HostList hl;
        BatchDevice d{};
        rc = make_list(&B, plans, &hl);
        if (rc == JUQCS_OK && hl.lay.total > lay.total - lay.o_list)
          rc = fail(JUQCS_ERR_SIZE, "branch round list larger than its workspace share");
        if (rc == JUQCS_OK) rc = bind_list(hl, dlist, &d, s);
        if (rc == JUQCS_OK) rc = run_device(states, d, s);
        if (rc == JUQCS_OK) {
          // the host image must outlive its upload
          e = hipStreamSynchronize(s);
          if (e != hipSuccess) rc = hip_fail(e, "branch batch");
        }
      }
    }
    if (rc == JUQCS_OK) {
      const bool last = gi + 1 == ngroups;
      const double scale = std::ldexp(1.0, -m);
      if (lds) {
        BranchParts bp{};
        for (int p = 0; p <= P; ++p) bp.first[p] = lay.first[p];
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
  if (rc == JUQCS_OK) g_branch_stats = stats;
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// The decomposition without a caller workspace: everything beyond the
// caller's bitstrings and result lives in one file-scope device array of
// JUQCS_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  Host
// code never passes the array's name to a kernel or a copy: it takes the
// array's device address on each device from hipGetSymbolAddress (once per
// device, with that device current) and passes that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[JUQCS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;           // one call at a time per process: calls share the array
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of the scratch array on the current device.
juqcs_status scratch_on_current_device(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return fail(JUQCS_ERR_UNSUPPORTED, "device index above 63");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return JUQCS_OK;
}

}  // namespace

extern "C" juqcs_status juqcs_branch_amplitudes_noalloc(int n, const juqcs_gate* gates,
                                                        size_t gate_count, const uint8_t* side,
                                                        const uint64_t* d_z, int words, size_t count,
                                                        int group_size, double* d_out,
                                                        void* hip_stream) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  size_t need = 0;
  if (count > 0) {
    auto J = std::make_unique<BranchJob>();
    if (juqcs_status rc = branch_prepare(n, gates, gate_count, side, words, count, false, J.get()))
      return rc;
    need = branch_layout(*J, group_size > 0 ? group_bits(J->m, group_size) : J->m).total;
    if (need > (size_t)JUQCS_NOALLOC_SCRATCH_BYTES)
      return fail(JUQCS_ERR_SIZE, "the decomposition needs " + std::to_string(need) +
                                      " bytes of workspace; the static scratch holds " +
                                      std::to_string((size_t)JUQCS_NOALLOC_SCRATCH_BYTES));
  }
  void* ws = nullptr;
  if (count > 0)
    if (juqcs_status rc = scratch_on_current_device(&ws)) return rc;
  return branch_amplitudes(n, gates, gate_count, side, d_z, words, count, group_size, d_out, ws,
                           count > 0 ? (size_t)JUQCS_NOALLOC_SCRATCH_BYTES : 0, (hipStream_t)hip_stream,
                           true);
}

extern "C" juqcs_status juqcs_branch_last_stats(juqcs_branch_stats* out) {
  if (!out) return fail(JUQCS_ERR_ARG, "null output");
  *out = g_branch_stats;
  return JUQCS_OK;
}

extern "C" juqcs_status juqcs_branch_bytes(int n, const juqcs_gate* gates, size_t gate_count,
                                           const uint8_t* side, int words, size_t count,
                                           int group_size, int host_io, size_t* min_bytes,
                                           size_t* bytes) {
  if (!min_bytes || !bytes) return fail(JUQCS_ERR_ARG, "null output");
  auto J = std::make_unique<BranchJob>();
  if (juqcs_status rc = branch_prepare(n, gates, gate_count, side, words, count, host_io != 0, J.get()))
    return rc;
  *min_bytes = branch_layout(*J, J->m).total;
  *bytes = branch_layout(*J, group_bits(J->m, group_size)).total;
  return JUQCS_OK;
}

extern "C" juqcs_status juqcs_branch_amplitudes(int n, const juqcs_gate* gates, size_t gate_count,
                                                const uint8_t* side, const uint64_t* z,
                                                size_t count, int group_size, double* out,
                                                void* d_work, size_t work_bytes,
                                                void* hip_stream) {
  if (n < 2 || n > 62) return fail(JUQCS_ERR_ARG, "n must be in [2, 62]");
  return branch_amplitudes(n, gates, gate_count, side, z, 1, count, group_size, out, d_work, work_bytes,
                           (hipStream_t)hip_stream, false);
}

extern "C" juqcs_status juqcs_branch_amplitudes_wide(int n, const juqcs_gate* gates, size_t gate_count,
                                                     const uint8_t* side, const uint64_t* z, int words,
                                                     size_t count, int group_size, double* out,
                                                     void* d_work, size_t work_bytes,
                                                     void* hip_stream) {
  return branch_amplitudes(n, gates, gate_count, side, z, words, count, group_size, out, d_work,
                           work_bytes, (hipStream_t)hip_stream, false);
}

extern "C" juqcs_status juqcs_branch_amplitudes_device(int n, const juqcs_gate* gates,
                                                       size_t gate_count, const uint8_t* side,
                                                       const uint64_t* d_z, int words, size_t count,
                                                       int group_size, double* d_out,
                                                       void* d_work, size_t work_bytes,
                                                       void* hip_stream) {
  return branch_amplitudes(n, gates, gate_count, side, d_z, words, count, group_size, d_out, d_work,
                           work_bytes, (hipStream_t)hip_stream, true);
}
