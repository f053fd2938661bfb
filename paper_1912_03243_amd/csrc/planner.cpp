// Host-side planning: gate decoding, tile-pass selection with on-chip fusion,
// and dense k-qubit block fusion.  Pure C++ (no device code).
//
// Reordering rule used everywhere: a gate may move earlier past any gate that
// acts on none of its qubits (gates on disjoint qubits commute), so every
// plan computes the same product as the circuit order, up to rounding.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "juqcs_internal.hpp"

namespace juqcs {

namespace {

using C = cplx<double>;

inline C cx(double re, double im) { return C{re, im}; }
inline C cadd(C a, C b) { return C{a.re + b.re, a.im + b.im}; }

bool finite(C z) { return std::isfinite(z.re) && std::isfinite(z.im); }

// One nonzero entry per row, in distinct columns: row r reads column
// sigma(r), packed 3 bits per row (dim <= 8).
bool monomial(const C* m, int dim, int* sigma) {
  int packed = 0, used = 0;
  for (int r = 0; r < dim; ++r) {
    int col = -1;
    for (int c = 0; c < dim; ++c) {
      const C z = m[r * dim + c];
      if (z.re != 0.0 || z.im != 0.0) {
        if (col >= 0) return false;
        col = c;
      }
    }
    if (col < 0 || (used >> col) & 1) return false;
    used |= 1 << col;
    packed |= col << (3 * r);
  }
  *sigma = packed;
  return true;
}

bool is_diag(const C* m, int dim) {
  for (int r = 0; r < dim; ++r)
    for (int c = 0; c < dim; ++c)
      if (r != c && (m[r * dim + c].re != 0.0 || m[r * dim + c].im != 0.0)) return false;
  return true;
}

// A fused cluster: qubit list + dense matrix over it (index sum_j b_{q[j]} 2^j).
struct Cluster {
  std::vector<int> q;
  std::vector<C> m;
  std::vector<int> gates;  // merge order
};

bool touches(const Cluster& c, const Gate& g) {
  for (int x : c.q)
    for (int j = 0; j < g.nq; ++j)
      if (x == g.q[j]) return true;
  return false;
}

// Qubits of a cluster and a gate together.
int union_size(const Cluster& c, const Gate& g) {
  int k = (int)c.q.size();
  for (int j = 0; j < g.nq; ++j)
    if (std::find(c.q.begin(), c.q.end(), g.q[j]) == c.q.end()) ++k;
  return k;
}

// Fold gate g into cluster c (g applied after c), re-expressed on the union
// of their qubits (the cluster's order, then the gate's new qubits): the
// cluster matrix is widened by identities on the new qubits, and g's rows
// are combined over the index bits of its qubits, column by column.
void merge_into(Cluster& c, const Gate& g) {
  int u[8];
  const int kold = (int)c.q.size();
  int k = kold;
  for (int i = 0; i < kold; ++i) u[i] = c.q[i];
  for (int j = 0; j < g.nq; ++j)
    if (std::find(u, u + k, g.q[j]) == u + k) u[k++] = g.q[j];
  const int dim = 1 << k, dold = 1 << kold;
  std::vector<C> a((size_t)dim * dim, cx(0, 0));
  for (int r = 0; r < dim; ++r)
    for (int cc = 0; cc < dim; ++cc)
      if ((r >> kold) == (cc >> kold))
        a[(size_t)r * dim + cc] = kold == 0 ? cx(r == cc ? 1 : 0, 0)
                                            : c.m[(size_t)(r & (dold - 1)) * dold + (cc & (dold - 1))];
  int pos[2] = {0, 0}, gmask = 0;
  for (int j = 0; j < g.nq; ++j) {
    pos[j] = (int)(std::find(u, u + k, g.q[j]) - u);
    gmask |= 1 << pos[j];
  }
  const int gd = 1 << g.nq;
  int off[4];
  for (int t = 0; t < gd; ++t) {
    off[t] = 0;
    for (int j = 0; j < g.nq; ++j) off[t] |= ((t >> j) & 1) << pos[j];
  }
  std::vector<C> out(a);
  for (int r0 = 0; r0 < dim; ++r0) {
    if (r0 & gmask) continue;
    for (int cc = 0; cc < dim; ++cc) {
      C v[4];
      for (int t = 0; t < gd; ++t) v[t] = a[(size_t)(r0 | off[t]) * dim + cc];
      for (int t = 0; t < gd; ++t) {
        C acc = cx(0, 0);
        for (int t2 = 0; t2 < gd; ++t2) acc = cmad(g.m[t * gd + t2], v[t2], acc);
        out[(size_t)(r0 | off[t]) * dim + cc] = acc;
      }
    }
  }
  c.q.assign(u, u + k);
  c.m.swap(out);
}

// Greedy fusion: each gate joins the most recent cluster it may legally join
// (no later cluster touches its qubits) whose union with the gate has at most
// kmax qubits, preferring one that already shares a qubit; otherwise it opens
// a new cluster.  The backward scan is bounded to keep planning linear.
void fuse(const std::vector<Gate>& gates, const std::vector<int>& order, int kmax,
          std::vector<Cluster>* out) {
  constexpr int kScan = 64;
  std::vector<Cluster>& cl = *out;
  cl.clear();
  for (int gi : order) {
    const Gate& g = gates[gi];
    int chosen = -1, fallback = -1;
    for (int i = (int)cl.size() - 1; i >= 0 && (int)cl.size() - 1 - i < kScan; --i) {
      const bool t = touches(cl[i], g);
      const bool fits = union_size(cl[i], g) <= kmax;
      if (t) {
        if (fits) chosen = i;
        break;
      }
      if (fits && fallback < 0) fallback = i;
    }
    if (chosen < 0) chosen = fallback;
    if (chosen < 0) {
      cl.push_back(Cluster{});
      chosen = (int)cl.size() - 1;
    }
    merge_into(cl[chosen], g);
    cl[chosen].gates.push_back(gi);
  }
}

}  // namespace

bool decode_gate(const juqcs_gate& g, int n, Gate* out, std::string* err) {
  Gate r{};
  const double s2 = 1.0 / std::sqrt(2.0);
  auto set2 = [&](C a, C b, C c, C d) {
    r.nq = 1;
    r.m[0] = a;
    r.m[1] = b;
    r.m[2] = c;
    r.m[3] = d;
  };
  auto check_q = [&](int q) { return q >= 0 && q < n; };
  r.q[0] = g.q0;
  r.q[1] = g.q1;
  switch (g.op) {
    case JUQCS_OP_H: set2(cx(s2, 0), cx(s2, 0), cx(s2, 0), cx(-s2, 0)); break;
    case JUQCS_OP_X: set2(cx(0, 0), cx(1, 0), cx(1, 0), cx(0, 0)); break;
    case JUQCS_OP_Y: set2(cx(0, 0), cx(0, -1), cx(0, 1), cx(0, 0)); break;
    case JUQCS_OP_Z: set2(cx(1, 0), cx(0, 0), cx(0, 0), cx(-1, 0)); break;
    case JUQCS_OP_S: set2(cx(1, 0), cx(0, 0), cx(0, 0), cx(0, 1)); break;
    case JUQCS_OP_T:
      set2(cx(1, 0), cx(0, 0), cx(0, 0), cx(std::cos(M_PI / 4), std::sin(M_PI / 4)));
      break;
    case JUQCS_OP_U:
      set2(cx(g.u[0], g.u[1]), cx(g.u[2], g.u[3]), cx(g.u[4], g.u[5]), cx(g.u[6], g.u[7]));
      break;
    case JUQCS_OP_CNOT:
    case JUQCS_OP_CZ:
    case JUQCS_OP_CP: {
      r.nq = 2;
      for (int i = 0; i < 16; ++i) r.m[i] = cx(0, 0);
      if (g.op == JUQCS_OP_CNOT) {  // index b_control + 2 b_target
        r.m[0 * 4 + 0] = cx(1, 0);
        r.m[2 * 4 + 2] = cx(1, 0);
        r.m[1 * 4 + 3] = cx(1, 0);
        r.m[3 * 4 + 1] = cx(1, 0);
      } else {
        r.m[0] = r.m[5] = r.m[10] = cx(1, 0);
        r.m[15] = g.op == JUQCS_OP_CZ ? cx(-1, 0) : cx(std::cos(g.theta), std::sin(g.theta));
      }
      break;
    }
    default:
      *err = "unknown gate op " + std::to_string(g.op);
      return false;
  }
  if (!check_q(r.q[0]) || (r.nq == 2 && !check_q(r.q[1]))) {
    *err = "gate qubit out of range";
    return false;
  }
  if (r.nq == 2 && r.q[0] == r.q[1]) {
    *err = "two-qubit gate with equal qubits";
    return false;
  }
  if (r.nq == 1) r.q[1] = -1;
  const int dim = 1 << r.nq;
  for (int i = 0; i < dim * dim; ++i)
    if (!finite(r.m[i])) {
      *err = "non-finite matrix entry";
      return false;
    }
  r.diag = is_diag(r.m, dim);
  *out = r;
  return true;
}

// Algorithmic flops per state amplitude of a gate, counted on the matrix
// as given: a dense 2x2 is two complex products and a sum per amplitude
// (14); a diagonal touches a half (3 when its first entry is 1) or every
// amplitude (6); controlled forms touch a half (7) or, when diagonal, a
// quarter (1.5; 0.5 for a sign flip); a controlled X only moves data; a
// dense 4x4 is four complex products and three sums (30).
double gate_flops(const Gate& g) {
  const auto eq = [](C a, double re, double im) { return a.re == re && a.im == im; };
  if (g.nq == 1) {
    if (!g.diag) return 14.0;
    return eq(g.m[0], 1.0, 0.0) ? 3.0 : 6.0;
  }
  // controlled form (index b_q0 + 2 b_q1): rows and columns with b_q0 = 0 identity
  bool ctrl = true;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      if (((r & 1) == 0 || (c & 1) == 0) && !eq(g.m[4 * r + c], r == c ? 1.0 : 0.0, 0.0)) ctrl = false;
  if (!ctrl) return 30.0;
  const C u00 = g.m[5], u01 = g.m[7], u10 = g.m[13], u11 = g.m[15];
  if (eq(u00, 0, 0) && eq(u11, 0, 0) && eq(u01, 1, 0) && eq(u10, 1, 0)) return 0.0;  // CNOT
  if (eq(u01, 0, 0) && eq(u10, 0, 0) && eq(u00, 1, 0)) return eq(u11, -1, 0) ? 0.5 : 1.5;
  return 7.0;
}

// ---------------------------------------------------------------------------
// Tile planning
// ---------------------------------------------------------------------------
namespace {

// Qubit masks of the gates rem lists (n <= 40 qubits fit one word).
std::vector<uint64_t> rem_masks(const std::vector<Gate>& gates, const std::vector<int>& rem) {
  std::vector<uint64_t> m(rem.size());
  for (size_t i = 0; i < rem.size(); ++i) {
    const Gate& g = gates[rem[i]];
    uint64_t x = 0;
    for (int j = 0; j < g.nq; ++j) x |= uint64_t(1) << g.q[j];
    m[i] = x;
  }
  return m;
}

// Number of gates at the front of the remaining list (as qubit masks)
// absorbable by the tile: a gate is taken if its qubits are in the tile and
// none of them is blocked by an earlier gate that was not taken.
int absorb_count(const std::vector<uint64_t>& rm, uint64_t tile) {
  uint64_t blocked = 0;
  int cnt = 0;
  for (uint64_t m : rm) {
    if (!(m & ~tile) && !(m & blocked)) {
      ++cnt;
    } else {
      blocked |= m;
      if (!(tile & ~blocked)) break;  // every tile qubit blocked
    }
  }
  return cnt;
}

uint64_t tile_mask(const std::vector<char>& in_tile) {
  uint64_t t = 0;
  for (size_t q = 0; q < in_tile.size(); ++q)
    if (in_tile[q]) t |= uint64_t(1) << q;
  return t;
}

void emit_ops(const std::vector<Cluster>& cl, const TileGeom& geom, TilePlan* plan) {
  auto local = [&](int p) {
    if (p < geom.L) return p;
    for (int j = 0; j < geom.H; ++j)
      if (geom.hbits[j] == p) return geom.L + j;
    return -1;
  };
  for (const Cluster& c : cl) {
    TileOp op{};
    const int k = (int)c.q.size();
    const int dim = 1 << k;
    op.k = k;
    op.moff = (int64_t)plan->mats.size();
    int sigma = 0;
    if (is_diag(c.m.data(), dim) && k <= 2) {
      op.kind = TOP_DIAG2;
      op.a = local(c.q[0]);
      op.b = k == 2 ? local(c.q[1]) : -1;
      for (int r = 0; r < 4; ++r) plan->mats.push_back(c.m[(r % dim) * dim + (r % dim)]);
    } else if (k <= 3 && monomial(c.m.data(), dim, &sigma)) {
      // permutations with phases (CNOT, X, SWAP, CZ chains, ...): one
      // coefficient per row instead of a dense matrix
      op.kind = TOP_PERM;
      op.a = sigma;
      op.b = -1;
      for (int j = 0; j < k; ++j) op.bits[j] = local(c.q[j]);
      for (int r = 0; r < dim; ++r) plan->mats.push_back(c.m[r * dim + ((sigma >> (3 * r)) & 7)]);
    } else if (k == 1) {
      op.kind = TOP_DENSE1;
      op.a = local(c.q[0]);
      op.b = -1;
      for (int i = 0; i < 4; ++i) plan->mats.push_back(c.m[i]);
    } else if (k == 2) {
      op.kind = TOP_DENSE2;
      op.a = local(c.q[0]);
      op.b = local(c.q[1]);
      for (int i = 0; i < 16; ++i) plan->mats.push_back(c.m[i]);
    } else {
      op.kind = k == 3 ? TOP_DENSE3 : TOP_DENSE4;
      op.a = op.b = -1;
      for (int j = 0; j < k; ++j) op.bits[j] = local(c.q[j]);
      for (int i = 0; i < dim * dim; ++i) plan->mats.push_back(c.m[i]);
    }
    plan->ops.push_back(op);
    plan->op_gates.push_back(c.gates);
  }
}

}  // namespace

void select_tiles(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                  TileSchedule* sched, int max_take) {
  sched->passes.clear();
  sched->taken.clear();
  sched->gates = (int64_t)gates.size();
  if (n <= b) {
    L = n;
    b = n;
  }
  const int H = b - L;
  std::vector<int> rem(gates.size());
  for (size_t i = 0; i < gates.size(); ++i) rem[i] = (int)i;
  constexpr int kCandidates = 24;
  while (!rem.empty()) {
    std::vector<char> in_tile(n, 0);
    for (int q = 0; q < L; ++q) in_tile[q] = 1;
    std::vector<int> chosen;
    if (H > 0) {
      std::vector<int> cand;
      std::vector<char> seen(n, 0);
      for (int gi : rem) {
        const Gate& g = gates[gi];
        for (int j = 0; j < g.nq; ++j) {
          const int q = g.q[j];
          if (q >= L && !seen[q]) {
            seen[q] = 1;
            cand.push_back(q);
          }
        }
        if ((int)cand.size() >= kCandidates) break;
      }
      // greedy: add the candidate that lets the most gates through
      const std::vector<uint64_t> rm = rem_masks(gates, rem);
      for (int step = 0; step < H; ++step) {
        int best = -1, bc = -1;
        const uint64_t base = tile_mask(in_tile);
        for (int c : cand) {
          if (in_tile[c]) continue;
          const int v = absorb_count(rm, base | (uint64_t(1) << c));
          if (v > bc) {
            bc = v;
            best = c;
          }
        }
        if (best < 0) {
          // fewer candidates than slots: fill with unused high bits
          for (int q = n - 1; q >= L; --q)
            if (!in_tile[q]) {
              best = q;
              break;
            }
        }
        in_tile[best] = 1;
        chosen.push_back(best);
      }
    }
    std::sort(chosen.begin(), chosen.end());
    // absorb
    std::vector<int> taken, keep;
    std::vector<char> blocked(n, 0);
    for (int gi : rem) {
      const Gate& g = gates[gi];
      bool ok = max_take <= 0 || (int)taken.size() < max_take;
      for (int j = 0; j < g.nq; ++j)
        if (!in_tile[g.q[j]] || blocked[g.q[j]]) ok = false;
      if (ok) {
        taken.push_back(gi);
      } else {
        keep.push_back(gi);
        for (int j = 0; j < g.nq; ++j) blocked[g.q[j]] = 1;
      }
    }
    if (taken.empty()) {  // the front gate cannot fit any tile: give up
      sched->gates -= (int64_t)rem.size();
      return;
    }
    TilePass pass{};
    pass.g.n = n;
    pass.g.L = L;
    pass.g.H = H;
    pass.g.b = b;
    pass.g.block_bits = block_bits;
    for (int j = 0; j < H; ++j) pass.g.hbits[j] = chosen[j];
    pass.g.maxk = 1;
    sched->passes.push_back(pass);
    sched->taken.push_back(std::move(taken));
    rem.swap(keep);
  }
}

namespace {

// Greedy choice of a b-qubit tile for the front of rem.  Starts from the
// qubits marked in `fixed` (kept), then adds the candidate that lets the
// most gates through, one at a time; a qubit outside `near` may be added
// only while fewer than `far_cap` such qubits were taken.
std::vector<char> pick_tile(int n, int b, const std::vector<Gate>& gates, const std::vector<int>& rem,
                            const std::vector<char>& fixed, const std::vector<char>& near, int far_cap) {
  constexpr int kCandidates = 32;
  std::vector<char> in_tile(fixed);
  int count = 0, far = 0;
  for (int q = 0; q < n; ++q) count += in_tile[q] ? 1 : 0;
  std::vector<int> cand;
  std::vector<char> seen(n, 0);
  for (int gi : rem) {
    const Gate& g = gates[gi];
    for (int j = 0; j < g.nq; ++j) {
      const int q = g.q[j];
      if (!seen[q] && !in_tile[q]) {
        seen[q] = 1;
        cand.push_back(q);
      }
    }
    if ((int)cand.size() >= kCandidates) break;
  }
  const std::vector<uint64_t> rm = rem_masks(gates, rem);
  while (count < b) {
    int best = -1, bc = -1;
    const uint64_t base = tile_mask(in_tile);
    for (int c : cand) {
      if (in_tile[c] || (!near[c] && far >= far_cap)) continue;
      const int v = absorb_count(rm, base | (uint64_t(1) << c));
      if (v > bc) {
        bc = v;
        best = c;
      }
    }
    if (best < 0)  // candidates used up: any admissible qubit, nearby ones first
      for (int round = 0; round < 2 && best < 0; ++round)
        for (int q = n - 1; q >= 0; --q)
          if (!in_tile[q] && (near[q] || (round == 1 && far < far_cap))) {
            best = q;
            break;
          }
    in_tile[best] = 1;
    ++count;
    if (!near[best]) ++far;
  }
  return in_tile;
}

}  // namespace

namespace {

// Rank of the bank-slot directions the first w lanes of the write-back of a
// relabeling pass reach (local element swap(e) is read for destination e;
// the kernels' LDS slot map folds bits s.. and 2s.. onto the low s bits:
// s = 4 for 16-byte and 5 for 8-byte amplitudes; an access phase covers
// 2^w lanes, w = 3 and 4).  Full rank: no bank conflicts.
int writeback_slot_rank(const TileGeom& g, int s, int w) {
  int span = 1, rank = 0;
  for (int j = 0; j < w; ++j) {
    const int e = swap_local(1 << j, g);
    const int v = (e ^ (((e >> s) ^ (e >> (2 * s))) & ((1 << s) - 1))) & ((1 << w) - 1);
    if ((span >> v) & 1) continue;
    ++rank;
    int grown = span;
    for (int u = 0; u < (1 << w); ++u)
      if ((span >> u) & 1) grown |= 1 << (u ^ v);
    span = grown;
  }
  return rank;
}

}  // namespace

void select_tiles_relabel(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                          TileSchedule* sched, int max_take) {
  sched->final_pos.resize(n);
  for (int q = 0; q < n; ++q) sched->final_pos[q] = q;
  sched->tgates.clear();
  sched->tsrc.clear();
  if (n <= b) {
    select_tiles(n, L, b, block_bits, gates, sched, max_take);
    sched->tgates = gates;  // a single tile: nothing moves
    sched->tsrc.resize(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) sched->tsrc[i] = (int)i;
    return;
  }
  sched->passes.clear();
  sched->taken.clear();
  sched->gates = (int64_t)gates.size();
  const int H = b - L;
  // Qubits are named by their physical bit before the schedule ("wires");
  // pos[w] is the wire's current physical bit, at[p] the wire at bit p.
  std::vector<int> pos(n), at(n);
  for (int q = 0; q < n; ++q) pos[q] = at[q] = q;
  std::vector<int> rem(gates.size());
  for (size_t i = 0; i < gates.size(); ++i) rem[i] = (int)i;
  auto low_wires = [&]() {
    std::vector<char> m(n, 0);
    for (int p = 0; p < L; ++p) m[at[p]] = 1;
    return m;
  };
  const std::vector<char> none(n, 0), all(n, 1);
  std::vector<char> tile = pick_tile(n, b, gates, rem, low_wires(), all, n);
  while (!rem.empty()) {
    // absorb, in order, the gates whose qubits are all in the tile
    std::vector<int> taken, keep;
    std::vector<char> blocked(n, 0);
    for (int gi : rem) {
      const Gate& g = gates[gi];
      bool ok = max_take <= 0 || (int)taken.size() < max_take;
      for (int j = 0; j < g.nq; ++j)
        if (!tile[g.q[j]] || blocked[g.q[j]]) ok = false;
      if (ok) {
        Gate t = g;
        for (int j = 0; j < t.nq; ++j) t.q[j] = pos[t.q[j]];
        taken.push_back((int)sched->tgates.size());
        sched->tgates.push_back(t);
        sched->tsrc.push_back(gi);
      } else {
        keep.push_back(gi);
        for (int j = 0; j < g.nq; ++j) blocked[g.q[j]] = 1;
      }
    }
    if (taken.empty()) {  // the front gate cannot fit any tile: give up
      sched->gates -= (int64_t)rem.size();
      break;
    }
    TilePass pass{};
    pass.g.n = n;
    pass.g.L = L;
    pass.g.H = H;
    pass.g.b = b;
    pass.g.block_bits = block_bits;
    pass.g.maxk = 1;
    std::vector<int> hp;
    for (int w = 0; w < n; ++w)
      if (tile[w] && pos[w] >= L) hp.push_back(pos[w]);
    std::sort(hp.begin(), hp.end());
    for (int j = 0; j < H; ++j) pass.g.hbits[j] = hp[j];
    rem.swap(keep);
    if (!rem.empty()) {
      // next tile: the low qubits kept, or any b qubits with at most H from
      // outside this tile (its low L then come from this tile), whichever
      // lets more gates through (ties keep the low qubits: no swaps)
      std::vector<char> kept = pick_tile(n, b, gates, rem, low_wires(), all, n);
      std::vector<char> moved = pick_tile(n, b, gates, rem, none, tile, H);
      // new low wires if moving: those already low stay; the rest come from
      // moved & tile
      std::vector<char> nl(n, 0);
      int cnt = 0;
      for (int p = 0; p < L; ++p)
        if (moved[at[p]]) nl[at[p]] = 1, ++cnt;
      std::vector<int> in, out;
      for (int w = 0; w < n && cnt < L; ++w)
        if (moved[w] && tile[w] && !nl[w]) nl[w] = 1, ++cnt, in.push_back(w);
      for (int p = 0; p < L; ++p)
        if (!nl[at[p]]) out.push_back(at[p]);
      const std::vector<uint64_t> rm = rem_masks(gates, rem);
      if (cnt == L && in.size() == out.size() && (int)in.size() <= kSwapCap &&
          absorb_count(rm, tile_mask(moved)) > absorb_count(rm, tile_mask(kept))) {
        // wire in[i] (gathered in this pass) trades places with out[i] (low);
        // the pairing is free, pick the one whose write-back keeps the LDS
        // lanes of an access phase in distinct bank slots
        std::vector<int> lin(in.size());
        for (size_t i = 0; i < in.size(); ++i)
          lin[i] = L + (int)(std::lower_bound(hp.begin(), hp.end(), pos[in[i]]) - hp.begin());
        std::vector<int> perm(out.size()), best_perm;
        for (size_t i = 0; i < out.size(); ++i) perm[i] = (int)i;
        int best_score = -1;
        do {
          TileGeom t{};
          t.nswap = (int)in.size();
          for (size_t i = 0; i < in.size(); ++i) {
            t.swap_a[i] = (int8_t)pos[out[perm[i]]];
            t.swap_b[i] = (int8_t)lin[i];
          }
          const int score = 8 * writeback_slot_rank(t, 4, 3) + writeback_slot_rank(t, 5, 4);
          if (score > best_score) {
            best_score = score;
            best_perm = perm;
          }
        } while (std::next_permutation(perm.begin(), perm.end()));
        std::vector<int> out2(out.size());
        for (size_t i = 0; i < out.size(); ++i) out2[i] = out[best_perm[i]];
        out.swap(out2);
        for (size_t i = 0; i < in.size(); ++i) {
          const int x = in[i], y = out[i], px = pos[x], py = pos[y];
          const int lx = L + (int)(std::lower_bound(hp.begin(), hp.end(), px) - hp.begin());
          pass.g.swap_a[pass.g.nswap] = (int8_t)py;
          pass.g.swap_b[pass.g.nswap] = (int8_t)lx;
          ++pass.g.nswap;
          pos[x] = py;
          pos[y] = px;
          at[py] = x;
          at[px] = y;
        }
        tile = moved;
      } else {
        tile = kept;
      }
    }
    sched->passes.push_back(pass);
    sched->taken.push_back(std::move(taken));
  }
  sched->final_pos = pos;
}

// Whether emit_ops makes a cluster an 8x8 (TOP_DENSE3) op.
bool cluster_mma(const Cluster& c) {
  int sigma = 0;
  return c.q.size() == 3 && !monomial(c.m.data(), 8, &sigma);
}

// Coefficients emit_ops stores for a cluster.
int cluster_coefs(const Cluster& c) {
  const int k = (int)c.q.size();
  int sigma = 0;
  if (k <= 2 && is_diag(c.m.data(), 1 << k)) return 4;
  if (k <= 3 && monomial(c.m.data(), 1 << k, &sigma)) return 1 << k;
  return (1 << k) * (1 << k);
}

void emit_schedule(const TileSchedule& sched, const std::vector<Gate>& gates, int kin,
                   TilePlan* plan, int max_mats, int max_mma) {
  plan->passes.clear();
  plan->ops.clear();
  plan->mats.clear();
  plan->op_gates.clear();
  plan->gates = sched.gates;
  kin = std::max(1, std::min(kin, 4));  // on-chip fusion width
  const std::vector<Gate>& src = sched.tgates.empty() ? gates : sched.tgates;
  for (size_t i = 0; i < sched.passes.size(); ++i) {
    std::vector<Cluster> cl;
    fuse(src, sched.taken[i], kin, &cl);
    // consecutive runs of clusters whose coefficients fit max_mats and whose
    // 8x8 ops fit max_mma
    size_t c0 = 0;
    do {
      size_t c1 = c0;
      int coefs = 0, mma = 0;
      while (c1 < cl.size()) {
        const int w = cluster_coefs(cl[c1]);
        const int x = cluster_mma(cl[c1]) ? 1 : 0;
        if (c1 > c0 && ((max_mats > 0 && coefs + w > max_mats) || (max_mma > 0 && mma + x > max_mma) ||
                        (int)(c1 - c0) >= kPassOps))
          break;
        coefs += w;
        mma += x;
        ++c1;
      }
      const std::vector<Cluster> part(cl.begin() + c0, cl.begin() + c1);
      TilePass pass = sched.passes[i];
      if (c1 < cl.size()) pass.g.nswap = 0;  // swaps after the pass's last ops
      pass.op_begin = (int32_t)plan->ops.size();
      const int64_t m0 = (int64_t)plan->mats.size();
      emit_ops(part, pass.g, plan);
      pass.op_count = (int32_t)plan->ops.size() - pass.op_begin;
      pass.g.mat_count = (int32_t)((int64_t)plan->mats.size() - m0);
      pass.g.mma_count = mma;
      pass.g.maxk = 1;
      for (const Cluster& c : part) pass.g.maxk = std::max(pass.g.maxk, (int32_t)c.q.size());
      plan->passes.push_back(pass);
      c0 = c1;
    } while (c0 < cl.size());
  }
}

void plan_tiles(int n, int L, int b, int block_bits, const std::vector<Gate>& gates,
                TilePlan* plan, int kin, int max_mats, int max_take, int max_mma, bool relabel,
                std::vector<int>* final_pos) {
  TileSchedule sched;
  if (relabel) {
    select_tiles_relabel(n, L, b, block_bits, gates, &sched, max_take);
  } else {
    select_tiles(n, L, b, block_bits, gates, &sched, max_take);
    sched.final_pos.resize(n);
    for (int q = 0; q < n; ++q) sched.final_pos[q] = q;
  }
  emit_schedule(sched, gates, kin, plan, max_mats, max_mma);
  if (final_pos) *final_pos = sched.final_pos;
}

void rebuild_mats(const std::vector<Gate>& gates, TilePlan* plan) {
  for (size_t o = 0; o < plan->ops.size(); ++o) {
    Cluster c;
    for (int gi : plan->op_gates[o]) merge_into(c, gates[gi]);
    const TileOp& op = plan->ops[o];
    const int k = (int)c.q.size(), dim = 1 << k;
    C* dst = plan->mats.data() + op.moff;
    if (op.kind == TOP_DIAG2) {
      for (int r = 0; r < 4; ++r) dst[r] = c.m[(r % dim) * dim + (r % dim)];
    } else if (op.kind == TOP_PERM) {
      for (int r = 0; r < dim; ++r) dst[r] = c.m[r * dim + ((op.a >> (3 * r)) & 7)];
    } else {
      for (int i = 0; i < dim * dim; ++i) dst[i] = c.m[i];
    }
  }
}

void plan_fused(int n, int kmax, const std::vector<Gate>& gates, std::vector<FusedBlock>* blocks) {
  (void)n;
  std::vector<int> order(gates.size());
  for (size_t i = 0; i < gates.size(); ++i) order[i] = (int)i;
  std::vector<Cluster> cl;
  fuse(gates, order, kmax, &cl);
  blocks->clear();
  for (Cluster& c : cl) {
    FusedBlock fb;
    fb.targets = c.q;
    fb.m = c.m;
    blocks->push_back(std::move(fb));
  }
}

}  // namespace juqcs
