// LD-Leiden CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, single-threaded, deliberately unoptimised implementation of the LD-Leiden batch
// update (Algorithm 1 of the paper) used to check the GPU library result-for-result.  Only
// the tests, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
// code, header or constant with the GPU library.
//
// Paper references (LD-Leiden: Local Parallel Community Detection in Large Dynamic Networks):
//   Sec. II          problem statement, batch semantics, Eq. 1 (directed weighted modularity)
//   Sec. III-A       incremental hierarchy: levels G^r, parent maps pi_r, level labels P^r
//   Sec. III-B       per-level frontier (active nodes)
//   Sec. III-C       Algorithm 1 (Update / Levels / Move / Refine / Agg. / Stop blocks)
//   Sec. III-D       Eq. 2 one-step gain
//   Sec. III-E       decoupled moves: sort by gain, emitter/acceptor filter
//   Sec. III-F       Eq. 3 aggregate weights and subtract-add repair
// Where the paper leaves a step open, the reading taken is stated next to the code.
//
// Representation: an undirected graph is the symmetric matrix W (Sec. II); every level
// stores matrix entries, so m = sum_ij W_ij counts each undirected edge twice.  All weights,
// degrees, totals and gains are exact integers; gamma = gp/gq.  For a move of v from a to b
// the exact change of q*m^2*Q (Eq. 1, with a' = a minus v) is
//   directed:   G = q m (acc[b]-acc[a]) - p (kout_v (Kin_b-Kin_a+kin_v) + kin_v (Kout_b-Kout_a+kout_v))
//   undirected: G = q m (acc[b]-acc[a]) - p k_v (K_b - K_a + k_v)      (half of the directed value)
// where acc[c] sums the weights of v's entries to/from nodes u != v with label c (undirected:
// one row).  Eq. 2 differs from this only by terms independent of the target b.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace {

typedef int64_t i64;
typedef __int128 i128;

enum { OK = 0, EINVAL_ = -1, EDUP_ = -2, ENOEDGE_ = -3, EOVERFLOW_ = -4, ECHECK_ = -100 };

struct Cfg {
  int directed;
  int gp, gq;      // gamma = gp / gq
  int N, L, M;     // outer passes, top level index, move/refine iterations
  int an, ad;      // alpha = an / ad
  int bn, bd;      // beta = bn / bd
  int rn = 0, rd = 1;   // adaptive refresh threshold rho = rn / rd (0: never)
};

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", 2014):
// the output function applied to a 64-bit state.  Its first output for seed s is
// splitmix_mix(s + 0x9E3779B97F4A7C15).
uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef std::vector<std::pair<uint32_t, i64>> Row;  // sorted by column

struct Level {
  std::vector<uint8_t> alive;
  std::vector<Row> out, in;     // `in` is unused for undirected graphs (W symmetric)
  std::vector<i64> kout, kin;   // row / column sums of W (equal when undirected)
  std::vector<uint32_t> lab;    // P^r: move-community label
  std::vector<uint32_t> par;    // pi_r: refined community = level r+1 node id
};

struct NodeSet {
  std::vector<uint8_t> flag;
  std::vector<uint32_t> list;
  void init(uint32_t n) { flag.assign(n, 0); list.clear(); }
  bool add(uint32_t x) {
    if (flag[x]) return false;
    flag[x] = 1; list.push_back(x); return true;
  }
  bool has(uint32_t x) const { return flag[x] != 0; }
  void clear() { for (uint32_t x : list) flag[x] = 0; list.clear(); }
  size_t size() const { return list.size(); }
};

struct Cand {
  uint32_t v, a, b;
  i128 G;
  bool empty = false;   // b is the empty community labelled v (variant, see best_move)
};

struct TraceRec {
  int32_t pass, level, phase, iter;   // phase 0 = move, 1 = refine
  uint64_t nscan, ncand, nacc;
  i64 dq_hi;
  uint64_t dq_lo;
};

i64 row_get(const Row& r, uint32_t c) {
  auto it = std::lower_bound(r.begin(), r.end(), std::make_pair(c, (i64)INT64_MIN));
  if (it != r.end() && it->first == c) return it->second;
  return 0;
}
bool row_has(const Row& r, uint32_t c) {
  auto it = std::lower_bound(r.begin(), r.end(), std::make_pair(c, (i64)INT64_MIN));
  return it != r.end() && it->first == c;
}
struct Tup {
  uint32_t x, y;
  i64 d;
};

// Group tuples by (x, y), sum them and drop the zero sums (a grouped sum as in Eq. 3).
std::vector<Tup> reduce_tuples(std::vector<Tup> t) {
  std::sort(t.begin(), t.end(), [](const Tup& a, const Tup& b) { return a.x != b.x ? a.x < b.x : a.y < b.y; });
  std::vector<Tup> r;
  for (size_t i = 0; i < t.size();) {
    size_t j = i;
    i64 s = 0;
    while (j < t.size() && t[j].x == t[i].x && t[j].y == t[i].y) s += t[j++].d;
    if (s != 0) r.push_back({t[i].x, t[i].y, s});
    i = j;
  }
  return r;
}

// Add sorted, distinct column deltas to a sorted row in one merge pass; an entry that reaches
// zero is removed (Sec. II: zero-weight edges are removed).
void row_merge(Row& row, const std::vector<std::pair<uint32_t, i64>>& dl) {
  Row out;
  out.reserve(row.size() + dl.size());
  size_t i = 0, j = 0;
  while (i < row.size() || j < dl.size()) {
    if (j == dl.size() || (i < row.size() && row[i].first < dl[j].first)) {
      out.push_back(row[i++]);
    } else if (i == row.size() || dl[j].first < row[i].first) {
      out.push_back(dl[j++]);
    } else {
      i64 w = row[i].second + dl[j].second;
      if (w != 0) out.push_back(std::make_pair(row[i].first, w));
      ++i; ++j;
    }
  }
  row.swap(out);
}

struct Oracle {
  Cfg cfg;
  uint32_t n;
  int top = 0;
  std::vector<Level> lv;
  std::vector<i64> Kout, Kin;     // community totals (one table serves every level)
  i64 m = 0, Ein = 0;             // m = sum W; Ein = sum of W over same-label entries
  i128 SKK = 0;                   // sum_c Kout[c] * Kin[c]
  std::vector<NodeSet> D;         // pending seeds per level
  int pass_idx = 0;
  uint64_t refreshes = 0;         // batches that switched to full reoptimisation
  // debugging / checking modes
  int single_move = 0;            // accept only the best candidate per move iteration
  int check_moves = 0;            // recount Q from scratch around every move and refinement commit
  int empty_target = 0;           // variant: BestMove may also move v to an empty community
  int random_refine = 0;          // variant: BestRef picks a random target among improving ones
  uint64_t seed = 0;              // seed of that choice
  uint64_t batches = 0;           // batches accepted so far (creation's is batch 0)
  uint64_t cur_batch = 0;         // index of the batch being applied
  uint64_t rkey = 0;              // key of the current refinement iteration (random_refine)
  uint64_t checks[6] = {0, 0, 0, 0, 0, 0};   // recount checks done: moves, refinements, and of those
                                             // the single-move ones that compared a predicted gain;
                                             // empty-target moves accepted, and of those the
                                             // single-move ones compared with a recount
  std::string err;
  std::vector<TraceRec> trace;
  int tracing = 0;
  // scratch
  std::vector<i64> acc;
  std::vector<uint32_t> acc_touched;
  std::vector<uint8_t> acc_flag;
  static constexpr uint32_t NONE = 0xFFFFFFFFu;
  std::vector<uint32_t> mover_from;

  i128 qnum() const { return (i128)cfg.gq * m * Ein - (i128)cfg.gp * SKK; }

  const Row& inrow(const Level& L, uint32_t v) const { return cfg.directed ? L.in[v] : L.out[v]; }

  void alloc_level(int r) {
    Level& L = lv[r];
    L.alive.assign(n, 0);
    L.out.assign(n, Row());
    if (cfg.directed) L.in.assign(n, Row());
    L.kout.assign(n, 0);
    L.kin.assign(n, 0);
    L.lab.assign(n, 0);
    L.par.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) { L.lab[i] = i; L.par[i] = i; }
  }

  // Apply reduced tuples (distinct keys, nonzero) to level r.
  void apply_reduced(int r, const std::vector<Tup>& t, bool degrees) {
    Level& L = lv[r];
    std::vector<std::pair<uint32_t, i64>> dl;
    for (size_t i = 0; i < t.size();) {
      size_t j = i;
      dl.clear();
      while (j < t.size() && t[j].x == t[i].x) { dl.push_back(std::make_pair(t[j].y, t[j].d)); ++j; }
      row_merge(L.out[t[i].x], dl);
      i = j;
    }
    if (cfg.directed) {
      std::vector<Tup> tt(t.begin(), t.end());
      std::sort(tt.begin(), tt.end(), [](const Tup& a, const Tup& b) { return a.y != b.y ? a.y < b.y : a.x < b.x; });
      for (size_t i = 0; i < tt.size();) {
        size_t j = i;
        dl.clear();
        while (j < tt.size() && tt[j].y == tt[i].y) { dl.push_back(std::make_pair(tt[j].x, tt[j].d)); ++j; }
        row_merge(L.in[tt[i].y], dl);
        i = j;
      }
    }
    if (degrees)
      for (auto& e : t) { L.kout[e.x] += e.d; L.kin[e.y] += e.d; }
  }

  uint32_t anc(uint32_t u, int s) const {
    for (int t = 0; t < s; ++t) u = lv[t].par[u];
    return u;
  }

  void add_total(uint32_t c, i64 dout, i64 din) {
    SKK -= (i128)Kout[c] * Kin[c];
    Kout[c] += dout; Kin[c] += din;
    SKK += (i128)Kout[c] * Kin[c];
  }

  void record(int level, int phase, int iter, uint64_t nscan, uint64_t ncand, uint64_t nacc, i128 dq) {
    if (!tracing) return;
    TraceRec t;
    t.pass = pass_idx; t.level = level; t.phase = phase; t.iter = iter;
    t.nscan = nscan; t.ncand = ncand; t.nacc = nacc;
    t.dq_hi = (i64)(dq >> 64); t.dq_lo = (uint64_t)dq;
    trace.push_back(t);
  }

  // ---------------------------------------------------------------- Eq. 1 from scratch
  // Exact numerator q*m^2*Q of the current ground partition, recomputed from the level-0
  // matrix and the labels induced by level r (ground node u has label P^r(anc_r(u))).
  i128 recount_qnum(int r) const {
    const Level& L0 = lv[0];
    std::vector<i64> ko(n, 0), ki(n, 0);
    i64 mm = 0, ein = 0;
    std::vector<uint32_t> g(n);
    for (uint32_t u = 0; u < n; ++u) g[u] = lv[r].lab[anc(u, r)];
    for (uint32_t u = 0; u < n; ++u)
      for (auto& e : L0.out[u]) {
        mm += e.second;
        ko[g[u]] += e.second;
        ki[g[e.first]] += e.second;
        if (g[u] == g[e.first]) ein += e.second;
      }
    i128 skk = 0;
    for (uint32_t c = 0; c < n; ++c) skk += (i128)ko[c] * ki[c];
    return (i128)cfg.gq * mm * ein - (i128)cfg.gp * skk;
  }

  // Exact numerator of Eq. 1 for the refined partition of level r: ground node u belongs to
  // the refined community pi_r(anc_r(u)).  Refinement moves change this partition only.
  i128 recount_qnum_refined(int r) const {
    const Level& L0 = lv[0];
    std::vector<i64> ko(n, 0), ki(n, 0);
    i64 mm = 0, ein = 0;
    std::vector<uint32_t> g(n);
    for (uint32_t u = 0; u < n; ++u) g[u] = lv[r].par[anc(u, r)];
    for (uint32_t u = 0; u < n; ++u)
      for (auto& e : L0.out[u]) {
        mm += e.second;
        ko[g[u]] += e.second;
        ki[g[e.first]] += e.second;
        if (g[u] == g[e.first]) ein += e.second;
      }
    i128 skk = 0;
    for (uint32_t c = 0; c < n; ++c) skk += (i128)ko[c] * ki[c];
    return (i128)cfg.gq * mm * ein - (i128)cfg.gp * skk;
  }

  // ------------------------------------------------------------------- candidates
  // BestMove_r (Sec. III-D): best adjacent community by the exact gain, ties to the lowest
  // community id, kept only if the gain is strictly positive.
  //
  // Variant (empty_target; the paper considers adjacent communities only, Sec. III-C): v may
  // also move to an empty community, as in the Louvain and Leiden move phases.  The empty
  // community offered to v is the one labelled v itself, when v does not carry label v and the
  // totals of community v are zero (every member, if any, has no incident weight, so the move's
  // gain is that of moving to an empty community: no weight towards it and zero totals).  It is
  // one more candidate with its own id in the comparison above.
  bool best_move(int r, uint32_t v, Cand& out) {
    const Level& L = lv[r];
    const uint32_t a = L.lab[v];
    i64 acc_a = 0;
    acc_touched.clear();
    auto visit = [&](uint32_t u, i64 w) {
      if (u == v) return;
      uint32_t c = L.lab[u];
      if (c == a) { acc_a += w; return; }
      if (!acc_flag[c]) { acc_flag[c] = 1; acc[c] = 0; acc_touched.push_back(c); }
      acc[c] += w;
    };
    for (auto& e : L.out[v]) visit(e.first, e.second);
    if (cfg.directed) for (auto& e : L.in[v]) visit(e.first, e.second);
    bool found = false;
    i128 bestG = 0; uint32_t bestb = 0;
    const i128 qm = (i128)cfg.gq * m;
    for (uint32_t b : acc_touched) {
      i128 G;
      if (cfg.directed) {
        G = qm * (acc[b] - acc_a) -
            (i128)cfg.gp * ((i128)L.kout[v] * (Kin[b] - Kin[a] + L.kin[v]) +
                            (i128)L.kin[v] * (Kout[b] - Kout[a] + L.kout[v]));
      } else {
        G = qm * (acc[b] - acc_a) - (i128)cfg.gp * ((i128)L.kout[v] * (Kout[b] - Kout[a] + L.kout[v]));
      }
      if (!found || G > bestG || (G == bestG && b < bestb)) { found = true; bestG = G; bestb = b; }
    }
    for (uint32_t b : acc_touched) acc_flag[b] = 0;
    bool empty = false;
    if (empty_target && a != v && Kout[v] == 0 && Kin[v] == 0) {
      // the gain above with acc[b] = 0 and Kout[b] = Kin[b] = 0
      i128 G;
      if (cfg.directed)
        G = -qm * acc_a - (i128)cfg.gp * ((i128)L.kout[v] * (L.kin[v] - Kin[a]) + (i128)L.kin[v] * (L.kout[v] - Kout[a]));
      else
        G = -qm * acc_a - (i128)cfg.gp * ((i128)L.kout[v] * (L.kout[v] - Kout[a]));
      if (!found || G > bestG || (G == bestG && v < bestb)) { found = true; bestG = G; bestb = v; empty = true; }
    }
    if (!found || bestG <= 0) return false;
    out.v = v; out.a = a; out.b = bestb; out.G = bestG; out.empty = empty;
    return true;
  }

  // BestRef_r: a singleton refined community {u} joins an adjacent refined community y whose
  // members carry u's move label.  Gain on refined totals Kr (from a singleton there is no
  // acc[a] term): q m acc[y] - p (kout_u Krin_y + kin_u Krout_y); undirected q m acc[y] - p k_u Kr_y.
  //
  // Variant (random_refine): as in the Leiden refinement of Traag et al., the target is drawn at
  // random among the refined communities whose gain is strictly positive, here uniformly (the
  // limit of their exp(gain / theta) weights for large theta, which keeps the choice exact): each
  // such y gets the priority prio(u, y) of a counter-based hash (SplitMix64's output function
  // chained over seed, batch, pass, level, iteration, u and y) and the highest priority wins;
  // equal priorities go to the larger gain, then to the lower id.
  uint32_t prio(uint32_t u, uint32_t y) const { return ref_prio(rkey, u, y); }
  static uint32_t ref_prio(uint64_t key, uint32_t u, uint32_t y) {
    return (uint32_t)(splitmix_mix(splitmix_mix(key ^ u) ^ y) >> 32) | 1u;
  }
  // The choice among the evaluated targets ys with gains Gs: the largest gain (equal gains: the
  // lower id), or with random_refine the highest priority among strictly positive gains.
  // Returns the index of the chosen target, -1 when there is none.
  static int choose_ref(bool random, uint64_t key, uint32_t u, const std::vector<uint32_t>& ys,
                        const std::vector<i128>& Gs) {
    int best = -1;
    uint32_t bestP = 0;
    for (size_t i = 0; i < ys.size(); ++i) {
      const i128 G = Gs[i];
      const uint32_t y = ys[i];
      if (random) {
        if (G <= 0) continue;
        const uint32_t p = ref_prio(key, u, y);
        if (best < 0 || p > bestP || (p == bestP && (G > Gs[best] || (G == Gs[best] && y < ys[best])))) {
          best = (int)i;
          bestP = p;
        }
      } else if (best < 0 || G > Gs[best] || (G == Gs[best] && y < ys[best])) {
        best = (int)i;
      }
    }
    return best;
  }
  bool best_ref(int r, uint32_t u, const std::vector<i64>& Krout, const std::vector<i64>& Krin, Cand& out) {
    const Level& L = lv[r];
    const uint32_t lu = L.lab[u];
    acc_touched.clear();
    auto visit = [&](uint32_t x, i64 w) {
      if (x == u || L.lab[x] != lu) return;
      uint32_t y = L.par[x];
      if (!acc_flag[y]) { acc_flag[y] = 1; acc[y] = 0; acc_touched.push_back(y); }
      acc[y] += w;
    };
    for (auto& e : L.out[u]) visit(e.first, e.second);
    if (cfg.directed) for (auto& e : L.in[u]) visit(e.first, e.second);
    std::vector<i128> Gs;
    const i128 qm = (i128)cfg.gq * m;
    for (uint32_t y : acc_touched) {
      if (cfg.directed)
        Gs.push_back(qm * acc[y] - (i128)cfg.gp * ((i128)L.kout[u] * Krin[y] + (i128)L.kin[u] * Krout[y]));
      else
        Gs.push_back(qm * acc[y] - (i128)cfg.gp * ((i128)L.kout[u] * Krout[y]));
    }
    for (uint32_t y : acc_touched) acc_flag[y] = 0;
    const int k = choose_ref(random_refine != 0, rkey, u, acc_touched, Gs);
    if (k < 0 || Gs[k] <= 0) return false;
    out.v = u; out.a = u; out.b = acc_touched[k]; out.G = Gs[k];
    return true;
  }

  // Decouple (Sec. III-E): sort by decreasing gain (ties: lower node id first), then accept a
  // candidate iff its source is not already an acceptor and its target not already an emitter.
  std::vector<Cand> decouple(std::vector<Cand> c, bool only_first) {
    std::sort(c.begin(), c.end(), [](const Cand& x, const Cand& y) {
      if (x.G != y.G) return x.G > y.G;
      return x.v < y.v;
    });
    std::vector<Cand> acc_list;
    std::map<uint32_t, int> role;  // 1 = emitter, 2 = acceptor
    for (const Cand& x : c) {
      auto ia = role.find(x.a), ib = role.find(x.b);
      bool a_is_acc = ia != role.end() && ia->second == 2;
      bool b_is_emit = ib != role.end() && ib->second == 1;
      if (a_is_acc || b_is_emit) continue;
      role[x.a] = 1; role[x.b] = 2;
      acc_list.push_back(x);
      if (only_first) break;
    }
    return acc_list;
  }

  void neighbours(int r, uint32_t v, NodeSet& into) {
    const Level& L = lv[r];
    for (auto& e : L.out[v]) into.add(e.first);
    if (cfg.directed) for (auto& e : L.in[v]) into.add(e.first);
  }

  // Commit an accepted move batch at level r; returns the exact Delta(q m^2 Q).
  // Delta Ein counts every matrix entry incident to a mover once.
  i128 commit_moves(int r, const std::vector<Cand>& B) {
    Level& L = lv[r];
    for (auto& c : B) mover_from[c.v] = c.a;   // mover -> old label
    auto is_mover = [&](uint32_t x) { return mover_from[x] != NONE; };
    auto old_lab = [&](uint32_t x) { return is_mover(x) ? mover_from[x] : L.lab[x]; };
    const i128 q0 = qnum();
    // labels after the batch
    for (auto& c : B) L.lab[c.v] = c.b;
    i64 dein = 0;
    for (auto& c : B) {
      uint32_t v = c.v;
      for (auto& e : L.out[v]) {
        uint32_t u = e.first;
        int before = old_lab(v) == old_lab(u), after = L.lab[v] == L.lab[u];
        dein += e.second * (after - before);
      }
      for (auto& e : inrow(L, v)) {
        uint32_t u = e.first;
        if (is_mover(u)) continue;  // counted from u's out-row
        int before = old_lab(u) == old_lab(v), after = L.lab[u] == L.lab[v];
        dein += e.second * (after - before);
      }
    }
    for (auto& c : B) mover_from[c.v] = NONE;
    Ein += dein;
    for (auto& c : B) {
      add_total(c.a, -L.kout[c.v], -L.kin[c.v]);
      add_total(c.b, L.kout[c.v], L.kin[c.v]);
    }
    return qnum() - q0;
  }

  void rollback_moves(int r, const std::vector<Cand>& B, i128) {
    Level& L = lv[r];
    // recompute Ein change by reverse commit
    std::vector<Cand> rev;
    for (auto& c : B) { Cand x = c; std::swap(x.a, x.b); rev.push_back(x); }
    commit_moves(r, rev);
    (void)L;
  }

  // ---------------------------------------------------------------- process level r
  void process_level(int r) {
    Level& L = lv[r];
    std::vector<uint32_t> entry = D[r].list;
    D[r].clear();
    // closure (InitFrontier / per-level seeds): alive seeds plus all alive nodes whose label
    // is the label of an alive seed
    NodeSet U; U.init(n);
    {
      std::vector<uint8_t> cm(n, 0);
      for (uint32_t x : entry) if (L.alive[x]) cm[L.lab[x]] = 1;
      for (uint32_t u = 0; u < n; ++u) if (L.alive[u] && cm[L.lab[u]]) U.add(u);
    }
    const i128 Q0 = qnum();
    NodeSet Moved; Moved.init(n);
    for (int j = 1; j <= cfg.M; ++j) {
      // S = U u N_r(U)
      NodeSet S; S.init(n);
      for (uint32_t u : U.list) S.add(u);
      for (uint32_t u : U.list) neighbours(r, u, S);
      std::vector<Cand> cands;
      for (uint32_t v : S.list) { Cand c; if (best_move(r, v, c)) cands.push_back(c); }
      std::vector<Cand> B = decouple(cands, single_move != 0);
      for (auto& c : B) checks[4] += c.empty ? 1 : 0;
      i128 before = 0;
      if (check_moves) before = recount_qnum(r);
      i128 dq = commit_moves(r, B);
      if (check_moves) {
        i128 after = recount_qnum(r);
        if (after - before != dq && err.empty()) err = "batch gain differs from recount";
        if (single_move && B.size() == 1) {
          i128 expect = cfg.directed ? B[0].G : 2 * B[0].G;
          if (dq != expect && err.empty()) err = "single-move gain differs from predicted gain";
          checks[2]++;
          checks[5] += B[0].empty ? 1 : 0;
        }
        if (qnum() != after && err.empty()) err = "maintained Q numerator differs from recount";
        checks[0]++;
      }
      record(r, 0, j, S.size(), cands.size(), B.size(), dq);
      if (dq < 0) {  // negative batch gain (Algorithm 1): roll the whole mini-batch back and stop moving
        rollback_moves(r, B, dq);
        break;
      }
      // Expand_r (Sec. III-C): movers, their neighbours, members of touched communities
      U.clear();
      std::vector<uint8_t> cm(n, 0);
      for (auto& c : B) {
        Moved.add(c.v);
        U.add(c.v);
        neighbours(r, c.v, U);
        cm[c.a] = 1; cm[c.b] = 1;
      }
      if (!B.empty())
        for (uint32_t u = 0; u < n; ++u) if (L.alive[u] && cm[L.lab[u]]) U.add(u);
      // the alpha and beta stops of the move loop as exact rational comparisons
      if ((i128)cfg.ad * dq < (i128)cfg.an * Q0) break;
      if ((i128)cfg.bd * B.size() < (i128)cfg.bn * S.size()) break;
    }
    if (r < cfg.L) refine_and_aggregate(r, entry, Moved);
    if (r >= 1 && Moved.size() > 0) label_refresh(r);
  }

  // Refinement (Algorithm 1, BestRef) and aggregate repair (Eq. 3) at level r < L.
  void refine_and_aggregate(int r, const std::vector<uint32_t>& entry, NodeSet& Moved) {
    Level& L = lv[r];
    // TouchedRefined: refined communities of this level's seeds and movers
    std::vector<uint8_t> tref(n, 0);
    for (uint32_t x : entry) tref[L.par[x]] = 1;
    for (uint32_t x : Moved.list) tref[L.par[x]] = 1;
    std::vector<uint32_t> oldpar(n, 0);
    NodeSet Rset; Rset.init(n);
    std::vector<uint32_t> R;
    for (uint32_t u = 0; u < n; ++u)
      if (L.alive[u] && tref[L.par[u]]) { Rset.add(u); oldpar[u] = L.par[u]; R.push_back(u); }
    for (uint32_t u : R) L.par[u] = u;   // reset to singletons
    // refined totals from scratch
    std::vector<i64> Krout(n, 0), Krin(n, 0);
    std::vector<uint32_t> rsize(n, 0);
    for (uint32_t u = 0; u < n; ++u)
      if (L.alive[u]) { Krout[L.par[u]] += L.kout[u]; Krin[L.par[u]] += L.kin[u]; rsize[L.par[u]]++; }
    for (int j = 1; j <= cfg.M; ++j) {
      // key of this refinement iteration: SplitMix64's first output of the seed, chained with
      // the batch index, the pass, then level and iteration in one word
      rkey = splitmix_mix(splitmix_mix(splitmix_mix(splitmix_mix(seed + 0x9E3779B97F4A7C15ull) ^ cur_batch) ^
                                       (uint64_t)pass_idx) ^
                          (((uint64_t)r << 32) | (uint64_t)j)) | 1ull;
      std::vector<Cand> cands;
      for (uint32_t u : R) {
        if (!(L.par[u] == u && rsize[u] == 1)) continue;   // only singletons move
        Cand c; if (best_ref(r, u, Krout, Krin, c)) cands.push_back(c);
      }
      std::vector<Cand> B = decouple(cands, single_move != 0);
      i128 before = 0;
      if (check_moves) before = recount_qnum_refined(r);
      for (auto& c : B) {
        L.par[c.v] = c.b;
        Krout[c.b] += L.kout[c.v]; Krin[c.b] += L.kin[c.v]; rsize[c.b]++;
        Krout[c.v] -= L.kout[c.v]; Krin[c.v] -= L.kin[c.v]; rsize[c.v]--;
      }
      if (check_moves) {
        // A singleton {u} joining refined community y changes the refined partition's numerator
        // by exactly the predicted gain (directed; twice it for the symmetric matrix of an
        // undirected graph), and the maintained refined totals equal their recount.
        const i128 dq_ref = recount_qnum_refined(r) - before;
        if (single_move && B.size() == 1) {
          const i128 expect = cfg.directed ? B[0].G : 2 * B[0].G;
          if (dq_ref != expect && err.empty()) err = "single-move refinement gain differs from recount";
          checks[3]++;
        }
        std::vector<i64> ro(n, 0), ri(n, 0);
        std::vector<uint32_t> rs(n, 0);
        for (uint32_t u = 0; u < n; ++u)
          if (L.alive[u]) { ro[L.par[u]] += L.kout[u]; ri[L.par[u]] += L.kin[u]; rs[L.par[u]]++; }
        if ((ro != Krout || ri != Krin || rs != rsize) && err.empty()) err = "refined totals differ from recount";
        checks[1]++;
      }
      record(r, 1, j, R.size(), cands.size(), B.size(), 0);
      if ((i128)cfg.bd * B.size() < (i128)cfg.bn * R.size()) break;
      // SPExpand: singleton neighbours of movers carrying the mover's label
      NodeSet Rn; Rn.init(n);
      for (auto& c : B) {
        uint32_t v = c.v;
        auto consider = [&](uint32_t x) {
          if (x == v || !L.alive[x] || L.lab[x] != L.lab[v]) return;
          if (!(L.par[x] == x && rsize[x] == 1)) return;
          Rn.add(x);
        };
        for (auto& e : L.out[v]) consider(e.first);
        if (cfg.directed) for (auto& e : L.in[v]) consider(e.first);
      }
      R = Rn.list;
      for (uint32_t x : R) if (Rset.add(x)) oldpar[x] = L.par[x];
    }
    if (r == top) { materialise(r); return; }

    // ---- aggregate repair by subtract-add (Sec. III-F, Eq. 3)
    Level& H = lv[r + 1];
    NodeSet& Dn = D[r + 1];
    std::vector<uint8_t> inC(n, 0);
    std::vector<uint32_t> C;
    for (uint32_t u : Rset.list) if (L.par[u] != oldpar[u]) { inC[u] = 1; C.push_back(u); }
    auto op = [&](uint32_t x) { return inC[x] ? oldpar[x] : L.par[x]; };
    std::vector<Tup> delta;
    auto emit = [&](uint32_t xo, uint32_t yo, uint32_t xn, uint32_t yn, i64 w) {
      delta.push_back({xo, yo, -w});
      delta.push_back({xn, yn, w});
      Dn.add(xo); Dn.add(yo); Dn.add(xn); Dn.add(yn);
    };
    for (uint32_t u : C) {
      for (auto& e : L.out[u]) emit(op(u), op(e.first), L.par[u], L.par[e.first], e.second);
      for (auto& e : inrow(L, u)) {
        if (inC[e.first]) continue;
        emit(op(e.first), op(u), L.par[e.first], L.par[u], e.second);
      }
    }
    // NextFrontier: parents of seeds, movers and refined nodes; old parents of changed nodes
    for (uint32_t x : entry) Dn.add(L.par[x]);
    for (uint32_t x : Moved.list) Dn.add(L.par[x]);
    for (uint32_t x : Rset.list) Dn.add(L.par[x]);
    for (uint32_t x : C) Dn.add(oldpar[x]);
    // liveness and labels of level r+1, revival chains above
    std::vector<uint32_t> cnt(n, 0);
    for (uint32_t u = 0; u < n; ++u) if (L.alive[u]) cnt[L.par[u]]++;
    for (uint32_t x = 0; x < n; ++x) {
      uint8_t a = cnt[x] > 0;
      if (a && !H.alive[x] && r + 1 < cfg.L) H.par[x] = x;
      H.alive[x] = a;
    }
    for (uint32_t u : Rset.list) { uint32_t x = L.par[u]; if (H.alive[x]) H.lab[x] = L.lab[x]; }
    for (int s = r + 2; s <= top; ++s) {
      Level& B = lv[s - 1];
      Level& T = lv[s];
      std::vector<uint32_t> c2(n, 0);
      for (uint32_t x = 0; x < n; ++x) if (B.alive[x]) c2[B.par[x]]++;
      for (uint32_t x = 0; x < n; ++x) {
        uint8_t a = c2[x] > 0;
        if (a && !T.alive[x]) { if (s < cfg.L) T.par[x] = x; T.lab[x] = B.lab[x]; }
        T.alive[x] = a;
      }
    }
    // apply the grouped deltas at r+1 and cascade them up the hierarchy
    std::vector<Tup> cur = reduce_tuples(delta);
    for (int s = r + 1; s <= top; ++s) {
      apply_reduced(s, cur, true);
      if (s == top) break;
      for (auto& e : cur) { e.x = lv[s].par[e.x]; e.y = lv[s].par[e.y]; }
      cur = reduce_tuples(cur);
    }
  }

  // First visit of level r+1: build it from scratch by Eq. 3.
  void materialise(int r) {
    Level& L = lv[r];
    alloc_level(r + 1);
    Level& H = lv[r + 1];
    for (uint32_t u = 0; u < n; ++u) if (L.alive[u]) H.alive[L.par[u]] = 1;
    std::vector<Tup> agg;
    for (uint32_t u = 0; u < n; ++u)
      for (auto& e : L.out[u]) agg.push_back({L.par[u], L.par[e.first], e.second});
    apply_reduced(r + 1, reduce_tuples(agg), true);
    for (uint32_t x = 0; x < n; ++x) { H.lab[x] = H.alive[x] ? L.lab[x] : x; H.par[x] = x; }
    top = r + 1;
    for (uint32_t x = 0; x < n; ++x) if (H.alive[x]) D[r + 1].add(x);
  }

  // After moves at level r >= 1: P^s(u) <- P^{s+1}(pi_s(u)) for s < r; relabelled nodes are
  // seeds of their level for the next pass.
  void label_refresh(int r) {
    for (int s = r - 1; s >= 0; --s) {
      Level& L = lv[s];
      const Level& H = lv[s + 1];
      for (uint32_t u = 0; u < n; ++u) {
        if (!L.alive[u]) continue;
        uint32_t nl = H.lab[L.par[u]];
        if (nl != L.lab[u]) { L.lab[u] = nl; D[s].add(u); }
      }
    }
  }

  // ---------------------------------------------------------------- batch
  struct Upd { uint32_t u, v; int kind; i64 w; };   // kind 0 insert, 1 delete, 2 change

  int apply_batch(const uint32_t* ins, uint64_t n_ins, const uint32_t* del, uint64_t n_del,
                  const uint32_t* chg, uint64_t n_chg) {
    // ---- validation (atomic batch: nothing is modified before it passes)
    std::vector<Upd> ups;
    for (uint64_t i = 0; i < n_ins; ++i) ups.push_back({ins[3 * i], ins[3 * i + 1], 0, (i64)ins[3 * i + 2]});
    for (uint64_t i = 0; i < n_del; ++i) ups.push_back({del[2 * i], del[2 * i + 1], 1, 0});
    for (uint64_t i = 0; i < n_chg; ++i) ups.push_back({chg[3 * i], chg[3 * i + 1], 2, (i64)chg[3 * i + 2]});
    for (auto& x : ups) {
      if (x.u >= n || x.v >= n) return EINVAL_;
      if (x.kind != 1 && x.w == 0) return EINVAL_;
      if (!cfg.directed && x.u > x.v) std::swap(x.u, x.v);
    }
    {
      std::vector<std::pair<uint32_t, uint32_t>> keys;
      for (auto& x : ups) keys.push_back(std::make_pair(x.u, x.v));
      std::sort(keys.begin(), keys.end());
      for (size_t i = 1; i < keys.size(); ++i) if (keys[i] == keys[i - 1]) return EDUP_;
    }
    const Level& L0 = lv[0];
    std::vector<std::pair<std::pair<uint32_t, uint32_t>, i64>> net;  // (u,v) -> delta
    i64 dm = 0;
    for (auto& x : ups) {
      bool present = row_has(L0.out[x.u], x.v);
      i64 old = row_get(L0.out[x.u], x.v);
      i64 d;
      if (x.kind == 0) {
        d = x.w;
        if (old + x.w > (i64)0xFFFFFFFFll) return EOVERFLOW_;
      } else {
        if (!present) return ENOEDGE_;
        d = x.kind == 1 ? -old : x.w - old;
      }
      if (d == 0) continue;
      net.push_back(std::make_pair(std::make_pair(x.u, x.v), d));
      dm += (!cfg.directed && x.u != x.v) ? 2 * d : d;
    }
    if (m + dm >= ((i64)1 << 40)) return EOVERFLOW_;
    cur_batch = batches++;   // the batch is accepted

    // ---- batch ingest: apply to G^0 as matrix entries, repair m, degrees, totals, Ein, SKK
    std::vector<std::pair<std::pair<uint32_t, uint32_t>, i64>> ent;
    for (auto& kv : net) {
      ent.push_back(kv);
      if (!cfg.directed && kv.first.first != kv.first.second)
        ent.push_back(std::make_pair(std::make_pair(kv.first.second, kv.first.first), kv.second));
    }
    {
      std::vector<Tup> t0;
      for (auto& e : ent) t0.push_back({e.first.first, e.first.second, e.second});
      apply_reduced(0, reduce_tuples(t0), true);
    }
    for (auto& e : ent) {
      uint32_t x = e.first.first, y = e.first.second;
      i64 d = e.second;
      m += d;
      add_total(lv[0].lab[x], d, 0);
      add_total(lv[0].lab[y], 0, d);
      if (lv[0].lab[x] == lv[0].lab[y]) Ein += d;
    }
    // ---- seeds; cascade of the entry deltas through pi to every existing level
    for (auto& e : ent) { D[0].add(e.first.first); D[0].add(e.first.second); }
    for (int s = 1; s <= top; ++s) {
      std::vector<Tup> agg;
      for (auto& e : ent) {
        uint32_t X = anc(e.first.first, s), Y = anc(e.first.second, s);
        agg.push_back({X, Y, e.second});
        D[s].add(X); D[s].add(Y);
      }
      apply_reduced(s, reduce_tuples(agg), true);
    }
    // ---- adaptive refresh (a variant, off unless rho > 0): when the level-0 frontier A^0
    // (InitFrontier: alive seeds and every alive member of their communities) reaches rho n, the
    // update no longer has locality (Sec. IV-F, Sec. V), so the batch reoptimises from scratch:
    // the hierarchy and partition are discarded and static Leiden runs on the current graph.
    if (cfg.rn > 0) {
      const Level& L0 = lv[0];
      std::vector<uint8_t> cm(n, 0);
      for (uint32_t x : D[0].list) if (L0.alive[x]) cm[L0.lab[x]] = 1;
      uint64_t a0 = 0;
      for (uint32_t u = 0; u < n; ++u) if (L0.alive[u] && cm[L0.lab[u]]) ++a0;
      if ((i128)cfg.rd * a0 >= (i128)cfg.rn * n) {
        record(0, 2, 0, a0, 0, 0, 0);
        refresh();
      }
    }
    // ---- outer passes over levels
    for (int i = 1; i <= cfg.N; ++i) {
      pass_idx = i;
      const i128 Qp = qnum();
      bool any = false;
      for (int r = 0; r <= top && r <= cfg.L; ++r) {
        if (D[r].size() == 0) continue;
        any = true;
        process_level(r);
      }
      bool all_empty = true;
      for (int r = 0; r <= cfg.L; ++r) if (D[r].size()) all_empty = false;
      if (!any || all_empty) break;
      if ((i128)cfg.ad * (qnum() - Qp) < (i128)cfg.an * Qp) break;
    }
    for (int r = 0; r <= cfg.L; ++r) D[r].clear();
    return err.empty() ? OK : ECHECK_;
  }

  // Full reoptimisation of the current graph: the state static Leiden starts from (singleton
  // labels and parents at level 0, no aggregate level, totals equal to the degrees), seeded with
  // every vertex that has an entry -- the state ldl_create reaches before its passes.
  void refresh() {
    Level& L0 = lv[0];
    for (uint32_t u = 0; u < n; ++u) { L0.lab[u] = u; L0.par[u] = u; }
    for (int r = 1; r <= top; ++r) lv[r] = Level();
    top = 0;
    Ein = 0;
    SKK = 0;
    for (uint32_t u = 0; u < n; ++u) {
      Kout[u] = L0.kout[u];
      Kin[u] = L0.kin[u];
      SKK += (i128)Kout[u] * Kin[u];
      Ein += row_get(L0.out[u], u);
    }
    for (auto& d : D) d.clear();
    for (uint32_t u = 0; u < n; ++u)
      if (!L0.out[u].empty() || (cfg.directed && !L0.in[u].empty())) D[0].add(u);
    refreshes++;
  }

  // ---------------------------------------------------------------- invariants (recount)
  std::string check() const {
    // I5/I6/I7 at level 0 and every level; I1 aggregation; I2 labels; I3 roots
    std::vector<i64> ko(n, 0), ki(n, 0);
    i64 mm = 0, ein = 0;
    for (int r = 0; r <= top; ++r) {
      const Level& L = lv[r];
      std::vector<i64> a(n, 0), b(n, 0);
      for (uint32_t u = 0; u < n; ++u) {
        for (auto& e : L.out[u]) {
          if (e.second <= 0) return "non-positive weight";
          if (!L.alive[u] || !L.alive[e.first]) return "entry at dead node";
          a[u] += e.second; b[e.first] += e.second;
          if (cfg.directed && row_get(L.in[e.first], u) != e.second) return "in/out mismatch";
          if (!cfg.directed && row_get(L.out[e.first], u) != e.second) return "asymmetric";
        }
      }
      if (cfg.directed) {
        size_t no = 0, ni = 0;
        for (uint32_t u = 0; u < n; ++u) { no += L.out[u].size(); ni += L.in[u].size(); }
        if (no != ni) return "in/out entry count mismatch";
      }
      for (uint32_t u = 0; u < n; ++u) if (a[u] != L.kout[u] || b[u] != L.kin[u]) return "degree mismatch at level " + std::to_string(r);
      if (r < top) {
        const Level& H = lv[r + 1];
        std::map<std::pair<uint32_t, uint32_t>, i64> agg;
        std::vector<uint8_t> al(n, 0);
        for (uint32_t u = 0; u < n; ++u) if (L.alive[u]) al[L.par[u]] = 1;
        for (uint32_t x = 0; x < n; ++x) if (al[x] != H.alive[x]) return "liveness mismatch at level " + std::to_string(r + 1);
        for (uint32_t u = 0; u < n; ++u)
          for (auto& e : L.out[u]) agg[std::make_pair(L.par[u], L.par[e.first])] += e.second;
        size_t cntH = 0;
        for (uint32_t x = 0; x < n; ++x) cntH += H.out[x].size();
        size_t nz = 0;
        for (auto& kv : agg) {
          if (kv.second == 0) continue;
          ++nz;
          if (row_get(H.out[kv.first.first], kv.first.second) != kv.second) return "aggregate mismatch at level " + std::to_string(r + 1);
        }
        if (nz != cntH) return "aggregate entry count mismatch at level " + std::to_string(r + 1);
        for (uint32_t u = 0; u < n; ++u)
          if (L.alive[u] && L.lab[u] != H.lab[L.par[u]]) return "label nesting broken at level " + std::to_string(r);
        for (uint32_t x = 0; x < n; ++x)
          if (H.alive[x] && !(L.alive[x] && L.par[x] == x)) return "refined root missing at level " + std::to_string(r);
      }
    }
    const Level& L0 = lv[0];
    for (uint32_t u = 0; u < n; ++u)
      for (auto& e : L0.out[u]) {
        mm += e.second; ko[L0.lab[u]] += e.second; ki[L0.lab[e.first]] += e.second;
        if (L0.lab[u] == L0.lab[e.first]) ein += e.second;
      }
    if (mm != m) return "m mismatch";
    if (ein != Ein) return "Ein mismatch";
    i128 skk = 0;
    for (uint32_t c = 0; c < n; ++c) {
      if (ko[c] != Kout[c] || ki[c] != Kin[c]) return "community totals mismatch";
      skk += (i128)ko[c] * ki[c];
    }
    if (skk != SKK) return "SKK mismatch";
    return "";
  }
};

Cfg default_cfg(int directed) {
  Cfg c;
  c.directed = directed; c.gp = 1; c.gq = 1; c.N = 2; c.L = 4; c.M = 5;
  c.an = 1; c.ad = 1000; c.bn = 1; c.bd = 100;
  return c;
}

}  // namespace

extern "C" {

// cfg10 = {directed, gamma_num, gamma_den, N, L, M, alpha_num, alpha_den, beta_num, beta_den};
// null -> defaults (N=2, L=4, M=5, alpha=1/1000, beta=1/100, gamma=1) for an undirected graph.
int orc_create_ex(const int32_t* cfg10, uint32_t n, const uint32_t* edges, uint64_t n_edges, int flags,
                  uint64_t seed, void** out) {
  *out = nullptr;
  Cfg c = default_cfg(0);
  if (cfg10) {
    c.directed = cfg10[0] != 0; c.gp = cfg10[1]; c.gq = cfg10[2]; c.N = cfg10[3]; c.L = cfg10[4];
    c.M = cfg10[5]; c.an = cfg10[6]; c.ad = cfg10[7]; c.bn = cfg10[8]; c.bd = cfg10[9];
  }
  if (n == 0 || c.gp < 1 || c.gq < 1 || c.gp >= 65536 || c.gq >= 65536 || c.N < 1 || c.M < 1 || c.L < 0 ||
      c.L > 16 || c.an < 0 || c.ad < 1 || c.bn < 0 || c.bd < 1 || c.ad >= 65536 || c.bd >= 65536 ||
      c.an >= 65536 || c.bn >= 65536)
    return EINVAL_;
  Oracle* o = new Oracle();
  o->cfg = c; o->n = n;
  o->single_move = (flags & 1) != 0;
  o->check_moves = (flags & 2) != 0;
  o->tracing = (flags & 4) != 0;
  o->empty_target = (flags & 8) != 0;
  o->random_refine = (flags & 16) != 0;
  o->seed = seed;
  o->lv.resize(c.L + 1);
  o->alloc_level(0);
  for (uint32_t u = 0; u < n; ++u) o->lv[0].alive[u] = 1;
  o->Kout.assign(n, 0); o->Kin.assign(n, 0);
  o->D.resize(c.L + 1);
  for (auto& s : o->D) s.init(n);
  o->acc.assign(n, 0); o->acc_flag.assign(n, 0); o->mover_from.assign(n, 0xFFFFFFFFu);
  // static Leiden = the batch update applied to the empty singleton state
  int rc = o->apply_batch(edges, n_edges, nullptr, 0, nullptr, 0);
  if (rc != OK && rc != ECHECK_) { delete o; return rc; }
  *out = o;
  return rc;
}

int orc_create(const int32_t* cfg10, uint32_t n, const uint32_t* edges, uint64_t n_edges, int flags,
               void** out) {
  return orc_create_ex(cfg10, n, edges, n_edges, flags, 0, out);
}

void orc_destroy(void* h) { delete (Oracle*)h; }

uint64_t orc_splitmix_mix(uint64_t z) { return splitmix_mix(z); }

// The refinement target choice on given candidates (gains as hi/lo words): index or -1.
int orc_choose_ref(int random, uint64_t key, uint32_t u, uint64_t k, const uint32_t* ys, const int64_t* ghi,
                   const uint64_t* glo) {
  std::vector<uint32_t> y(ys, ys + k);
  std::vector<i128> g(k);
  for (uint64_t i = 0; i < k; ++i) g[i] = ((i128)ghi[i] << 64) | (i128)glo[i];
  return Oracle::choose_ref(random != 0, key, u, y, g);
}

// Adaptive refresh threshold rho = num / den for the following batches (num = 0: never);
// returns the number of batches so far that switched to full reoptimisation.
uint64_t orc_set_refresh(void* h, int32_t num, int32_t den) {
  Oracle* o = (Oracle*)h;
  if (num >= 0 && den >= 1) { o->cfg.rn = num; o->cfg.rd = den; }
  return o->refreshes;
}

int orc_apply_batch(void* h, const uint32_t* ins, uint64_t n_ins, const uint32_t* del, uint64_t n_del,
                    const uint32_t* chg, uint64_t n_chg) {
  return ((Oracle*)h)->apply_batch(ins, n_ins, del, n_del, chg, n_chg);
}

int orc_get_partition(void* h, uint32_t* labels) {
  Oracle* o = (Oracle*)h;
  std::memcpy(labels, o->lv[0].lab.data(), sizeof(uint32_t) * o->n);
  return OK;
}

// Q numerator (i128 as hi/lo) and the FP64 value Qnum / (q m^2).
int orc_modularity(void* h, int64_t* num_hi, uint64_t* num_lo, double* q) {
  Oracle* o = (Oracle*)h;
  i128 num = o->qnum();
  *num_hi = (int64_t)(num >> 64); *num_lo = (uint64_t)num;
  if (o->m == 0) { *q = 0.0; return OK; }
  *q = (double)num / ((double)o->cfg.gq * (double)o->m * (double)o->m);
  return OK;
}

int orc_scalars(void* h, int32_t* top, int64_t* m, int64_t* ein, int64_t* skk_hi, uint64_t* skk_lo) {
  Oracle* o = (Oracle*)h;
  *top = o->top; *m = o->m; *ein = o->Ein;
  *skk_hi = (int64_t)(o->SKK >> 64); *skk_lo = (uint64_t)o->SKK;
  return OK;
}

int orc_totals(void* h, int64_t* kout, int64_t* kin) {
  Oracle* o = (Oracle*)h;
  std::memcpy(kout, o->Kout.data(), 8 * o->n);
  std::memcpy(kin, o->Kin.data(), 8 * o->n);
  return OK;
}

// Per-level node arrays; par is meaningful only below the top level.
int orc_level_nodes(void* h, int r, uint8_t* alive, uint32_t* lab, uint32_t* par, int64_t* kout, int64_t* kin) {
  Oracle* o = (Oracle*)h;
  if (r < 0 || r > o->top) return EINVAL_;
  const Level& L = o->lv[r];
  std::memcpy(alive, L.alive.data(), o->n);
  std::memcpy(lab, L.lab.data(), 4 * o->n);
  std::memcpy(par, L.par.data(), 4 * o->n);
  std::memcpy(kout, L.kout.data(), 8 * o->n);
  std::memcpy(kin, L.kin.data(), 8 * o->n);
  return OK;
}

uint64_t orc_level_nnz(void* h, int r) {
  Oracle* o = (Oracle*)h;
  if (r < 0 || r > o->top) return 0;
  uint64_t c = 0;
  for (auto& row : o->lv[r].out) c += row.size();
  return c;
}

// Matrix entries of level r in (row, col) order.
int orc_level_entries(void* h, int r, uint32_t* rows, uint32_t* cols, int64_t* w) {
  Oracle* o = (Oracle*)h;
  if (r < 0 || r > o->top) return EINVAL_;
  uint64_t k = 0;
  for (uint32_t u = 0; u < o->n; ++u)
    for (auto& e : o->lv[r].out[u]) { rows[k] = u; cols[k] = e.first; w[k] = e.second; ++k; }
  return OK;
}

// Recount every invariant from scratch; returns 0 or ECHECK with a message.
int orc_check(void* h, char* msg, int cap) {
  Oracle* o = (Oracle*)h;
  std::string s = o->check();
  if (s.empty() && !o->err.empty()) s = o->err;
  if (msg && cap > 0) { std::strncpy(msg, s.c_str(), cap - 1); msg[cap - 1] = 0; }
  return s.empty() ? OK : ECHECK_;
}

// Recount checks done so far (FLAG_CHECK_MOVES): [0] move commits, [1] refinement commits,
// [2] single-move move commits compared with their predicted gain, [3] likewise for refinement.
void orc_check_counts(void* h, uint64_t* out6) {
  Oracle* o = (Oracle*)h;
  for (int i = 0; i < 6; ++i) out6[i] = o->checks[i];
}

uint64_t orc_trace_len(void* h) { return ((Oracle*)h)->trace.size(); }
// 8 int64 per record: pass, level, phase, iter, nscan, ncand, nacc, dq (low 64 bits, signed)
void orc_trace(void* h, int64_t* out) {
  Oracle* o = (Oracle*)h;
  for (size_t i = 0; i < o->trace.size(); ++i) {
    const TraceRec& t = o->trace[i];
    int64_t* p = out + 8 * i;
    p[0] = t.pass; p[1] = t.level; p[2] = t.phase; p[3] = t.iter;
    p[4] = (int64_t)t.nscan; p[5] = (int64_t)t.ncand; p[6] = (int64_t)t.nacc; p[7] = (int64_t)t.dq_lo;
  }
}
void orc_trace_clear(void* h) { ((Oracle*)h)->trace.clear(); }

// Eq. 1 evaluated from an edge list and a labelling: exact numerator q*m^2*Q (hi/lo) and m.
// Undirected edges become the two symmetric matrix entries (a self-loop one entry).
int orc_eval_modularity(int directed, int gp, int gq, uint32_t n, const uint32_t* edges, uint64_t n_edges,
                        const uint32_t* labels, int64_t* num_hi, uint64_t* num_lo, int64_t* m_out) {
  std::vector<i64> ko(n, 0), ki(n, 0);
  i64 mm = 0, ein = 0;
  auto entry = [&](uint32_t u, uint32_t v, i64 w) {
    mm += w; ko[labels[u]] += w; ki[labels[v]] += w;
    if (labels[u] == labels[v]) ein += w;
  };
  for (uint64_t i = 0; i < n_edges; ++i) {
    uint32_t u = edges[3 * i], v = edges[3 * i + 1];
    i64 w = edges[3 * i + 2];
    if (u >= n || v >= n) return EINVAL_;
    entry(u, v, w);
    if (!directed && u != v) entry(v, u, w);
  }
  i128 skk = 0;
  for (uint32_t c = 0; c < n; ++c) skk += (i128)ko[c] * ki[c];
  i128 num = (i128)gq * mm * ein - (i128)gp * skk;
  *num_hi = (int64_t)(num >> 64); *num_lo = (uint64_t)num; *m_out = mm;
  return OK;
}

// The serial decouple filter alone, for testing: cand = (v, a, b) rows with gains as hi/lo;
// writes 1/0 per candidate in `accepted` (input order).
int orc_decouple(uint64_t k, const uint32_t* vab, const int64_t* g_hi, const uint64_t* g_lo, uint8_t* accepted) {
  Oracle o;
  std::vector<Cand> c(k);
  for (uint64_t i = 0; i < k; ++i) {
    c[i].v = vab[3 * i]; c[i].a = vab[3 * i + 1]; c[i].b = vab[3 * i + 2];
    c[i].G = ((i128)g_hi[i] << 64) | (i128)g_lo[i];
  }
  std::vector<Cand> B = o.decouple(c, false);
  std::map<uint32_t, int> acc;
  for (auto& x : B) acc[x.v] = 1;
  for (uint64_t i = 0; i < k; ++i) accepted[i] = acc.count(c[i].v) ? 1 : 0;
  return OK;
}

}  // extern "C"
