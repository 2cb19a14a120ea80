// Seeded synthetic graph and update-stream generators.
//
// This module only draws random inputs: planted-partition graphs, R-MAT graphs and
// insert/delete/reweight update batches.  It contains none of the community-detection
// arithmetic; both the CPU oracle and the GPU library consume the arrays it writes.
//
// Random numbers: SplitMix64 seeds xoshiro256** (Blackman & Vigna, "Scrambled linear
// pseudorandom number generators", 2018).  Lognormal weights use the Box-Muller transform.
// Planted-partition pairs are drawn by geometric skipping over the pair index space
// (Batagelj & Brandes, "Efficient generation of large random networks", 2005).
// R-MAT follows Chakrabarti, Zhan & Faloutsos, "R-MAT: a recursive model for graph
// mining", SDM 2004.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

struct Rng {
  uint64_t s[4];
  static uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  explicit Rng(uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) s[i] = splitmix(x);
  }
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  uint64_t next() {
    uint64_t r = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return r;
  }
  // uniform integer in [0, k) by the multiply-high map
  uint64_t below(uint64_t k) { return (uint64_t)(((unsigned __int128)next() * k) >> 64); }
  // uniform double in [0, 1)
  double unit() { return (double)(next() >> 11) * 0x1.0p-53; }
  double normal() {
    double u1 = unit(), u2 = unit();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// Open-addressing edge set: key -> index into parallel (keys, weights) arrays.
struct EdgeSet {
  std::vector<uint64_t> slot_key;  // 0 = empty (key+1 stored)
  std::vector<uint64_t> slot_idx;
  uint64_t mask = 0;
  std::vector<uint64_t> keys;
  std::vector<uint32_t> w;

  static uint64_t mix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull; k ^= k >> 33;
    return k;
  }
  void reserve(uint64_t n) {
    uint64_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    if (cap - 1 <= mask) return;
    std::vector<uint64_t> ok(cap, 0), oi(cap, 0);
    slot_key.swap(ok); slot_idx.swap(oi);
    mask = cap - 1;
    for (uint64_t i = 0; i < keys.size(); ++i) place(keys[i], i);
  }
  void place(uint64_t key, uint64_t idx) {
    uint64_t h = mix(key) & mask;
    while (slot_key[h]) h = (h + 1) & mask;
    slot_key[h] = key + 1; slot_idx[h] = idx;
  }
  int64_t find_slot(uint64_t key) const {
    if (slot_key.empty()) return -1;
    uint64_t h = mix(key) & mask;
    while (slot_key[h]) {
      if (slot_key[h] == key + 1) return (int64_t)h;
      h = (h + 1) & mask;
    }
    return -1;
  }
  bool contains(uint64_t key) const { return find_slot(key) >= 0; }
  uint64_t index_of(uint64_t key) const { return slot_idx[find_slot(key)]; }
  void insert(uint64_t key, uint32_t weight) {
    reserve(keys.size() + 1);
    place(key, keys.size());
    keys.push_back(key); w.push_back(weight);
  }
  void erase_slot(uint64_t h) {
    // backward-shift deletion for linear probing
    slot_key[h] = 0;
    uint64_t j = h;
    for (;;) {
      j = (j + 1) & mask;
      if (!slot_key[j]) break;
      uint64_t home = mix(slot_key[j] - 1) & mask;
      bool between = (h <= j) ? (h < home && home <= j) : (h < home || home <= j);
      if (between) continue;
      slot_key[h] = slot_key[j]; slot_idx[h] = slot_idx[j]; slot_key[j] = 0; h = j;
    }
  }
  void erase(uint64_t key) {
    int64_t h = find_slot(key);
    uint64_t i = slot_idx[h];
    erase_slot((uint64_t)h);
    uint64_t last = keys.size() - 1;
    if (i != last) {
      keys[i] = keys[last]; w[i] = w[last];
      slot_idx[find_slot(keys[i])] = i;
    }
    keys.pop_back(); w.pop_back();
  }
};

struct Gen {
  Rng rng;
  uint32_t n;
  int directed;
  EdgeSet es;
  Gen(uint64_t seed, uint32_t n_, int d) : rng(seed), n(n_), directed(d) {}
  uint64_t key(uint32_t u, uint32_t v) const {
    if (!directed && u > v) std::swap(u, v);
    return ((uint64_t)u << 32) | v;
  }
  uint32_t draw_weight(int kind, double p1, double p2) {
    if (kind == 0) {
      uint64_t lo = (uint64_t)p1, hi = (uint64_t)p2;
      return (uint32_t)(lo + rng.below(hi - lo + 1));
    }
    double x = std::exp(p1 + p2 * rng.normal());
    long long r = std::llround(x);
    if (r < 1) r = 1;
    if (r > 0xFFFFFFFFll) r = 0xFFFFFFFFll;
    return (uint32_t)r;
  }
};

// geometric skip length for success probability p (number of failures before a success)
inline uint64_t geo_skip(Rng& r, double p) {
  if (p >= 1.0) return 0;
  double u = r.unit();
  double k = std::floor(std::log1p(-u) / std::log1p(-p));
  if (k > 1.8e19) return UINT64_MAX;
  return (uint64_t)k;
}

}  // namespace

extern "C" {

void* syn_new(uint64_t seed, uint32_t n, int directed) { return new Gen(seed, n, directed); }
void syn_free(void* g) { delete (Gen*)g; }
uint64_t syn_num_edges(void* g) { return ((Gen*)g)->es.keys.size(); }

// Copy the current edge set (u, v, w) triples in storage order.
void syn_get_edges(void* gp, uint32_t* uvw) {
  Gen* g = (Gen*)gp;
  for (uint64_t i = 0; i < g->es.keys.size(); ++i) {
    uvw[3 * i] = (uint32_t)(g->es.keys[i] >> 32);
    uvw[3 * i + 1] = (uint32_t)g->es.keys[i];
    uvw[3 * i + 2] = g->es.w[i];
  }
}

// Planted partition: vertex u is in block u / block_size.  Each unordered pair (undirected)
// or ordered pair u != v (directed) is an edge with probability p_in inside a block and
// p_out across blocks.  Weights uniform in [wmin, wmax].
int syn_planted(void* gp, uint32_t block_size, double p_in, double p_out, uint32_t wmin, uint32_t wmax) {
  Gen* g = (Gen*)gp;
  const uint64_t n = g->n;
  if (block_size == 0 || n < 2) return -1;
  auto add = [&](uint32_t u, uint32_t v) {
    g->es.insert(g->key(u, v), (uint32_t)(wmin + g->rng.below((uint64_t)wmax - wmin + 1)));
  };
  // inside blocks
  for (uint64_t b0 = 0; b0 < n; b0 += block_size) {
    uint64_t s = std::min<uint64_t>(block_size, n - b0);
    uint64_t total = g->directed ? s * (s - 1) : s * (s - 1) / 2;
    if (p_in <= 0 || total == 0) continue;
    uint64_t idx = geo_skip(g->rng, p_in);
    while (idx < total) {
      uint32_t u, v;
      if (g->directed) {
        u = (uint32_t)(idx / (s - 1));
        uint32_t o = (uint32_t)(idx % (s - 1));
        v = o >= u ? o + 1 : o;
      } else {
        // row-major over u < v: row u holds s-1-u pairs
        uint64_t rem = idx; uint64_t uu = 0;
        // closed-form start then integer correction
        double ds = (double)s;
        double est = std::floor(ds - 0.5 - std::sqrt((ds - 0.5) * (ds - 0.5) - 2.0 * (double)idx));
        if (est < 0) est = 0;
        uu = (uint64_t)est;
        auto start = [&](uint64_t r) { return r * (2 * s - r - 1) / 2; };
        while (uu > 0 && start(uu) > idx) --uu;
        while (start(uu + 1) <= idx) ++uu;
        rem = idx - start(uu);
        u = (uint32_t)uu; v = (uint32_t)(uu + 1 + rem);
      }
      add((uint32_t)(b0 + u), (uint32_t)(b0 + v));
      uint64_t k = geo_skip(g->rng, p_in);
      if (k == UINT64_MAX || idx + 1 + k < idx) break;
      idx += 1 + k;
    }
  }
  // across blocks: walk the full pair space and skip same-block pairs
  if (p_out > 0) {
    uint64_t total = g->directed ? n * (n - 1) : n * (n - 1) / 2;
    uint64_t idx = geo_skip(g->rng, p_out);
    auto start = [&](uint64_t r) { return r * (2 * n - r - 1) / 2; };
    while (idx < total) {
      uint64_t u, v;
      if (g->directed) {
        u = idx / (n - 1);
        uint64_t o = idx % (n - 1);
        v = o >= u ? o + 1 : o;
      } else {
        double dn = (double)n;
        double est = std::floor(dn - 0.5 - std::sqrt((dn - 0.5) * (dn - 0.5) - 2.0 * (double)idx));
        if (est < 0) est = 0;
        uint64_t uu = (uint64_t)est;
        while (uu > 0 && start(uu) > idx) --uu;
        while (start(uu + 1) <= idx) ++uu;
        u = uu; v = uu + 1 + (idx - start(uu));
      }
      if (u / block_size != v / block_size) add((uint32_t)u, (uint32_t)v);
      uint64_t k = geo_skip(g->rng, p_out);
      if (k == UINT64_MAX || idx + 1 + k < idx) break;
      idx += 1 + k;
    }
  }
  return 0;
}

// R-MAT with quadrant probabilities a, b, c (d = 1-a-b-c) on 2^scale ids, ids >= n rejected,
// self-loops and duplicates dropped until exactly n_edges unique edges exist; then a seeded
// random vertex permutation is applied.  weight_kind 0: uniform integers [p1, p2];
// weight_kind 1: lognormal exp(p1 + p2 Z) rounded to the nearest integer, at least 1.
int syn_rmat(void* gp, uint64_t n_edges, double a, double b, double c, int weight_kind, double p1,
             double p2, int permute) {
  Gen* g = (Gen*)gp;
  const uint64_t n = g->n;
  if (n < 2) return -1;
  uint64_t maxpairs = g->directed ? n * (n - 1) : n * (n - 1) / 2;
  if (n_edges > maxpairs / 2) return -2;
  int scale = 0;
  while ((1ull << scale) < n) ++scale;
  g->es.reserve(n_edges);
  std::vector<uint32_t> perm;
  if (permute) {
    perm.resize(n);
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (uint64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[g->rng.below(i + 1)]);
  }
  const double ab = a + b, abc = a + b + c;
  while (g->es.keys.size() < n_edges) {
    uint64_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      double r = g->rng.unit();
      u <<= 1; v <<= 1;
      if (r < a) {
      } else if (r < ab) {
        v |= 1;
      } else if (r < abc) {
        u |= 1;
      } else {
        u |= 1; v |= 1;
      }
    }
    if (u >= n || v >= n || u == v) continue;
    uint32_t pu = permute ? perm[u] : (uint32_t)u, pv = permute ? perm[v] : (uint32_t)v;
    uint64_t k = g->key(pu, pv);
    if (g->es.contains(k)) continue;
    g->es.insert(k, g->draw_weight(weight_kind, p1, p2));
  }
  return 0;
}

// One update batch of `size` updates: round(f_ins*size) inserts of uniform random non-edge
// pairs, round(f_del*size) deletions drawn uniformly without replacement from current edges,
// the rest reweights of other current edges to a new weight != old.  Every pair appears at
// most once per batch.  The batch is applied to the generator's edge set.
// Output arrays: ins (u,v,w) triples, del (u,v) pairs, chg (u,v,w) triples.
int syn_batch(void* gp, uint64_t size, double f_ins, double f_del, int weight_kind, double p1, double p2,
              uint32_t* ins, uint64_t* n_ins, uint32_t* del, uint64_t* n_del, uint32_t* chg,
              uint64_t* n_chg) {
  Gen* g = (Gen*)gp;
  uint64_t ni = (uint64_t)std::llround(f_ins * (double)size);
  uint64_t nd = (uint64_t)std::llround(f_del * (double)size);
  if (ni > size) ni = size;
  if (nd > size - ni) nd = size - ni;
  uint64_t nc = size - ni - nd;
  uint64_t E = g->es.keys.size();
  if (nd > E) nd = E;
  if (nc > E - nd) nc = E - nd;
  // deletions: partial Fisher-Yates over the key array (moves picks to the tail)
  std::vector<uint64_t> pick_del, pick_chg;
  {
    std::vector<uint64_t>& K = g->es.keys;
    std::vector<uint32_t>& W = g->es.w;
    uint64_t m = K.size();
    for (uint64_t t = 0; t < nd + nc; ++t) {
      uint64_t j = g->rng.below(m - t);
      uint64_t last = m - 1 - t;
      std::swap(K[j], K[last]); std::swap(W[j], W[last]);
      g->es.slot_idx[g->es.find_slot(K[j])] = j;
      g->es.slot_idx[g->es.find_slot(K[last])] = last;
    }
    for (uint64_t t = 0; t < nd + nc; ++t) {
      uint64_t i = m - 1 - t;
      if (t < nd) pick_del.push_back(K[i]); else pick_chg.push_back(K[i]);
    }
  }
  for (uint64_t t = 0; t < nd; ++t) {
    uint64_t k = pick_del[t];
    del[2 * t] = (uint32_t)(k >> 32); del[2 * t + 1] = (uint32_t)k;
  }
  uint64_t cc = 0;
  for (uint64_t t = 0; t < nc; ++t) {
    uint64_t k = pick_chg[t];
    uint64_t idx = g->es.index_of(k);
    uint32_t old = g->es.w[idx], nw = old;
    int tries = 0;
    while (nw == old && tries < 64) { nw = g->draw_weight(weight_kind, p1, p2); ++tries; }
    if (nw == old) continue;
    chg[3 * cc] = (uint32_t)(k >> 32); chg[3 * cc + 1] = (uint32_t)k; chg[3 * cc + 2] = nw;
    g->es.w[idx] = nw;
    ++cc;
  }
  for (uint64_t t = 0; t < nd; ++t) g->es.erase(pick_del[t]);
  // inserts: uniform non-edge pairs, u != v, distinct within the batch (and not a pair that
  // was deleted in this batch, so that no pair appears twice)
  EdgeSet fresh;
  std::vector<uint64_t> deleted(pick_del.begin(), pick_del.end());
  std::sort(deleted.begin(), deleted.end());
  uint64_t ic = 0;
  uint64_t guard = 0;
  while (ic < ni && guard < 100 * (ni + 10)) {
    ++guard;
    uint32_t u = (uint32_t)g->rng.below(g->n), v = (uint32_t)g->rng.below(g->n);
    if (u == v) continue;
    uint64_t k = g->key(u, v);
    if (g->es.contains(k) || fresh.contains(k)) continue;
    if (std::binary_search(deleted.begin(), deleted.end(), k)) continue;
    uint32_t w = g->draw_weight(weight_kind, p1, p2);
    fresh.insert(k, w);
    ins[3 * ic] = u; ins[3 * ic + 1] = v; ins[3 * ic + 2] = w;
    ++ic;
  }
  for (uint64_t t = 0; t < ic; ++t) g->es.insert(g->key(ins[3 * t], ins[3 * t + 1]), ins[3 * t + 2]);
  *n_ins = ic; *n_del = nd; *n_chg = cc;
  return 0;
}

}  // extern "C"
