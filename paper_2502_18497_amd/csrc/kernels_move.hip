// Local-move and refinement kernels (Alg. 1 l.8-12 and l.16-21; gain of Sec. III-D), the
// exact decoupling filter of Sec. III-E as parallel rounds, and the commit / rollback /
// expansion kernels.
//
// BestMove for vertex v with label a scans v's out-entries (and in-entries when directed),
// sums acc[c] over neighbours u != v by label c = P(u), and evaluates for every b != a the
// exact integer gain
//   directed:   G = qm (acc[b]-acc[a]) - p (kout_v (Kin_b-Kin_a+kin_v) + kin_v (Kout_b-Kout_a+kout_v))
//   undirected: G = qm (acc[b]-acc[a]) - p k_v (K_b-K_a+k_v)
// (qm = q*m, gamma = p/q), keeping the largest G with ties to the lowest b, if G > 0.
// BestRef for a singleton u sums acc[y] over neighbours x with P(x) = P(u) by y = pi(x) and
// uses G = qm acc[y] - p (kout_u Krin_y + kin_u Krout_y) (undirected: qm acc[y] - p k_u Kr_y).
//
// Vertices are binned by their entry count T: groups of 8 or 32 lanes hold one entry per
// lane and sum equal keys with lane shuffles; wavefront and workgroup teams accumulate in an
// LDS hash table; hubs use a workgroup with a hash table in global memory.
#include "ldl_dev.h"
#include "ldl_kernels.h"

namespace ldl {

namespace {

constexpr int kTpb = 256;

inline unsigned grid_for(uint64_t n, uint64_t per_block = kTpb) {
  uint64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (1u << 20)) g = 1u << 20;
  return (unsigned)g;
}
inline unsigned grid_waves(uint64_t items) { return grid_for(items, kTpb / kWave); }

__device__ __forceinline__ uint64_t gtid() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ uint64_t gwave() { return ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; }
__device__ __forceinline__ uint64_t gwstride() { return (uint64_t)gridDim.x * blockDim.x / kWave; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int64_t wget(const CsrRef& c, uint64_t i) {
  return c.wide ? ((const int64_t*)c.w)[i] : (int64_t)((const uint32_t*)c.w)[i];
}

template <typename WT>
__device__ __forceinline__ int64_t wload(const CsrRef& c, uint64_t i) {
  return (int64_t)((const WT*)c.w)[i];
}

// Entry j of vertex v's combined out/in list: (neighbour, weight).
template <typename WT, bool DIR>
__device__ __forceinline__ void entry_at(const MoveView& mv, uint64_t oo, uint32_t dout, uint64_t oi, uint32_t j,
                                         uint32_t& x, int64_t& w) {
  if (!DIR || j < dout) {
    x = mv.out.nbr[oo + j];
    w = wload<WT>(mv.out, oo + j);
  } else {
    x = mv.in.nbr[oi + (j - dout)];
    w = wload<WT>(mv.in, oi + (j - dout));
  }
}

// key of neighbour x for vertex v: its label (move) or its refined community when it shares
// v's label (refinement); kEmpty for entries that do not count
template <bool REF>
__device__ __forceinline__ uint32_t entry_key(const MoveView& mv, uint32_t v, uint32_t labv, uint32_t x) {
  if (x == v) return kEmpty;
  if (!REF) return mv.lab[x];
  return mv.lab[x] == labv ? mv.par[x] : kEmpty;
}

struct VInfo {
  int64_t ko, ki, Koa, Kia;
  uint32_t lab;
};

template <bool DIR, bool REF>
__device__ __forceinline__ i128 gain(const MoveView& mv, const VInfo& vi, uint32_t b, int64_t accb, int64_t acca) {
  if (!REF) {
    const int64_t Kob = mv.Kout[b];
    if (DIR) {
      const int64_t Kib = mv.Kin[b];
      return (i128)mv.qm * (accb - acca) -
             (i128)mv.p * ((i128)vi.ko * (Kib - vi.Kia + vi.ki) + (i128)vi.ki * (Kob - vi.Koa + vi.ko));
    }
    return (i128)mv.qm * (accb - acca) - (i128)mv.p * ((i128)vi.ko * (Kob - vi.Koa + vi.ko));
  } else {
    const int64_t Kob = mv.Kout[b];
    if (DIR) {
      const int64_t Kib = mv.Kin[b];
      return (i128)mv.qm * accb - (i128)mv.p * ((i128)vi.ko * Kib + (i128)vi.ki * Kob);
    }
    return (i128)mv.qm * accb - (i128)mv.p * ((i128)vi.ko * Kob);
  }
}

template <bool DIR, bool REF>
__device__ __forceinline__ VInfo vinfo(const MoveView& mv, uint32_t v) {
  VInfo vi;
  vi.lab = mv.lab[v];
  vi.ko = mv.kout[v];
  vi.ki = DIR ? mv.kin[v] : vi.ko;
  if (!REF) {
    vi.Koa = mv.Kout[vi.lab];
    vi.Kia = DIR ? mv.Kin[vi.lab] : vi.Koa;
  } else {
    vi.Koa = vi.Kia = 0;
  }
  return vi;
}

__device__ __forceinline__ void emit_cand_at(const CandBuf& cb, uint32_t at, uint32_t v, uint32_t a, const Best& b) {
  cb.v[at] = v;
  cb.a[at] = a;
  cb.b[at] = b.id;
  cb.glo[at] = b.lo;
  cb.ghi[at] = b.hi;
}

// ------------------------------------------------------------------ binning
__global__ void k_bin(MoveView mv, const uint32_t* list, uint32_t count, int refine, uint32_t* b0, uint32_t* b1,
                      uint32_t* b2, uint32_t* b3, uint32_t* b4, uint32_t* bc) {
  for (uint64_t i = gtid(); i < count; i += gstride()) {
    const uint32_t v = list[i];
    if (refine && !(mv.par[v] == v && mv.rsize[v] == 1)) continue;   // only singletons move
    const uint64_t T = (uint64_t)mv.out.deg[v] + (mv.directed ? (uint64_t)mv.in.deg[v] : 0ull);
    if (T == 0) continue;
    int b = 4;
    if (T <= kBinLimit[0]) b = 0;
    else if (T <= kBinLimit[1]) b = 1;
    else if (T <= kBinLimit[2]) b = 2;
    else if (T <= kBinLimit[3]) b = 3;
    uint32_t* dsts[kNumBins] = {b0, b1, b2, b3, b4};
#pragma unroll
    for (int t = 0; t < kNumBins; ++t) {
      const uint32_t at = wave_reserve(&bc[t], b == t);
      if (b == t) dsts[t][at] = v;
    }
  }
}

// ------------------------------------------------------------------ binning without atomics
__device__ __forceinline__ int bin_of(const MoveView& mv, uint32_t v, int refine) {
  if (refine && !(mv.par[v] == v && mv.rsize[v] == 1)) return -1;   // only singletons move
  const uint64_t T = (uint64_t)mv.out.deg[v] + (mv.directed ? (uint64_t)mv.in.deg[v] : 0ull);
  if (T == 0) return -1;
  if (T <= kBinLimit[0]) return 0;
  if (T <= kBinLimit[1]) return 1;
  if (T <= kBinLimit[2]) return 2;
  if (T <= kBinLimit[3]) return 3;
  return 4;
}

// block b owns list[b*chunk, (b+1)*chunk); hist[bin * gridDim + b] = its count per bin
__global__ void k_bin_count(MoveView mv, const uint32_t* list, uint32_t count, int refine, uint32_t* hist) {
  __shared__ uint32_t h[kNumBins];
  if (threadIdx.x < kNumBins) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t chunk = ((uint64_t)count + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int b = bin_of(mv, list[i], refine);
    if (b >= 0) atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kNumBins) hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_bin_fill(MoveView mv, const uint32_t* list, uint32_t count, int refine, const uint32_t* offs,
                           uint32_t* out, uint32_t* bin_start, uint32_t* bin_count) {
  __shared__ uint32_t pos[kNumBins];
  const unsigned nb = gridDim.x;
  if (threadIdx.x < kNumBins) pos[threadIdx.x] = offs[threadIdx.x * nb + blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x < kNumBins) {
    const uint32_t start = offs[threadIdx.x * nb];
    const uint32_t end = threadIdx.x + 1 < kNumBins ? offs[(threadIdx.x + 1) * nb] : offs[kNumBins * nb];
    bin_start[threadIdx.x] = start;
    bin_count[threadIdx.x] = end - start;
  }
  __syncthreads();
  const uint64_t chunk = ((uint64_t)count + nb - 1) / nb;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const uint32_t v = list[i];
    const int b = bin_of(mv, v, refine);
    if (b >= 0) out[atomicAdd(&pos[b], 1u)] = v;
  }
}

// movers and their neighbours marked with plain stores
__global__ void k_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, uint32_t na, CandBuf cand,
                                      CsrRef out, CsrRef in, int directed) {
  const int lane = lane_id();
  for (uint64_t t = gwave(); t < na; t += gwstride()) {
    const uint32_t v = cand.v[acc[t]];
    if (lane == 0) stamp[v] = ep;
    const uint64_t o = out.off[v];
    const uint32_t d = out.deg[v];
    for (uint32_t j = lane; j < d; j += kWave) stamp[out.nbr[o + j]] = ep;
    if (directed) {
      const uint64_t oi = in.off[v];
      const uint32_t di = in.deg[v];
      for (uint32_t j = lane; j < di; j += kWave) stamp[in.nbr[oi + j]] = ep;
    }
  }
}

// ------------------------------------------------------------------ candidate staging
// The candidate kernels run persistent grids (a few workgroups per CU, block-uniform loops).
// Candidates are staged in LDS and appended to the global list in bulk, and the statistics
// are kept in registers until the block exits, so global atomics on the shared counters are
// a handful per workgroup rather than several per wavefront.
constexpr unsigned kPersistBlocks = 2048;

template <int CAP>
struct Stage {
  uint32_t v[CAP], a[CAP], b[CAP];
  uint64_t lo[CAP];
  int64_t hi[CAP];
  uint32_t n, base;
};

template <int CAP>
__device__ __forceinline__ void stage_push(Stage<CAP>& s, uint32_t v, uint32_t a, const Best& b) {
  const uint32_t i = atomicAdd(&s.n, 1u);
  s.v[i] = v;
  s.a[i] = a;
  s.b[i] = b.id;
  s.lo[i] = b.lo;
  s.hi[i] = b.hi;
}

// every thread of the block calls this
template <int CAP>
__device__ __forceinline__ void stage_flush(Stage<CAP>& s, const CandBuf& cand) {
  __syncthreads();
  const uint32_t k = s.n;
  if (k) {
    if (threadIdx.x == 0) s.base = atomicAdd(cand.count, k);
    __syncthreads();
    const uint32_t base = s.base;
    for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
      cand.v[base + i] = s.v[i];
      cand.a[base + i] = s.a[i];
      cand.b[base + i] = s.b[i];
      cand.glo[base + i] = s.lo[i];
      cand.ghi[base + i] = s.hi[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) s.n = 0;
  }
  __syncthreads();
}

struct LocalStats {
  unsigned long long entries = 0, distinct = 0, vertices = 0, cands = 0;
};

// every thread of the block calls this once, at exit
__device__ __forceinline__ void stats_flush(LocalStats ls, const MoveStats& st, unsigned long long* red) {
  if (!st.entries) return;
  unsigned long long v[4] = {ls.entries, ls.distinct, ls.vertices, ls.cands};
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (unsigned long long)wave_sum_i64((int64_t)v[k]);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[4 * w + k] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long t = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += red[4 * i + threadIdx.x];
    u64a* dst = threadIdx.x == 0 ? st.entries : threadIdx.x == 1 ? st.distinct : threadIdx.x == 2 ? st.vertices
                                                                                                 : st.cands;
    if (t) atomicAdd(dst, t);
  }
}

// ------------------------------------------------------------------ small degrees: lane groups
template <typename WT, int G, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_best_group(MoveView mv, const uint32_t* list, uint32_t count,
                                                     CandBuf cand, MoveStats st) {
  constexpr int VPB = kTpb / G;            // vertices per block iteration
  __shared__ Stage<256> stage;
  __shared__ unsigned long long red[4 * (kTpb / kWave)];
  if (threadIdx.x == 0) stage.n = 0;
  __syncthreads();
  LocalStats ls;
  const int li = threadIdx.x & (G - 1);
  for (uint64_t base = (uint64_t)blockIdx.x * VPB; base < count; base += (uint64_t)gridDim.x * VPB) {
    const uint64_t gid = base + threadIdx.x / G;
    const bool active = gid < count;        // every lane stays for the shuffles
    uint32_t v = 0, key = kEmpty;
    int64_t w = 0;
    VInfo vi{};
    uint32_t T = 0;
    if (active) {
      v = list[gid];
      vi = vinfo<DIR, REF>(mv, v);
      const uint32_t dout = mv.out.deg[v];
      const uint32_t din = DIR ? mv.in.deg[v] : 0;
      T = dout + din;
      if ((uint32_t)li < T) {
        uint32_t x;
        entry_at<WT, DIR>(mv, mv.out.off[v], dout, DIR ? mv.in.off[v] : 0, (uint32_t)li, x, w);
        key = entry_key<REF>(mv, v, vi.lab, x);
      }
    }
    // weight towards the own community (move only)
    int64_t own = (!REF && key != kEmpty && key == vi.lab) ? w : 0;
#pragma unroll
    for (int o = G >> 1; o > 0; o >>= 1) own += __shfl_xor(own, o, G);
    // sum equal keys across the group; the lowest lane of each key represents it
    int64_t acc = 0;
    bool rep = key != kEmpty && (REF || key != vi.lab);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint32_t kj = (uint32_t)__shfl((int)key, j, G);
      const int64_t wj = __shfl(w, j, G);
      if (kj == key) {
        acc += wj;
        if (j < li) rep = false;
      }
    }
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
    if (active && rep) b = make_best(gain<DIR, REF>(mv, vi, key, acc, own), key);
    ls.distinct += (active && rep) ? 1 : 0;
    b = group_best(b, G);
    if (active && li == 0) {
      ls.entries += T;
      ls.vertices += 1;
      if (b.valid && best_gain(b) > 0) {
        stage_push(stage, v, REF ? v : vi.lab, b);
        ls.cands += 1;
      }
    }
    __syncthreads();
    if (stage.n + VPB > 256) stage_flush(stage, cand);
  }
  stage_flush(stage, cand);
  stats_flush(ls, st, red);
}

// ------------------------------------------------------------------ hash-table teams
template <int TEAM>
__device__ __forceinline__ int64_t team_sum(int64_t x, int64_t* red) {
  x = wave_sum_i64(x);
  if (TEAM == kWave) return x;
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  int64_t s = 0;
  for (int i = 0; i < TEAM / kWave; ++i) s += red[i];
  return s;
}

template <int TEAM>
__device__ __forceinline__ Best team_best(Best b, Best* red) {
  b = group_best(b, kWave);
  if (TEAM == kWave) return b;
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = b;
  __syncthreads();
  Best r = red[0];
  for (int i = 1; i < TEAM / kWave; ++i)
    if (better(red[i], r)) r = red[i];
  return r;
}

__device__ __forceinline__ void table_insert(uint32_t* keys, u64a* vals, uint32_t mask, uint32_t key, int64_t w) {
  uint32_t h = hash32(key) & mask;
  for (;;) {
    const uint32_t prev = atomicCAS(&keys[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&vals[h], (u64a)w);
      return;
    }
    h = (h + 1) & mask;
  }
}

// TEAM lanes per vertex with a private LDS table of SLOTS (>= 2 T) entries
template <typename WT, int TEAM, int SLOTS, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_best_hash(MoveView mv, const uint32_t* list, uint32_t count, CandBuf cand,
                                                    MoveStats st) {
  constexpr int TEAMS = kTpb / TEAM;
  __shared__ uint32_t skey[TEAMS][SLOTS];
  __shared__ u64a sval[TEAMS][SLOTS];
  __shared__ int64_t red_i[kTpb / kWave];
  __shared__ Best red_b[kTpb / kWave];
  __shared__ Stage<64> stage;
  __shared__ unsigned long long red_s[4 * (kTpb / kWave)];
  if (threadIdx.x == 0) stage.n = 0;
  const int t = threadIdx.x / TEAM;
  const int li = threadIdx.x % TEAM;
  LocalStats ls;
  for (uint64_t base = (uint64_t)blockIdx.x * TEAMS; base < count; base += (uint64_t)gridDim.x * TEAMS) {
    const uint64_t slot = base + t;
    const bool active = slot < count;
    const uint32_t v = active ? list[slot] : 0;
    for (int s = li; s < SLOTS; s += TEAM) {
      skey[t][s] = kEmpty;
      sval[t][s] = 0;
    }
    __syncthreads();
    VInfo vi{};
    int64_t own = 0;
    uint32_t T = 0;
    if (active) {
      vi = vinfo<DIR, REF>(mv, v);
      const uint32_t dout = mv.out.deg[v];
      const uint32_t din = DIR ? mv.in.deg[v] : 0;
      const uint64_t oo = mv.out.off[v], oi = DIR ? mv.in.off[v] : 0;
      T = dout + din;
      for (uint32_t j = li; j < T; j += TEAM) {
        uint32_t x;
        int64_t w;
        entry_at<WT, DIR>(mv, oo, dout, oi, j, x, w);
        const uint32_t key = entry_key<REF>(mv, v, vi.lab, x);
        if (key == kEmpty) continue;
        if (!REF && key == vi.lab) {
          own += w;
          continue;
        }
        table_insert(skey[t], sval[t], SLOTS - 1, key, w);
      }
    }
    __syncthreads();
    own = team_sum<TEAM>(own, red_i);
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
    if (active) {
      for (int s = li; s < SLOTS; s += TEAM) {
        const uint32_t key = skey[t][s];
        if (key == kEmpty) continue;
        ls.distinct += 1;
        const Best c = make_best(gain<DIR, REF>(mv, vi, key, (int64_t)sval[t][s], own), key);
        if (better(c, b)) b = c;
      }
    }
    b = team_best<TEAM>(b, red_b);
    if (active && li == 0) {
      ls.entries += T;
      ls.vertices += 1;
      if (b.valid && best_gain(b) > 0) {
        stage_push(stage, v, REF ? v : vi.lab, b);
        ls.cands += 1;
      }
    }
    __syncthreads();
    if (stage.n + TEAMS > 64) stage_flush(stage, cand);
  }
  stage_flush(stage, cand);
  stats_flush(ls, st, red_s);
}

// hubs: one workgroup per vertex, table of pow2 >= 2T slots carved from a global pool; a
// vertex that finds the pool full is deferred to the overflow list for a later launch
template <typename WT, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_best_hub(MoveView mv, const uint32_t* list, uint32_t count, CandBuf cand,
                                                   HubPool hub, MoveStats st) {
  __shared__ int64_t red_i[kTpb / kWave];
  __shared__ Best red_b[kTpb / kWave];
  __shared__ uint64_t s_base;
  __shared__ int s_ok;
  __shared__ Stage<32> stage;
  __shared__ unsigned long long red_s[4 * (kTpb / kWave)];
  if (threadIdx.x == 0) stage.n = 0;
  LocalStats ls;
  for (uint64_t slot = blockIdx.x; slot < count; slot += gridDim.x) {
    const uint32_t v = list[slot];
    const uint32_t dout = mv.out.deg[v];
    const uint32_t din = DIR ? mv.in.deg[v] : 0;
    const uint32_t T = dout + din;
    uint64_t size = 1;
    while (size < 2ull * T) size <<= 1;
    __syncthreads();
    if (threadIdx.x == 0) {
      const u64a o = atomicAdd(hub.top, (u64a)size);
      s_ok = (o + size <= hub.cap) ? 1 : 0;
      s_base = o;
      if (!s_ok) hub.over[atomicAdd(hub.over_count, 1u)] = v;
    }
    __syncthreads();
    if (!s_ok) continue;
    uint32_t* keys = hub.keys + s_base;
    u64a* vals = hub.vals + s_base;
    const uint32_t mask = (uint32_t)(size - 1);
    for (uint64_t s = threadIdx.x; s < size; s += kTpb) {
      keys[s] = kEmpty;
      vals[s] = 0;
    }
    __threadfence();
    __syncthreads();
    const VInfo vi = vinfo<DIR, REF>(mv, v);
    const uint64_t oo = mv.out.off[v], oi = DIR ? mv.in.off[v] : 0;
    int64_t own = 0;
    for (uint32_t j = threadIdx.x; j < T; j += kTpb) {
      uint32_t x;
      int64_t w;
      entry_at<WT, DIR>(mv, oo, dout, oi, j, x, w);
      const uint32_t key = entry_key<REF>(mv, v, vi.lab, x);
      if (key == kEmpty) continue;
      if (!REF && key == vi.lab) {
        own += w;
        continue;
      }
      table_insert(keys, vals, mask, key, w);
    }
    __threadfence();
    __syncthreads();
    own = team_sum<kTpb>(own, red_i);
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
    for (uint64_t s = threadIdx.x; s < size; s += kTpb) {
      const uint32_t key = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (key == kEmpty) continue;
      ls.distinct += 1;
      const int64_t a = (int64_t)__hip_atomic_load(&vals[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const Best c = make_best(gain<DIR, REF>(mv, vi, key, a, own), key);
      if (better(c, b)) b = c;
    }
    b = team_best<kTpb>(b, red_b);
    if (threadIdx.x == 0) {
      ls.entries += T;
      ls.vertices += 1;
      if (b.valid && best_gain(b) > 0) {
        stage_push(stage, v, REF ? v : vi.lab, b);
        ls.cands += 1;
      }
    }
    __syncthreads();
    if (stage.n + 1 > 32) stage_flush(stage, cand);
  }
  stage_flush(stage, cand);
  stats_flush(ls, st, red_s);
}

// ---- hubs split over many workgroups.  Each hub vertex i owns a table of hsize[i] =
// pow2 >= 2 T_i slots at hoff[i] in the pool; entry chunks insert in parallel, slot chunks
// evaluate gains into partial bests, and one wavefront per hub reduces the partials.
constexpr uint32_t kHubChunk = 4096;   // entries per insert workgroup
constexpr uint32_t kHubScan = kHubScanSlots;

__global__ void k_hub_prep(MoveView mv, const uint32_t* list, uint32_t h, uint64_t* hsize, u64a* maxT) {
  u64a mt = 0;
  for (uint64_t i = gtid(); i <= h; i += gstride()) {
    if (i == h) {
      hsize[h] = 0;
      continue;
    }
    const uint32_t v = list[i];
    const uint64_t T = (uint64_t)mv.out.deg[v] + (mv.directed ? (uint64_t)mv.in.deg[v] : 0ull);
    uint64_t size = 64;
    while (size < 2 * T) size <<= 1;
    hsize[i] = size;
    if (T > mt) mt = T;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const u64a t = (u64a)__shfl_xor((long long)mt, o, 64);
    if (t > mt) mt = t;
  }
  if ((threadIdx.x & 63) == 0 && mt) atomicMax(maxT, mt);
}

template <typename WT, bool DIR, bool REF>
__global__ __launch_bounds__(256) void k_hub_insert(MoveView mv, const uint32_t* list, uint32_t i0,
                                                    const uint64_t* hoff, uint64_t base0, HubPool hub, int64_t* own,
                                                    MoveStats st) {
  __shared__ int64_t red[kTpb / kWave];
  const uint32_t i = i0 + blockIdx.y;
  const uint32_t v = list[i];
  const uint32_t dout = mv.out.deg[v];
  const uint32_t din = DIR ? mv.in.deg[v] : 0;
  const uint32_t T = dout + din;
  const uint64_t e0 = (uint64_t)blockIdx.x * kHubChunk;
  if (e0 >= T) return;                      // whole workgroup leaves together
  const uint64_t e1 = e0 + kHubChunk < T ? e0 + kHubChunk : T;
  const uint64_t base = hoff[i] - base0;
  const uint32_t mask = (uint32_t)(hoff[i + 1] - hoff[i] - 1);
  uint32_t* keys = hub.keys + base;
  u64a* vals = hub.vals + base;
  const uint32_t labv = mv.lab[v];
  const uint64_t oo = mv.out.off[v], oi = DIR ? mv.in.off[v] : 0;
  int64_t ow = 0;
  for (uint64_t j = e0 + threadIdx.x; j < e1; j += blockDim.x) {
    uint32_t x;
    int64_t w;
    entry_at<WT, DIR>(mv, oo, dout, oi, (uint32_t)j, x, w);
    const uint32_t key = entry_key<REF>(mv, v, labv, x);
    if (key == kEmpty) continue;
    if (!REF && key == labv) {
      ow += w;
      continue;
    }
    table_insert(keys, vals, mask, key, w);
  }
  ow = team_sum<kTpb>(ow, red);
  if (threadIdx.x == 0) {
    if (ow) atomic_add_i64(&own[blockIdx.y], ow);
    if (st.entries) atomicAdd(st.entries, (u64a)(e1 - e0));
  }
}

template <typename WT, bool DIR, bool REF>
__global__ __launch_bounds__(256) void k_hub_scan(MoveView mv, const uint32_t* list, uint32_t i0,
                                                  const uint64_t* hoff, uint64_t base0, HubPool hub,
                                                  const int64_t* own, uint32_t max_parts, int64_t* phi, uint64_t* plo,
                                                  uint32_t* pid, int* pvalid, MoveStats st) {
  __shared__ Best red_b[kTpb / kWave];
  __shared__ int64_t red_i[kTpb / kWave];
  const uint32_t i = i0 + blockIdx.y;
  const uint64_t size = hoff[i + 1] - hoff[i];
  const uint64_t s0 = (uint64_t)blockIdx.x * kHubScan;
  if (s0 >= size) return;
  const uint64_t s1 = s0 + kHubScan < size ? s0 + kHubScan : size;
  const uint64_t base = hoff[i] - base0;
  const uint32_t v = list[i];
  const VInfo vi = vinfo<DIR, REF>(mv, v);
  const int64_t ow = own[blockIdx.y];
  Best b;
  b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
  int64_t nd = 0;
  for (uint64_t sl = s0 + threadIdx.x; sl < s1; sl += blockDim.x) {
    const uint32_t key = __hip_atomic_load(&hub.keys[base + sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (key == kEmpty) continue;
    ++nd;
    const int64_t a = (int64_t)__hip_atomic_load(&hub.vals[base + sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Best c = make_best(gain<DIR, REF>(mv, vi, key, a, ow), key);
    if (better(c, b)) b = c;
  }
  nd = team_sum<kTpb>(nd, red_i);
  b = team_best<kTpb>(b, red_b);
  if (threadIdx.x == 0) {
    const uint64_t at = (uint64_t)blockIdx.y * max_parts + blockIdx.x;
    phi[at] = b.hi;
    plo[at] = b.lo;
    pid[at] = b.id;
    pvalid[at] = b.valid;
    if (st.entries && nd) atomicAdd(st.distinct, (u64a)nd);
  }
}

template <bool REF>
__global__ void k_hub_final(const uint32_t* list, uint32_t i0, uint32_t ng, const uint64_t* hoff,
                            const uint32_t* lab, uint32_t max_parts, const int64_t* phi, const uint64_t* plo,
                            const uint32_t* pid, const int* pvalid, CandBuf cand, MoveStats st) {
  const int lane = lane_id();
  for (uint64_t g = gwave(); g < ng; g += gwstride()) {
    const uint32_t i = i0 + (uint32_t)g;
    const uint64_t size = hoff[i + 1] - hoff[i];
    const uint32_t np = (uint32_t)((size + kHubScan - 1) / kHubScan);
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
    for (uint32_t p = lane; p < np; p += kWave) {
      const uint64_t at = g * max_parts + p;
      Best c;
      c.hi = phi[at]; c.lo = plo[at]; c.id = pid[at]; c.valid = pvalid[at];
      if (better(c, b)) b = c;
    }
    b = group_best(b, kWave);
    if (lane == 0) {
      const uint32_t v = list[i];
      if (st.entries) atomicAdd(st.vertices, 1ull);
      if (b.valid && best_gain(b) > 0) {
        emit_cand_at(cand, atomicAdd(cand.count, 1u), v, REF ? v : lab[v], b);
        if (st.cands) atomicAdd(st.cands, 1ull);
      }
    }
  }
}

__global__ void k_hub_clear(uint32_t* keys, u64a* vals, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) {
    keys[i] = kEmpty;
    vals[i] = 0;
  }
}

template <typename WT, bool DIR, bool REF>
void hub_group_dispatch(const MoveView& mv, const uint32_t* list, uint32_t i0, uint32_t ng, const uint64_t* hoff,
                        uint64_t base0, uint64_t span, uint64_t maxT, HubPool hub, int64_t* own, uint32_t max_parts,
                        int64_t* phi, uint64_t* plo, uint32_t* pid, int* pvalid, CandBuf cand, MoveStats st,
                        hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  k_hub_clear<<<grid_for(span), kTpb, 0, s>>>(hub.keys, hub.vals, span);
  if (ev_a) (void)hipEventRecord(ev_a, s);
  dim3 gi((unsigned)((maxT + kHubChunk - 1) / kHubChunk), ng);
  k_hub_insert<WT, DIR, REF><<<gi, kTpb, 0, s>>>(mv, list, i0, hoff, base0, hub, own, st);
  if (ev_b) (void)hipEventRecord(ev_b, s);
  dim3 gs(max_parts, ng);
  k_hub_scan<WT, DIR, REF><<<gs, kTpb, 0, s>>>(mv, list, i0, hoff, base0, hub, own, max_parts, phi, plo, pid, pvalid,
                                              st);
  k_hub_final<REF><<<grid_waves(ng), kTpb, 0, s>>>(list, i0, ng, hoff, mv.lab, max_parts, phi, plo, pid, pvalid,
                                                   cand, st);
}

inline unsigned persist_grid(uint64_t items_per_block_units) {
  uint64_t g = items_per_block_units;
  if (g < 1) g = 1;
  if (g > kPersistBlocks) g = kPersistBlocks;
  return (unsigned)g;
}

template <typename WT, bool DIR, bool REF>
void best_dispatch(const MoveView& mv, int bin, const uint32_t* list, uint32_t count, CandBuf cand, HubPool hub,
                   MoveStats st, hipStream_t s) {
  switch (bin) {
    case 0:
      k_best_group<WT, 8, DIR, REF><<<persist_grid((count + 31) / 32), kTpb, 0, s>>>(mv, list, count, cand, st);
      break;
    case 1:
      k_best_group<WT, 32, DIR, REF><<<persist_grid((count + 7) / 8), kTpb, 0, s>>>(mv, list, count, cand, st);
      break;
    case 2:
      k_best_hash<WT, 64, 256, DIR, REF><<<persist_grid((count + 3) / 4), kTpb, 0, s>>>(mv, list, count, cand, st);
      break;
    case 3:
      k_best_hash<WT, 256, 4096, DIR, REF><<<persist_grid(count), kTpb, 0, s>>>(mv, list, count, cand, st);
      break;
    default:
      k_best_hub<WT, DIR, REF><<<persist_grid(count), kTpb, 0, s>>>(mv, list, count, cand, hub, st);
  }
}

// ------------------------------------------------------------------ decouple rounds
// Candidates in rank order (gain descending, vertex ascending).  Candidate i conflicts with j
// when a_i == b_j or b_i == a_j.  The sequential filter accepts a candidate iff no earlier
// accepted candidate conflicts with it, i.e. it returns the lexicographically first maximal
// independent set of the conflict graph; each round accepts every live candidate without an
// earlier live conflict and drops the live candidates that conflict with an accepted one.

__global__ void k_rank_from_order(const uint32_t* order, uint32_t k, uint32_t* rank) {
  for (uint64_t i = gtid(); i < k; i += gstride()) rank[order[i]] = (uint32_t)i;
}
__global__ void k_gather_u64(const uint64_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst, int invert) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t x = src[idx[i]];
    dst[i] = invert ? ~x : x;
  }
}
__global__ void k_gather_u32_as_u64(const uint32_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst) {
  for (uint64_t i = gtid(); i < k; i += gstride()) dst[i] = idx ? src[idx[i]] : src[i];
}
__global__ void k_lf_reset(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, uint32_t* minE,
                           uint32_t* minA) {
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    minE[a[i]] = kEmpty; minA[a[i]] = kEmpty;
    minE[b[i]] = kEmpty; minA[b[i]] = kEmpty;
  }
}
__global__ void k_lf_min(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b,
                         const uint32_t* rank, uint32_t* minE, uint32_t* minA) {
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    atomicMin(&minE[a[i]], rank[i]);
    atomicMin(&minA[b[i]], rank[i]);
  }
}
__global__ void k_lf_accept(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b,
                            const uint32_t* rank, const uint32_t* minE, const uint32_t* minA, uint32_t* accE,
                            uint32_t* accA, uint32_t ep, uint8_t* flag, uint32_t* acc_list, uint32_t* acc_count) {
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    const uint32_t r = rank[i];
    // no live earlier candidate enters my source or leaves my target
    const bool ok = minA[a[i]] > r && minE[b[i]] > r;
    const uint32_t at = wave_reserve(acc_count, ok);
    if (ok) {
      flag[i] = 1;
      accE[a[i]] = ep;
      accA[b[i]] = ep;
      acc_list[at] = i;
    }
  }
}
__global__ void k_lf_reject(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b,
                            const uint32_t* accE, const uint32_t* accA, uint32_t ep, const uint8_t* flag,
                            uint32_t* live2, uint32_t* live2_count) {
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    const bool keep = !flag[i] && !(accA[a[i]] == ep || accE[b[i]] == ep);
    const uint32_t at = wave_reserve(live2_count, keep);
    if (keep) live2[at] = i;
  }
}

// ------------------------------------------------------------------ commit / rollback
__global__ void k_commit_mark(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* mov_stamp, uint32_t mov_ep,
                              uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin, SetRef touched,
                              int64_t* tko, int64_t* tki) {
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    const uint32_t v = cand.v[i];
    mov_stamp[v] = mov_ep;
    oldlab[v] = cand.a[i];
    const uint32_t cs[2] = {cand.a[i], cand.b[i]};
    for (int k = 0; k < 2; ++k) {
      const uint32_t c = cs[k];
      const bool claimed = set_claim(touched.stamp, touched.epoch, c);
      const uint32_t at = wave_reserve(touched.count, claimed);
      if (claimed) {
        touched.list[at] = c;
        tko[at] = Kout[c];
        tki[at] = Kin[c];
      }
    }
  }
}

__global__ void k_commit_apply(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* lab, const int64_t* kout,
                               const int64_t* kin, int64_t* Kout, int64_t* Kin, int forward) {
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    const uint32_t v = cand.v[i];
    const uint32_t from = forward ? cand.a[i] : cand.b[i];
    const uint32_t to = forward ? cand.b[i] : cand.a[i];
    lab[v] = to;
    atomic_add_i64(&Kout[from], -kout[v]);
    atomic_add_i64(&Kout[to], kout[v]);
    if (Kin) {
      atomic_add_i64(&Kin[from], -kin[v]);
      atomic_add_i64(&Kin[to], kin[v]);
    }
  }
}

// wave per mover: exact change of the same-label weight over matrix entries incident to
// movers, each entry once (entries between two movers from the out side)
__global__ void k_commit_dein(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                              const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep,
                              const uint32_t* oldlab, i64a* dein) {
  const int lane = lane_id();
  for (uint64_t t = gwave(); t < na; t += gwstride()) {
    const uint32_t v = cand.v[acc[t]];
    const uint32_t lv_new = lab[v], lv_old = oldlab[v];
    int64_t s = 0;
    {
      const uint64_t o = out.off[v];
      const uint32_t d = out.deg[v];
      for (uint32_t j = lane; j < d; j += kWave) {
        const uint32_t u = out.nbr[o + j];
        const int64_t w = wget(out, o + j);
        const uint32_t lu_new = lab[u];
        const uint32_t lu_old = mov_stamp[u] == mov_ep ? oldlab[u] : lu_new;
        s += w * ((int64_t)(lv_new == lu_new) - (int64_t)(lv_old == lu_old));
      }
    }
    {
      const CsrRef& c = directed ? in : out;
      const uint64_t o = c.off[v];
      const uint32_t d = c.deg[v];
      for (uint32_t j = lane; j < d; j += kWave) {
        const uint32_t u = c.nbr[o + j];
        if (mov_stamp[u] == mov_ep) continue;
        const int64_t w = wget(c, o + j);
        const uint32_t lu = lab[u];
        s += w * ((int64_t)(lv_new == lu) - (int64_t)(lv_old == lu));
      }
    }
    s = wave_sum_i64(s);
    if (lane == 0 && s != 0) atomicAdd((u64a*)dein, (u64a)s);
  }
}

__global__ void k_mark_acc_comms(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* stamp, uint32_t ep) {
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    set_claim(stamp, ep, cand.a[i]);
    set_claim(stamp, ep, cand.b[i]);
  }
}

__global__ void k_set_add_acc_v(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand) {
  for (uint64_t t = gtid(); t < na; t += gstride())
    set_add(set.stamp, set.epoch, set.list, set.count, cand.v[acc[t]]);
}

__global__ void k_neighbours_acc(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in,
                                 int directed) {
  const int lane = lane_id();
  for (uint64_t t = gwave(); t < na; t += gwstride()) {
    const uint32_t v = cand.v[acc[t]];
    if (lane == 0) set_add(set.stamp, set.epoch, set.list, set.count, v);
    const uint64_t o = out.off[v];
    const uint32_t d = out.deg[v];
    for (uint32_t j = lane; j < d; j += kWave) set_add(set.stamp, set.epoch, set.list, set.count, out.nbr[o + j]);
    if (directed) {
      const uint64_t oi = in.off[v];
      const uint32_t di = in.deg[v];
      for (uint32_t j = lane; j < di; j += kWave) set_add(set.stamp, set.epoch, set.list, set.count, in.nbr[oi + j]);
    }
  }
}

__global__ void k_ref_commit(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* par, const int64_t* kout,
                             const int64_t* kin, int64_t* Krout, int64_t* Krin, uint32_t* rsize) {
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    const uint32_t u = cand.v[i], y = cand.b[i];
    par[u] = y;
    atomic_add_i64(&Krout[y], kout[u]);
    atomic_add_i64(&Krout[u], -kout[u]);
    if (Krin) {
      atomic_add_i64(&Krin[y], kin[u]);
      atomic_add_i64(&Krin[u], -kin[u]);
    }
    atomicAdd(&rsize[y], 1u);
    atomicSub(&rsize[u], 1u);
  }
}

// SPExpand: singleton neighbours of refinement movers that carry the mover's label
__global__ void k_spexpand(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                           const uint32_t* lab, const uint32_t* par, const uint32_t* rsize, SetRef rcur, SetRef rset,
                           uint32_t* oldpar) {
  const int lane = lane_id();
  for (uint64_t t = gwave(); t < na; t += gwstride()) {
    const uint32_t v = cand.v[acc[t]];
    const uint32_t lv = lab[v];
    for (int side = 0; side < (directed ? 2 : 1); ++side) {
      const CsrRef& c = side == 0 ? out : in;
      const uint64_t o = c.off[v];
      const uint32_t d = c.deg[v];
      for (uint32_t j = lane; j < d; j += kWave) {
        const uint32_t x = c.nbr[o + j];
        const bool ok = x != v && lab[x] == lv && par[x] == x && rsize[x] == 1;
        set_add(rcur.stamp, rcur.epoch, rcur.list, rcur.count, x, ok);
        const bool claimed = ok && set_claim(rset.stamp, rset.epoch, x);
        const uint32_t at = wave_reserve(rset.count, claimed);
        if (claimed) {
          rset.list[at] = x;
          oldpar[x] = x;
        }
      }
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_bin_count(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, uint32_t* hist,
                      hipStream_t s) {
  k_bin_count<<<kBinBlocks, kTpb, 0, s>>>(mv, list, count, refine, hist);
}
void launch_bin_fill(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, const uint32_t* offs,
                     uint32_t* out, uint32_t* bin_start, uint32_t* bin_count, hipStream_t s) {
  k_bin_fill<<<kBinBlocks, kTpb, 0, s>>>(mv, list, count, refine, offs, out, bin_start, bin_count);
}
void launch_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, uint32_t na, CandBuf cand,
                                CsrRef out, CsrRef in, int directed, hipStream_t s) {
  if (na) k_mark_neighbours_acc<<<grid_waves(na), kTpb, 0, s>>>(stamp, ep, acc, na, cand, out, in, directed);
}
void launch_hub_prep(const MoveView& mv, const uint32_t* list, uint32_t h, uint64_t* hsize, u64a* maxT,
                     hipStream_t s) {
  k_hub_prep<<<grid_for((uint64_t)h + 1), kTpb, 0, s>>>(mv, list, h, hsize, maxT);
}
void launch_hub_group(const MoveView& mv, const uint32_t* list, uint32_t i0, uint32_t ng, const uint64_t* hoff,
                      uint64_t base0, uint64_t span, uint64_t maxT, int refine, HubPool hub, int64_t* own,
                      uint32_t max_parts, int64_t* phi, uint64_t* plo, uint32_t* pid, int* pvalid, CandBuf cand,
                      MoveStats st, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  const bool dir = mv.directed != 0;
#define LDL_HUB(WT, D, R)                                                                                          \
  hub_group_dispatch<WT, D, R>(mv, list, i0, ng, hoff, base0, span, maxT, hub, own, max_parts, phi, plo, pid,      \
                               pvalid, cand, st, s, ev_a, ev_b)
  if (!mv.out.wide) {
    if (dir) { if (refine) LDL_HUB(uint32_t, true, true); else LDL_HUB(uint32_t, true, false); }
    else { if (refine) LDL_HUB(uint32_t, false, true); else LDL_HUB(uint32_t, false, false); }
  } else {
    if (dir) { if (refine) LDL_HUB(int64_t, true, true); else LDL_HUB(int64_t, true, false); }
    else { if (refine) LDL_HUB(int64_t, false, true); else LDL_HUB(int64_t, false, false); }
  }
#undef LDL_HUB
}
void launch_bin(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, uint32_t* const* bins,
                uint32_t* bin_counts, hipStream_t s) {
  if (count)
    k_bin<<<grid_for(count), kTpb, 0, s>>>(mv, list, count, refine, bins[0], bins[1], bins[2], bins[3], bins[4],
                                           bin_counts);
}

void launch_best(const MoveView& mv, int bin, const uint32_t* list, uint32_t count, int refine, CandBuf cand,
                 HubPool hub, MoveStats st, hipStream_t s) {
  if (!count) return;
  const bool dir = mv.directed != 0;
  if (!mv.out.wide) {
    if (dir) {
      if (refine) best_dispatch<uint32_t, true, true>(mv, bin, list, count, cand, hub, st, s);
      else best_dispatch<uint32_t, true, false>(mv, bin, list, count, cand, hub, st, s);
    } else {
      if (refine) best_dispatch<uint32_t, false, true>(mv, bin, list, count, cand, hub, st, s);
      else best_dispatch<uint32_t, false, false>(mv, bin, list, count, cand, hub, st, s);
    }
  } else {
    if (dir) {
      if (refine) best_dispatch<int64_t, true, true>(mv, bin, list, count, cand, hub, st, s);
      else best_dispatch<int64_t, true, false>(mv, bin, list, count, cand, hub, st, s);
    } else {
      if (refine) best_dispatch<int64_t, false, true>(mv, bin, list, count, cand, hub, st, s);
      else best_dispatch<int64_t, false, false>(mv, bin, list, count, cand, hub, st, s);
    }
  }
}

void launch_rank_from_order(const uint32_t* order, uint32_t k, uint32_t* rank, hipStream_t s) {
  if (k) k_rank_from_order<<<grid_for(k), kTpb, 0, s>>>(order, k, rank);
}
void launch_gather_u64(const uint64_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst, int invert,
                       hipStream_t s) {
  if (k) k_gather_u64<<<grid_for(k), kTpb, 0, s>>>(src, idx, k, dst, invert);
}
void launch_gather_u32_as_u64(const uint32_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst, hipStream_t s) {
  if (k) k_gather_u32_as_u64<<<grid_for(k), kTpb, 0, s>>>(src, idx, k, dst);
}
void launch_lf_reset(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, uint32_t* minE,
                     uint32_t* minA, hipStream_t s) {
  if (nl) k_lf_reset<<<grid_for(nl), kTpb, 0, s>>>(live, nl, a, b, minE, minA);
}
void launch_lf_min(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* rank,
                   uint32_t* minE, uint32_t* minA, hipStream_t s) {
  if (nl) k_lf_min<<<grid_for(nl), kTpb, 0, s>>>(live, nl, a, b, rank, minE, minA);
}
void launch_lf_accept(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* rank,
                      const uint32_t* minE, const uint32_t* minA, uint32_t* accE, uint32_t* accA, uint32_t ep,
                      uint8_t* flag, uint32_t* acc_list, uint32_t* acc_count, hipStream_t s) {
  if (nl)
    k_lf_accept<<<grid_for(nl), kTpb, 0, s>>>(live, nl, a, b, rank, minE, minA, accE, accA, ep, flag, acc_list,
                                              acc_count);
}
void launch_lf_reject(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* accE,
                      const uint32_t* accA, uint32_t ep, const uint8_t* flag, uint32_t* live2, uint32_t* live2_count,
                      hipStream_t s) {
  if (nl) k_lf_reject<<<grid_for(nl), kTpb, 0, s>>>(live, nl, a, b, accE, accA, ep, flag, live2, live2_count);
}
void launch_commit_mark(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* mov_stamp, uint32_t mov_ep,
                        uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin, SetRef touched, int64_t* tko,
                        int64_t* tki, hipStream_t s) {
  if (na)
    k_commit_mark<<<grid_for(na), kTpb, 0, s>>>(acc, na, cand, mov_stamp, mov_ep, oldlab, Kout, Kin, touched, tko,
                                                tki);
}
void launch_commit_apply(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* lab, const int64_t* kout,
                         const int64_t* kin, int64_t* Kout, int64_t* Kin_or_null, int forward, hipStream_t s) {
  if (na) k_commit_apply<<<grid_for(na), kTpb, 0, s>>>(acc, na, cand, lab, kout, kin, Kout, Kin_or_null, forward);
}
void launch_commit_dein(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                        const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep, const uint32_t* oldlab,
                        i64a* dein, hipStream_t s) {
  if (na)
    k_commit_dein<<<grid_waves(na), kTpb, 0, s>>>(acc, na, cand, out, in, directed, lab, mov_stamp, mov_ep, oldlab,
                                                  dein);
}
void launch_mark_acc_comms(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* stamp, uint32_t ep,
                           hipStream_t s) {
  if (na) k_mark_acc_comms<<<grid_for(na), kTpb, 0, s>>>(acc, na, cand, stamp, ep);
}
void launch_set_add_acc_v(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand, hipStream_t s) {
  if (na) k_set_add_acc_v<<<grid_for(na), kTpb, 0, s>>>(set, acc, na, cand);
}
void launch_neighbours_acc(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in,
                           int directed, hipStream_t s) {
  if (na) k_neighbours_acc<<<grid_waves(na), kTpb, 0, s>>>(set, acc, na, cand, out, in, directed);
}
void launch_ref_commit(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* par, const int64_t* kout,
                       const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s) {
  if (na) k_ref_commit<<<grid_for(na), kTpb, 0, s>>>(acc, na, cand, par, kout, kin, Krout, Krin_or_null, rsize);
}
void launch_spexpand(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                     const uint32_t* lab, const uint32_t* par, const uint32_t* rsize, SetRef rcur, SetRef rset,
                     uint32_t* oldpar, hipStream_t s) {
  if (na)
    k_spexpand<<<grid_waves(na), kTpb, 0, s>>>(acc, na, cand, out, in, directed, lab, par, rsize, rcur, rset,
                                               oldpar);
}

}  // namespace ldl
