// Local-move and refinement kernels (Algorithm 1; gain of Sec. III-D), the
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
#include <hip/hip_ext.h>

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
  return (int64_t)__builtin_nontemporal_load(&((const WT*)c.w)[i]);
}

// Entry j of vertex v's combined out/in list: (neighbour, weight).  The adjacency is read once per
// search, so it is loaded nontemporally: the caches are left to the label and total gathers.
template <typename WT, bool DIR>
__device__ __forceinline__ void entry_at(const MoveView& mv, uint64_t oo, uint32_t dout, uint64_t oi, uint32_t j,
                                         uint32_t& x, int64_t& w) {
  if (!DIR || j < dout) {
    x = __builtin_nontemporal_load(&mv.out.nbr[oo + j]);
    w = wload<WT>(mv.out, oo + j);
  } else {
    x = __builtin_nontemporal_load(&mv.in.nbr[oi + (j - dout)]);
    w = wload<WT>(mv.in, oi + (j - dout));
  }
}

// key of neighbour x for vertex v: its label (move) or its refined community when it shares
// v's label (refinement); kEmpty for entries that do not count
template <bool REF>
__device__ __forceinline__ uint32_t entry_key(const MoveView& mv, uint32_t v, uint32_t labv, uint32_t x) {
  if (x == v) return kEmpty;
  if (!REF) return mv.lab[x];
  const uint2 q = mv.lp[x];                        // label and parent in one gather
  return q.x == labv ? q.y : kEmpty;
}

struct VInfo {
  int64_t ko, ki, Koa, Kia;
  uint32_t lab;
};

// gain of moving to b given b's totals (Kob, Kib) and the weights towards b and the own community
template <bool DIR, bool REF>
__device__ __forceinline__ i128 gain_t(const MoveView& mv, const VInfo& vi, int64_t Kob, int64_t Kib, int64_t accb,
                                       int64_t acca) {
  if (!REF) {
    if (DIR)
      return (i128)mv.qm * (accb - acca) -
             (i128)mv.p * ((i128)vi.ko * (Kib - vi.Kia + vi.ki) + (i128)vi.ki * (Kob - vi.Koa + vi.ko));
    return (i128)mv.qm * (accb - acca) - (i128)mv.p * ((i128)vi.ko * (Kob - vi.Koa + vi.ko));
  } else {
    if (DIR) return (i128)mv.qm * accb - (i128)mv.p * ((i128)vi.ko * Kib + (i128)vi.ki * Kob);
    return (i128)mv.qm * accb - (i128)mv.p * ((i128)vi.ko * Kob);
  }
}
template <bool DIR, bool REF>
__device__ __forceinline__ i128 gain(const MoveView& mv, const VInfo& vi, uint32_t b, int64_t accb, int64_t acca) {
  const int64_t Kob = mv.Kout[b];
  const int64_t Kib = DIR ? mv.Kin[b] : 0;
  return gain_t<DIR, REF>(mv, vi, Kob, Kib, accb, acca);
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

// Variant (mv.empty_target, moves only): the empty community labelled v is one more target when v
// does not carry label v and that community's totals are zero; its gain is gain_t with no weight
// towards it and zero totals.  Every lane that calls this with the same arguments gets the same b.
template <bool DIR, bool REF>
__device__ __forceinline__ Best with_empty(const MoveView& mv, const VInfo& vi, uint32_t v, int64_t own, Best b) {
  if (REF || !mv.empty_target || vi.lab == v) return b;
  if (mv.Kout[v] != 0 || (DIR && mv.Kin[v] != 0)) return b;
  const Best e = make_best(gain_t<DIR, REF>(mv, vi, 0, 0, 0, own), v);
  return better(e, b) ? e : b;
}

// A target's entry in the reductions: its exact gain and id; with the randomised refinement
// (mv.rkey != 0) only strictly positive gains count, ranked by their draw priority.
template <bool REF>
__device__ __forceinline__ Best cand_best(const MoveView& mv, uint32_t v, i128 g, uint32_t id) {
  Best b = make_best(g, id);
  if (REF && mv.rkey) b.valid = g > 0 ? (int)draw_priority(mv.rkey, v, id) : 0;
  return b;
}

__device__ __forceinline__ void emit_cand_at(const CandBuf& cb, uint32_t at, uint32_t v, uint32_t a, const Best& b) {
  cb.v[at] = v;
  cb.a[at] = a;
  cb.b[at] = b.id;
  cb.glo[at] = b.lo;
  cb.ghi[at] = b.hi;
}

// ------------------------------------------------------------------ binning without atomics
__device__ __forceinline__ int bin_of(const MoveView& mv, uint32_t v, int refine) {
  if (refine && !(mv.par[v] == v && mv.rsize[v] == 1)) return -1;   // only singletons move
  const uint64_t T = (uint64_t)mv.out.deg[v] + (mv.directed ? (uint64_t)mv.in.deg[v] : 0ull);
  if (T == 0) return -1;
#pragma unroll
  for (int b = 0; b < kNumBins - 1; ++b)
    if (T <= mv.lim[b]) return b;
  return kNumBins - 1;
}

// block b owns list[b*chunk, (b+1)*chunk); hist[bin * gridDim + b] = its count per bin
__global__ void k_bin_count(MoveView mv, const uint32_t* list, const uint32_t* countp, int refine, uint32_t* hist,
                            uint32_t* zero_words, uint32_t nzero) {
  __shared__ uint32_t h[kNumBins];
  if (blockIdx.x == 0)
    for (uint32_t t = threadIdx.x; t < nzero; t += blockDim.x) zero_words[t] = 0;
  if (threadIdx.x < kNumBins) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t count = *countp;
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

// every block reduces the per-block histograms itself (kBinBlocks words per bin): its start in
// each bin is the sum of the earlier bins plus the earlier blocks' counts of that bin
__global__ __launch_bounds__(kTpb) void k_bin_fill(MoveView mv, const uint32_t* list, const uint32_t* countp,
                                                   int refine, const uint32_t* hist, uint32_t* out,
                                                   uint32_t* bin_start, uint32_t* bin_count) {
  __shared__ uint32_t red[2 * kNumBins][kTpb / kWave];
  __shared__ uint32_t pos[kNumBins];
  const unsigned nb = gridDim.x;   // == kBinBlocks <= kTpb
  const uint32_t count = *countp;
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int t = 0; t < kNumBins; ++t) {
    const uint32_t x = threadIdx.x < nb ? hist[t * nb + threadIdx.x] : 0u;
    const uint32_t all = (uint32_t)wave_sum_i64((int64_t)x);
    const uint32_t before = (uint32_t)wave_sum_i64(threadIdx.x < blockIdx.x ? (int64_t)x : 0);
    if (lane_id() == 0) {
      red[2 * t][w] = all;
      red[2 * t + 1][w] = before;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t base = 0;
    for (int t = 0; t < kNumBins; ++t) {
      uint32_t all = 0, before = 0;
      for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
        all += red[2 * t][q];
        before += red[2 * t + 1][q];
      }
      pos[t] = base + before;
      if (blockIdx.x == 0) {
        bin_start[t] = base;
        bin_count[t] = all;
      }
      base += all;
    }
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
__global__ void k_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, const uint32_t* nap,
                                      CandBuf cand, CsrRef out, CsrRef in, int directed) {
  const int lane = lane_id();
  const uint32_t na = *nap;
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

// Launch with the optional start / stop events attached to the kernel's own dispatch, so that
// their elapsed time is the kernel's execution time and not the gaps around it.
template <typename... KArgs, typename... Args>
inline void launch_timed(void (*kern)(KArgs...), unsigned grid, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b,
                         Args... args) {
  if (ev_a) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kTpb), 0, s, ev_a, ev_b, 0, args...);
  else hipLaunchKernelGGL(kern, dim3(grid), dim3(kTpb), 0, s, args...);
}

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
  unsigned long long maxhi = 0;   // gains of candidates are positive, so their high words are >= 0
};

__device__ __forceinline__ void note_cand(LocalStats& ls, const Best& b) {
  ls.cands += 1;
  if ((unsigned long long)b.hi > ls.maxhi) ls.maxhi = (unsigned long long)b.hi;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = (unsigned long long)__shfl_xor((long long)v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}

// every thread of the block calls this once, at exit; red holds 5 words per wavefront
__device__ __forceinline__ void stats_flush(LocalStats ls, const MoveStats& st, unsigned long long* red) {
  unsigned long long v[5] = {ls.entries, ls.distinct, ls.vertices, ls.cands, ls.maxhi};
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (unsigned long long)wave_sum_i64((int64_t)v[k]);
  v[4] = wave_max_u64(v[4]);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 5; ++k) red[5 * w + k] = v[k];
  __syncthreads();
  if (threadIdx.x < 5) {
    unsigned long long t = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
      const unsigned long long x = red[5 * i + threadIdx.x];
      if (threadIdx.x < 4) t += x;
      else t = x > t ? x : t;
    }
    if (threadIdx.x == 4) {
      if (t) atomicMax(st.maxhi, t);
    } else if (st.entries && t) {
      u64a* dst = threadIdx.x == 0 ? st.entries : threadIdx.x == 1 ? st.distinct : threadIdx.x == 2 ? st.vertices
                                                                                                   : st.cands;
      atomicAdd(dst, t);
    }
  }
}

// ------------------------------------------------------------------ small degrees: lane groups
// G lanes per vertex, one entry per lane; every lane group works on U vertices at once and
// issues each phase's loads for all of them before using any (the kernel is bound by the
// latency of its dependent gathers: vertex -> row -> neighbour -> label -> community totals).
template <typename WT, int G, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_best_group(MoveView mv, BinRef br, CandBuf cand, MoveStats st) {
  constexpr int VPB = kTpb / G;            // vertices per block and set
  constexpr int U = 2;                     // vertex sets per block iteration
  static_assert(U * VPB <= 256, "stage capacity");
  __shared__ Stage<256> stage;
  __shared__ unsigned long long red[5 * (kTpb / kWave)];
  if (threadIdx.x == 0) stage.n = 0;
  __syncthreads();
  const uint32_t count = *br.count;
  const uint32_t* list = br.base + *br.start;
  LocalStats ls;
  const int li = threadIdx.x & (G - 1);
  for (uint64_t base = (uint64_t)blockIdx.x * VPB * U; base < count; base += (uint64_t)gridDim.x * VPB * U) {
    bool act[U];
    uint32_t v[U], T[U], dout[U];
    uint64_t oo[U], oi[U];
    VInfo vi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t gid = base + (uint64_t)u * VPB + threadIdx.x / G;
      act[u] = gid < count;                  // every lane stays for the shuffles
      v[u] = act[u] ? list[gid] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      dout[u] = 0; T[u] = 0; oo[u] = 0; oi[u] = 0;
      vi[u] = VInfo{};
      if (act[u]) {
        dout[u] = mv.out.deg[v[u]];
        T[u] = dout[u] + (DIR ? mv.in.deg[v[u]] : 0);
        oo[u] = mv.out.off[v[u]];
        if (DIR) oi[u] = mv.in.off[v[u]];
        vi[u].lab = mv.lab[v[u]];
        vi[u].ko = mv.kout[v[u]];
        vi[u].ki = DIR ? mv.kin[v[u]] : 0;
      }
    }
    uint32_t x[U];
    int64_t w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!DIR) vi[u].ki = vi[u].ko;
      if (!REF && act[u]) {
        vi[u].Koa = mv.Kout[vi[u].lab];
        vi[u].Kia = DIR ? mv.Kin[vi[u].lab] : vi[u].Koa;
      }
      x[u] = v[u];                           // the vertex itself does not count
      w[u] = 0;
      if (act[u] && (uint32_t)li < T[u]) entry_at<WT, DIR>(mv, oo[u], dout[u], oi[u], (uint32_t)li, x[u], w[u]);
    }
    uint32_t key[U];
#pragma unroll
    for (int u = 0; u < U; ++u) key[u] = act[u] ? entry_key<REF>(mv, v[u], vi[u].lab, x[u]) : kEmpty;
    // sum equal keys across the group; the lowest lane of each key represents it
    int64_t acc[U], own[U];
    bool rep[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      own[u] = (!REF && key[u] != kEmpty && key[u] == vi[u].lab) ? w[u] : 0;
#pragma unroll
      for (int o = G >> 1; o > 0; o >>= 1) own[u] += __shfl_xor(own[u], o, G);
      acc[u] = 0;
      rep[u] = key[u] != kEmpty && (REF || key[u] != vi[u].lab);
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint32_t kj = (uint32_t)__shfl((int)key[u], j, G);
        const int64_t wj = __shfl(w[u], j, G);
        if (kj == key[u]) {
          acc[u] += wj;
          if (j < li) rep[u] = false;
        }
      }
    }
    int64_t Kob[U], Kib[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      Kob[u] = 0; Kib[u] = 0;
      if (act[u] && rep[u]) {
        Kob[u] = mv.Kout[key[u]];
        if (DIR) Kib[u] = mv.Kin[key[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      Best b;
      b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
      if (act[u] && rep[u]) b = cand_best<REF>(mv, v[u], gain_t<DIR, REF>(mv, vi[u], Kob[u], Kib[u], acc[u], own[u]), key[u]);
      ls.distinct += (act[u] && rep[u]) ? 1 : 0;
      b = group_best(b, G);
      if (act[u] && li == 0) {
        ls.entries += T[u];
        ls.vertices += 1;
        b = with_empty<DIR, REF>(mv, vi[u], v[u], own[u], b);
        if (b.valid && best_gain(b) > 0) {
          stage_push(stage, v[u], REF ? v[u] : vi[u].lab, b);
          note_cand(ls, b);
        }
      }
    }
    __syncthreads();
    if (stage.n + U * VPB > 256) stage_flush(stage, cand);
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

// ------------------------------------------------------------------ wavefront teams

// Insert (key, w) into an LDS table that is empty between vertices.  Returns the slot when
// this call created the key's entry (the calling lane then owns it), else kNoSlot.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t table_insert_own(uint32_t* keys, u64a* vals, uint32_t mask, uint32_t key,
                                                     int64_t w) {
  uint32_t h = hash32(key) & mask;
  for (;;) {
    const uint32_t prev = atomicCAS(&keys[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&vals[h], (u64a)w);
      return prev == kEmpty ? h : kNoSlot;
    }
    h = (h + 1) & mask;
  }
}

// Row of one vertex for the LDS-table kernels: degrees, row offsets and the vertex's own label,
// degrees and (move) community totals.
struct HashRow {
  uint32_t v, dout, din;
  uint64_t oo, oi;
  VInfo vi;
  bool active;
};

// first dependent level: everything read at the vertex's own index
template <bool DIR>
__device__ __forceinline__ HashRow hash_row_head(const MoveView& mv, bool active, uint32_t v) {
  HashRow r;
  r.active = active;
  r.v = v;
  r.dout = r.din = 0;
  r.oo = r.oi = 0;
  r.vi.lab = 0;
  r.vi.ko = r.vi.ki = r.vi.Koa = r.vi.Kia = 0;
  if (active) {
    r.dout = mv.out.deg[v];
    r.oo = mv.out.off[v];
    if (DIR) {
      r.din = mv.in.deg[v];
      r.oi = mv.in.off[v];
    }
    r.vi.lab = mv.lab[v];
    r.vi.ko = mv.kout[v];
    r.vi.ki = DIR ? mv.kin[v] : r.vi.ko;
  }
  return r;
}

// second dependent level: the entries of lane li (j = li + q TEAM) and the own community's totals
template <typename WT, int TEAM, int EPL, bool DIR, bool REF>
__device__ __forceinline__ void hash_row_entries(const MoveView& mv, HashRow& r, int li, uint32_t* xs, int64_t* ws) {
  const uint32_t T = r.dout + r.din;
#pragma unroll
  for (int q = 0; q < EPL; ++q) {
    const uint32_t j = (uint32_t)li + (uint32_t)q * TEAM;
    xs[q] = r.v;                              // the vertex itself does not count
    ws[q] = 0;
    if (r.active && j < T) entry_at<WT, DIR>(mv, r.oo, r.dout, r.oi, j, xs[q], ws[q]);
  }
  if (!REF && r.active) {
    r.vi.Koa = mv.Kout[r.vi.lab];
    r.vi.Kia = DIR ? mv.Kin[r.vi.lab] : r.vi.Koa;
  }
}

// One wavefront per vertex with a private LDS table of SLOTS slots (load factor <= 1/2), kept
// empty between vertices: the lane that creates a key's slot owns it, evaluates that
// community after the wavefront has inserted everything and empties the slot afterwards, so
// no cycle is spent on empty slots.  A lane loads all of its entries (at most SLOTS / 128),
// then all their keys, then inserts; the totals of all its owned communities are gathered
// together.  The wavefronts of a workgroup run independently (no workgroup barrier inside the
// loop); candidates are staged per wavefront.  The loop over the wavefront's vertices is
// software-pipelined as in k_best_hash below.
template <typename WT, int SLOTS, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_best_wave(MoveView mv, BinRef br, CandBuf cand, MoveStats st) {
  constexpr int W = kTpb / kWave;
  constexpr int EPL = SLOTS / 2 / kWave;   // entries per lane, T <= SLOTS / 2
  constexpr uint32_t SCAP = 32;            // staged candidates per wavefront
  __shared__ uint32_t skey[W][SLOTS];
  __shared__ u64a sval[W][SLOTS];
  __shared__ uint32_t cv[W][SCAP], ca[W][SCAP], cb[W][SCAP];
  __shared__ uint64_t clo[W][SCAP];
  __shared__ int64_t chi[W][SCAP];
  __shared__ unsigned long long red_s[5 * W];
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  const uint32_t count = *br.count;
  const uint32_t* list = br.base + *br.start;
  uint32_t* keys = skey[wv];
  u64a* vals = sval[wv];
  LocalStats ls;
  uint32_t ns = 0;   // staged candidates of this wavefront (same in every lane)
  auto flush = [&]() {
    wave_sync();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(cand.count, ns);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    if ((uint32_t)lane < ns) {
      cand.v[base + lane] = cv[wv][lane];
      cand.a[base + lane] = ca[wv][lane];
      cand.b[base + lane] = cb[wv][lane];
      cand.glo[base + lane] = clo[wv][lane];
      cand.ghi[base + lane] = chi[wv][lane];
    }
    wave_sync();
    ns = 0;
  };
  uint64_t i = (uint64_t)blockIdx.x * W + wv;
  const uint64_t step = (uint64_t)gridDim.x * W;
  if (i < count) {
    for (uint32_t s = lane; s < (uint32_t)SLOTS; s += kWave) {
      keys[s] = kEmpty;
      vals[s] = 0;
    }
  }
  // pipeline state: the current vertex's row and entries, the next vertex's id
  HashRow cur = hash_row_head<DIR>(mv, i < count, i < count ? list[i] : 0);
  uint32_t xs[EPL];
  int64_t ws[EPL];
  hash_row_entries<WT, kWave, EPL, DIR, REF>(mv, cur, lane, xs, ws);
  uint32_t vnext = i + step < count ? list[i + step] : 0;
  for (; i < count; i += step) {
    const uint32_t v = cur.v;
    uint32_t ks[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) ks[q] = entry_key<REF>(mv, v, cur.vi.lab, xs[q]);
    HashRow nxt = hash_row_head<DIR>(mv, i + step < count, vnext);
    const uint32_t vnext2 = i + 2 * step < count ? list[i + 2 * step] : 0;
    wave_sync();                              // the previous vertex's slots are empty
    int64_t own = 0;
    uint32_t mine[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const uint32_t key = ks[q];
      mine[q] = kNoSlot;
      if (key == kEmpty) continue;
      if (!REF && key == cur.vi.lab) {
        own += ws[q];
        continue;
      }
      mine[q] = table_insert_own(keys, vals, (uint32_t)SLOTS - 1, key, ws[q]);
    }
    wave_sync();                              // every insert done
    own = wave_sum_i64(own);
    int64_t Kb[EPL], Kib[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      Kb[q] = 0; Kib[q] = 0;
      if (mine[q] != kNoSlot) {
        Kb[q] = mv.Kout[ks[q]];
        if (DIR) Kib[q] = mv.Kin[ks[q]];
      }
    }
    uint32_t xn[EPL];
    int64_t wn[EPL];
    hash_row_entries<WT, kWave, EPL, DIR, REF>(mv, nxt, lane, xn, wn);
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      if (mine[q] == kNoSlot) continue;
      ls.distinct += 1;
      const int64_t av = (int64_t)vals[mine[q]];
      const Best c = cand_best<REF>(mv, v, gain_t<DIR, REF>(mv, cur.vi, Kb[q], Kib[q], av, own), ks[q]);
      if (better(c, b)) b = c;
    }
    // each slot is read and emptied by its owner only; the barrier at the top of the next
    // vertex orders the resets before any insert
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      if (mine[q] != kNoSlot) {
        keys[mine[q]] = kEmpty;
        vals[mine[q]] = 0;
      }
    }
    b = group_best(b, kWave);                 // every lane holds the wavefront's best
    b = with_empty<DIR, REF>(mv, cur.vi, v, own, b);
    if (lane == 0) {
      ls.entries += cur.dout + cur.din;
      ls.vertices += 1;
    }
    if (b.valid && best_gain(b) > 0) {
      if (lane == 0) {
        cv[wv][ns] = v;
        ca[wv][ns] = REF ? v : cur.vi.lab;
        cb[wv][ns] = b.id;
        clo[wv][ns] = b.lo;
        chi[wv][ns] = b.hi;
        note_cand(ls, b);
      }
      if (++ns == SCAP) flush();
    }
    cur = nxt;
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      xs[q] = xn[q];
      ws[q] = wn[q];
    }
    vnext = vnext2;
  }
  if (ns) flush();
  stats_flush(ls, st, red_s);
}

// TEAM lanes per vertex with a private LDS table of SLOTS slots (load factor <= 1/2), empty
// between vertices: as in k_best_wave, the lane that creates a key's slot evaluates that
// community and empties the slot.  A lane loads all of its entries (at most SLOTS / (2 TEAM)),
// then all their keys, then inserts; the totals of its owned communities are gathered together.
// The loop is software-pipelined over the team's vertices: the next vertex's header is read
// while the current one's keys are, and its entries while the current one's community totals
// are, so each vertex waits on two dependent gathers instead of five (list, header, entries,
// keys, totals).
template <typename WT, int TEAM, int SLOTS, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) __attribute__((amdgpu_waves_per_eu(3)))   // LDS holds 3 workgroups per CU
void k_best_hash(MoveView mv, BinRef br, CandBuf cand, MoveStats st) {
  constexpr int TEAMS = kTpb / TEAM;
  constexpr int EPL = SLOTS / 2 / TEAM;    // entries per lane, T <= SLOTS / 2
  __shared__ uint32_t skey[TEAMS][SLOTS];
  __shared__ u64a sval[TEAMS][SLOTS];
  __shared__ int64_t red_i[kTpb / kWave];
  __shared__ Best red_b[kTpb / kWave];
  __shared__ Stage<64> stage;
  __shared__ unsigned long long red_s[5 * (kTpb / kWave)];
  if (threadIdx.x == 0) stage.n = 0;
  const uint32_t count = *br.count;
  const uint32_t* list = br.base + *br.start;
  const int t = threadIdx.x / TEAM;
  const int li = threadIdx.x % TEAM;
  const uint64_t step = (uint64_t)gridDim.x * TEAMS;
  LocalStats ls;
  uint64_t base = (uint64_t)blockIdx.x * TEAMS;
  if (base < count) {
    for (uint32_t s = li; s < (uint32_t)SLOTS; s += TEAM) {
      skey[t][s] = kEmpty;
      sval[t][s] = 0;
    }
  }
  // pipeline state: the current vertex's row and entries, the next vertex's id
  HashRow cur;
  uint32_t xs[EPL];
  int64_t ws[EPL];
  uint32_t vnext = 0;
  {
    const uint64_t s0 = base + t, s1 = base + step + t;
    cur = hash_row_head<DIR>(mv, s0 < count, s0 < count ? list[s0] : 0);
    hash_row_entries<WT, TEAM, EPL, DIR, REF>(mv, cur, li, xs, ws);
    if (s1 < count) vnext = list[s1];
  }
  for (; base < count; base += step) {
    const uint64_t s1 = base + step + t, s2 = base + 2 * step + t;
    uint32_t ks[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) ks[q] = cur.active ? entry_key<REF>(mv, cur.v, cur.vi.lab, xs[q]) : kEmpty;
    HashRow nxt = hash_row_head<DIR>(mv, s1 < count, vnext);
    const uint32_t vnext2 = s2 < count ? list[s2] : 0;
    __syncthreads();                          // the previous vertex's slots are empty
    int64_t own = 0;
    uint32_t mine[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const uint32_t key = ks[q];
      mine[q] = kNoSlot;
      if (key == kEmpty) continue;
      if (!REF && key == cur.vi.lab) {
        own += ws[q];
        continue;
      }
      mine[q] = table_insert_own(skey[t], sval[t], (uint32_t)SLOTS - 1, key, ws[q]);
    }
    __syncthreads();                          // every insert done
    own = team_sum<TEAM>(own, red_i);
    int64_t Kb[EPL], Kib[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      Kb[q] = 0; Kib[q] = 0;
      if (mine[q] != kNoSlot) {
        Kb[q] = mv.Kout[ks[q]];
        if (DIR) Kib[q] = mv.Kin[ks[q]];
      }
    }
    uint32_t xn[EPL];
    int64_t wn[EPL];
    hash_row_entries<WT, TEAM, EPL, DIR, REF>(mv, nxt, li, xn, wn);
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      if (mine[q] == kNoSlot) continue;
      ls.distinct += 1;
      const int64_t av = (int64_t)sval[t][mine[q]];
      const Best c = cand_best<REF>(mv, cur.v, gain_t<DIR, REF>(mv, cur.vi, Kb[q], Kib[q], av, own), ks[q]);
      if (better(c, b)) b = c;
    }
    b = team_best<TEAM>(b, red_b);
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      if (mine[q] != kNoSlot) {
        skey[t][mine[q]] = kEmpty;
        sval[t][mine[q]] = 0;
      }
    }
    if (cur.active && li == 0) {
      ls.entries += cur.dout + cur.din;
      ls.vertices += 1;
      b = with_empty<DIR, REF>(mv, cur.vi, cur.v, own, b);
      if (b.valid && best_gain(b) > 0) {
        stage_push(stage, cur.v, REF ? cur.v : cur.vi.lab, b);
        note_cand(ls, b);
      }
    }
    __syncthreads();
    if (stage.n + TEAMS > 64) stage_flush(stage, cand);
    cur = nxt;
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      xs[q] = xn[q];
      ws[q] = wn[q];
    }
    vnext = vnext2;
  }
  stage_flush(stage, cand);
  stats_flush(ls, st, red_s);
}

// ---- hubs split over many workgroups, driven from device counts.  Hub i (of the bin's h
// vertices, T_i entries) has ceil(T_i / kHubChunk) chunk items and P_i hash partitions of its
// neighbour communities (P_i = ceil(T_i 2^pshift / kPartEntries), at most ceil(T_i / 16)); one
// exclusive scan of (entries, chunks, partitions) places the hub's slice of the bucket pool, its
// items and its partitions.  The keys pass computes every entry's community key (the own
// community's weight is summed apart) and counts the entries per partition; a per-hub scan turns
// the counts into bucket offsets; the scatter pass writes (key, weight) into the buckets; one
// workgroup per partition then sums its bucket by key in an LDS table and evaluates the gains
// into a partial best; one wavefront per hub reduces its partials.  Every key of a hub lands in
// exactly one partition, so the sums are complete without global atomics on them.  Hubs whose
// entries end beyond the pool are skipped and reported (bit 0 of *over, with the entries needed
// in *need); more than `bound` hubs is bit 1; a partition with more distinct keys than its LDS
// table is bit 2 (the host then redoes the pass with more partitions).
constexpr uint32_t kHubChunk = 2048;
constexpr uint32_t kPartHist = 4096;   // partitions counted in LDS per chunk (more: global atomics)

__device__ __forceinline__ uint32_t hub_count(const BinRef& br, uint32_t bound) {
  const uint32_t c = *br.count;
  return c < bound ? c : bound;
}

__device__ __forceinline__ uint64_t entries_of(const MoveView& mv, uint32_t v) {
  return (uint64_t)mv.out.deg[v] + (mv.directed ? (uint64_t)mv.in.deg[v] : 0ull);
}

// partition of a key among P: the high bits of a second hash (the LDS tables use the low bits
// of hash32, so keys of one partition do not crowd one end of its table)
__device__ __forceinline__ uint32_t part_of(uint32_t key, uint32_t P) {
  return (uint32_t)(((uint64_t)hash32(key * 0x9E3779B1u + 0x7F4A7C15u) * P) >> 32);
}

// largest i in [0, h) with off[i].F <= it, for off non-decreasing in F with off[h].F > it
template <int F>
__device__ __forceinline__ uint32_t item_owner(const U64x3* off, uint32_t h, uint64_t it) {
  uint32_t lo = 0, hi = h;   // off[lo] <= it < off[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    const uint64_t x = F == 1 ? off[mid].y : off[mid].z;
    if (x <= it) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_hub_size(MoveView mv, BinRef br, uint32_t bound, int pshift, U64x3* cnt, int64_t* own,
                           uint32_t* over) {
  const uint32_t c = *br.count;
  const uint32_t h = c < bound ? c : bound;
  const uint32_t* list = br.base + *br.start;
  if (gtid() == 0 && c > bound) atomicOr(over, 2u);
  for (uint64_t i = gtid(); i <= bound; i += gstride()) {
    U64x3 x{0, 0, 0};
    if (i < h) {
      const uint64_t T = entries_of(mv, list[i]);
      uint64_t P = ((T << pshift) + kPartEntries - 1) / kPartEntries;
      const uint64_t Pmax = (T + 15) / 16;
      if (P > Pmax) P = Pmax;
      if (P < 1) P = 1;
      x.x = T;
      x.y = (T + kHubChunk - 1) / kHubChunk;
      x.z = P;
      own[i] = 0;
    }
    cnt[i] = x;
  }
}

// chunk items: the chunk's entries summed by key in LDS (each chunk of kHubChunk entries leaves
// its distinct (key, weight) pairs at the start of its own stretch of the pool), the weight
// towards the own community, and the pairs per partition.  The scatter and partition passes then
// handle distinct pairs only: a hub's neighbours crowd into few communities.
constexpr uint32_t kChunkSlots = 2 * kHubChunk;   // load factor <= 1/2
constexpr uint32_t kKeysHist = 1024;              // partitions counted in LDS (more: global atomics)
template <typename WT, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_hub_keys(MoveView mv, BinRef br, uint32_t bound, const U64x3* off,
                                                   HubPool hub, HubWork hw, MoveStats st) {
  __shared__ int64_t red[kTpb / kWave];
  __shared__ uint32_t lh[kKeysHist];
  __shared__ uint32_t tk[kChunkSlots];
  __shared__ u64a tv[kChunkSlots];
  __shared__ uint32_t s_nd;
  const uint32_t h = hub_count(br, bound);
  const uint32_t* list = br.base + *br.start;
  const uint64_t total = off[h].y;
  // the table starts empty and every chunk leaves it empty (each slot is reset by its reader)
  for (uint32_t t = threadIdx.x; t < kChunkSlots; t += blockDim.x) {
    tk[t] = kEmpty;
    tv[t] = 0;
  }
  if (threadIdx.x == 0) s_nd = 0;
  __syncthreads();
  uint64_t nent = 0;
  for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const uint32_t i = item_owner<1>(off, h, it);
    const uint64_t base = off[i].x;
    if (off[i + 1].x > hub.cap) continue;      // beyond the pool: reported by k_hub_final
    const uint32_t v = list[i];
    const uint32_t dout = mv.out.deg[v];
    const uint32_t T = dout + (DIR ? mv.in.deg[v] : 0);
    const uint32_t P = (uint32_t)(off[i + 1].z - off[i].z);
    const uint64_t pbase = off[i].z;
    const uint64_t e0 = (it - off[i].y) * kHubChunk;
    const uint64_t e1 = e0 + kHubChunk < T ? e0 + kHubChunk : T;
    const uint32_t labv = mv.lab[v];
    const uint64_t oo = mv.out.off[v], oi = DIR ? mv.in.off[v] : 0;
    const bool local = P <= kKeysHist;
    if (local)
      for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) lh[t] = 0;
    int64_t ow = 0;
    // four entries per thread at a time: their loads, then their key gathers, then the inserts,
    // so four gathers are in flight before any is used
    for (uint64_t jb = e0 + threadIdx.x; jb < e1; jb += 4 * (uint64_t)blockDim.x) {
      uint32_t xs[4], ks[4];
      int64_t wv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = jb + (uint64_t)k * blockDim.x;
        xs[k] = v;   // a key of kEmpty for slots past the chunk
        wv[k] = 0;
        if (j < e1) entry_at<WT, DIR>(mv, oo, dout, oi, (uint32_t)j, xs[k], wv[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) ks[k] = entry_key<REF>(mv, v, labv, xs[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t key = ks[k];
        if (key == kEmpty) continue;
        if (!REF && key == labv) {
          ow += wv[k];
          continue;
        }
        table_insert(tk, tv, kChunkSlots - 1, key, wv[k]);
      }
    }
    __syncthreads();   // every insert done (and lh cleared)
    // the chunk's distinct pairs to the start of its stretch of the pool, counted per partition
    for (uint32_t t = threadIdx.x; t < kChunkSlots; t += blockDim.x) {
      const uint32_t key = tk[t];
      if (key == kEmpty) continue;
      const uint32_t at = atomicAdd(&s_nd, 1u);
      hub.ekey[base + e0 + at] = key;
      hub.ew[base + e0 + at] = (int64_t)tv[t];
      tk[t] = kEmpty;
      tv[t] = 0;
      const uint32_t p = part_of(key, P);
      if (local) atomicAdd(&lh[p], 1u);
      else atomicAdd(&hw.pcount[pbase + p], 1u);
    }
    __syncthreads();
    if (local)
      for (uint32_t t = threadIdx.x; t < P; t += blockDim.x)
        if (lh[t]) atomicAdd(&hw.pcount[pbase + t], lh[t]);
    if (threadIdx.x == 0) {
      hw.icnt[it] = s_nd;
      s_nd = 0;
    }
    ow = team_sum<kTpb>(ow, red);   // its barriers also order the lh reads and s_nd before reuse
    if (threadIdx.x == 0 && ow) atomic_add_i64(&hw.own[i], ow);
    nent += e1 - e0;
    __syncthreads();
  }
  if (threadIdx.x == 0 && st.entries && nent) atomicAdd(st.entries, (u64a)nent);
}

// per hub: bucket offsets of its partitions (exclusive scan of the counts); counts return to 0
__global__ __launch_bounds__(kTpb) void k_hub_poff(BinRef br, uint32_t bound, const U64x3* off, HubPool hub,
                                                   HubWork hw) {
  __shared__ uint64_t wsum[kTpb / kWave];
  const uint32_t h = hub_count(br, bound);
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (uint32_t i = blockIdx.x; i < h; i += gridDim.x) {
    if (off[i + 1].x > hub.cap) continue;
    const uint64_t p0 = off[i].z, p1 = off[i + 1].z;
    uint64_t carry = off[i].x;
    for (uint64_t b = p0; b < p1; b += blockDim.x) {
      const uint64_t q = b + threadIdx.x;
      const uint64_t c = q < p1 ? hw.pcount[q] : 0;
      uint64_t incl = c;   // inclusive scan within the wavefront
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t t = (uint64_t)__shfl_up((long long)incl, o, kWave);
        if (lane >= o) incl += t;
      }
      if (lane == kWave - 1) wsum[w] = incl;
      __syncthreads();
      uint64_t before = 0, all = 0;
      for (int k = 0; k < kTpb / kWave; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
      }
      if (q < p1) {
        hw.poff[q] = carry + before + incl - c;
        hw.pcnt[q] = (uint32_t)c;
        hw.pcount[q] = 0;
      }
      carry += all;
      __syncthreads();
    }
  }
}

// chunk items: each distinct (key, weight) pair the keys pass left into its partition's bucket
template <typename WT, bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_hub_scatter(MoveView mv, BinRef br, uint32_t bound, const U64x3* off,
                                                      HubPool hub, HubWork hw) {
  __shared__ uint32_t lh[kPartHist];
  __shared__ uint32_t lb[kPartHist];
  const uint32_t h = hub_count(br, bound);
  const uint64_t total = off[h].y;
  for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const uint32_t i = item_owner<1>(off, h, it);
    if (off[i + 1].x > hub.cap) continue;
    const uint32_t P = (uint32_t)(off[i + 1].z - off[i].z);
    const uint64_t pbase = off[i].z;
    const uint64_t p0 = off[i].x + (it - off[i].y) * kHubChunk;   // the chunk's pairs
    const uint32_t nd = hw.icnt[it];
    const bool local = P <= kPartHist;
    if (local) {
      for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) lh[t] = 0;
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < nd; j += blockDim.x) atomicAdd(&lh[part_of(hub.ekey[p0 + j], P)], 1u);
      __syncthreads();
      // one global reservation per partition of the chunk; lh becomes the chunk's local cursor
      for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) {
        if (lh[t]) lb[t] = atomicAdd(&hw.pcur[pbase + t], lh[t]);
        lh[t] = 0;
      }
      __syncthreads();
    }
    for (uint32_t j = threadIdx.x; j < nd; j += blockDim.x) {
      const uint32_t key = hub.ekey[p0 + j];
      const int64_t w = hub.ew[p0 + j];
      const uint32_t p = part_of(key, P);
      const uint32_t at = local ? lb[p] + atomicAdd(&lh[p], 1u) : atomicAdd(&hw.pcur[pbase + p], 1u);
      const uint64_t pos = hw.poff[pbase + p] + at;
      hub.bkey[pos] = key;
      hub.bw[pos] = w;
    }
    __syncthreads();
  }
}

// workgroup per partition: sum its bucket by key in LDS, evaluate every key's gain, keep the
// partition's best; the scatter cursor returns to 0
template <bool DIR, bool REF>
__global__ __launch_bounds__(kTpb) void k_hub_part(MoveView mv, BinRef br, uint32_t bound, const U64x3* off,
                                                   HubPool hub, HubWork hw, MoveStats st) {
  __shared__ uint32_t tk[kPartSlots];
  __shared__ u64a tv[kPartSlots];
  __shared__ Best red_b[kTpb / kWave];
  __shared__ int64_t red_i[kTpb / kWave];
  __shared__ int s_over;
  const uint32_t h = hub_count(br, bound);
  const uint32_t* list = br.base + *br.start;
  const uint64_t total = off[h].z;
  uint64_t ndist = 0;
  for (uint64_t q = blockIdx.x; q < total; q += gridDim.x) {
    const uint32_t i = item_owner<2>(off, h, q);
    if (off[i + 1].x > hub.cap) continue;
    const uint64_t b0 = hw.poff[q], nb = hw.pcnt[q];
    uint32_t size = 64;   // pow2 >= 2 nb slots (at most the table), cleared and scanned
    while (size < 2 * nb && size < hw.tslots) size <<= 1;
    if (size > hw.tslots) size = hw.tslots;
    const uint32_t mask = size - 1;
    for (uint32_t t = threadIdx.x; t < size; t += blockDim.x) {
      tk[t] = kEmpty;
      tv[t] = 0;
    }
    if (threadIdx.x == 0) s_over = 0;
    __syncthreads();
    // four bucket entries per thread at a time: keys and weights loaded together, then inserted
    for (uint64_t jb = threadIdx.x; jb < nb; jb += 4 * (uint64_t)blockDim.x) {
      uint32_t ks[4];
      int64_t wv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = jb + (uint64_t)k * blockDim.x;
        ks[k] = kEmpty;
        wv[k] = 0;
        if (j < nb) {
          ks[k] = hub.bkey[b0 + j];
          wv[k] = hub.bw[b0 + j];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t key = ks[k];
        if (key == kEmpty) continue;
        uint32_t slot = hash32(key) & mask;
        uint32_t probes = 0;
        for (;;) {
          const uint32_t prev = atomicCAS(&tk[slot], kEmpty, key);
          if (prev == kEmpty || prev == key) {
            atomicAdd(&tv[slot], (u64a)wv[k]);
            break;
          }
          slot = (slot + 1) & mask;
          if (++probes == size) {   // table full: more distinct keys than slots
            s_over = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    const uint32_t v = list[i];
    const VInfo vi = vinfo<DIR, REF>(mv, v);
    const int64_t ow = hw.own[i];
    Best b;
    b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
    int64_t nd = 0;
    for (uint32_t t = threadIdx.x; t < size; t += blockDim.x) {
      const uint32_t key = tk[t];
      if (key == kEmpty) continue;
      ++nd;
      const Best c = cand_best<REF>(mv, v, gain<DIR, REF>(mv, vi, key, (int64_t)tv[t], ow), key);
      if (better(c, b)) b = c;
    }
    nd = team_sum<kTpb>(nd, red_i);
    b = team_best<kTpb>(b, red_b);
    if (threadIdx.x == 0) {
      if (q == off[i].z) b = with_empty<DIR, REF>(mv, vi, v, ow, b);   // once per hub
      if (s_over) {
        atomicOr(hub.over_count, 4u);
        b.valid = 0;
      }
      hw.phi[q] = b.hi;
      hw.plo[q] = b.lo;
      hw.pid[q] = b.id;
      hw.pvalid[q] = b.valid;
      hw.pcur[q] = 0;
      ndist += (uint64_t)nd;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && st.entries && ndist) atomicAdd(st.distinct, (u64a)ndist);
}

// wavefront per hub: the best of its partitions' bests is its candidate.  Candidates and counts
// are gathered per workgroup (one global atomic per 64 candidates): the hubs of a full-frontier
// scan number in the millions.
template <bool REF>
__global__ __launch_bounds__(kTpb) void k_hub_final(BinRef br, uint32_t bound, const U64x3* off, uint64_t cap,
                                                    const uint32_t* lab, const int64_t* phi, const uint64_t* plo,
                                                    const uint32_t* pid, const int* pvalid, CandBuf cand, MoveStats st,
                                                    u64a* need, uint32_t* over) {
  constexpr int W = kTpb / kWave;
  __shared__ Stage<64> stage;
  __shared__ unsigned long long red_s[5 * W];
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const uint32_t h = hub_count(br, bound);
  const uint32_t* list = br.base + *br.start;
  if (gtid() == 0) {
    const uint64_t total = off[h].x;
    *need = total;
    if (total > cap) atomicOr(over, 1u);
  }
  if (threadIdx.x == 0) stage.n = 0;
  __syncthreads();
  LocalStats ls;
  // every wavefront of a workgroup takes one hub per round, so all of them reach its barriers
  for (uint64_t base = (uint64_t)blockIdx.x * W; base < h; base += (uint64_t)gridDim.x * W) {
    const uint64_t i = base + wv;
    if (i < h && off[i + 1].x <= cap) {       // else skipped: entries beyond the pool
      const uint64_t p0 = off[i].z, p1 = off[i + 1].z;
      Best b;
      b.valid = 0; b.hi = 0; b.lo = 0; b.id = 0;
      for (uint64_t p = p0 + lane; p < p1; p += kWave) {
        Best c;
        c.hi = phi[p]; c.lo = plo[p]; c.id = pid[p]; c.valid = pvalid[p];
        if (better(c, b)) b = c;
      }
      b = group_best(b, kWave);
      if (lane == 0) {
        const uint32_t v = list[i];
        ls.vertices += 1;
        if (b.valid && best_gain(b) > 0) {
          stage_push(stage, v, REF ? v : lab[v], b);
          note_cand(ls, b);
        }
      }
    }
    __syncthreads();
    if (stage.n + W > 64) stage_flush(stage, cand);
  }
  stage_flush(stage, cand);
  stats_flush(ls, st, red_s);
}

template <typename WT, bool DIR, bool REF>
int hub_dispatch(const MoveView& mv, BinRef br, uint32_t bound, HubPool hub, HubWork hw, CandBuf cand, MoveStats st,
                 void** tmp, size_t* tmp_bytes, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  k_hub_size<<<cap_blocks(grid_for((uint64_t)bound + 1), LDL_RESIDENT(k_hub_size, kTpb)), kTpb, 0, s>>>(
      mv, br, bound, hw.pshift, hw.cnt, hw.own, hub.over_count);
  const int rc = prim_exclusive_sum_u64x3(tmp, tmp_bytes, hw.cnt, hw.off, (uint64_t)bound + 1, s);
  if (rc) return rc;
  launch_timed(k_hub_keys<WT, DIR, REF>, cap_blocks(kPersistBlocks, LDL_RESIDENT((k_hub_keys<WT, DIR, REF>), kTpb)), s,
               ev_a, ev_b, mv, br, bound, (const U64x3*)hw.off, hub, hw, st);
  k_hub_poff<<<cap_blocks(bound, LDL_RESIDENT(k_hub_poff, kTpb)), kTpb, 0, s>>>(br, bound, hw.off, hub, hw);
  k_hub_scatter<WT, DIR, REF><<<cap_blocks(kPersistBlocks, LDL_RESIDENT((k_hub_scatter<WT, DIR, REF>), kTpb)), kTpb,
                                0, s>>>(mv, br, bound, hw.off, hub, hw);
  k_hub_part<DIR, REF><<<cap_blocks(kPersistBlocks, LDL_RESIDENT((k_hub_part<DIR, REF>), kTpb)), kTpb, 0, s>>>(
      mv, br, bound, hw.off, hub, hw, st);
  k_hub_final<REF><<<cap_blocks(grid_waves(bound), LDL_RESIDENT(k_hub_final<REF>, kTpb)), kTpb, 0, s>>>(
      br, bound, hw.off, hub.cap, mv.lab, hw.phi, hw.plo, hw.pid, hw.pvalid, cand, st, hub.top, hub.over_count);
  return 0;
}

template <typename WT, bool DIR, bool REF>
void best_dispatch(const MoveView& mv, int bin, BinRef br, uint32_t max_count, CandBuf cand, MoveStats st,
                   hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  const uint64_t c = max_count;
  switch (bin) {
    case 0:
      launch_timed(k_best_group<WT, 8, DIR, REF>,
                   cap_blocks((c + 31) / 32, LDL_RESIDENT((k_best_group<WT, 8, DIR, REF>), kTpb)), s, ev_a, ev_b, mv,
                   br, cand, st);
      break;
    case 1:
      launch_timed(k_best_group<WT, 32, DIR, REF>,
                   cap_blocks((c + 7) / 8, LDL_RESIDENT((k_best_group<WT, 32, DIR, REF>), kTpb)), s, ev_a, ev_b, mv,
                   br, cand, st);
      break;
    case 2:
      launch_timed(k_best_wave<WT, 256, DIR, REF>,
                   cap_blocks((c + 3) / 4, LDL_RESIDENT((k_best_wave<WT, 256, DIR, REF>), kTpb)), s, ev_a, ev_b, mv,
                   br, cand, st);
      break;
    case 3:
      launch_timed(k_best_wave<WT, 1024, DIR, REF>,
                   cap_blocks((c + 3) / 4, LDL_RESIDENT((k_best_wave<WT, 1024, DIR, REF>), kTpb)), s, ev_a, ev_b, mv,
                   br, cand, st);
      break;
    default:
      launch_timed(k_best_hash<WT, 256, 4096, DIR, REF>,
                   cap_blocks(c, LDL_RESIDENT((k_best_hash<WT, 256, 4096, DIR, REF>), kTpb)), s, ev_a, ev_b, mv, br,
                   cand, st);
  }
}

// ------------------------------------------------------------------ decouple rounds
// Candidates are ordered by gain (descending), then vertex id (ascending).  Candidate i
// conflicts with j when a_i == b_j or b_i == a_j.  The sequential filter accepts a candidate
// iff no earlier accepted candidate conflicts with it, i.e. it returns the lexicographically
// first maximal independent set of the conflict graph.  Each round accepts every live
// candidate that precedes all live candidates entering its source and all live candidates
// leaving its target, then drops the live candidates that conflict with an accepted one.
// The first live candidate leaving (E) and entering (A) each community is found exactly,
// without a sort, by three atomic passes: max of the gain's high word, max of the low word
// among those with that high word, min of the vertex among those with both.  The
// per-community words are empty between rounds: each round's reject kernel clears the ones
// its live candidates wrote.
__device__ __forceinline__ uint32_t dev_count(const uint32_t* p, uint32_t bound) {
  const uint32_t c = *p;
  return c < bound ? c : bound;
}

__global__ void k_lf_init(const uint32_t* kp, uint32_t bound, uint32_t* live, uint8_t* flag, uint32_t* nlive,
                          uint32_t* nacc) {
  const uint32_t K = dev_count(kp, bound);
  if (gtid() == 0) {
    *nlive = K;
    *nacc = 0;
  }
  for (uint64_t i = gtid(); i < K; i += gstride()) {
    live[i] = (uint32_t)i;
    flag[i] = 0;
  }
}

template <int PASS>
__global__ void k_lf_pass(const uint32_t* live, const uint32_t* nlp, uint32_t bound, CandBuf cand, LfFirst E,
                          LfFirst A) {
  const uint32_t nl = dev_count(nlp, bound);
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    const uint32_t a = cand.a[i], b = cand.b[i];
    const u64a hi = (u64a)cand.ghi[i], lo = cand.glo[i];
    if (PASS == 0) {
      atomicMax(&E.hi[a], hi);
      atomicMax(&A.hi[b], hi);
    } else if (PASS == 1) {
      if (E.hi[a] == hi) atomicMax(&E.lo[a], lo);
      if (A.hi[b] == hi) atomicMax(&A.lo[b], lo);
    } else {
      const uint32_t v = cand.v[i];
      if (E.hi[a] == hi && E.lo[a] == lo) atomicMin(&E.v[a], v);
      if (A.hi[b] == hi && A.lo[b] == lo) atomicMin(&A.v[b], v);
    }
  }
}

// candidate (hi, lo, v) precedes the first of a set (empty sets have v == kEmpty)
__device__ __forceinline__ bool precedes_first(u64a hi, u64a lo, uint32_t v, const LfFirst& F, uint32_t c) {
  const uint32_t fv = F.v[c];
  if (fv == kEmpty) return true;
  const u64a fh = F.hi[c], fl = F.lo[c];
  if (hi != fh) return hi > fh;
  if (lo != fl) return lo > fl;
  return v < fv;
}

__global__ void k_lf_accept(const uint32_t* live, const uint32_t* nlp, uint32_t bound, CandBuf cand, LfFirst E,
                            LfFirst A, uint32_t* accE, uint32_t* accA, uint32_t ep, uint8_t* flag, uint32_t* acc_list,
                            uint32_t* acc_count, uint32_t* next_count) {
  const uint32_t nl = dev_count(nlp, bound);
  if (gtid() == 0) *next_count = 0;   // the reject kernel appends the survivors
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    const uint32_t a = cand.a[i], b = cand.b[i];
    const u64a hi = (u64a)cand.ghi[i], lo = cand.glo[i];
    const uint32_t v = cand.v[i];
    // no live candidate entering my source or leaving my target comes first
    const bool ok = precedes_first(hi, lo, v, A, a) && precedes_first(hi, lo, v, E, b);
    const uint32_t at = wave_reserve(acc_count, ok);
    if (ok) {
      flag[i] = 1;
      accE[a] = ep;
      accA[b] = ep;
      acc_list[at] = i;
    }
  }
}

// drops the live candidates that conflict with an accepted one and returns the per-community
// words of this round's communities to their empty state for the next round
__global__ void k_lf_reject(const uint32_t* live, const uint32_t* nlp, uint32_t bound, CandBuf cand, LfFirst E,
                            LfFirst A, const uint32_t* accE, const uint32_t* accA, uint32_t ep, const uint8_t* flag,
                            uint32_t* live2, uint32_t* live2_count) {
  const uint32_t nl = dev_count(nlp, bound);
  for (uint64_t t = gtid(); t < nl; t += gstride()) {
    const uint32_t i = live[t];
    const uint32_t a = cand.a[i], b = cand.b[i];
    const bool keep = !flag[i] && !(accA[a] == ep || accE[b] == ep);
    const uint32_t at = wave_reserve(live2_count, keep);
    if (keep) live2[at] = i;
    E.hi[a] = 0; E.lo[a] = 0; E.v[a] = kEmpty;
    A.hi[b] = 0; A.lo[b] = 0; A.v[b] = kEmpty;
  }
}

// ---- the same filter in one workgroup for at most kLfSmall candidates.  The candidates are
// ranked by a bitonic sort in LDS on (gain descending, vertex ascending); their source and target
// communities get LDS slots from a hash table (at most 2 kLfSmall communities in kLfSlots slots);
// then the rounds run on ranks: per community the first live candidate leaving it and the first
// entering it by an LDS atomic min, acceptance of every live candidate that precedes both firsts
// that concern it, and removal of the live candidates that conflict with an accepted one, with
// workgroup barriers between the steps, until no candidate is live.  Each round accepts at least
// the first live candidate.
constexpr uint32_t kLfSlots = 4096;

__device__ __forceinline__ bool lf_precedes(int64_t h1, uint64_t l1, uint32_t v1, int64_t h2, uint64_t l2,
                                            uint32_t v2) {
  if (h1 != h2) return h1 > h2;
  if (l1 != l2) return l1 > l2;
  return v1 < v2;
}

__device__ __forceinline__ uint32_t lf_slot(uint32_t* keys, uint32_t c) {
  uint32_t h = hash32(c) & (kLfSlots - 1);
  for (;;) {   // at most 2 kLfSmall keys in kLfSlots >= 4 kLfSmall slots: a free slot exists
    const uint32_t prev = atomicCAS(&keys[h], kEmpty, c);
    if (prev == kEmpty || prev == c) return h;
    h = (h + 1) & (kLfSlots - 1);
  }
}

__global__ __launch_bounds__(kLfSmall) void k_lf_small(CandBuf cand, uint32_t* acc, uint32_t* nacc, uint32_t* nlive) {
  static_assert(kLfSlots >= 4 * kLfSmall, "load factor of the community table");
  __shared__ int64_t shi[kLfSmall];
  __shared__ uint64_t slo[kLfSmall];
  __shared__ uint32_t sv[kLfSmall];
  __shared__ uint16_t sid[kLfSmall];
  __shared__ uint32_t rank[kLfSmall];
  __shared__ uint32_t ckey[kLfSlots], emin[kLfSlots], amin[kLfSlots];
  __shared__ uint8_t accE[kLfSlots], accA[kLfSlots];
  __shared__ uint32_t s_nacc;
  const uint32_t K = *cand.count;
  const uint32_t t = threadIdx.x;
  if (K > kLfSmall) {
    if (t == 0) {
      *nacc = 0;
      *nlive = 0;
    }
    return;
  }
  // padding has gain 0 and sorts after every candidate (candidate gains are positive)
  if (t < K) {
    shi[t] = cand.ghi[t];
    slo[t] = cand.glo[t];
    sv[t] = cand.v[t];
  } else {
    shi[t] = 0;
    slo[t] = 0;
    sv[t] = kEmpty;
  }
  sid[t] = (uint16_t)t;
  for (uint32_t q = t; q < kLfSlots; q += blockDim.x) {
    ckey[q] = kEmpty;
    emin[q] = kEmpty;
    amin[q] = kEmpty;
    accE[q] = 0;
    accA[q] = 0;
  }
  if (t == 0) s_nacc = 0;
  __syncthreads();
  for (uint32_t k = 2; k <= kLfSmall; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint32_t p = t ^ j;
      if (p > t) {
        const bool first_is_t = (t & k) == 0;   // this pair is ordered t before p
        const bool sw = first_is_t ? lf_precedes(shi[p], slo[p], sv[p], shi[t], slo[t], sv[t])
                                   : lf_precedes(shi[t], slo[t], sv[t], shi[p], slo[p], sv[p]);
        if (sw) {
          const int64_t h = shi[t]; shi[t] = shi[p]; shi[p] = h;
          const uint64_t l = slo[t]; slo[t] = slo[p]; slo[p] = l;
          const uint32_t v = sv[t]; sv[t] = sv[p]; sv[p] = v;
          const uint16_t d = sid[t]; sid[t] = sid[p]; sid[p] = d;
        }
      }
      __syncthreads();
    }
  }
  rank[sid[t]] = t;   // position t of the order holds candidate sid[t]
  __syncthreads();
  bool live = t < K;
  uint32_t sa = 0, sb = 0, rk = 0;
  if (live) {
    sa = lf_slot(ckey, cand.a[t]);
    sb = lf_slot(ckey, cand.b[t]);
    rk = rank[t];
  }
  __syncthreads();
  for (;;) {
    if (live) {
      atomicMin(&emin[sa], rk);   // first live candidate leaving the community
      atomicMin(&amin[sb], rk);   // first live candidate entering it
    }
    __syncthreads();
    const bool ok = live && rk < amin[sa] && rk < emin[sb];
    __syncthreads();
    if (ok) {
      accE[sa] = 1;
      accA[sb] = 1;
      acc[atomicAdd(&s_nacc, 1u)] = t;
    }
    __syncthreads();
    if (live) {
      emin[sa] = kEmpty;
      amin[sb] = kEmpty;
    }
    live = live && !ok && !(accA[sa] || accE[sb]);
    if (!__syncthreads_or(live)) break;
  }
  if (t == 0) {
    *nacc = s_nacc;
    *nlive = 0;
  }
}

// ------------------------------------------------------------------ commit / rollback
__global__ void k_commit_mark(const uint32_t* acc, const uint32_t* nap, CandBuf cand, uint32_t* mov_stamp,
                              uint32_t mov_ep, uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin,
                              SetRef touched, int64_t* tko, int64_t* tki) {
  const uint32_t na = *nap;
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

__global__ void k_commit_apply(const uint32_t* acc, const uint32_t* nap, CandBuf cand, uint32_t* lab,
                               const int64_t* kout, const int64_t* kin, int64_t* Kout, int64_t* Kin, int forward) {
  const uint32_t na = *nap;
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

// Exact change of the same-label weight over the matrix entries incident to movers, each entry
// once: mover v's out entries (with the neighbour's old label when the neighbour moved too),
// then its in entries whose other end did not move (for undirected graphs the out entries
// again, standing for the mirrored matrix entries).  One wavefront per mover; a mover with more
// than kDeinBig entries is listed instead and taken by a whole workgroup in k_commit_dein_big.
constexpr uint32_t kDeinBig = 4096;

__device__ __forceinline__ int64_t dein_entry(const CsrRef& out, const CsrRef& second, uint32_t dout, uint64_t oo,
                                              uint64_t os, uint64_t j, uint32_t lv_new, uint32_t lv_old,
                                              const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep,
                                              const uint32_t* oldlab) {
  if (j < dout) {
    const uint32_t u = out.nbr[oo + j];
    const int64_t w = wget(out, oo + j);
    const uint32_t lu_new = lab[u];
    const uint32_t lu_old = mov_stamp[u] == mov_ep ? oldlab[u] : lu_new;
    return w * ((int64_t)(lv_new == lu_new) - (int64_t)(lv_old == lu_old));
  }
  const uint64_t e = os + (j - dout);
  const uint32_t u = second.nbr[e];
  if (mov_stamp[u] == mov_ep) return 0;
  const int64_t w = wget(second, e);
  const uint32_t lu = lab[u];
  return w * ((int64_t)(lv_new == lu) - (int64_t)(lv_old == lu));
}

__global__ void k_commit_dein(const uint32_t* acc, const uint32_t* nap, CandBuf cand, CsrRef out, CsrRef second,
                              const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep, const uint32_t* oldlab,
                              uint32_t* big, uint32_t* nbig, i64a* dein) {
  const int lane = lane_id();
  const uint32_t na = *nap;
  int64_t s = 0;
  for (uint64_t t = gwave(); t < na; t += gwstride()) {
    const uint32_t v = cand.v[acc[t]];
    const uint32_t dout = out.deg[v];
    const uint64_t sl = (uint64_t)dout + second.deg[v];
    if (sl > kDeinBig) {
      if (lane == 0) big[atomicAdd(nbig, 1u)] = v;
      continue;
    }
    const uint32_t lv_new = lab[v], lv_old = oldlab[v];
    const uint64_t oo = out.off[v], os = second.off[v];
    for (uint64_t j = lane; j < sl; j += kWave)
      s += dein_entry(out, second, dout, oo, os, j, lv_new, lv_old, lab, mov_stamp, mov_ep, oldlab);
  }
  s = wave_sum_i64(s);
  if (lane == 0 && s != 0) atomicAdd((u64a*)dein, (u64a)s);
}

// the listed movers: one workgroup of kDeinTpb threads per mover
constexpr int kDeinTpb = 1024;
__global__ __launch_bounds__(kDeinTpb) void k_commit_dein_big(const uint32_t* big, const uint32_t* nbig, CsrRef out,
                                                              CsrRef second, const uint32_t* lab,
                                                              const uint32_t* mov_stamp, uint32_t mov_ep,
                                                              const uint32_t* oldlab, i64a* dein) {
  const uint32_t nb = *nbig;
  int64_t s = 0;
  for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint32_t v = big[b];
    const uint32_t dout = out.deg[v];
    const uint64_t sl = (uint64_t)dout + second.deg[v];
    const uint32_t lv_new = lab[v], lv_old = oldlab[v];
    const uint64_t oo = out.off[v], os = second.off[v];
    for (uint64_t j = threadIdx.x; j < sl; j += blockDim.x)
      s += dein_entry(out, second, dout, oo, os, j, lv_new, lv_old, lab, mov_stamp, mov_ep, oldlab);
  }
  s = wave_sum_i64(s);
  if (lane_id() == 0 && s != 0) atomicAdd((u64a*)dein, (u64a)s);
}

__global__ void k_mark_acc_comms(const uint32_t* acc, const uint32_t* nap, CandBuf cand, uint32_t* stamp,
                                 uint32_t ep) {
  const uint32_t na = *nap;
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    stamp[cand.a[i]] = ep;
    stamp[cand.b[i]] = ep;
  }
}

__global__ void k_set_add_acc_v(SetRef set, const uint32_t* acc, const uint32_t* nap, CandBuf cand) {
  const uint32_t na = *nap;
  for (uint64_t t = gtid(); t < na; t += gstride())
    set_add(set.stamp, set.epoch, set.list, set.count, cand.v[acc[t]]);
}

// singleton u joins refined community y (forward) or returns to itself (undo)
__global__ void k_ref_commit(const uint32_t* acc, const uint32_t* nap, CandBuf cand, uint32_t* par, uint2* lp,
                             const int64_t* kout, const int64_t* kin, int64_t* Krout, int64_t* Krin, uint32_t* rsize,
                             int forward) {
  const uint32_t na = *nap;
  for (uint64_t t = gtid(); t < na; t += gstride()) {
    const uint32_t i = acc[t];
    const uint32_t u = cand.v[i], y = cand.b[i];
    const int64_t sg = forward ? 1 : -1;
    par[u] = forward ? y : u;
    lp[u].y = forward ? y : u;
    atomic_add_i64(&Krout[y], sg * kout[u]);
    atomic_add_i64(&Krout[u], -sg * kout[u]);
    if (Krin) {
      atomic_add_i64(&Krin[y], sg * kin[u]);
      atomic_add_i64(&Krin[u], -sg * kin[u]);
    }
    if (forward) {
      atomicAdd(&rsize[y], 1u);
      atomicSub(&rsize[u], 1u);
    } else {
      atomicSub(&rsize[y], 1u);
      atomicAdd(&rsize[u], 1u);
    }
  }
}

__global__ void k_pack_lab_par(uint32_t n, const uint32_t* lab, const uint32_t* par, uint2* lp) {
  for (uint64_t u = gtid(); u < n; u += gstride()) lp[u] = make_uint2(lab[u], par[u]);
}

__global__ void k_stride_sample(const uint32_t* src, const uint32_t* countp, uint32_t bound, uint32_t stride,
                                uint32_t* out, uint32_t* out_count) {
  const uint32_t c0 = *countp;
  const uint32_t c = c0 < bound ? c0 : bound;
  const uint32_t k = (c + stride - 1) / stride;
  if (gtid() == 0) *out_count = k;
  for (uint64_t i = gtid(); i < k; i += gstride()) out[i] = src[i * (uint64_t)stride];
}

}  // namespace

// ------------------------------------------------------------------ launchers
// Kernels that read their item count from device memory get a grid sized from a host-side
// upper bound (the grid-stride loops cover any count up to it).

void launch_bin_count(const MoveView& mv, const uint32_t* list, const uint32_t* count, int refine, uint32_t* hist,
                      uint32_t* zero_words, uint32_t nzero, hipStream_t s) {
  k_bin_count<<<kBinBlocks, kTpb, 0, s>>>(mv, list, count, refine, hist, zero_words, nzero);
}
void launch_bin_fill(const MoveView& mv, const uint32_t* list, const uint32_t* count, int refine, const uint32_t* hist,
                     uint32_t* out, uint32_t* bin_start, uint32_t* bin_count, hipStream_t s) {
  static_assert(kBinBlocks <= kTpb, "one histogram word per thread");
  k_bin_fill<<<kBinBlocks, kTpb, 0, s>>>(mv, list, count, refine, hist, out, bin_start, bin_count);
}
void launch_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, const uint32_t* na,
                                uint32_t na_max, CandBuf cand, CsrRef out, CsrRef in, int directed, hipStream_t s) {
  if (na_max)
    k_mark_neighbours_acc<<<grid_waves(na_max), kTpb, 0, s>>>(stamp, ep, acc, na, cand, out, in, directed);
}

#define LDL_TYPED(CALL)                                                                                             \
  do {                                                                                                             \
    const bool dir_ = mv.directed != 0;                                                                            \
    if (!mv.out.wide) {                                                                                            \
      if (dir_) { if (refine) CALL(uint32_t, true, true); else CALL(uint32_t, true, false); }                      \
      else { if (refine) CALL(uint32_t, false, true); else CALL(uint32_t, false, false); }                         \
    } else {                                                                                                       \
      if (dir_) { if (refine) CALL(int64_t, true, true); else CALL(int64_t, true, false); }                        \
      else { if (refine) CALL(int64_t, false, true); else CALL(int64_t, false, false); }                           \
    }                                                                                                              \
  } while (0)

void launch_best(const MoveView& mv, int bin, BinRef br, uint32_t max_count, int refine, CandBuf cand, MoveStats st,
                 hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  if (!max_count) return;
#define LDL_BEST(WT, D, R) best_dispatch<WT, D, R>(mv, bin, br, max_count, cand, st, s, ev_a, ev_b)
  LDL_TYPED(LDL_BEST);
#undef LDL_BEST
}

int launch_hub(const MoveView& mv, BinRef br, uint32_t bound, int refine, HubPool hub, HubWork hw, CandBuf cand,
               MoveStats st, void** tmp, size_t* tmp_bytes, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  if (!bound) return 0;
  int rc = 0;
#define LDL_HUB(WT, D, R) rc = hub_dispatch<WT, D, R>(mv, br, bound, hub, hw, cand, st, tmp, tmp_bytes, s, ev_a, ev_b)
  LDL_TYPED(LDL_HUB);
#undef LDL_HUB
  return rc;
}
#undef LDL_TYPED

void launch_lf_init(const uint32_t* K, uint32_t bound, uint32_t* live, uint8_t* flag, uint32_t* nlive, uint32_t* nacc,
                    hipStream_t s) {
  k_lf_init<<<kLfBlocks, kTpb, 0, s>>>(K, bound, live, flag, nlive, nacc);
}
void launch_lf_small(CandBuf cand, uint32_t* acc, uint32_t* nacc, uint32_t* nlive, hipStream_t s) {
  k_lf_small<<<1, kLfSmall, 0, s>>>(cand, acc, nacc, nlive);
}
void launch_lf_round(const uint32_t* live, const uint32_t* nl, uint32_t bound, CandBuf cand, LfFirst E, LfFirst A,
                     uint32_t* accE, uint32_t* accA, uint32_t ep, uint8_t* flag, uint32_t* acc_list,
                     uint32_t* acc_count, uint32_t* live2, uint32_t* live2_count, hipStream_t s) {
  k_lf_pass<0><<<kLfBlocks, kTpb, 0, s>>>(live, nl, bound, cand, E, A);
  k_lf_pass<1><<<kLfBlocks, kTpb, 0, s>>>(live, nl, bound, cand, E, A);
  k_lf_pass<2><<<kLfBlocks, kTpb, 0, s>>>(live, nl, bound, cand, E, A);
  k_lf_accept<<<kLfBlocks, kTpb, 0, s>>>(live, nl, bound, cand, E, A, accE, accA, ep, flag, acc_list, acc_count,
                                        live2_count);
  k_lf_reject<<<kLfBlocks, kTpb, 0, s>>>(live, nl, bound, cand, E, A, accE, accA, ep, flag, live2, live2_count);
}
// grids for counts read on the device: at most kLfBlocks workgroups (grid-stride loops)
inline unsigned cap_grid(unsigned g) { return g < kLfBlocks ? g : kLfBlocks; }

void launch_commit_mark(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* mov_stamp,
                        uint32_t mov_ep, uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin, SetRef touched,
                        int64_t* tko, int64_t* tki, hipStream_t s) {
  if (na_max)
    k_commit_mark<<<cap_grid(grid_for(na_max)), kTpb, 0, s>>>(acc, na, cand, mov_stamp, mov_ep, oldlab, Kout, Kin,
                                                              touched, tko, tki);
}
void launch_commit_apply(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* lab,
                         const int64_t* kout, const int64_t* kin, int64_t* Kout, int64_t* Kin_or_null, int forward,
                         hipStream_t s) {
  if (na_max)
    k_commit_apply<<<cap_grid(grid_for(na_max)), kTpb, 0, s>>>(acc, na, cand, lab, kout, kin, Kout, Kin_or_null,
                                                               forward);
}
void launch_commit_dein(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, CsrRef out, CsrRef in,
                        int directed, const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep,
                        const uint32_t* oldlab, uint32_t* big, uint32_t* nbig, i64a* dein, hipStream_t s) {
  if (!na_max) return;
  const CsrRef second = directed ? in : out;
  k_commit_dein<<<cap_grid(grid_waves(na_max)), kTpb, 0, s>>>(acc, na, cand, out, second, lab, mov_stamp, mov_ep,
                                                              oldlab, big, nbig, dein);
  k_commit_dein_big<<<cap_blocks(kPersistBlocks, LDL_RESIDENT(k_commit_dein_big, kDeinTpb)), kDeinTpb, 0, s>>>(
      big, nbig, out, second, lab, mov_stamp, mov_ep, oldlab, dein);
}
void launch_mark_acc_comms(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* stamp,
                           uint32_t ep, hipStream_t s) {
  if (na_max) k_mark_acc_comms<<<cap_grid(grid_for(na_max)), kTpb, 0, s>>>(acc, na, cand, stamp, ep);
}
void launch_set_add_acc_v(SetRef set, const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand,
                          hipStream_t s) {
  if (na_max) k_set_add_acc_v<<<cap_grid(grid_for(na_max)), kTpb, 0, s>>>(set, acc, na, cand);
}
void launch_ref_commit(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* par,
                       uint2* lp, const int64_t* kout, const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null,
                       uint32_t* rsize, int forward, hipStream_t s) {
  if (na_max)
    k_ref_commit<<<cap_grid(grid_for(na_max)), kTpb, 0, s>>>(acc, na, cand, par, lp, kout, kin, Krout, Krin_or_null,
                                                             rsize, forward);
}
void launch_pack_lab_par(uint32_t n, const uint32_t* lab, const uint32_t* par, uint2* lp, hipStream_t s) {
  if (n) k_pack_lab_par<<<grid_for(n), kTpb, 0, s>>>(n, lab, par, lp);
}
void launch_stride_sample(const uint32_t* src, const uint32_t* count, uint32_t bound, uint32_t stride, uint32_t* out,
                          uint32_t* out_count, hipStream_t s) {
  if (bound && stride) k_stride_sample<<<cap_grid(grid_for(bound)), kTpb, 0, s>>>(src, count, bound, stride, out,
                                                                                   out_count);
}

}  // namespace ldl
