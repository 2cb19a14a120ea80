// Graph-maintenance kernels: stamped sets, dynamic CSR edits, batch ingest and statistic
// repair (Alg. 1 l.1-3), aggregate-repair tuples and hierarchy liveness (Alg. 1 l.23-24,
// Eq. 3), label refresh.
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
__device__ __forceinline__ void wset(const CsrRef& c, uint64_t i, int64_t v) {
  if (c.wide) ((int64_t*)c.w)[i] = v;
  else ((uint32_t*)c.w)[i] = (uint32_t)v;
}

// lanes below me in the wave with `pred` set
__device__ __forceinline__ uint32_t rank_in_wave(bool pred) {
  const uint64_t m = __ballot(pred);
  const uint64_t below = m & ((1ull << lane_id()) - 1ull);
  return (uint32_t)__popcll(below);
}

// ------------------------------------------------------------------ generic helpers

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, uint8_t v, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t v, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void k_iota(uint32_t* p, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = (uint32_t)i;
}
__global__ void k_copy_i64(int64_t* d, const int64_t* s, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) d[i] = s[i];
}

__global__ void k_set_add_list(SetRef set, const uint32_t* list, uint32_t count) {
  for (uint64_t i = gtid(); i < count; i += gstride()) set_add(set.stamp, set.epoch, set.list, set.count, list[i]);
}
__global__ void k_set_add_mapped(SetRef set, const uint32_t* list, uint32_t count, const uint32_t* key,
                                 const uint8_t* alive) {
  for (uint64_t i = gtid(); i < count; i += gstride()) {
    uint32_t x = list[i];
    if (alive && !alive[x]) continue;
    uint32_t k = key[x];
    if (set.list) set_add(set.stamp, set.epoch, set.list, set.count, k);
    else set_claim(set.stamp, set.epoch, k);
  }
}
__global__ void k_members(SetRef set, uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* mark,
                          uint32_t ep) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    if (!alive[u]) continue;
    if (mark[key[u]] == ep) set_add(set.stamp, set.epoch, set.list, set.count, (uint32_t)u);
  }
}

// wave per listed vertex: the vertex and every out/in neighbour join the set
__global__ void k_neighbours(SetRef set, const uint32_t* list, uint32_t count, CsrRef out, CsrRef in, int directed) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < count; i += gwstride()) {
    const uint32_t v = list[i];
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

// ------------------------------------------------------------------ dynamic CSR

// wave per record: locate col in row; update in place, tombstone (w = 0) on a zero result,
// or flag an insertion.  Rows that lose or gain entries join `dirty`.
__global__ void k_csr_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, uint8_t* insflag,
                           uint32_t* rowdel, uint32_t* rowins, SetRef dirty) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < k; i += gwstride()) {
    const int64_t d = delta[i];
    if (d == 0) {
      if (lane == 0) insflag[i] = 0;
      continue;
    }
    const uint32_t row = (uint32_t)(keys[i] >> 32), col = (uint32_t)keys[i];
    const uint64_t o = c.off[row];
    const uint32_t deg = c.deg[row];
    int64_t slot = -1;
    for (uint32_t base = 0; base < deg; base += kWave) {
      const uint32_t j = base + lane;
      const bool hit = j < deg && c.nbr[o + j] == col;
      const uint64_t m = __ballot(hit);
      if (m) {
        slot = (int64_t)(o + base + (uint32_t)__ffsll((long long)m) - 1);
        break;
      }
    }
    if (lane == 0) {
      if (slot >= 0) {
        const int64_t nw = wget(c, (uint64_t)slot) + d;
        wset(c, (uint64_t)slot, nw);
        insflag[i] = 0;
        if (nw == 0) {
          atomicAdd(&rowdel[row], 1u);
          set_add(dirty.stamp, dirty.epoch, dirty.list, dirty.count, row);
        }
      } else {
        insflag[i] = 1;
        atomicAdd(&rowins[row], 1u);
        set_add(dirty.stamp, dirty.epoch, dirty.list, dirty.count, row);
      }
    }
  }
}

// Row segments of sorted record keys: one entry (first record index) per distinct row.
__global__ void k_segments(const uint64_t* keys, uint64_t k, uint64_t* seg_lo, uint32_t* nseg) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const bool head = i == 0 || (keys[i] >> 32) != (keys[i - 1] >> 32);
    const uint32_t at = wave_reserve(nseg, head);
    if (head) seg_lo[at] = i;
  }
}

__device__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key);

// Workgroup per row segment: the segment's records (up to 2048 at a time) go into an LDS
// hash table keyed by column, then the row is streamed once and every entry probes the
// table, so the cost is O(degree + records) per row.
// MODE 0: write the slot (or -1) of every record.  MODE 1: apply the deltas in place
// (a zero result leaves a w = 0 tombstone), flag insertions, count per-row deletions and
// insertions and collect the rows that change shape in `dirty`.
constexpr int kSegChunk = 2048;
template <int MODE>
__global__ __launch_bounds__(256) void k_seg_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k,
                                                  const uint64_t* seg_lo, const uint32_t* nseg_ptr, int64_t* slot_out,
                                                  uint8_t* insflag, uint32_t* rowdel, uint32_t* rowins,
                                                  SetRef dirty) {
  __shared__ uint32_t tkey[2 * kSegChunk];
  __shared__ uint32_t tval[2 * kSegChunk];
  __shared__ int64_t sslot[kSegChunk];
  __shared__ uint64_t s_hi;
  __shared__ uint32_t s_cnt[2];
  const uint32_t nseg = *nseg_ptr;
  for (uint32_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const uint64_t lo = seg_lo[seg];
    const uint32_t row = (uint32_t)(keys[lo] >> 32);
    if (threadIdx.x == 0) {
      s_hi = lower_bound_u64(keys, k, ((uint64_t)row + 1) << 32);
      s_cnt[0] = 0;
      s_cnt[1] = 0;
    }
    __syncthreads();
    const uint64_t hi = s_hi;
    const uint64_t off = c.off[row];
    const uint32_t deg = c.deg[row];
    uint32_t ndel = 0, nins = 0;
    for (uint64_t clo = lo; clo < hi; clo += kSegChunk) {
      const uint32_t kk = (uint32_t)((hi - clo) < (uint64_t)kSegChunk ? (hi - clo) : (uint64_t)kSegChunk);
      uint32_t size = 64;
      while (size < 2 * kk) size <<= 1;
      const uint32_t mask = size - 1;
      for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) tkey[i] = kEmpty;
      for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) sslot[i] = -1;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) {
        const uint32_t col = (uint32_t)keys[clo + i];
        uint32_t h = hash32(col) & mask;
        for (;;) {
          const uint32_t prev = atomicCAS(&tkey[h], kEmpty, col);
          if (prev == kEmpty) {
            tval[h] = i;
            break;
          }
          h = (h + 1) & mask;
        }
      }
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < deg; j += blockDim.x) {
        const uint32_t x = c.nbr[off + j];
        uint32_t h = hash32(x) & mask;
        for (;;) {
          const uint32_t kx = tkey[h];
          if (kx == kEmpty) break;
          if (kx == x) {
            sslot[tval[h]] = (int64_t)(off + j);
            break;
          }
          h = (h + 1) & mask;
        }
      }
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) {
        const int64_t sl = sslot[i];
        if (MODE == 0) {
          slot_out[clo + i] = sl;
        } else {
          const int64_t d = delta[clo + i];
          if (d == 0) {
            insflag[clo + i] = 0;
          } else if (sl >= 0) {
            const int64_t nw = wget(c, (uint64_t)sl) + d;
            wset(c, (uint64_t)sl, nw);
            insflag[clo + i] = 0;
            if (nw == 0) ++ndel;
          } else {
            insflag[clo + i] = 1;
            ++nins;
          }
        }
      }
      __syncthreads();
    }
    if (MODE == 1) {
      if (ndel) atomicAdd(&s_cnt[0], ndel);
      if (nins) atomicAdd(&s_cnt[1], nins);
      __syncthreads();
      if (threadIdx.x == 0) {
        rowdel[row] = s_cnt[0];
        rowins[row] = s_cnt[1];
        if (s_cnt[0] + s_cnt[1]) dirty.list[atomicAdd(dirty.count, 1u)] = row;
      }
    }
    __syncthreads();
  }
}

// ---- row-segment lookup split into (segment, record chunk, row slice) work items, so a
// huge row is streamed by many workgroups and a row with many records by several tables.
constexpr uint32_t kSlice = 16384;

__global__ void k_seg_items(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo,
                            const uint32_t* nseg_ptr, uint64_t* seg_hi, uint64_t* items) {
  const uint32_t nseg = *nseg_ptr;
  for (uint64_t s = gtid(); s <= k; s += gstride()) {
    if (s >= nseg) {
      items[s] = 0;
      continue;
    }
    const uint64_t lo = seg_lo[s];
    const uint32_t row = (uint32_t)(keys[lo] >> 32);
    const uint64_t hi = lower_bound_u64(keys, k, ((uint64_t)row + 1) << 32);
    seg_hi[s] = hi;
    const uint64_t deg = c.deg[row];
    const uint64_t nsl = deg == 0 ? 1 : (deg + kSlice - 1) / kSlice;
    const uint64_t nrc = (hi - lo + kSegChunk - 1) / kSegChunk;
    items[s] = nsl * nrc;
  }
}

__device__ __forceinline__ uint32_t upper_bound_u64(const uint64_t* a, uint32_t n, uint64_t key) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// workgroup per work item: LDS table of the item's record chunk, stream the item's row slice,
// write the slot of every record found (each record matches at most one entry)
__global__ __launch_bounds__(256) void k_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k,
                                                    const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                    const uint32_t* nseg_ptr, const uint64_t* item_off,
                                                    int64_t* slot_out) {
  __shared__ uint32_t tkey[2 * kSegChunk];
  __shared__ uint32_t tval[2 * kSegChunk];
  const uint32_t nseg = *nseg_ptr;
  const uint64_t total = item_off[nseg];
  for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const uint32_t sg = upper_bound_u64(item_off, nseg + 1, it) - 1;
    const uint64_t sub = it - item_off[sg];
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    const uint32_t row = (uint32_t)(keys[lo] >> 32);
    const uint64_t deg = c.deg[row];
    const uint64_t nsl = deg == 0 ? 1 : (deg + kSlice - 1) / kSlice;
    const uint64_t rc = sub / nsl, sl = sub % nsl;
    const uint64_t clo = lo + rc * kSegChunk;
    const uint32_t kk = (uint32_t)((hi - clo) < (uint64_t)kSegChunk ? (hi - clo) : (uint64_t)kSegChunk);
    uint32_t size = 64;
    while (size < 2 * kk) size <<= 1;
    const uint32_t mask = size - 1;
    for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) tkey[i] = kEmpty;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) {
      const uint32_t col = (uint32_t)keys[clo + i];
      uint32_t h = hash32(col) & mask;
      for (;;) {
        const uint32_t prev = atomicCAS(&tkey[h], kEmpty, col);
        if (prev == kEmpty) {
          tval[h] = i;
          break;
        }
        h = (h + 1) & mask;
      }
    }
    __syncthreads();
    const uint64_t off = c.off[row];
    const uint64_t e0 = sl * kSlice;
    const uint64_t e1 = e0 + kSlice < deg ? e0 + kSlice : deg;
    for (uint64_t j = e0 + threadIdx.x; j < e1; j += blockDim.x) {
      const uint32_t x = c.nbr[off + j];
      uint32_t h = hash32(x) & mask;
      for (;;) {
        const uint32_t kx = tkey[h];
        if (kx == kEmpty) break;
        if (kx == x) {
          slot_out[clo + tval[h]] = (int64_t)(off + j);
          break;
        }
        h = (h + 1) & mask;
      }
    }
    __syncthreads();
  }
}

// workgroup per segment: apply the row's deltas at the looked-up slots (a zero result leaves a
// w = 0 tombstone), flag insertions, count deletions / insertions, add the row's delta sum to
// its degree (when deg != null) and collect rows that change shape in `dirty`
__global__ __launch_bounds__(256) void k_seg_apply(CsrRef c, const uint64_t* keys, const int64_t* delta,
                                                   const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                   const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* insflag,
                                                   uint32_t* rowdel, uint32_t* rowins, int64_t* deg_arr,
                                                   uint32_t* dirty_list, uint32_t* dirty_count) {
  __shared__ int64_t red[3 * 4];
  const uint32_t nseg = *nseg_ptr;
  for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    const uint32_t row = (uint32_t)(keys[lo] >> 32);
    int64_t ndel = 0, nins = 0, dsum = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const int64_t d = delta[i];
      const int64_t sl = slot[i];
      dsum += d;
      if (d == 0) {
        insflag[i] = 0;
      } else if (sl >= 0) {
        const int64_t nw = wget(c, (uint64_t)sl) + d;
        wset(c, (uint64_t)sl, nw);
        insflag[i] = 0;
        if (nw == 0) ++ndel;
      } else {
        insflag[i] = 1;
        ++nins;
      }
    }
    ndel = wave_sum_i64(ndel);
    nins = wave_sum_i64(nins);
    dsum = wave_sum_i64(dsum);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & 63) == 0) {
      red[3 * w] = ndel;
      red[3 * w + 1] = nins;
      red[3 * w + 2] = dsum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t a = 0, b = 0, d = 0;
      for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
        a += red[3 * i];
        b += red[3 * i + 1];
        d += red[3 * i + 2];
      }
      rowdel[row] = (uint32_t)a;
      rowins[row] = (uint32_t)b;
      if (deg_arr) deg_arr[row] += d;
      if (a + b) dirty_list[atomicAdd(dirty_count, 1u)] = row;
    }
    __syncthreads();
  }
}

__global__ void k_fill_i64_dev(int64_t* p, int64_t v, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// Per sorted ingest record: duplicate check, validation and delta from the looked-up slot.
__global__ void k_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot,
                                  uint64_t k, const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd,
                                  const uint32_t* chg, int directed, int64_t* delta, uint32_t* err,
                                  uint32_t* first_bad, i64a* dm) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t key = keys[i];
    if (i > 0 && keys[i - 1] == key) atomicOr(err, 2u);
    const uint32_t u = (uint32_t)(key >> 32), v = (uint32_t)key;
    const int64_t sl = slot[i];
    const uint32_t src = idx[i];
    const int64_t old = sl >= 0 ? (int64_t)((const uint32_t*)out0.w)[sl] : 0;
    int64_t d = 0;
    bool bad = false;
    if (src < ni) {
      const int64_t w = ins[3 * (uint64_t)src + 2];
      if (old + w > 0xFFFFFFFFll) { bad = true; atomicOr(err, 8u); }
      d = w;
    } else if (src < ni + nd) {
      if (sl < 0) { bad = true; atomicOr(err, 4u); }
      d = -old;
    } else {
      const int64_t w = chg[3 * ((uint64_t)src - ni - nd) + 2];
      if (sl < 0) { bad = true; atomicOr(err, 4u); }
      d = w - old;
    }
    if (bad) {
      atomicMin(first_bad, src);
      d = 0;
    }
    delta[i] = d;
    if (d != 0) atomicAdd((u64a*)dm, (u64a)((!directed && u != v) ? 2 * d : d));
  }
}

__global__ void k_csr_plan(CsrRef c, const uint32_t* dirty, uint32_t nd, const uint32_t* rowdel,
                           const uint32_t* rowins, uint64_t* plan_off, uint32_t* plan_cap, u64a* pool_top,
                           uint64_t pool_cap, uint32_t* overflow) {
  for (uint64_t j = gtid(); j < nd; j += gstride()) {
    const uint32_t row = dirty[j];
    const uint64_t need = (uint64_t)c.deg[row] - rowdel[row] + rowins[row];
    if (need <= c.cap[row]) {
      plan_off[j] = c.off[row];
      plan_cap[j] = c.cap[row];
      continue;
    }
    uint64_t nc = need + (need >> 2);
    if (nc < need + 4) nc = need + 4;
    if (nc > 0xFFFFFFFFull) nc = 0xFFFFFFFFull;
    const u64a o = atomicAdd(pool_top, (u64a)nc);
    if (o + nc > pool_cap) {
      atomicOr(overflow, 1u);
      plan_off[j] = ~0ull;
      plan_cap[j] = 0;
    } else {
      plan_off[j] = o;
      plan_cap[j] = (uint32_t)nc;
    }
  }
}

__device__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// wave per dirty row: compact survivors (w != 0) to the planned location, then append the
// row's flagged insertions (records of the row are contiguous in the sorted keys)
__global__ void k_csr_rewrite(CsrRef c, const uint32_t* dirty, uint32_t nd, uint32_t* rowdel, uint32_t* rowins,
                              const uint64_t* plan_off, const uint32_t* plan_cap, const uint64_t* keys,
                              const int64_t* delta, const uint8_t* insflag, uint64_t k) {
  const int lane = lane_id();
  for (uint64_t j = gwave(); j < nd; j += gwstride()) {
    const uint32_t row = dirty[j];
    const uint64_t src = c.off[row];
    const uint32_t deg = c.deg[row];
    const uint64_t dst = plan_off[j];
    uint32_t written = 0;
    for (uint32_t base = 0; base < deg; base += kWave) {
      const uint32_t i = base + lane;
      uint32_t nb = 0;
      int64_t w = 0;
      if (i < deg) {
        nb = c.nbr[src + i];
        w = wget(c, src + i);
      }
      const bool keep = i < deg && w != 0;
      const uint32_t r = rank_in_wave(keep);
      const uint32_t tot = (uint32_t)__popcll(__ballot(keep));
      // every lane has read its element before any lane writes (writes land at or below reads)
      __builtin_amdgcn_wave_barrier();
      if (keep) {
        c.nbr[dst + written + r] = nb;
        wset(c, dst + written + r, w);
      }
      __builtin_amdgcn_wave_barrier();
      written += tot;
    }
    const uint64_t lo = lower_bound_u64(keys, k, (uint64_t)row << 32);
    const uint64_t hi = lower_bound_u64(keys, k, ((uint64_t)row + 1) << 32);
    for (uint64_t base = lo; base < hi; base += kWave) {
      const uint64_t i = base + lane;
      const bool ins = i < hi && insflag[i];
      const uint32_t r = rank_in_wave(ins);
      const uint32_t tot = (uint32_t)__popcll(__ballot(ins));
      if (ins) {
        c.nbr[dst + written + r] = (uint32_t)keys[i];
        wset(c, dst + written + r, delta[i]);
      }
      written += tot;
    }
    if (lane == 0) {
      c.off[row] = dst;
      c.cap[row] = plan_cap[j];
      c.deg[row] = written;
      rowdel[row] = 0;
      rowins[row] = 0;
    }
  }
}

__global__ void k_csr_degrees(int64_t* kout, int64_t* kin, const uint64_t* keys, const int64_t* delta, uint64_t k) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const int64_t d = delta[i];
    if (d == 0) continue;
    atomic_add_i64(&kout[keys[i] >> 32], d);
    if (kin) atomic_add_i64(&kin[(uint32_t)keys[i]], d);
  }
}

__global__ void k_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    uint64_t d = deg[u];
    uint64_t nc = d + (d >> 2);
    if (nc < d + 2) nc = d + 2;
    if (nc > 0xFFFFFFFFull) nc = 0xFFFFFFFFull;
    newcap[u] = (uint32_t)nc;
    newcap64[u] = nc;
  }
}

__global__ void k_csr_move_rows(CsrRef from, CsrRef to, const uint64_t* new_off, const uint32_t* new_cap,
                                uint32_t n) {
  const int lane = lane_id();
  for (uint64_t u = gwave(); u < n; u += gwstride()) {
    const uint64_t s = from.off[u], d = new_off[u];
    const uint32_t deg = from.deg[u];
    for (uint32_t i = lane; i < deg; i += kWave) {
      to.nbr[d + i] = from.nbr[s + i];
      wset(to, d + i, wget(from, s + i));
    }
    if (lane == 0) {
      to.off[u] = d;
      to.cap[u] = new_cap[u];
      to.deg[u] = deg;
    }
  }
}

__global__ void k_csr_entries(CsrRef c, uint32_t n, uint64_t* out_keys, int64_t* out_w, u64a* counter) {
  const int lane = lane_id();
  for (uint64_t u = gwave(); u < n; u += gwstride()) {
    const uint64_t o = c.off[u];
    const uint32_t deg = c.deg[u];
    u64a base = 0;
    if (lane == 0 && deg) base = atomicAdd(counter, (u64a)deg);
    base = __shfl(base, 0, kWave);
    for (uint32_t i = lane; i < deg; i += kWave) {
      out_keys[base + i] = ((uint64_t)u << 32) | c.nbr[o + i];
      out_w[base + i] = wget(c, o + i);
    }
  }
}

// ------------------------------------------------------------------ batch ingest

__global__ void k_ingest_records(const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd,
                                 const uint32_t* chg, uint64_t nc, uint32_t n, int directed, uint64_t* keys,
                                 uint32_t* idx, uint32_t* err) {
  const uint64_t total = ni + nd + nc;
  for (uint64_t i = gtid(); i < total; i += gstride()) {
    uint32_t u, v, w;
    bool needw;
    if (i < ni) {
      u = ins[3 * i]; v = ins[3 * i + 1]; w = ins[3 * i + 2]; needw = true;
    } else if (i < ni + nd) {
      const uint64_t j = i - ni;
      u = del[2 * j]; v = del[2 * j + 1]; w = 1; needw = false;
    } else {
      const uint64_t j = i - ni - nd;
      u = chg[3 * j]; v = chg[3 * j + 1]; w = chg[3 * j + 2]; needw = true;
    }
    if (u >= n || v >= n || (needw && w == 0)) {
      atomicOr(err, 1u);
      u = 0; v = 0;
    }
    if (!directed && u > v) { uint32_t t = u; u = v; v = t; }
    keys[i] = ((uint64_t)u << 32) | v;
    idx[i] = (uint32_t)i;
  }
}

// wave per sorted record: duplicate check, existing weight, delta and validation
__global__ void k_ingest_check(CsrRef out0, const uint64_t* keys, const uint32_t* idx, uint64_t k,
                               const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd,
                               const uint32_t* chg, int directed, int64_t* delta, uint32_t* err,
                               uint32_t* first_bad, i64a* dm) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < k; i += gwstride()) {
    const uint64_t key = keys[i];
    if (lane == 0 && i > 0 && keys[i - 1] == key) atomicOr(err, 2u);
    const uint32_t u = (uint32_t)(key >> 32), v = (uint32_t)key;
    const uint64_t o = out0.off[u];
    const uint32_t deg = out0.deg[u];
    int64_t slot = -1;
    for (uint32_t base = 0; base < deg; base += kWave) {
      const uint32_t j = base + lane;
      const bool hit = j < deg && out0.nbr[o + j] == v;
      const uint64_t m = __ballot(hit);
      if (m) {
        slot = (int64_t)(o + base + (uint32_t)__ffsll((long long)m) - 1);
        break;
      }
    }
    if (lane != 0) continue;
    const uint32_t src = idx[i];
    const int64_t old = slot >= 0 ? (int64_t)((const uint32_t*)out0.w)[slot] : 0;
    int64_t d = 0;
    bool bad = false;
    if (src < ni) {
      const int64_t w = ins[3 * (uint64_t)src + 2];
      if (old + w > 0xFFFFFFFFll) { bad = true; atomicOr(err, 8u); }
      d = w;
    } else if (src < ni + nd) {
      if (slot < 0) { bad = true; atomicOr(err, 4u); }
      d = -old;
    } else {
      const int64_t w = chg[3 * ((uint64_t)src - ni - nd) + 2];
      if (slot < 0) { bad = true; atomicOr(err, 4u); }
      d = w - old;
    }
    if (bad) {
      atomicMin(first_bad, src);
      d = 0;
    }
    delta[i] = d;
    if (d != 0) atomicAdd((u64a*)dm, (u64a)((!directed && u != v) ? 2 * d : d));
  }
}

__global__ void k_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed,
                                 uint64_t* ekeys, int64_t* edelta, u64a* count) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const int64_t d = delta[i];
    if (d == 0) continue;
    const uint64_t key = keys[i];
    const uint32_t u = (uint32_t)(key >> 32), v = (uint32_t)key;
    const bool mirror = !directed && u != v;
    const u64a at = atomicAdd(count, (u64a)(mirror ? 2 : 1));
    ekeys[at] = key;
    edelta[at] = d;
    if (mirror) {
      ekeys[at + 1] = ((uint64_t)v << 32) | u;
      edelta[at + 1] = d;
    }
  }
}

__global__ void k_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                              const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = (uint32_t)(ekeys[i] >> 32), y = (uint32_t)ekeys[i];
    set_add(seeds0.stamp, seeds0.epoch, seeds0.list, seeds0.count, x);
    set_add(seeds0.stamp, seeds0.epoch, seeds0.list, seeds0.count, y);
    const uint32_t cs[2] = {lab0[x], lab0[y]};
    for (int t = 0; t < 2; ++t) {
      const uint32_t c = cs[t];
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

__global__ void k_ingest_totals(const uint64_t* ekeys, const int64_t* edelta, uint64_t k, const uint32_t* lab0,
                                int64_t* Kout, int64_t* Kin, i64a* dein) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = (uint32_t)(ekeys[i] >> 32), y = (uint32_t)ekeys[i];
    const int64_t d = edelta[i];
    const uint32_t cx = lab0[x], cy = lab0[y];
    atomic_add_i64(&Kout[cx], d);
    if (Kin) atomic_add_i64(&Kin[cy], d);
    if (cx == cy) atomicAdd((u64a*)dein, (u64a)d);
  }
}

__global__ void k_dskk(const uint32_t* touched, uint32_t nt, const int64_t* Kout, const int64_t* Kin,
                       const int64_t* tko, const int64_t* tki, u64a* lo, i64a* hi) {
  for (uint64_t t = gtid(); t < nt; t += gstride()) {
    const uint32_t c = touched[t];
    const i128 d = (i128)Kout[c] * Kin[c] - (i128)tko[t] * tki[t];
    if (d != 0) atomic_add_i128(lo, hi, d);
  }
}

__global__ void k_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                              uint64_t* keys, int64_t* vals, SetRef seeds) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = par[ex[i]], y = par[ey[i]];
    ex[i] = x;
    ey[i] = y;
    if (seeds.stamp) {
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, x);
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, y);
    }
    keys[i] = ((uint64_t)x << 32) | y;
    vals[i] = ed[i];
  }
}

__global__ void k_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    ex[i] = (uint32_t)(keys[i] >> 32);
    ey[i] = (uint32_t)keys[i];
  }
}

__global__ void k_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k) {
  for (uint64_t i = gtid(); i < k; i += gstride()) tkeys[i] = (keys[i] << 32) | (keys[i] >> 32);
}

// ------------------------------------------------------------------ refinement bookkeeping

__global__ void k_ref_init_top(uint32_t n, const uint8_t* alive, const int64_t* kout, const int64_t* kin,
                               int64_t* Krout, int64_t* Krin, uint32_t* rsize) {
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const bool a = alive[x] != 0;
    Krout[x] = a ? kout[x] : 0;
    if (Krin) Krin[x] = a ? kin[x] : 0;
    rsize[x] = a ? 1u : 0u;
  }
}

// phase 0: record the old parent and take the node out of it; phase 1: make it a singleton
__global__ void k_ref_reset(const uint32_t* R, uint32_t nr, uint32_t* par, uint32_t* oldpar, const int64_t* kout,
                            const int64_t* kin, int64_t* Krout, int64_t* Krin, uint32_t* rsize, int phase) {
  for (uint64_t i = gtid(); i < nr; i += gstride()) {
    const uint32_t u = R[i];
    if (phase == 0) {
      const uint32_t x = par[u];
      oldpar[u] = x;
      atomic_add_i64(&Krout[x], -kout[u]);
      if (Krin) atomic_add_i64(&Krin[x], -kin[u]);
      atomicSub(&rsize[x], 1u);
    } else {
      par[u] = u;
      atomic_add_i64(&Krout[u], kout[u]);
      if (Krin) atomic_add_i64(&Krin[u], kin[u]);
      atomicAdd(&rsize[u], 1u);
    }
  }
}

// ------------------------------------------------------------------ aggregate repair

__global__ void k_changed(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint32_t* oldpar,
                          SetRef C) {
  for (uint64_t i = gtid(); i < nr; i += gstride()) {
    const uint32_t u = rset[i];
    if (par[u] != oldpar[u]) set_add(C.stamp, C.epoch, C.list, C.count, u);
  }
}

__global__ void k_tuple_count(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, u64a* total) {
  u64a local = 0;
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t u = list[i];
    local += 2ull * ((u64a)out.deg[u] + (directed ? (u64a)in.deg[u] : (u64a)out.deg[u]));
  }
  if (local) atomicAdd(total, local);
}

// wave per node.  repair == 0 (materialise): one tuple (par(u), par(v), w) per out-entry.
// repair == 1: for u in C, each matrix entry incident to u once: (oldpar, oldpar, -w) and
// (par, par, +w); entries whose other end is also in C are taken from the out side only.
__global__ void k_tuples(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* par,
                         const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep, int repair, uint64_t* tkeys,
                         int64_t* tvals, u64a* tcount, uint64_t tcap, SetRef seeds) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < k; i += gwstride()) {
    const uint32_t u = list[i];
    const uint32_t pu = par[u];
    const uint32_t ou = repair ? oldpar[u] : pu;
    // out side
    {
      const uint64_t o = out.off[u];
      const uint32_t d = out.deg[u];
      for (uint32_t base = 0; base < d; base += kWave) {
        const uint32_t j = base + lane;
        const bool act = j < d;
        uint32_t v = 0;
        int64_t w = 0;
        if (act) {
          v = out.nbr[o + j];
          w = wget(out, o + j);
        }
        const uint32_t per = repair ? 2u : 1u;
        const uint32_t r = rank_in_wave(act);
        const uint32_t tot = (uint32_t)__popcll(__ballot(act));
        u64a at = 0;
        if (lane == 0 && tot) at = atomicAdd(tcount, (u64a)tot * per);
        at = __shfl(at, 0, kWave);
        if (act) {
          const uint32_t pv = par[v];
          const uint64_t pos = at + (u64a)r * per;
          if (!repair) {
            if (pos < tcap) {
              tkeys[pos] = ((uint64_t)pu << 32) | pv;
              tvals[pos] = w;
            }
          } else {
            const uint32_t ov = cstamp[v] == cep ? oldpar[v] : pv;
            if (pos + 1 < tcap) {
              tkeys[pos] = ((uint64_t)ou << 32) | ov;
              tvals[pos] = -w;
              tkeys[pos + 1] = ((uint64_t)pu << 32) | pv;
              tvals[pos + 1] = w;
            }
            set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, ov);
            set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, pv);
          }
        }
      }
    }
    if (!repair) continue;
    if (lane == 0) {
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, ou);
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, pu);
    }
    // in side: entries (v, u) with v outside C
    {
      const CsrRef& c = directed ? in : out;
      const uint64_t o = c.off[u];
      const uint32_t d = c.deg[u];
      for (uint32_t base = 0; base < d; base += kWave) {
        const uint32_t j = base + lane;
        bool act = j < d;
        uint32_t v = 0;
        int64_t w = 0;
        if (act) {
          v = c.nbr[o + j];
          w = wget(c, o + j);
          if (cstamp[v] == cep) act = false;
        }
        const uint32_t r = rank_in_wave(act);
        const uint32_t tot = (uint32_t)__popcll(__ballot(act));
        u64a at = 0;
        if (lane == 0 && tot) at = atomicAdd(tcount, (u64a)tot * 2);
        at = __shfl(at, 0, kWave);
        if (act) {
          const uint32_t pv = par[v];
          const uint64_t pos = at + (u64a)r * 2;
          if (pos + 1 < tcap) {
            tkeys[pos] = ((uint64_t)pv << 32) | ou;
            tvals[pos] = -w;
            tkeys[pos + 1] = ((uint64_t)pv << 32) | pu;
            tvals[pos + 1] = w;
          }
          set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, pv);
        }
      }
    }
  }
}

// liveness of level-(r+1) candidates from child counts; revivals get an identity parent
// (when the level has one) and their child's label
__global__ void k_live_update(const uint32_t* cand, uint32_t k, const uint32_t* rsize_below, uint8_t* alive,
                              uint32_t* par, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                              SetRef revived) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = cand[i];
    const uint8_t a = rsize_below[x] > 0 ? 1 : 0;
    if (a == alive[x]) continue;
    alive[x] = a;
    if (a) {
      if (par) par[x] = x;
      lab[x] = lab_below[x];
      set_add(revived.stamp, revived.epoch, revived.list, revived.count, x);
    } else {
      set_add(died.stamp, died.epoch, died.list, died.count, x);
    }
  }
}

__global__ void k_live_prop(const uint32_t* died, uint32_t nd, const uint32_t* revived, uint32_t nr,
                            const uint32_t* par, uint32_t* rsize, SetRef cand) {
  for (uint64_t i = gtid(); i < (uint64_t)nd + nr; i += gstride()) {
    if (i < nd) {
      const uint32_t y = par[died[i]];
      atomicSub(&rsize[y], 1u);
      set_add(cand.stamp, cand.epoch, cand.list, cand.count, y);
    } else {
      const uint32_t x = revived[i - nd];
      atomicAdd(&rsize[x], 1u);
      set_add(cand.stamp, cand.epoch, cand.list, cand.count, x);
    }
  }
}

__global__ void k_label_up(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint8_t* alive_up,
                           const uint32_t* lab, uint32_t* lab_up) {
  for (uint64_t i = gtid(); i < nr; i += gstride()) {
    const uint32_t x = par[rset[i]];
    if (alive_up[x]) lab_up[x] = lab[x];
  }
}

__global__ void k_alive_list(uint32_t n, const uint8_t* alive, SetRef set) {
  for (uint64_t x = gtid(); x < n; x += gstride())
    if (alive[x]) set_add(set.stamp, set.epoch, set.list, set.count, (uint32_t)x);
}

__global__ void k_materialise_nodes(uint32_t n, const uint32_t* rsize, uint8_t* alive_up, const uint32_t* lab,
                                    uint32_t* lab_up, uint32_t* par_up) {
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const bool a = rsize[x] > 0;
    alive_up[x] = a ? 1 : 0;
    lab_up[x] = a ? lab[x] : (uint32_t)x;
    if (par_up) par_up[x] = (uint32_t)x;
  }
}

__global__ void k_label_refresh(uint32_t n, const uint8_t* alive, const uint32_t* par, const uint32_t* lab_up,
                                uint32_t* lab, SetRef seeds) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    if (!alive[u]) continue;
    const uint32_t nl = lab_up[par[u]];
    if (nl != lab[u]) {
      lab[u] = nl;
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, (uint32_t)u);
    }
  }
}

__global__ void k_recount_degrees(CsrRef c, uint32_t n, int64_t* deg_out) {
  const int lane = lane_id();
  for (uint64_t u = gwave(); u < n; u += gwstride()) {
    const uint64_t o = c.off[u];
    const uint32_t d = c.deg[u];
    int64_t s = 0;
    for (uint32_t i = lane; i < d; i += kWave) s += wget(c, o + i);
    s = wave_sum_i64(s);
    if (lane == 0) deg_out[u] = s;
  }
}

__global__ void k_mark_members(uint32_t* stamp, uint32_t ep, uint32_t n, const uint8_t* alive, const uint32_t* key,
                               const uint32_t* mark, uint32_t mark_ep) {
  for (uint64_t u = gtid(); u < n; u += gstride())
    if (alive[u] && mark[key[u]] == mark_ep) stamp[u] = ep;
}

// wave per listed vertex; plain stores (every writer stores the same epoch)
__global__ void k_mark_neighbours(uint32_t* stamp, uint32_t ep, const uint32_t* list, uint32_t count, CsrRef out,
                                  CsrRef in, int directed) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < count; i += gwstride()) {
    const uint32_t v = list[i];
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

__global__ void k_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t nr, const uint32_t* par,
                               const uint32_t* oldpar) {
  for (uint64_t i = gtid(); i < nr; i += gstride()) {
    const uint32_t u = rset[i];
    if (par[u] != oldpar[u]) stamp[u] = ep;
  }
}

// number of tuples node u emits (materialise: its out-entries; repair: twice its out-entries
// plus twice its in-side entries whose other end is outside C)
__global__ void k_tuple_counts(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed,
                               const uint32_t* cstamp, uint32_t cep, int repair, uint64_t* counts) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < k; i += gwstride()) {
    const uint32_t u = list[i];
    const uint32_t dout = out.deg[u];
    if (!repair) {
      if (lane == 0) counts[i] = dout;
      continue;
    }
    const CsrRef& c = directed ? in : out;
    const uint64_t o = c.off[u];
    const uint32_t d = c.deg[u];
    int64_t outside = 0;
    for (uint32_t j = lane; j < d; j += kWave) outside += cstamp[c.nbr[o + j]] != cep ? 1 : 0;
    outside = wave_sum_i64(outside);
    if (lane == 0) counts[i] = 2ull * dout + 2ull * (uint64_t)outside;
  }
}

// tuples of node list[i] written from offs[i] on, in entry order (see k_tuples)
__global__ void k_tuples_at(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed,
                            const uint32_t* par, const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep,
                            int repair, const uint64_t* offs, uint64_t* tkeys, int64_t* tvals, SetRef seeds) {
  const int lane = lane_id();
  for (uint64_t i = gwave(); i < k; i += gwstride()) {
    const uint32_t u = list[i];
    const uint32_t pu = par[u];
    const uint32_t ou = repair ? oldpar[u] : pu;
    uint64_t pos = offs[i];
    {
      const uint64_t o = out.off[u];
      const uint32_t d = out.deg[u];
      for (uint32_t j = lane; j < d; j += kWave) {
        const uint32_t v = out.nbr[o + j];
        const int64_t w = wget(out, o + j);
        const uint32_t pv = par[v];
        if (!repair) {
          tkeys[pos + j] = ((uint64_t)pu << 32) | pv;
          tvals[pos + j] = w;
        } else {
          const uint32_t ov = cstamp[v] == cep ? oldpar[v] : pv;
          tkeys[pos + 2 * j] = ((uint64_t)ou << 32) | ov;
          tvals[pos + 2 * j] = -w;
          tkeys[pos + 2 * j + 1] = ((uint64_t)pu << 32) | pv;
          tvals[pos + 2 * j + 1] = w;
          set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, ov);
          set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, pv);
        }
      }
      pos += repair ? 2ull * d : (uint64_t)d;
    }
    if (!repair) continue;
    if (lane == 0) {
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, ou);
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, pu);
    }
    const CsrRef& c = directed ? in : out;
    const uint64_t o = c.off[u];
    const uint32_t d = c.deg[u];
    for (uint32_t base = 0; base < d; base += kWave) {
      const uint32_t j = base + lane;
      bool act = j < d;
      uint32_t v = 0;
      int64_t w = 0;
      if (act) {
        v = c.nbr[o + j];
        w = wget(c, o + j);
        if (cstamp[v] == cep) act = false;
      }
      const uint32_t r = rank_in_wave(act);
      const uint32_t tot = (uint32_t)__popcll(__ballot(act));
      if (act) {
        const uint32_t pv = par[v];
        const uint64_t p2 = pos + 2ull * r;
        tkeys[p2] = ((uint64_t)pv << 32) | ou;
        tvals[p2] = -w;
        tkeys[p2 + 1] = ((uint64_t)pv << 32) | pu;
        tvals[p2 + 1] = w;
      }
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, act ? par[v] : 0u, act);
      pos += 2ull * tot;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_mark_members(uint32_t* stamp, uint32_t ep, uint32_t n, const uint8_t* alive, const uint32_t* key,
                         const uint32_t* mark, uint32_t mark_ep, hipStream_t s) {
  if (n) k_mark_members<<<grid_for(n), kTpb, 0, s>>>(stamp, ep, n, alive, key, mark, mark_ep);
}
void launch_mark_neighbours(uint32_t* stamp, uint32_t ep, const uint32_t* list, uint32_t count, CsrRef out, CsrRef in,
                            int directed, hipStream_t s) {
  if (count) k_mark_neighbours<<<grid_waves(count), kTpb, 0, s>>>(stamp, ep, list, count, out, in, directed);
}
void launch_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t nr, const uint32_t* par,
                         const uint32_t* oldpar, hipStream_t s) {
  if (nr) k_mark_changed<<<grid_for(nr), kTpb, 0, s>>>(stamp, ep, rset, nr, par, oldpar);
}
void launch_tuple_counts(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* cstamp,
                         uint32_t cep, int repair, uint64_t* counts, hipStream_t s) {
  if (k) k_tuple_counts<<<grid_waves(k), kTpb, 0, s>>>(list, k, out, in, directed, cstamp, cep, repair, counts);
}
void launch_tuples_at(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* par,
                      const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep, int repair, const uint64_t* offs,
                      uint64_t* tkeys, int64_t* tvals, SetRef seeds_or_null, hipStream_t s) {
  if (k)
    k_tuples_at<<<grid_waves(k), kTpb, 0, s>>>(list, k, out, in, directed, par, oldpar, cstamp, cep, repair, offs,
                                               tkeys, tvals, seeds_or_null);
}
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n) k_fill_u32<<<grid_for(n), kTpb, 0, s>>>(p, v, n);
}
void launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s) {
  if (n) k_fill_u8<<<grid_for(n), kTpb, 0, s>>>(p, v, n);
}
void launch_fill_i64(int64_t* p, int64_t v, uint64_t n, hipStream_t s) {
  if (n) k_fill_i64<<<grid_for(n), kTpb, 0, s>>>(p, v, n);
}
void launch_iota(uint32_t* p, uint64_t n, hipStream_t s) {
  if (n) k_iota<<<grid_for(n), kTpb, 0, s>>>(p, n);
}
void launch_copy_i64(int64_t* dst, const int64_t* src, uint64_t n, hipStream_t s) {
  if (n) k_copy_i64<<<grid_for(n), kTpb, 0, s>>>(dst, src, n);
}
void launch_set_add_list(SetRef set, const uint32_t* list, uint32_t count, hipStream_t s) {
  if (count) k_set_add_list<<<grid_for(count), kTpb, 0, s>>>(set, list, count);
}
void launch_set_add_mapped(SetRef set, const uint32_t* list, uint32_t count, const uint32_t* key,
                           const uint8_t* alive_or_null, hipStream_t s) {
  if (count) k_set_add_mapped<<<grid_for(count), kTpb, 0, s>>>(set, list, count, key, alive_or_null);
}
void launch_members(SetRef set, uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* mark,
                    uint32_t mark_epoch, hipStream_t s) {
  if (n) k_members<<<grid_for(n), kTpb, 0, s>>>(set, n, alive, key, mark, mark_epoch);
}
void launch_neighbours(SetRef set, const uint32_t* list, uint32_t count, CsrRef out, CsrRef in, int directed,
                       hipStream_t s) {
  if (count) k_neighbours<<<grid_waves(count), kTpb, 0, s>>>(set, list, count, out, in, directed);
}
void launch_csr_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, uint8_t* insflag,
                     uint32_t* rowdel, uint32_t* rowins, SetRef dirty, hipStream_t s) {
  if (k) k_csr_find<<<grid_waves(k), kTpb, 0, s>>>(c, keys, delta, k, insflag, rowdel, rowins, dirty);
}
void launch_segments(const uint64_t* keys, uint64_t k, uint64_t* seg_lo, uint32_t* nseg, hipStream_t s) {
  if (k) k_segments<<<grid_for(k), kTpb, 0, s>>>(keys, k, seg_lo, nseg);
}
void launch_seg_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                     const uint32_t* nseg_ptr, uint32_t nseg_max, int64_t* slot_out, uint8_t* insflag,
                     uint32_t* rowdel, uint32_t* rowins, SetRef dirty, int apply, hipStream_t s) {
  if (!k) return;
  unsigned g = nseg_max < 8192 ? (nseg_max ? nseg_max : 1) : 8192;
  if (apply)
    k_seg_find<1><<<g, 256, 0, s>>>(c, keys, delta, k, seg_lo, nseg_ptr, slot_out, insflag, rowdel, rowins, dirty);
  else
    k_seg_find<0><<<g, 256, 0, s>>>(c, keys, delta, k, seg_lo, nseg_ptr, slot_out, insflag, rowdel, rowins, dirty);
}
void launch_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot, uint64_t k,
                            const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                            int directed, int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm,
                            hipStream_t s) {
  if (k)
    k_ingest_validate<<<grid_for(k), kTpb, 0, s>>>(out0, keys, idx, slot, k, ins, ni, del, nd, chg, directed, delta,
                                                   err, first_bad, dm);
}
void launch_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo, const uint32_t* nseg_ptr,
                       uint64_t* seg_hi, uint64_t* items, uint64_t* item_off, int64_t* slot_out, void** tmp,
                       size_t* tmp_bytes, hipStream_t s) {
  if (!k) return;
  k_seg_items<<<grid_for(k + 1), kTpb, 0, s>>>(c, keys, k, seg_lo, nseg_ptr, seg_hi, items);
  prim_exclusive_sum_u64(tmp, tmp_bytes, items, item_off, k + 1, s);
  k_fill_i64_dev<<<grid_for(k), kTpb, 0, s>>>(slot_out, -1, k);
  const unsigned g = k < 8192 ? (unsigned)k : 8192u;
  k_seg_lookup<<<g, 256, 0, s>>>(c, keys, k, seg_lo, seg_hi, nseg_ptr, item_off, slot_out);
}
void launch_seg_apply(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                      const uint64_t* seg_hi, const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* insflag,
                      uint32_t* rowdel, uint32_t* rowins, int64_t* deg_arr, uint32_t* dirty_list, uint32_t* dirty_count,
                      hipStream_t s) {
  if (!k) return;
  const unsigned g = k < 8192 ? (unsigned)k : 8192u;
  k_seg_apply<<<g, 256, 0, s>>>(c, keys, delta, seg_lo, seg_hi, nseg_ptr, slot, insflag, rowdel, rowins, deg_arr,
                                dirty_list, dirty_count);
}
void launch_csr_plan(CsrRef c, const uint32_t* dirty, uint32_t nd, const uint32_t* rowdel, const uint32_t* rowins,
                     uint64_t* plan_off, uint32_t* plan_cap, u64a* pool_top, uint64_t pool_cap, uint32_t* overflow,
                     hipStream_t s) {
  if (nd)
    k_csr_plan<<<grid_for(nd), kTpb, 0, s>>>(c, dirty, nd, rowdel, rowins, plan_off, plan_cap, pool_top, pool_cap,
                                             overflow);
}
void launch_csr_rewrite(CsrRef c, const uint32_t* dirty, uint32_t nd, uint32_t* rowdel, uint32_t* rowins,
                        const uint64_t* plan_off, const uint32_t* plan_cap, const uint64_t* keys, const int64_t* delta,
                        const uint8_t* insflag, uint64_t k, hipStream_t s) {
  if (nd)
    k_csr_rewrite<<<grid_waves(nd), kTpb, 0, s>>>(c, dirty, nd, rowdel, rowins, plan_off, plan_cap, keys, delta,
                                                  insflag, k);
}
void launch_csr_degrees(int64_t* kout, int64_t* kin_or_null, const uint64_t* keys, const int64_t* delta, uint64_t k,
                        hipStream_t s) {
  if (k) k_csr_degrees<<<grid_for(k), kTpb, 0, s>>>(kout, kin_or_null, keys, delta, k);
}
void launch_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n, hipStream_t s) {
  if (n) k_csr_newcap<<<grid_for(n), kTpb, 0, s>>>(deg, newcap, newcap64, n);
}
void launch_csr_move_rows(CsrRef from, CsrRef to, const uint64_t* new_off, const uint32_t* new_cap, uint32_t n,
                          hipStream_t s) {
  if (n) k_csr_move_rows<<<grid_waves(n), kTpb, 0, s>>>(from, to, new_off, new_cap, n);
}
void launch_csr_entries(CsrRef c, uint32_t n, uint64_t* out_keys, int64_t* out_w, u64a* counter, hipStream_t s) {
  if (n) k_csr_entries<<<grid_waves(n), kTpb, 0, s>>>(c, n, out_keys, out_w, counter);
}
void launch_ingest_records(const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                           uint64_t nc, uint32_t n, int directed, uint64_t* keys, uint32_t* idx, uint32_t* err,
                           hipStream_t s) {
  const uint64_t t = ni + nd + nc;
  if (t) k_ingest_records<<<grid_for(t), kTpb, 0, s>>>(ins, ni, del, nd, chg, nc, n, directed, keys, idx, err);
}
void launch_ingest_check(CsrRef out0, const uint64_t* keys, const uint32_t* idx, uint64_t k, const uint32_t* ins,
                         uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg, int directed,
                         int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm, hipStream_t s) {
  if (k)
    k_ingest_check<<<grid_waves(k), kTpb, 0, s>>>(out0, keys, idx, k, ins, ni, del, nd, chg, directed, delta, err,
                                                  first_bad, dm);
}
void launch_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed, uint64_t* ekeys,
                           int64_t* edelta, u64a* count, hipStream_t s) {
  if (k) k_ingest_entries<<<grid_for(k), kTpb, 0, s>>>(keys, delta, k, directed, ekeys, edelta, count);
}
void launch_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                        const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, hipStream_t s) {
  if (k) k_ingest_mark<<<grid_for(k), kTpb, 0, s>>>(ekeys, k, lab0, Kout, Kin, touched, tko, tki, seeds0);
}
void launch_ingest_totals(const uint64_t* ekeys, const int64_t* edelta, uint64_t k, const uint32_t* lab0,
                          int64_t* Kout, int64_t* Kin_or_null, i64a* dein, hipStream_t s) {
  if (k) k_ingest_totals<<<grid_for(k), kTpb, 0, s>>>(ekeys, edelta, k, lab0, Kout, Kin_or_null, dein);
}
void launch_dskk(const uint32_t* touched, uint32_t nt, const int64_t* Kout, const int64_t* Kin, const int64_t* tko,
                 const int64_t* tki, u64a* lo, i64a* hi, hipStream_t s) {
  if (nt) k_dskk<<<grid_for(nt), kTpb, 0, s>>>(touched, nt, Kout, Kin, tko, tki, lo, hi);
}
void launch_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                        uint64_t* keys, int64_t* vals, SetRef seeds, hipStream_t s) {
  if (k) k_cascade_map<<<grid_for(k), kTpb, 0, s>>>(ex, ey, ed, k, par, keys, vals, seeds);
}
void launch_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey, hipStream_t s) {
  if (k) k_split_keys<<<grid_for(k), kTpb, 0, s>>>(keys, k, ex, ey);
}
void launch_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k, hipStream_t s) {
  if (k) k_transpose_keys<<<grid_for(k), kTpb, 0, s>>>(keys, tkeys, k);
}
void launch_ref_init_top(uint32_t n, const uint8_t* alive, const int64_t* kout, const int64_t* kin, int64_t* Krout,
                         int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s) {
  if (n) k_ref_init_top<<<grid_for(n), kTpb, 0, s>>>(n, alive, kout, kin, Krout, Krin_or_null, rsize);
}
void launch_ref_reset(const uint32_t* R, uint32_t nr, uint32_t* par, uint32_t* oldpar, const int64_t* kout,
                      const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, int phase,
                      hipStream_t s) {
  if (nr) k_ref_reset<<<grid_for(nr), kTpb, 0, s>>>(R, nr, par, oldpar, kout, kin, Krout, Krin_or_null, rsize, phase);
}
void launch_changed(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint32_t* oldpar, SetRef C,
                    hipStream_t s) {
  if (nr) k_changed<<<grid_for(nr), kTpb, 0, s>>>(rset, nr, par, oldpar, C);
}
void launch_tuple_count(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, u64a* total,
                        hipStream_t s) {
  if (k) k_tuple_count<<<grid_for(k), kTpb, 0, s>>>(list, k, out, in, directed, total);
}
void launch_tuples(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* par,
                   const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep, int repair, uint64_t* tkeys,
                   int64_t* tvals, u64a* tcount, uint64_t tcap, SetRef seeds_or_null, hipStream_t s) {
  if (k)
    k_tuples<<<grid_waves(k), kTpb, 0, s>>>(list, k, out, in, directed, par, oldpar, cstamp, cep, repair, tkeys, tvals,
                                            tcount, tcap, seeds_or_null);
}
void launch_live_update(const uint32_t* cand, uint32_t k, const uint32_t* rsize_below, uint8_t* alive,
                        uint32_t* par_or_null, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                        SetRef revived, hipStream_t s) {
  if (k)
    k_live_update<<<grid_for(k), kTpb, 0, s>>>(cand, k, rsize_below, alive, par_or_null, lab, lab_below, died,
                                               revived);
}
void launch_live_prop(const uint32_t* died, uint32_t nd, const uint32_t* revived, uint32_t nr, const uint32_t* par,
                      uint32_t* rsize, SetRef cand, hipStream_t s) {
  if (nd + nr) k_live_prop<<<grid_for((uint64_t)nd + nr), kTpb, 0, s>>>(died, nd, revived, nr, par, rsize, cand);
}
void launch_label_up(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint8_t* alive_up,
                     const uint32_t* lab, uint32_t* lab_up, hipStream_t s) {
  if (nr) k_label_up<<<grid_for(nr), kTpb, 0, s>>>(rset, nr, par, alive_up, lab, lab_up);
}
void launch_alive_list(uint32_t n, const uint8_t* alive, SetRef set, hipStream_t s) {
  if (n) k_alive_list<<<grid_for(n), kTpb, 0, s>>>(n, alive, set);
}
void launch_materialise_nodes(uint32_t n, const uint32_t* rsize, uint8_t* alive_up, const uint32_t* lab,
                              uint32_t* lab_up, uint32_t* par_up_or_null, hipStream_t s) {
  if (n) k_materialise_nodes<<<grid_for(n), kTpb, 0, s>>>(n, rsize, alive_up, lab, lab_up, par_up_or_null);
}
void launch_label_refresh(uint32_t n, const uint8_t* alive, const uint32_t* par, const uint32_t* lab_up,
                          uint32_t* lab, SetRef seeds, hipStream_t s) {
  if (n) k_label_refresh<<<grid_for(n), kTpb, 0, s>>>(n, alive, par, lab_up, lab, seeds);
}
void launch_recount_degrees(CsrRef c, uint32_t n, int64_t* deg_out, hipStream_t s) {
  if (n) k_recount_degrees<<<grid_waves(n), kTpb, 0, s>>>(c, n, deg_out);
}

}  // namespace ldl
