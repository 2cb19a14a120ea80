// Graph-maintenance kernels: stamped sets, dynamic CSR edits, batch ingest and statistic
// repair (Algorithm 1), aggregate-repair tuples and hierarchy liveness (Eq. 3), label
// refresh.
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
// a list length given on the host (bound) or, when countp is set, read on the device and capped
__device__ __forceinline__ uint32_t list_len(const uint32_t* countp, uint32_t bound) {
  if (!countp) return bound;
  const uint32_t c = *countp;
  return c < bound ? c : bound;
}
// grid of a launch whose length may be read on the device (grid-stride loops)
inline unsigned list_grid(uint32_t bound, const uint32_t* countp) {
  const unsigned g = grid_for(bound);
  return countp && g > 1024u ? 1024u : g;
}

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

// rank of the calling thread among the block's threads with `pred` (thread order) and their
// total; every thread of the block calls it (lds: one word per wavefront)
__device__ __forceinline__ uint32_t block_rank(bool pred, uint32_t* lds, uint32_t& total) {
  const uint64_t m = __ballot(pred);
  const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) lds[w] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
    const uint32_t c = lds[i];
    if (i < w) before += c;
    tot += c;
  }
  total = tot;
  return before + r;
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
__global__ void k_set_add_mapped(SetRef set, const uint32_t* list, uint32_t bound, const uint32_t* countp,
                                 const uint32_t* key, const uint8_t* alive) {
  const uint32_t count = list_len(countp, bound);
  for (uint64_t i = gtid(); i < count; i += gstride()) {
    uint32_t x = list[i];
    if (alive && !alive[x]) continue;
    uint32_t k = key[x];
    if (set.list) set_add(set.stamp, set.epoch, set.list, set.count, k);
    else set_claim(set.stamp, set.epoch, k);
  }
}
// Row segments of sorted record keys: one entry (first record index) per distinct row.
__device__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key);

// ---- row lookup of sorted records.  The records of one row (a segment) go into an LDS hash
// table keyed by column and the row is streamed once per table, each entry probing it.  A
// segment of at most kSegChunk records is one table: its work items are (segment, row slice of
// kSlice entries), each taken by a single wavefront without workgroup barriers.  A longer
// segment is cut into tables of kBigChunk records, each streamed over the row by a 256-lane
// workgroup in slices of kBigSlice entries: O(degree x records / kBigChunk + records) per row.
constexpr uint32_t kSegChunk = 512;     // records of a wavefront table
constexpr uint32_t kSlice = 4096;       // row entries per wavefront item
constexpr uint32_t kSegSlots = 2 * kSegChunk;
constexpr uint32_t kBigChunk = 4096;    // records of a workgroup table
constexpr uint32_t kBigSlice = 16384;   // row entries per workgroup item

__global__ void k_seg_items(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo,
                            const uint32_t* nseg_ptr, uint64_t* seg_hi, uint64_t* items, uint64_t* items_big,
                            int ks) {
  const uint32_t nseg = *nseg_ptr;
  for (uint64_t s = gtid(); s <= k; s += gstride()) {
    if (s >= nseg) {
      items[s] = 0;
      items_big[s] = 0;
      continue;
    }
    const uint64_t lo = seg_lo[s];
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t hi = s + 1 < nseg ? seg_lo[s + 1] : k;   // heads are selected in key order
    seg_hi[s] = hi;
    const uint64_t deg = c.deg[row];
    if (hi - lo <= kSegChunk) {
      items[s] = deg == 0 ? 1 : (deg + kSlice - 1) / kSlice;
      items_big[s] = 0;
    } else {
      items[s] = 0;
      items_big[s] = (deg == 0 ? 1 : (deg + kBigSlice - 1) / kBigSlice) * ((hi - lo + kBigChunk - 1) / kBigChunk);
    }
  }
}

// largest s in [0, n] with off[s] <= it, for off non-decreasing with off[0] <= it < off[n]; a
// 64-ary search by the whole wavefront (every lane returns the same value)
__device__ __forceinline__ uint32_t wave_owner(const uint64_t* off, uint32_t n, uint64_t it) {
  uint32_t lo = 0, hi = n;   // off[lo] <= it < off[hi]
  const uint32_t lane = (uint32_t)lane_id();
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + kWave - 1) / kWave;
    const uint32_t p = lo + lane * step;
    const bool ok = p < hi && off[p] <= it;   // a prefix of the lanes, lane 0 always
    const uint64_t m = __ballot(ok);
    const uint32_t last = 63u - (uint32_t)__clzll((long long)m);
    const uint32_t nlo = lo + last * step;
    hi = nlo + step < hi ? nlo + step : hi;
    lo = nlo;
  }
  return lo;
}

// Row entries jb, jb + stride, ... (U of them, those below e1) probed against an LDS table of
// record columns: all U neighbour loads are issued before the first probe, so each lane keeps U
// loads in flight.  A found entry's slot goes to the record that holds its column.
constexpr int kStreamU = 4;
template <int U>
__device__ __forceinline__ void probe_entries(const uint32_t* nbr, uint64_t off, uint64_t jb, uint64_t stride,
                                              uint64_t e1, const uint32_t* tkey, const uint32_t* tval,
                                              uint32_t mask, int64_t* slot_out) {
  uint32_t xs[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t j = jb + (uint64_t)u * stride;
    xs[u] = j < e1 ? nbr[off + j] : 0u;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t j = jb + (uint64_t)u * stride;
    if (j >= e1) continue;
    const uint32_t x = xs[u];
    uint32_t h = hash32(x) & mask;
    for (;;) {
      const uint32_t kx = tkey[h];
      if (kx == kEmpty) break;
      if (kx == x) {
        slot_out[tval[h]] = (int64_t)(off + j);
        break;
      }
      h = (h + 1) & mask;
    }
  }
}

// wavefront per work item: LDS table of the item's record chunk, stream the item's row slice,
// write the slot of every record found (each record matches at most one entry)
__global__ __launch_bounds__(256) void k_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k,
                                                    const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                    const uint32_t* nseg_ptr, const uint64_t* item_off,
                                                    int64_t* slot_out, int ks) {
  __shared__ uint32_t tkey_s[256 / kWave][kSegSlots];
  __shared__ uint32_t tval_s[256 / kWave][kSegSlots];
  const int lane = lane_id();
  uint32_t* tkey = tkey_s[threadIdx.x / kWave];
  uint32_t* tval = tval_s[threadIdx.x / kWave];
  const uint32_t nseg = *nseg_ptr;
  const uint64_t total = item_off[nseg];
  for (uint64_t it = gwave(); it < total; it += gwstride()) {
    const uint32_t sg = wave_owner(item_off, nseg, it);
    const uint64_t sl = it - item_off[sg];
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t deg = c.deg[row];
    const uint64_t clo = lo;
    const uint32_t kk = (uint32_t)(hi - lo);   // at most kSegChunk (small segment)
    uint32_t size = 64;
    while (size < 2 * kk) size <<= 1;
    const uint32_t mask = size - 1;
    for (uint32_t i = lane; i < size; i += kWave) tkey[i] = kEmpty;
    wave_sync();
    for (uint32_t i = lane; i < kk; i += kWave) {
      const uint32_t col = kcol(keys[clo + i], ks);
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
    wave_sync();
    const uint64_t off = c.off[row];
    const uint64_t e0 = sl * kSlice;
    const uint64_t e1 = e0 + kSlice < deg ? e0 + kSlice : deg;
    for (uint64_t jb = e0 + lane; jb < e1; jb += kStreamU * kWave)
      probe_entries<kStreamU>(c.nbr, off, jb, kWave, e1, tkey, tval, mask, slot_out + clo);
    wave_sync();   // table reads done before the next item clears it
  }
}

// workgroup per big-segment item: LDS table of a kBigChunk-record chunk, stream one row slice
__global__ __launch_bounds__(256) void k_seg_lookup_big(CsrRef c, const uint64_t* keys, uint64_t k,
                                                        const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                        const uint32_t* nseg_ptr, const uint64_t* item_off,
                                                        int64_t* slot_out, int ks) {
  __shared__ uint32_t tkey[2 * kBigChunk];
  __shared__ uint32_t tval[2 * kBigChunk];
  const uint32_t nseg = *nseg_ptr;
  const uint64_t total = item_off[nseg];
  for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const uint32_t sg = wave_owner(item_off, nseg, it);   // every wavefront finds the same segment
    const uint64_t sub = it - item_off[sg];
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t deg = c.deg[row];
    const uint64_t nsl = deg == 0 ? 1 : (deg + kBigSlice - 1) / kBigSlice;
    const uint64_t rc = sub / nsl, sl = sub % nsl;
    const uint64_t clo = lo + rc * kBigChunk;
    const uint32_t kk = (uint32_t)((hi - clo) < (uint64_t)kBigChunk ? (hi - clo) : (uint64_t)kBigChunk);
    uint32_t size = 64;
    while (size < 2 * kk) size <<= 1;
    const uint32_t mask = size - 1;
    for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) tkey[i] = kEmpty;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) {
      const uint32_t col = kcol(keys[clo + i], ks);
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
    const uint64_t e0 = sl * kBigSlice;
    const uint64_t e1 = e0 + kBigSlice < deg ? e0 + kBigSlice : deg;
    for (uint64_t jb = e0 + threadIdx.x; jb < e1; jb += kStreamU * (uint64_t)blockDim.x)
      probe_entries<kStreamU>(c.nbr, off, jb, blockDim.x, e1, tkey, tval, mask, slot_out + clo);
    __syncthreads();
  }
}

// ---- in-place row update, O(records + deletions) per row.  Workgroup per segment (one row's
// records): apply every delta at its looked-up slot; a weight that reaches 0 is a deletion, a
// record without a slot an insertion.  When the new degree fits the row's capacity the row is
// repaired in place: with t0 = deg - ndel, the surviving entries among the last ndel slots
// move into the deletion holes below t0 (the two counts are equal), and insertions are
// written from t0 on.  Entry order within a row carries no meaning.  Rows that outgrow their
// capacity are listed for k_seg_move.
constexpr uint64_t kSegWaveMax = 1024;   // segments updated by one wavefront
constexpr int kSegTpb = 1024;            // threads of the workgroup that updates a larger segment

// Orders the global-memory accesses of one wavefront's lanes with respect to each other (a
// workgroup-scope fence waits for the wavefront's own stores; no other wavefront takes part).
__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
constexpr uint8_t kRecNone = 0, kRecUpd = 1, kRecDel = 2, kRecIns = 3;

__global__ __launch_bounds__(kSegTpb) void k_seg_update(CsrRef c, const uint64_t* keys, const int64_t* delta,
                                                     const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                     const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* rtype,
                                                     uint64_t* hole, int64_t* deg_arr, uint32_t* rowdel,
                                                     uint32_t* rowins, uint32_t* move_list, uint32_t* move_count, int ks) {
  __shared__ int64_t red[3 * (kSegTpb / kWave)];
  __shared__ uint32_t lds[kSegTpb / kWave];
  const uint32_t nseg = *nseg_ptr;
  for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    if (hi - lo <= kSegWaveMax) continue;   // k_seg_update_wave's segment
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t off = c.off[row];
    const uint32_t deg = c.deg[row];
    const uint32_t cap = c.cap[row];
    int64_t ndel = 0, nins = 0, dsum = 0;
    // four records per thread at a time: their deltas and slots, then the old weights at the slots
    // (the records of a segment have distinct columns, hence distinct slots)
    for (uint64_t ib = lo + threadIdx.x; ib < hi; ib += 4 * (uint64_t)blockDim.x) {
      int64_t dd[4], sl[4], ow[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t i = ib + (uint64_t)q * blockDim.x;
        dd[q] = 0;
        sl[q] = -1;
        if (i < hi) {
          dd[q] = delta[i];
          sl[q] = slot[i];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) ow[q] = (dd[q] != 0 && sl[q] >= 0) ? wget(c, (uint64_t)sl[q]) : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t i = ib + (uint64_t)q * blockDim.x;
        if (i >= hi) continue;
        const int64_t d = dd[q];
        dsum += d;
        uint8_t t = kRecNone;
        if (d != 0) {
          if (sl[q] >= 0) {
            const int64_t nw = ow[q] + d;
            wset(c, (uint64_t)sl[q], nw);
            t = nw == 0 ? kRecDel : kRecUpd;
            if (nw == 0) ++ndel;
          } else {
            t = kRecIns;
            ++nins;
          }
        }
        rtype[i] = t;
      }
    }
    ndel = wave_sum_i64(ndel);
    nins = wave_sum_i64(nins);
    dsum = wave_sum_i64(dsum);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) {
      red[3 * w] = ndel;
      red[3 * w + 1] = nins;
      red[3 * w + 2] = dsum;
    }
    __syncthreads();
    ndel = nins = dsum = 0;
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
      ndel += red[3 * q];
      nins += red[3 * q + 1];
      dsum += red[3 * q + 2];
    }
    if (threadIdx.x == 0 && deg_arr && dsum) deg_arr[row] += dsum;
    if (ndel + nins == 0) continue;                       // uniform over the workgroup
    const uint64_t ndeg = (uint64_t)deg - (uint64_t)ndel + (uint64_t)nins;
    if (ndeg > cap) {
      if (threadIdx.x == 0) {
        rowdel[row] = (uint32_t)ndel;
        rowins[row] = (uint32_t)nins;
        move_list[atomicAdd(move_count, 1u)] = sg;
      }
      continue;
    }
    const uint32_t t0 = deg - (uint32_t)ndel;
    // holes below t0, in record order (at most ndel <= hi - lo of them)
    uint32_t nh = 0;
    for (uint64_t b = lo; b < hi; b += blockDim.x) {
      const uint64_t i = b + threadIdx.x;
      bool f = false;
      uint64_t sl = 0;
      if (i < hi && rtype[i] == kRecDel) {
        sl = (uint64_t)slot[i];
        f = sl - off < t0;
      }
      uint32_t tot;
      const uint32_t r = block_rank(f, lds, tot);
      if (f) hole[lo + nh + r] = sl;
      nh += tot;
    }
    __syncthreads();
    // survivors among the last ndel slots fill the holes
    uint32_t ns = 0;
    for (uint32_t b = t0; b < deg; b += blockDim.x) {
      const uint32_t p = b + threadIdx.x;
      bool f = false;
      uint32_t x = 0;
      int64_t wv = 0;
      if (p < deg) {
        wv = wget(c, off + p);
        f = wv != 0;
        if (f) x = c.nbr[off + p];
      }
      uint32_t tot;
      const uint32_t r = block_rank(f, lds, tot);
      if (f && ns + r < nh) {
        const uint64_t dst = hole[lo + ns + r];
        c.nbr[dst] = x;
        wset(c, dst, wv);
      }
      ns += tot;
    }
    __syncthreads();
    // insertions from t0 on
    uint32_t ni = 0;
    for (uint64_t b = lo; b < hi; b += blockDim.x) {
      const uint64_t i = b + threadIdx.x;
      const bool f = i < hi && rtype[i] == kRecIns;
      uint32_t tot;
      const uint32_t r = block_rank(f, lds, tot);
      if (f) {
        const uint64_t dst = off + t0 + ni + r;
        c.nbr[dst] = kcol(keys[i], ks);
        wset(c, dst, delta[i]);
      }
      ni += tot;
    }
    if (threadIdx.x == 0) c.deg[row] = (uint32_t)ndeg;
    __syncthreads();
  }
}


// The same update with one wavefront per segment, for segments of at most kSegWaveMax records
// (the common case at aggregate levels): ranks come from ballots, no workgroup barrier.
__global__ __launch_bounds__(kTpb) void k_seg_update_wave(CsrRef c, const uint64_t* keys, const int64_t* delta,
                                                          const uint64_t* seg_lo, const uint64_t* seg_hi,
                                                          const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* rtype,
                                                          uint64_t* hole, int64_t* deg_arr, uint32_t* rowdel,
                                                          uint32_t* rowins, uint32_t* move_list, uint32_t* move_count,
                                                          int ks) {
  const int lane = lane_id();
  const uint32_t nseg = *nseg_ptr;
  for (uint64_t sg = gwave(); sg < nseg; sg += gwstride()) {
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    if (hi - lo > kSegWaveMax) continue;   // k_seg_update's segment
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t off = c.off[row];
    const uint32_t deg = c.deg[row];
    const uint32_t cap = c.cap[row];
    int64_t ndel = 0, nins = 0, dsum = 0;
    for (uint64_t i = lo + lane; i < hi; i += kWave) {
      const int64_t d = delta[i];
      const int64_t sl = slot[i];
      dsum += d;
      uint8_t t = kRecNone;
      if (d != 0) {
        if (sl >= 0) {
          const int64_t nw = wget(c, (uint64_t)sl) + d;
          wset(c, (uint64_t)sl, nw);
          t = nw == 0 ? kRecDel : kRecUpd;
          if (nw == 0) ++ndel;
        } else {
          t = kRecIns;
          ++nins;
        }
      }
      rtype[i] = t;
    }
    ndel = wave_sum_i64(ndel);
    nins = wave_sum_i64(nins);
    dsum = wave_sum_i64(dsum);
    wave_sync_global();                                  // weights and record types written above
    if (lane == 0 && deg_arr && dsum) deg_arr[row] += dsum;
    if (ndel + nins == 0) continue;                       // uniform over the wavefront
    const uint64_t ndeg = (uint64_t)deg - (uint64_t)ndel + (uint64_t)nins;
    if (ndeg > cap) {
      if (lane == 0) {
        rowdel[row] = (uint32_t)ndel;
        rowins[row] = (uint32_t)nins;
        move_list[atomicAdd(move_count, 1u)] = (uint32_t)sg;
      }
      continue;
    }
    const uint32_t t0 = deg - (uint32_t)ndel;
    // holes below t0, in record order (at most ndel <= hi - lo of them)
    uint32_t nh = 0;
    for (uint64_t b = lo; b < hi; b += kWave) {
      const uint64_t i = b + lane;
      bool f = false;
      uint64_t sl = 0;
      if (i < hi && rtype[i] == kRecDel) {
        sl = (uint64_t)slot[i];
        f = sl - off < t0;
      }
      const uint64_t m = __ballot(f);
      if (f) hole[lo + nh + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = sl;
      nh += (uint32_t)__popcll(m);
    }
    wave_sync_global();
    // survivors among the last ndel slots fill the holes
    uint32_t ns = 0;
    for (uint32_t b = t0; b < deg; b += kWave) {
      const uint32_t p = b + (uint32_t)lane;
      bool f = false;
      uint32_t x = 0;
      int64_t wv = 0;
      if (p < deg) {
        wv = wget(c, off + p);
        f = wv != 0;
        if (f) x = c.nbr[off + p];
      }
      const uint64_t m = __ballot(f);
      const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (f && ns + r < nh) {
        const uint64_t dst = hole[lo + ns + r];
        c.nbr[dst] = x;
        wset(c, dst, wv);
      }
      ns += (uint32_t)__popcll(m);
    }
    wave_sync_global();
    // insertions from t0 on
    uint32_t ni = 0;
    for (uint64_t b = lo; b < hi; b += kWave) {
      const uint64_t i = b + lane;
      const bool f = i < hi && rtype[i] == kRecIns;
      const uint64_t m = __ballot(f);
      if (f) {
        const uint64_t dst = off + t0 + ni + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        c.nbr[dst] = kcol(keys[i], ks);
        wset(c, dst, delta[i]);
      }
      ni += (uint32_t)__popcll(m);
    }
    if (lane == 0) c.deg[row] = (uint32_t)ndeg;
  }
}

// workgroup per listed row: a region of 1.25x its new degree is taken from the pool, the
// surviving entries and the insertions are copied there.  A row that finds the pool full
// stays listed (the caller grows the pool and launches again); done entries become kEmpty.
__global__ __launch_bounds__(kTpb) void k_seg_move(CsrRef c, const uint64_t* keys, const int64_t* delta,
                                                   const uint64_t* seg_lo, const uint64_t* seg_hi, const uint8_t* rtype,
                                                   const uint32_t* rowdel, const uint32_t* rowins, uint32_t* move_list,
                                                   const uint32_t* move_count, u64a* pool_top, uint64_t pool_cap,
                                                   uint32_t* overflow, int tight, int ks) {
  __shared__ uint32_t lds[kTpb / kWave];
  __shared__ uint64_t s_dst;
  const uint32_t nm = *move_count;
  for (uint32_t j = blockIdx.x; j < nm; j += gridDim.x) {
    const uint32_t sg = move_list[j];
    if (sg == kEmpty) continue;
    const uint64_t lo = seg_lo[sg], hi = seg_hi[sg];
    const uint32_t row = krow(keys[lo], ks);
    const uint64_t src = c.off[row];
    const uint32_t deg = c.deg[row];
    const uint64_t ndeg = (uint64_t)deg - rowdel[row] + rowins[row];
    uint64_t nc = tight ? ndeg : ndeg + (ndeg >> 2);
    if (!tight && nc < ndeg + 4) nc = ndeg + 4;
    if (nc > 0xFFFFFFFFull) nc = 0xFFFFFFFFull;
    __syncthreads();
    if (threadIdx.x == 0) {
      const u64a o = atomicAdd(pool_top, (u64a)nc);
      if (o + nc > pool_cap) {
        atomicOr(overflow, 1u);
        s_dst = ~0ull;
      } else {
        s_dst = o;
      }
    }
    __syncthreads();
    const uint64_t dst = s_dst;
    if (dst == ~0ull) continue;
    uint32_t written = 0;
    for (uint32_t b = 0; b < deg; b += blockDim.x) {
      const uint32_t p = b + threadIdx.x;
      bool f = false;
      uint32_t x = 0;
      int64_t wv = 0;
      if (p < deg) {
        wv = wget(c, src + p);
        f = wv != 0;
        if (f) x = c.nbr[src + p];
      }
      uint32_t tot;
      const uint32_t r = block_rank(f, lds, tot);
      if (f) {
        c.nbr[dst + written + r] = x;
        wset(c, dst + written + r, wv);
      }
      written += tot;
    }
    for (uint64_t b = lo; b < hi; b += blockDim.x) {
      const uint64_t i = b + threadIdx.x;
      const bool f = i < hi && rtype[i] == kRecIns;
      uint32_t tot;
      const uint32_t r = block_rank(f, lds, tot);
      if (f) {
        c.nbr[dst + written + r] = kcol(keys[i], ks);
        wset(c, dst + written + r, delta[i]);
      }
      written += tot;
    }
    if (threadIdx.x == 0) {
      c.off[row] = dst;
      c.cap[row] = (uint32_t)nc;
      c.deg[row] = written;
      move_list[j] = kEmpty;
    }
  }
}

__global__ void k_fill_i64_dev(int64_t* p, int64_t v, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// Per sorted ingest record: duplicate check, validation and delta from the looked-up slot.
__global__ void k_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot,
                                  uint64_t k, const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd,
                                  const uint32_t* chg, int directed, int64_t* delta, uint32_t* err,
                                  uint32_t* first_bad, i64a* dm, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t key = keys[i];
    if (i > 0 && keys[i - 1] == key) atomicOr(err, 2u);
    const uint32_t u = krow(key, ks), v = kcol(key, ks);
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

__device__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n, int tight) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    uint64_t d = deg[u];
    uint64_t nc = tight ? d : d + (d >> 2);
    if (!tight && nc < d + 2) nc = d + 2;
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
                                 uint32_t* idx, uint32_t* err, int ks) {
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
    keys[i] = kpack(u, v, ks);
    idx[i] = (uint32_t)i;
  }
}

__global__ void k_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed,
                                 uint64_t* ekeys, int64_t* edelta, u64a* count, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const int64_t d = delta[i];
    if (d == 0) continue;
    const uint64_t key = keys[i];
    const uint32_t u = krow(key, ks), v = kcol(key, ks);
    const bool mirror = !directed && u != v;
    const u64a at = atomicAdd(count, (u64a)(mirror ? 2 : 1));
    ekeys[at] = key;
    edelta[at] = d;
    if (mirror) {
      ekeys[at + 1] = kpack(v, u, ks);
      edelta[at + 1] = d;
    }
  }
}

__global__ void k_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                              const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = krow(ekeys[i], ks), y = kcol(ekeys[i], ks);
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
                                int64_t* Kout, int64_t* Kin, i64a* dein, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = krow(ekeys[i], ks), y = kcol(ekeys[i], ks);
    const int64_t d = edelta[i];
    const uint32_t cx = lab0[x], cy = lab0[y];
    atomic_add_i64(&Kout[cx], d);
    if (Kin) atomic_add_i64(&Kin[cy], d);
    if (cx == cy) atomicAdd((u64a*)dein, (u64a)d);
  }
}

__global__ void k_dskk(const uint32_t* touched, const uint32_t* nt_ptr, const int64_t* Kout, const int64_t* Kin,
                       const int64_t* tko, const int64_t* tki, u64a* lo, i64a* hi) {
  const uint32_t nt = *nt_ptr;
  i128 d = 0;
  for (uint64_t t = gtid(); t < nt; t += gstride()) {
    const uint32_t c = touched[t];
    d += (i128)Kout[c] * Kin[c] - (i128)tko[t] * tki[t];
  }
  d = wave_sum_i128(d);   // every lane of the wave is active here
  if ((threadIdx.x & (kWave - 1)) == 0 && d != 0) atomic_add_i128(lo, hi, d);
}

__global__ void k_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                              uint64_t* keys, int64_t* vals, SetRef seeds, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t x = par[ex[i]], y = par[ey[i]];
    ex[i] = x;
    ey[i] = y;
    if (seeds.stamp) {
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, x);
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, y);
    }
    keys[i] = kpack(x, y, ks);
    vals[i] = ed[i];
  }
}

// Degree deltas of records (row, col, d): out-degree of the row, and in-degree of the column
// when a separate in-degree array is given (directed graphs).  Deferred aggregate records often
// concentrate on a few rows (large communities), so each workgroup first sums its chunk per
// node in an LDS table and issues one global atomic per distinct node; a key that finds no free
// slot within kDegProbe probes goes straight to the global atomic.
constexpr uint32_t kDegSlots = 4096;
constexpr uint32_t kDegChunk = 8192;
constexpr int kDegProbe = 32;

__device__ __forceinline__ void deg_local_add(uint32_t* tk, u64a* tv, uint32_t key, int64_t d, int64_t* glob) {
  uint32_t h = hash32(key) & (kDegSlots - 1);
  for (int p = 0; p < kDegProbe; ++p) {
    const uint32_t prev = atomicCAS(&tk[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&tv[h], (u64a)d);
      return;
    }
    h = (h + 1) & (kDegSlots - 1);
  }
  atomic_add_i64(&glob[key], d);
}

__global__ __launch_bounds__(kTpb) void k_record_degrees(const uint64_t* keys, const int64_t* vals, uint64_t k,
                                                         int64_t* kout, int64_t* kin, int ks) {
  __shared__ uint32_t rk[kDegSlots];
  __shared__ u64a rv[kDegSlots];
  __shared__ uint32_t ck[kDegSlots];
  __shared__ u64a cv[kDegSlots];
  for (uint64_t c0 = (uint64_t)blockIdx.x * kDegChunk; c0 < k; c0 += (uint64_t)gridDim.x * kDegChunk) {
    for (uint32_t t = threadIdx.x; t < kDegSlots; t += blockDim.x) {
      rk[t] = kEmpty;
      rv[t] = 0;
      if (kin) {
        ck[t] = kEmpty;
        cv[t] = 0;
      }
    }
    __syncthreads();
    const uint64_t c1 = c0 + kDegChunk < k ? c0 + kDegChunk : k;
    // four records per thread at a time, all loaded before the first is added
    for (uint64_t ib = c0 + threadIdx.x; ib < c1; ib += 4 * (uint64_t)blockDim.x) {
      int64_t ds[4];
      uint64_t kk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t i = ib + (uint64_t)q * blockDim.x;
        ds[q] = 0;
        kk[q] = 0;
        if (i < c1) {
          ds[q] = vals[i];
          kk[q] = keys[i];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (ds[q] == 0) continue;
        deg_local_add(rk, rv, krow(kk[q], ks), ds[q], kout);
        if (kin) deg_local_add(ck, cv, kcol(kk[q], ks), ds[q], kin);
      }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < kDegSlots; t += blockDim.x) {
      if (rk[t] != kEmpty && rv[t]) atomic_add_i64(&kout[rk[t]], (int64_t)rv[t]);
      if (kin && ck[t] != kEmpty && cv[t]) atomic_add_i64(&kin[ck[t]], (int64_t)cv[t]);
    }
    __syncthreads();
  }
}
__global__ void k_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    ex[i] = krow(keys[i], ks);
    ey[i] = kcol(keys[i], ks);
  }
}

__global__ void k_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) tkeys[i] = kpack(kcol(keys[i], ks), krow(keys[i], ks), ks);
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
__global__ void k_ref_reset(const uint32_t* R, uint32_t bound, const uint32_t* countp, uint32_t* par,
                            uint32_t* oldpar, const int64_t* kout, const int64_t* kin, int64_t* Krout, int64_t* Krin,
                            uint32_t* rsize, int phase) {
  const uint32_t nr = list_len(countp, bound);
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

// liveness of level-(r+1) candidates from child counts; revivals get an identity parent
// (when the level has one) and their child's label
__global__ void k_live_update(const uint32_t* cand, uint32_t bound, const uint32_t* countp, const uint32_t* rsize_below,
                              uint8_t* alive, uint32_t* par, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                              SetRef revived) {
  const uint32_t k = list_len(countp, bound);
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

// alive nodes not yet in the set join it; every id is read by one thread only, so its stamp is
// tested and set without atomics, and each workgroup reserves its list slots with one atomic
__global__ __launch_bounds__(kTpb) void k_alive_list(uint32_t n, const uint8_t* alive, SetRef set) {
  __shared__ uint32_t lds[kTpb / kWave];
  __shared__ uint32_t s_base;
  for (uint64_t x0 = (uint64_t)blockIdx.x * kTpb; x0 < n; x0 += (uint64_t)gridDim.x * kTpb) {
    const uint64_t x = x0 + threadIdx.x;
    const bool add = x < n && alive[x] && set.stamp[x] != set.epoch;
    if (add) set.stamp[x] = set.epoch;
    uint32_t total = 0;
    const uint32_t r = block_rank(add, lds, total);
    if (threadIdx.x == 0 && total) s_base = atomicAdd(set.count, total);
    __syncthreads();
    if (add) set.list[s_base + r] = (uint32_t)x;
  }
}

// *count += alive nodes u < n whose key is marked (stamp[key[u]] == ep): the size of a frontier
// closure without listing it
__global__ void k_count_members(uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* stamp,
                                uint32_t ep, u64a* count) {
  uint64_t c = 0;
  for (uint64_t u = gtid(); u < n; u += gstride())
    if (alive[u] && stamp[key[u]] == ep) ++c;
  c = (uint64_t)wave_sum_i64((int64_t)c);
  if (lane_id() == 0 && c) atomicAdd(count, (u64a)c);
}

// Refresh: seeds = nodes with an entry; the intra-community weight of the singleton partition
// (the self-loops) and sum kout kin (exact), one wavefront per node
__global__ void k_refresh_scalars(CsrRef out, CsrRef in, uint32_t n, const int64_t* kout, const int64_t* kin,
                                  SetRef seeds, i64a* ein, u64a* skk_lo, i64a* skk_hi) {
  const int lane = lane_id();
  for (uint64_t u = gwave(); u < n; u += gwstride()) {
    const uint32_t d = out.deg[u];
    const uint64_t o = out.off[u];
    int64_t self = 0;
    for (uint32_t i = lane; i < d; i += kWave)
      if (out.nbr[o + i] == (uint32_t)u) self += wget(out, o + i);
    self = wave_sum_i64(self);
    if (lane == 0) {
      if (self) atomicAdd((u64a*)ein, (u64a)self);
      const i128 p = (i128)kout[u] * (i128)kin[u];
      if (p) atomic_add_i128(skk_lo, skk_hi, p);
      if (d || (in.off && in.deg[u])) seeds.stamp[u] = seeds.epoch;
    }
  }
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
    // the node's own words are read together; only the label gather depends on them
    const uint8_t al = alive[u];
    const uint32_t pu = par[u], lu = lab[u];
    if (!al) continue;
    const uint32_t nl = lab_up[pu];
    if (nl != lu) {
      lab[u] = nl;
      set_add(seeds.stamp, seeds.epoch, seeds.list, seeds.count, (uint32_t)u);
    }
  }
}

// *total += sum of a[0..n) (one atomic per wavefront)
__global__ void k_sum_u32(const uint32_t* a, uint32_t n, u64a* total) {
  uint64_t t = 0;
  for (uint64_t i = gtid(); i < n; i += gstride()) t += a[i];
  t = (uint64_t)wave_sum_i64((int64_t)t);
  if (lane_id() == 0 && t) atomicAdd(total, (u64a)t);
}

// kout_up[par[u]] += kout[u] (and kin) over the alive nodes u < n: degrees of the level above as
// sums over its children (zeroed beforehand)
__global__ void k_degrees_up(uint32_t n, const uint8_t* alive, const uint32_t* par, const int64_t* kout,
                             const int64_t* kin, int64_t* kout_up, int64_t* kin_up) {
  for (uint64_t u = gtid(); u < n; u += gstride()) {
    if (!alive[u]) continue;
    const uint32_t x = par[u];
    if (kout[u]) atomic_add_i64(&kout_up[x], kout[u]);
    if (kin_up && kin[u]) atomic_add_i64(&kin_up[x], kin[u]);
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
__global__ void k_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t bound,
                               const uint32_t* countp, const uint32_t* par, const uint32_t* oldpar) {
  const uint32_t nr = list_len(countp, bound);
  for (uint64_t i = gtid(); i < nr; i += gstride()) {
    const uint32_t u = rset[i];
    if (par[u] != oldpar[u]) stamp[u] = ep;
  }
}

// number of tuples node u emits (materialise: its out-entries; repair: twice its out-entries
// plus twice its in-side entries whose other end is outside C)
// ---- node lists split into wavefront items.  Node i of a list has s_i entries, its out
// entries followed by its in entries (when in.off is set); it is split into ceil(s_i / kItem)
// items and ioff is the exclusive prefix of the item counts.  Every wavefront takes a
// contiguous range of items (one binary search, then a linear walk), so a hub node is spread
// over many wavefronts and a run of small nodes over few.
__device__ __forceinline__ uint64_t node_slots(const CsrRef& out, const CsrRef& in, uint32_t u) {
  return (uint64_t)out.deg[u] + (in.off ? (uint64_t)in.deg[u] : 0ull);
}

// entry j of node u (out entries first)
__device__ __forceinline__ void node_entry(const CsrRef& out, const CsrRef& in, uint32_t u, uint32_t dout, uint64_t j,
                                           uint32_t& x, int64_t& w) {
  if (j < dout) {
    const uint64_t e = out.off[u] + j;
    x = out.nbr[e];
    w = wget(out, e);
  } else {
    const uint64_t e = in.off[u] + (j - dout);
    x = in.nbr[e];
    w = wget(in, e);
  }
}

// node i of a list, through an optional index list
__device__ __forceinline__ uint32_t list_node(const uint32_t* list, const uint32_t* idx, uint64_t i) {
  return idx ? list[idx[i]] : list[i];
}

// ---- item counts and their exclusive prefix over positions [0, cnt] of a list (cnt read on the
// device): a fixed grid of kScanBlocks workgroups, each owning one contiguous chunk of at least
// kScanMinChunk positions, writes the counts and its chunk's sum, then a second launch scans each
// chunk offset by the sums of the chunks before it.  The work follows the device count, not the
// host bound.
constexpr unsigned kScanBlocks = kItemScanBlocks;
constexpr uint64_t kScanMinChunk = 1024;
constexpr int kScanPer = 4;   // consecutive positions per thread in one scan tile

__device__ __forceinline__ void scan_chunk(uint32_t cnt, uint64_t& b0, uint64_t& b1) {
  const uint64_t total = (uint64_t)cnt + 1;
  uint64_t per = (total + kScanBlocks - 1) / kScanBlocks;
  if (per < kScanMinChunk) per = kScanMinChunk;
  b0 = (uint64_t)blockIdx.x * per;
  b1 = b0 + per < total ? b0 + per : total;
  if (b0 > b1) b0 = b1;
}

// sum over the workgroup; every thread calls it and gets the sum (lds: one word per wavefront)
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* lds) {
  v = (uint64_t)wave_sum_i64((int64_t)v);
  __syncthreads();
  if (lane_id() == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  uint64_t t = 0;
  for (unsigned w = 0; w < blockDim.x / kWave; ++w) t += lds[w];
  return t;
}

// inclusive prefix over the workgroup in thread order, and the workgroup total; every thread calls it
__device__ __forceinline__ uint64_t block_incl_scan_u64(uint64_t v, uint64_t* lds, uint64_t& total) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t t = (uint64_t)__shfl_up((long long)v, o, kWave);
    if (lane >= o) v += t;
  }
  const unsigned me = threadIdx.x / kWave;
  __syncthreads();
  if (lane == kWave - 1) lds[me] = v;
  __syncthreads();
  uint64_t before = 0;
  total = 0;
  for (unsigned w = 0; w < blockDim.x / kWave; ++w) {
    if (w < me) before += lds[w];
    total += lds[w];
  }
  return v + before;
}

__global__ __launch_bounds__(kTpb) void k_item_counts(const uint32_t* list, const uint32_t* idx,
                                                      const uint32_t* countp, uint32_t bound, CsrRef out, CsrRef in,
                                                      uint64_t* icnt, uint64_t* zero_a, uint64_t* zero_b,
                                                      uint64_t* csum) {
  __shared__ uint64_t lds[kTpb / kWave];
  const uint32_t cnt = list_len(countp, bound);
  uint64_t b0, b1;
  scan_chunk(cnt, b0, b1);
  uint64_t sum = 0;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    uint64_t c = 0;
    if (i < cnt) c = (node_slots(out, in, list_node(list, idx, i)) + kItem - 1) / kItem;
    icnt[i] = c;
    sum += c;
    if (zero_a) zero_a[i] = 0;
    if (zero_b) zero_b[i] = 0;
  }
  sum = block_sum_u64(sum, lds);
  if (threadIdx.x == 0) csum[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kTpb) void k_item_offsets(const uint32_t* countp, uint32_t bound, const uint64_t* icnt,
                                                       const uint64_t* csum, uint64_t* ioff) {
  __shared__ uint64_t lds[kTpb / kWave];
  const uint32_t cnt = list_len(countp, bound);
  uint64_t b0, b1;
  scan_chunk(cnt, b0, b1);
  if (b0 >= b1) return;   // the whole workgroup: its chunk is empty (so are those after it)
  uint64_t pre = 0;
  for (unsigned j = threadIdx.x; j < blockIdx.x; j += blockDim.x) pre += csum[j];
  pre = block_sum_u64(pre, lds);
  const uint64_t tile = (uint64_t)blockDim.x * kScanPer;
  for (uint64_t base = b0; base < b1; base += tile) {
    const uint64_t i0 = base + (uint64_t)threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = i0 + k < b1 ? icnt[i0 + k] : 0;
      mine += v[k];
    }
    uint64_t total = 0;
    uint64_t run = pre + block_incl_scan_u64(mine, lds, total) - mine;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < b1) ioff[i0 + k] = run;
      run += v[k];
    }
    pre += total;
  }
}

// f(i, q): item q of list node i; called with the whole wavefront
template <class F>
__device__ __forceinline__ void wave_items(const uint64_t* ioff, uint32_t cnt, F&& f) {
  const uint64_t total = ioff[cnt];
  const uint64_t W = gwstride();
  const uint64_t per = (total + W - 1) / W;
  uint64_t it = gwave() * per;
  const uint64_t end = it + per < total ? it + per : total;
  if (it >= end) return;
  uint32_t lo = 0, hi = cnt;   // ioff[lo] <= it < ioff[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ioff[mid] <= it) lo = mid;
    else hi = mid;
  }
  uint32_t i = lo;
  for (; it < end; ++it) {
    while (ioff[i + 1] <= it) ++i;
    f(i, it - ioff[i]);
  }
}

// stamp[x] = ep for every listed node (with or without entries) and each of its entries'
// neighbours
__global__ void k_mark_items(uint32_t* stamp, uint32_t ep, const uint32_t* list, const uint32_t* countp, uint32_t bound,
                             const uint64_t* ioff, CsrRef out, CsrRef in, uint32_t pull_from) {
  const int lane = lane_id();
  const uint32_t c0 = *countp;
  if (c0 >= pull_from) return;   // a dense list: k_mark_pull builds the set instead
  const uint32_t cnt = c0 < bound ? c0 : bound;
  for (uint64_t i = gtid(); i < cnt; i += gstride()) stamp[list[i]] = ep;
  if (c0 >= bound) return;   // every id of [0, bound) is listed: the neighbours are listed nodes
  wave_items(ioff, cnt, [&](uint32_t i, uint64_t q) {
    const uint32_t u = list[i];
    const uint32_t dout = out.deg[u];
    const uint64_t s = node_slots(out, in, u);
    const uint64_t j0 = q * kItem, j1 = j0 + kItem < s ? j0 + kItem : s;
    // four neighbour loads in flight per lane before their stamps are written
    for (uint64_t jb = j0 + lane; jb < j1; jb += 4 * kWave) {
      uint32_t xs[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = jb + (uint64_t)k * kWave;
        xs[k] = 0;
        if (j < j1) xs[k] = j < dout ? out.nbr[out.off[u] + j] : in.nbr[in.off[u] + (j - dout)];
      }
      // neighbours shared by many listed nodes are stamped once: a stamp already set is not
      // written again, so its cache line stays clean
      uint32_t cur[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[k] = jb + (uint64_t)k * kWave < j1 ? stamp[xs[k]] : ep;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (cur[k] != ep) stamp[xs[k]] = ep;
    }
  });
}

// The same set pulled instead of pushed, for a dense list (at least pull_from nodes; the list is
// the nodes whose ustamp equals uep): an alive node x joins when it is listed or when one of its
// out- or in-neighbours is (the in-rows hold the transpose, so x is a neighbour of a listed u iff
// u is a neighbour of x).  Each node stops reading its rows at the first listed neighbour, so a
// dense list costs about one gather per node instead of a write per entry of every listed node.
__global__ void k_mark_pull(uint32_t* stamp, uint32_t ep, const uint32_t* ustamp, uint32_t uep,
                            const uint32_t* countp, uint32_t pull_from, uint32_t n, const uint8_t* alive, CsrRef out,
                            CsrRef in) {
  if (*countp < pull_from) return;
  const int lane = lane_id();
  // one wavefront per node: 64 entries per step, a ballot ends the walk at the first listed one
  // (a long row of a node with few listed neighbours is read by the whole wavefront, not one lane)
  for (uint64_t x = gwave(); x < n; x += gwstride()) {
    if (!alive[x]) continue;
    bool hit = ustamp[x] == uep;
    const uint32_t dout = out.deg[x];
    const uint64_t s = node_slots(out, in, (uint32_t)x);
    for (uint64_t jb = 0; jb < s && !hit; jb += kWave) {
      const uint64_t j = jb + lane;
      bool h = false;
      if (j < s) {
        const uint32_t y = j < dout ? out.nbr[out.off[x] + j] : in.nbr[in.off[x] + (j - dout)];
        h = ustamp[y] == uep;
      }
      hit = __ballot(h) != 0;
    }
    if (hit && lane == 0) stamp[x] = ep;
  }
}

// Subtract-add tuples of Eq. 3.  Materialise (REPAIR false): (P(u), P(x), w) for every out entry.
// Repair over the changed nodes C (cstamp == cep): for an out entry (u, x) of u in C, the
// old pair (oldpar u, oldpar x) loses w and the new pair (par u, par x) gains it (x outside C
// keeps its parent); for an in entry (v, u) with v outside C, (par v, oldpar u) loses w and
// (par v, par u) gains it (entries between two C nodes come from the out side).  Node i's
// tuples start at toffs[i]: out tuples in entry order, then in tuples at a per-node cursor.
// po[x] = (pi(x), old pi(x) if x changed parent else pi(x)): the neighbour's both parents in one
// gather for the repair tuples (x changed iff the two differ)
__global__ void k_pack_parents(uint32_t n, const uint32_t* par, const uint32_t* oldpar, const uint32_t* cstamp,
                               uint32_t cep, uint2* po) {
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const uint32_t p = par[x];
    po[x] = make_uint2(p, cstamp[x] == cep ? oldpar[x] : p);
  }
}

template <bool REPAIR>
__global__ void k_tuples_count(const uint32_t* list, const uint32_t* countp, uint32_t bound, const uint64_t* ioff,
                               CsrRef out, CsrRef in, const uint2* po, u64a* counts) {
  const int lane = lane_id();
  const uint32_t c0 = *countp;
  const uint32_t cnt = c0 < bound ? c0 : bound;
  wave_items(ioff, cnt, [&](uint32_t i, uint64_t q) {
    const uint32_t u = list[i];
    const uint32_t dout = out.deg[u];
    const uint64_t s = node_slots(out, in, u);
    const uint64_t j0 = q * kItem, j1 = j0 + kItem < s ? j0 + kItem : s;
    int64_t c = 0;
    // four entries per lane at a time: the in-entries' neighbour loads, then their parent gathers
    for (uint64_t jb = j0 + lane; jb < j1; jb += 4 * kWave) {
      uint32_t xs[4];
      int kind[4];   // 0: past the item, 1: out entry, 2: in entry
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = jb + (uint64_t)k * kWave;
        kind[k] = j >= j1 ? 0 : (j < dout ? 1 : 2);
        xs[k] = kind[k] == 2 ? in.nbr[in.off[u] + (j - dout)] : 0u;
      }
      uint2 qs[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) qs[k] = kind[k] == 2 ? po[xs[k]] : make_uint2(0u, 0u);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (kind[k] == 1) c += REPAIR ? 2 : 1;
        else if (kind[k] == 2 && qs[k].x == qs[k].y) c += 2;   // the neighbour keeps its parent
      }
    }
    c = wave_sum_i64(c);
    if (lane == 0 && c) atomicAdd(&counts[i], (u64a)c);
  });
}

// WRITE = false (repair only): no tuples are written, only the seeds their endpoints would mark
// (used when the level above is rebuilt from scratch instead of repaired).
template <bool REPAIR, bool WRITE>
__global__ void k_tuples_gen(const uint32_t* list, const uint32_t* countp, uint32_t bound, const uint64_t* ioff,
                             CsrRef out, CsrRef in, const uint32_t* par, const uint2* po, const uint64_t* toffs,
                             u64a* cur, uint64_t* tkeys, int64_t* tvals, uint32_t* seed_stamp, uint32_t seed_ep,
                             int ks) {
  const int lane = lane_id();
  const uint32_t c0 = *countp;
  const uint32_t cnt = c0 < bound ? c0 : bound;
  wave_items(ioff, cnt, [&](uint32_t i, uint64_t q) {
    const uint32_t u = list[i];
    uint32_t pu, ou;
    if (REPAIR) {
      const uint2 qu = po[u];
      pu = qu.x;
      ou = qu.y;
    } else {
      pu = ou = par[u];
    }
    const uint32_t dout = out.deg[u];
    const uint64_t s = node_slots(out, in, u);
    const uint64_t j0 = q * kItem, j1 = j0 + kItem < s ? j0 + kItem : s;
    const uint64_t base = toffs[i];
    if (REPAIR && q == 0 && lane == 0) {
      seed_stamp[ou] = seed_ep;
      seed_stamp[pu] = seed_ep;
    }
    for (uint64_t jb = j0; jb < j1; jb += kWave) {   // wavefront-uniform steps
      const uint64_t j = jb + lane;
      const bool valid = j < j1;
      uint32_t x = 0;
      int64_t w = 0;
      if (valid) node_entry(out, in, u, dout, j, x, w);
      uint2 qx = make_uint2(0u, 0u);
      if (REPAIR && valid) qx = po[x];
      if (valid && j < dout) {
        if (!REPAIR) {
          const uint32_t px = par[x];
          tkeys[base + j] = kpack(pu, px, ks);
          tvals[base + j] = w;
        } else {
          const uint32_t px = qx.x, ox = qx.y;
          if (WRITE) {
            tkeys[base + 2 * j] = kpack(ou, ox, ks);
            tvals[base + 2 * j] = -w;
            tkeys[base + 2 * j + 1] = kpack(pu, px, ks);
            tvals[base + 2 * j + 1] = w;
          }
          seed_stamp[ox] = seed_ep;
          seed_stamp[px] = seed_ep;
        }
      }
      if (REPAIR && !WRITE && jb + kWave > dout) {
        if (valid && j >= dout && qx.x == qx.y) seed_stamp[qx.x] = seed_ep;
      } else if (REPAIR && jb + kWave > dout) {
        const bool act = valid && j >= dout && qx.x == qx.y;   // neighbour keeps its parent
        const uint64_t m = __ballot(act);
        if (m) {
          const uint32_t tot = (uint32_t)__popcll(m);
          const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
          u64a b = 0;
          if (lane == 0) b = atomicAdd(&cur[i], 2ull * tot);
          const uint32_t blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
          const uint32_t bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
          b = ((u64a)bhi << 32) | blo;
          if (act) {
            const uint32_t pv = qx.x;
            const uint64_t p2 = base + 2ull * dout + b + 2ull * r;
            tkeys[p2] = kpack(pv, ou, ks);
            tvals[p2] = -w;
            tkeys[p2 + 1] = kpack(pv, pu, ks);
            tvals[p2 + 1] = w;
            seed_stamp[pv] = seed_ep;
          }
        }
      }
    }
  });
}

// SPExpand over wavefront items of the refinement movers: their singleton neighbours with the
// mover's label join Rcur; those new to Rset join it too, with their old parent (themselves)
// recorded.  Plain-store marks (every writer of a word stores the same value); the lists
// come from a select.  Label and parent come from one packed (label, parent) gather.
__global__ void k_spexpand_items(const uint32_t* movers, const uint32_t* idx, const uint32_t* countp, uint32_t bound,
                                 const uint64_t* ioff, CsrRef out, CsrRef in, const uint2* lp, const uint32_t* rsize,
                                 uint32_t* rcur_stamp, uint32_t rcur_ep, uint32_t* rset_stamp, uint32_t rset_ep,
                                 uint32_t* oldpar) {
  const int lane = lane_id();
  const uint32_t c0 = *countp;
  const uint32_t cnt = c0 < bound ? c0 : bound;
  wave_items(ioff, cnt, [&](uint32_t i, uint64_t q) {
    const uint32_t v = list_node(movers, idx, i);
    const uint32_t lv = lp[v].x;
    const uint32_t dout = out.deg[v];
    const uint64_t s = node_slots(out, in, v);
    const uint64_t j0 = q * kItem, j1 = j0 + kItem < s ? j0 + kItem : s;
    // four entries per lane at a time: their neighbour loads, then their label gathers, then the
    // parent and size gathers of those in v's community, each group issued before any is used
    for (uint64_t jb = j0 + lane; jb < j1; jb += 4 * kWave) {
      uint32_t xs[4];
      bool ok[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = jb + (uint64_t)k * kWave;
        ok[k] = j < j1;
        xs[k] = v;
        if (ok[k]) xs[k] = j < dout ? out.nbr[out.off[v] + j] : in.nbr[in.off[v] + (j - dout)];
      }
      uint32_t px[4], rx[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint2 e = ok[k] && xs[k] != v ? lp[xs[k]] : make_uint2(~lv, 0u);
        ok[k] = e.x == lv;
        px[k] = e.y;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) rx[k] = ok[k] && px[k] == xs[k] ? rsize[xs[k]] : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t x = xs[k];
        if (!ok[k] || px[k] != x || rx[k] != 1) continue;
        rcur_stamp[x] = rcur_ep;
        if (rset_stamp[x] != rset_ep) {
          oldpar[x] = x;
          rset_stamp[x] = rset_ep;
        }
      }
    }
  });
}

// ------------------------------------------------------------------ bulk load
// An insert-only batch into a level-0 graph that has never held an entry (the first batch of a
// graph, batch ingest on the all-singleton state) builds its rows directly from the sorted
// records: the slot of a record is its row's first slot plus its rank within the row.

// Insert records of a bulk load: key (canonical pair for undirected graphs) and weight; an id
// >= n or a zero weight sets err bit 0
__global__ void k_bulk_records(const uint32_t* ins, uint64_t k, uint32_t n, int directed, uint64_t* keys,
                               uint32_t* wts, uint32_t* err, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    uint32_t u = ins[3 * i], v = ins[3 * i + 1];
    const uint32_t w = ins[3 * i + 2];
    if (u >= n || v >= n || w == 0) {
      atomicOr(err, 1u);
      u = 0;
      v = 0;
    }
    if (!directed && u > v) {
      const uint32_t t = u;
      u = v;
      v = t;
    }
    keys[i] = kpack(u, v, ks);
    wts[i] = w;
  }
}

// Sorted records: duplicate check (err bit 1) and the batch's matrix sum (each undirected pair
// u != v counts twice) into *dm as an unsigned sum.
__global__ void k_bulk_check(const uint64_t* keys, const uint32_t* wts, uint64_t k, int directed, uint32_t* err,
                             u64a* dm, int ks) {
  uint64_t sum = 0;
  bool dup = false;
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t key = keys[i];
    if (i > 0 && keys[i - 1] == key) dup = true;
    const uint32_t w = wts[i];
    sum += (!directed && krow(key, ks) != kcol(key, ks)) ? 2ull * w : (uint64_t)w;
  }
  // one atomic per workgroup (a launch of at most kItemBlocks workgroups)
  __shared__ uint64_t part[kTpb / kWave];
  __shared__ int pdup[kTpb / kWave];
  const bool any_dup = __ballot(dup) != 0;
  sum = (uint64_t)wave_sum_i64((int64_t)sum);   // two's-complement sums are exact modulo 2^64
  if (lane_id() == 0) {
    part[threadIdx.x / kWave] = sum;
    pdup[threadIdx.x / kWave] = any_dup;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    int d = 0;
    for (int w = 0; w < kTpb / kWave; ++w) {
      t += part[w];
      d |= pdup[w];
    }
    if (d) atomicOr(err, 2u);
    if (t) atomicAdd(dm, (u64a)t);
  }
}

// Mirror entries of sorted canonical undirected records (u <= v): (u, v) and, for u != v, (v, u).
__global__ void k_bulk_mirror(const uint64_t* keys, const uint32_t* wts, uint64_t k, uint64_t* ekeys, uint32_t* ew,
                              u64a* count, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t key = keys[i];
    const uint32_t u = krow(key, ks), v = kcol(key, ks);
    const uint32_t w = wts[i];
    const unsigned long long a = wave_reserve64(count, true, 1);
    ekeys[a] = key;
    ew[a] = w;
    const unsigned long long b = wave_reserve64(count, u != v, 1);
    if (u != v) {
      ekeys[b] = kpack(v, u, ks);
      ew[b] = w;
    }
  }
}

// in-degree of every column of a directed bulk load (deg zero at launch)
__global__ void k_bulk_count_cols(const uint64_t* keys, uint64_t k, uint32_t* deg, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) atomicAdd(&deg[kcol(keys[i], ks)], 1u);
}

// every record (u, v, w) into the in-row of v at the row's next free slot (cursor zero at launch;
// exactly deg[v] records have column v), its weight added to kin[v]
__global__ void k_bulk_scatter_in(const uint64_t* keys, const uint32_t* wts, uint64_t k, CsrRef in, uint32_t* cursor,
                                  int64_t* kin, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint64_t key = keys[i];
    const uint32_t u = krow(key, ks), v = kcol(key, ks);
    const uint32_t w = wts[i];
    const uint64_t slot = in.off[v] + atomicAdd(&cursor[v], 1u);
    in.nbr[slot] = u;
    ((uint32_t*)in.w)[slot] = w;
    atomic_add_i64(&kin[v], (int64_t)w);
  }
}

// first and one-past-last position of every row in a sorted entry list (rows without entries
// keep the zeros they were given)
__global__ void k_bulk_bounds(const uint64_t* keys, uint64_t k, uint64_t* start, uint64_t* end, int ks) {
  for (uint64_t i = gtid(); i < k; i += gstride()) {
    const uint32_t r = krow(keys[i], ks);
    if (i == 0 || krow(keys[i - 1], ks) != r) start[r] = i;
    if (i + 1 == k || krow(keys[i + 1], ks) != r) end[r] = i + 1;
  }
}

__global__ void k_bulk_deg(const uint64_t* start, const uint64_t* end, uint32_t n, uint32_t* deg) {
  for (uint64_t u = gtid(); u < n; u += gstride()) deg[u] = (uint32_t)(end[u] - start[u]);
}

// Entry i of the sorted list goes to slot off[row] + (i - start[row]) of a level-0 (uint32
// weight) CSR whose rows have room for their degree.  Each row's weight sum is added to
// rowsum[row] (one atomic per run of the row within a wavefront: the entries of a row are
// contiguous, so a segmented scan over the wavefront's lanes forms the runs).  With lab, the
// weight of entries whose endpoints share a community is added to *dein.
__global__ void k_bulk_place(const uint64_t* keys, const uint32_t* wts, uint64_t k, const uint64_t* start, CsrRef c,
                             int64_t* rowsum, const uint32_t* lab, i64a* dein, int ks) {
  const int lane = lane_id();
  int64_t in_sum = 0;
  for (uint64_t base = gwave() * kWave; base < k; base += gwstride() * kWave) {
    const uint64_t i = base + lane;
    const bool valid = i < k;
    uint32_t r = kEmpty;
    int64_t w = 0;
    if (valid) {
      const uint64_t key = keys[i];
      const uint32_t col = kcol(key, ks);
      r = krow(key, ks);
      w = wts[i];
      const uint64_t slot = c.off[r] + (i - start[r]);
      c.nbr[slot] = col;
      ((uint32_t*)c.w)[slot] = (uint32_t)w;
      if (lab && lab[r] == lab[col]) in_sum += w;
    }
    int64_t run = w;   // inclusive segmented scan by row (rows are non-decreasing over the lanes)
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t t = __shfl_up(run, o, kWave);
      const uint32_t ro = (uint32_t)__shfl_up((int)r, o, kWave);
      if (lane >= o && ro == r) run += t;
    }
    const uint32_t rn = (uint32_t)__shfl_down((int)r, 1, kWave);
    const bool last = lane == kWave - 1 || rn != r;
    if (valid && last && run) atomic_add_i64(&rowsum[r], run);
  }
  in_sum = wave_sum_i64(in_sum);
  if (lane == 0 && in_sum) atomicAdd((u64a*)dein, (u64a)in_sum);
}

// entries of the vertices with more than `lim` entries (out + in): the hub entries of a full scan
__global__ void k_hub_entries(const uint32_t* dout, const uint32_t* din_or_null, uint32_t n, uint32_t lim,
                              u64a* total) {
  __shared__ uint64_t part[kTpb / kWave];
  uint64_t sum = 0;
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const uint64_t t = (uint64_t)dout[x] + (din_or_null ? din_or_null[x] : 0u);
    if (t > lim) sum += t;
  }
  sum = (uint64_t)wave_sum_i64((int64_t)sum);
  if (lane_id() == 0) part[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kTpb / kWave; ++w) t += part[w];
    if (t) atomicAdd(total, (u64a)t);
  }
}

// Seeds and touched communities of a bulk load: every vertex with an entry is an endpoint of
// the batch; its community is touched (old totals recorded before any total changes).
__global__ void k_bulk_mark(uint32_t n, CsrRef out, CsrRef in, const uint32_t* lab0, const int64_t* Kout,
                            const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0) {
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const uint32_t u = (uint32_t)x;
    const bool e = out.deg[u] != 0 || (in.deg && in.deg[u] != 0);
    set_add(seeds0.stamp, seeds0.epoch, seeds0.list, seeds0.count, u, e);
    const uint32_t c = e ? lab0[u] : 0u;
    const bool claimed = e && set_claim(touched.stamp, touched.epoch, c);
    const uint32_t at = wave_reserve(touched.count, claimed);
    if (claimed) {
      touched.list[at] = c;
      tko[at] = Kout[c];
      tki[at] = Kin[c];
    }
  }
}

// Community totals of a bulk load: the degrees of the loaded rows (zero before the load) are
// added to the totals of each vertex's community.
__global__ void k_bulk_totals(uint32_t n, const uint32_t* lab0, const int64_t* kout, const int64_t* kin_or_null,
                              int64_t* Kout, int64_t* Kin_or_null) {
  for (uint64_t x = gtid(); x < n; x += gstride()) {
    const uint32_t c = lab0[x];
    if (kout[x]) atomic_add_i64(&Kout[c], kout[x]);
    if (kin_or_null && kin_or_null[x]) atomic_add_i64(&Kin_or_null[c], kin_or_null[x]);
  }
}

}  // namespace

// ids x < n with stamp[x] == ep appended to list (ascending within each 4096-id chunk, chunks in
// any order), one global atomic per chunk; *count must be 0 at launch
constexpr uint32_t kSelChunk = 4096;
__global__ __launch_bounds__(kTpb) void k_select_stamp(const uint32_t* stamp, uint32_t ep, uint32_t n, uint32_t* list,
                                                       uint32_t* count) {
  constexpr uint32_t PER = kSelChunk / kTpb;
  __shared__ uint32_t wsum[kTpb / kWave];
  __shared__ uint32_t s_base;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (uint64_t c0 = (uint64_t)blockIdx.x * kSelChunk; c0 < n; c0 += (uint64_t)gridDim.x * kSelChunk) {
    // thread t owns ids c0 + t*PER .. + PER (contiguous, so the chunk's output stays ascending)
    const uint64_t b = c0 + (uint64_t)threadIdx.x * PER;
    uint32_t sv[PER];
    if (b + PER <= n) {   // 64 contiguous bytes per lane (b is a multiple of 16 ids)
      const uint4* p4 = reinterpret_cast<const uint4*>(stamp + b);
#pragma unroll
      for (uint32_t k = 0; k < PER / 4; ++k) {
        const uint4 v4 = p4[k];
        sv[4 * k] = v4.x;
        sv[4 * k + 1] = v4.y;
        sv[4 * k + 2] = v4.z;
        sv[4 * k + 3] = v4.w;
      }
    } else {
#pragma unroll
      for (uint32_t q = 0; q < PER; ++q) sv[q] = b + q < n ? stamp[b + q] : ~ep;
    }
    uint32_t mine = 0;
    uint32_t flags = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
      const bool f = sv[q] == ep;
      flags |= (f ? 1u : 0u) << q;
      mine += f ? 1u : 0u;
    }
    uint32_t incl = mine;   // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = (uint32_t)__shfl_up((int)incl, o, kWave);
      if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int k = 0; k < kTpb / kWave; ++k) {
      if (k < w) before += wsum[k];
      total += wsum[k];
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(count, total) : 0u;
    __syncthreads();
    uint32_t at = s_base + before + incl - mine;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q)
      if (flags & (1u << q)) list[at++] = (uint32_t)(b + q);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers
void launch_select_stamp(const uint32_t* stamp, uint32_t ep, uint32_t n, uint32_t* list, uint32_t* count,
                         hipStream_t s) {
  (void)hipMemsetAsync(count, 0, sizeof(uint32_t), s);
  if (n)
    k_select_stamp<<<cap_blocks((n + kSelChunk - 1) / kSelChunk, LDL_RESIDENT(k_select_stamp, kTpb)), kTpb, 0, s>>>(
        stamp, ep, n, list, count);
}

void launch_mark_members(uint32_t* stamp, uint32_t ep, uint32_t n, const uint8_t* alive, const uint32_t* key,
                         const uint32_t* mark, uint32_t mark_ep, hipStream_t s) {
  if (n) k_mark_members<<<grid_for(n), kTpb, 0, s>>>(stamp, ep, n, alive, key, mark, mark_ep);
}
void launch_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t nr, const uint32_t* par,
                         const uint32_t* oldpar, hipStream_t s, const uint32_t* countp) {
  if (nr) k_mark_changed<<<list_grid(nr, countp), kTpb, 0, s>>>(stamp, ep, rset, nr, countp, par, oldpar);
}
void launch_items(const uint32_t* list, const uint32_t* idx, const uint32_t* count, uint32_t bound, CsrRef out,
                  CsrRef in, uint64_t* icnt, uint64_t* ioff, uint64_t* csum, uint64_t* zero_a, uint64_t* zero_b,
                  hipStream_t s) {
  const uint64_t need = ((uint64_t)bound + kScanMinChunk) / kScanMinChunk;   // chunks of bound + 1 positions
  const unsigned g = need < kScanBlocks ? (unsigned)need : kScanBlocks;
  k_item_counts<<<g, kTpb, 0, s>>>(list, idx, count, bound, out, in, icnt, zero_a, zero_b, csum);
  k_item_offsets<<<g, kTpb, 0, s>>>(count, bound, icnt, csum, ioff);
}
void launch_spexpand(const uint32_t* movers, const uint32_t* idx, const uint32_t* count, uint32_t bound,
                     const uint64_t* ioff, CsrRef out, CsrRef in, const uint2* lp, const uint32_t* rsize,
                     uint32_t* rcur_stamp, uint32_t rcur_ep, uint32_t* rset_stamp, uint32_t rset_ep, uint32_t* oldpar,
                     hipStream_t s) {
  k_spexpand_items<<<kItemBlocks, kTpb, 0, s>>>(movers, idx, count, bound, ioff, out, in, lp, rsize, rcur_stamp,
                                                rcur_ep, rset_stamp, rset_ep, oldpar);
}
void launch_mark_items(uint32_t* stamp, uint32_t ep, const uint32_t* list, const uint32_t* count, uint32_t bound,
                       const uint64_t* ioff, CsrRef out, CsrRef in, hipStream_t s, const uint32_t* ustamp,
                       uint32_t uep, const uint8_t* alive) {
  // dense lists (1/64 of the nodes or more) are pulled when the list's stamps are given: on the
  // full-method batches a pull already wins there (measured against 1/4, 1/16 and 1/256)
  const uint32_t pull_from = ustamp ? (uint32_t)(((uint64_t)bound + 63) / 64) : 0xFFFFFFFFu;
  k_mark_items<<<kItemBlocks, kTpb, 0, s>>>(stamp, ep, list, count, bound, ioff, out, in, pull_from);
  if (ustamp)
    k_mark_pull<<<grid_waves(bound) < 8192u ? grid_waves(bound) : 8192u, kTpb, 0, s>>>(stamp, ep, ustamp, uep, count,
                                                                                     pull_from, bound, alive, out, in);
}
void launch_pack_parents(uint32_t n, const uint32_t* par, const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep,
                         uint2* po, hipStream_t s) {
  if (n) k_pack_parents<<<grid_for(n), kTpb, 0, s>>>(n, par, oldpar, cstamp, cep, po);
}
void launch_tuples_count(const uint32_t* list, const uint32_t* count, uint32_t bound, const uint64_t* ioff, CsrRef out,
                         CsrRef in, const uint2* po, int repair, u64a* counts, hipStream_t s) {
  if (repair) k_tuples_count<true><<<kItemBlocks, kTpb, 0, s>>>(list, count, bound, ioff, out, in, po, counts);
  else k_tuples_count<false><<<kItemBlocks, kTpb, 0, s>>>(list, count, bound, ioff, out, in, po, counts);
}
void launch_tuples_gen(const uint32_t* list, const uint32_t* count, uint32_t bound, const uint64_t* ioff, CsrRef out,
                       CsrRef in, const uint32_t* par, const uint2* po, int repair, const uint64_t* toffs, u64a* cur,
                       uint64_t* tkeys, int64_t* tvals, uint32_t* seed_stamp, uint32_t seed_ep, int ks, hipStream_t s) {
  if (repair && !tkeys)
    k_tuples_gen<true, false><<<kItemBlocks, kTpb, 0, s>>>(list, count, bound, ioff, out, in, par, po, toffs, cur,
                                                           tkeys, tvals, seed_stamp, seed_ep, ks);
  else if (repair)
    k_tuples_gen<true, true><<<kItemBlocks, kTpb, 0, s>>>(list, count, bound, ioff, out, in, par, po, toffs, cur,
                                                          tkeys, tvals, seed_stamp, seed_ep, ks);
  else
    k_tuples_gen<false, true><<<kItemBlocks, kTpb, 0, s>>>(list, count, bound, ioff, out, in, par, po, toffs, cur,
                                                           tkeys, tvals, seed_stamp, seed_ep, ks);
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
                           const uint8_t* alive_or_null, hipStream_t s, const uint32_t* countp) {
  if (count)
    k_set_add_mapped<<<list_grid(count, countp), kTpb, 0, s>>>(set, list, count, countp, key, alive_or_null);
}
void launch_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot, uint64_t k,
                            const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                            int directed, int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm,
                            int ks, hipStream_t s) {
  if (k)
    k_ingest_validate<<<grid_for(k), kTpb, 0, s>>>(out0, keys, idx, slot, k, ins, ni, del, nd, chg, directed, delta,
                                                   err, first_bad, dm, ks);
}
int launch_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo, const uint32_t* nseg_ptr,
                      uint64_t* seg_hi, uint64_t* items, uint64_t* item_off, uint64_t* items_big,
                      uint64_t* item_off_big, int64_t* slot_out, void** tmp, size_t* tmp_bytes, int ks,
                      hipStream_t s) {
  if (!k) return 0;
  k_seg_items<<<grid_for(k + 1), kTpb, 0, s>>>(c, keys, k, seg_lo, nseg_ptr, seg_hi, items, items_big, ks);
  int rc = prim_exclusive_sum_u64(tmp, tmp_bytes, items, item_off, k + 1, s);
  if (rc) return rc;
  k_fill_i64_dev<<<grid_for(k), kTpb, 0, s>>>(slot_out, -1, k);
  const unsigned g = cap_blocks(k < 8192 ? k : 8192u, LDL_RESIDENT(k_seg_lookup, 256));
  k_seg_lookup<<<g, 256, 0, s>>>(c, keys, k, seg_lo, seg_hi, nseg_ptr, item_off, slot_out, ks);
  if (k > kSegChunk) {   // a segment above the wavefront limit exists only then
    rc = prim_exclusive_sum_u64(tmp, tmp_bytes, items_big, item_off_big, k + 1, s);
    if (rc) return rc;
    const unsigned gb = cap_blocks(k < 8192 ? k : 8192u, LDL_RESIDENT(k_seg_lookup_big, 256));
    k_seg_lookup_big<<<gb, 256, 0, s>>>(c, keys, k, seg_lo, seg_hi, nseg_ptr, item_off_big, slot_out, ks);
  }
  return 0;
}
void launch_seg_update(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                       const uint64_t* seg_hi, const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* rtype,
                       uint64_t* hole, int64_t* deg_arr, uint32_t* rowdel, uint32_t* rowins, uint32_t* move_list,
                       uint32_t* move_count, int ks, hipStream_t s) {
  if (!k) return;
  const unsigned gw = cap_blocks((k + 3) / 4, LDL_RESIDENT(k_seg_update_wave, kTpb));
  k_seg_update_wave<<<gw, kTpb, 0, s>>>(c, keys, delta, seg_lo, seg_hi, nseg_ptr, slot, rtype, hole, deg_arr, rowdel,
                                        rowins, move_list, move_count, ks);
  if (k > kSegWaveMax) {   // a segment above the wavefront limit exists only then
    const unsigned g = cap_blocks(k < 8192 ? k : 8192u, LDL_RESIDENT(k_seg_update, kSegTpb));
    k_seg_update<<<g, kSegTpb, 0, s>>>(c, keys, delta, seg_lo, seg_hi, nseg_ptr, slot, rtype, hole, deg_arr, rowdel,
                                    rowins, move_list, move_count, ks);
  }
}
void launch_seg_move(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                     const uint64_t* seg_hi, const uint8_t* rtype, const uint32_t* rowdel, const uint32_t* rowins,
                     uint32_t* move_list, const uint32_t* move_count, u64a* pool_top, uint64_t pool_cap,
                     uint32_t* overflow, int tight, int ks, hipStream_t s) {
  if (!k) return;
  const unsigned g = cap_blocks(k < 1024 ? k : 1024u, LDL_RESIDENT(k_seg_move, kTpb));
  k_seg_move<<<g, kTpb, 0, s>>>(c, keys, delta, seg_lo, seg_hi, rtype, rowdel, rowins, move_list, move_count, pool_top,
                                pool_cap, overflow, tight, ks);
}
void launch_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n, int tight, hipStream_t s) {
  if (n) k_csr_newcap<<<grid_for(n), kTpb, 0, s>>>(deg, newcap, newcap64, n, tight);
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
                           int ks, hipStream_t s) {
  const uint64_t t = ni + nd + nc;
  if (t) k_ingest_records<<<grid_for(t), kTpb, 0, s>>>(ins, ni, del, nd, chg, nc, n, directed, keys, idx, err, ks);
}
void launch_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed, uint64_t* ekeys,
                           int64_t* edelta, u64a* count, int ks, hipStream_t s) {
  if (k) k_ingest_entries<<<grid_for(k), kTpb, 0, s>>>(keys, delta, k, directed, ekeys, edelta, count, ks);
}
void launch_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                        const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, int ks, hipStream_t s) {
  if (k) k_ingest_mark<<<grid_for(k), kTpb, 0, s>>>(ekeys, k, lab0, Kout, Kin, touched, tko, tki, seeds0, ks);
}
void launch_ingest_totals(const uint64_t* ekeys, const int64_t* edelta, uint64_t k, const uint32_t* lab0,
                          int64_t* Kout, int64_t* Kin_or_null, i64a* dein, int ks, hipStream_t s) {
  if (k) k_ingest_totals<<<grid_for(k), kTpb, 0, s>>>(ekeys, edelta, k, lab0, Kout, Kin_or_null, dein, ks);
}
void launch_dskk(const uint32_t* touched, const uint32_t* nt, uint32_t nt_max, const int64_t* Kout, const int64_t* Kin,
                 const int64_t* tko, const int64_t* tki, u64a* lo, i64a* hi, hipStream_t s) {
  if (!nt_max) return;
  const unsigned g = grid_for(nt_max) < 1024u ? grid_for(nt_max) : 1024u;
  k_dskk<<<g, kTpb, 0, s>>>(touched, nt, Kout, Kin, tko, tki, lo, hi);
}
void launch_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                        uint64_t* keys, int64_t* vals, SetRef seeds, int ks, hipStream_t s) {
  if (k) k_cascade_map<<<grid_for(k), kTpb, 0, s>>>(ex, ey, ed, k, par, keys, vals, seeds, ks);
}
void launch_record_degrees(const uint64_t* keys, const int64_t* vals, uint64_t k, int64_t* kout, int64_t* kin_or_null,
                           int ks, hipStream_t s) {
  if (k)
    k_record_degrees<<<cap_blocks((k + kDegChunk - 1) / kDegChunk, LDL_RESIDENT(k_record_degrees, kTpb)), kTpb, 0,
                       s>>>(keys, vals, k, kout, kin_or_null, ks);
}
void launch_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey, int ks, hipStream_t s) {
  if (k) k_split_keys<<<grid_for(k), kTpb, 0, s>>>(keys, k, ex, ey, ks);
}
void launch_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k, int ks, hipStream_t s) {
  if (k) k_transpose_keys<<<grid_for(k), kTpb, 0, s>>>(keys, tkeys, k, ks);
}
void launch_ref_init_top(uint32_t n, const uint8_t* alive, const int64_t* kout, const int64_t* kin, int64_t* Krout,
                         int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s) {
  if (n) k_ref_init_top<<<grid_for(n), kTpb, 0, s>>>(n, alive, kout, kin, Krout, Krin_or_null, rsize);
}
void launch_ref_reset(const uint32_t* R, uint32_t nr, uint32_t* par, uint32_t* oldpar, const int64_t* kout,
                      const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, int phase,
                      hipStream_t s, const uint32_t* countp) {
  if (nr)
    k_ref_reset<<<list_grid(nr, countp), kTpb, 0, s>>>(R, nr, countp, par, oldpar, kout, kin, Krout, Krin_or_null,
                                                        rsize, phase);
}
void launch_live_update(const uint32_t* cand, uint32_t k, const uint32_t* rsize_below, uint8_t* alive,
                        uint32_t* par_or_null, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                        SetRef revived, hipStream_t s, const uint32_t* countp) {
  if (k)
    k_live_update<<<list_grid(k, countp), kTpb, 0, s>>>(cand, k, countp, rsize_below, alive, par_or_null, lab,
                                                         lab_below, died, revived);
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
  if (n) k_alive_list<<<grid_for(n) < 2048u ? grid_for(n) : 2048u, kTpb, 0, s>>>(n, alive, set);
}
void launch_materialise_nodes(uint32_t n, const uint32_t* rsize, uint8_t* alive_up, const uint32_t* lab,
                              uint32_t* lab_up, uint32_t* par_up_or_null, hipStream_t s) {
  if (n) k_materialise_nodes<<<grid_for(n), kTpb, 0, s>>>(n, rsize, alive_up, lab, lab_up, par_up_or_null);
}
void launch_label_refresh(uint32_t n, const uint8_t* alive, const uint32_t* par, const uint32_t* lab_up,
                          uint32_t* lab, SetRef seeds, hipStream_t s) {
  if (n) k_label_refresh<<<grid_for(n), kTpb, 0, s>>>(n, alive, par, lab_up, lab, seeds);
}
void launch_bulk_records(const uint32_t* ins, uint64_t k, uint32_t n, int directed, uint64_t* keys, uint32_t* wts,
                         uint32_t* err, int ks, hipStream_t s) {
  if (k) k_bulk_records<<<grid_for(k), kTpb, 0, s>>>(ins, k, n, directed, keys, wts, err, ks);
}
void launch_bulk_check(const uint64_t* keys, const uint32_t* wts, uint64_t k, int directed, uint32_t* err, u64a* dm,
                       int ks, hipStream_t s) {
  if (k) {
    const unsigned g = grid_for(k) < kItemBlocks ? grid_for(k) : kItemBlocks;
    k_bulk_check<<<g, kTpb, 0, s>>>(keys, wts, k, directed, err, dm, ks);
  }
}
void launch_bulk_mirror(const uint64_t* keys, const uint32_t* wts, uint64_t k, uint64_t* ekeys, uint32_t* ew,
                        u64a* count, int ks, hipStream_t s) {
  if (k) k_bulk_mirror<<<grid_for(k), kTpb, 0, s>>>(keys, wts, k, ekeys, ew, count, ks);
}
void launch_bulk_count_cols(const uint64_t* keys, uint64_t k, uint32_t* deg, int ks, hipStream_t s) {
  if (k) k_bulk_count_cols<<<grid_for(k), kTpb, 0, s>>>(keys, k, deg, ks);
}
void launch_bulk_scatter_in(const uint64_t* keys, const uint32_t* wts, uint64_t k, CsrRef in, uint32_t* cursor,
                            int64_t* kin, int ks, hipStream_t s) {
  if (k) k_bulk_scatter_in<<<grid_for(k), kTpb, 0, s>>>(keys, wts, k, in, cursor, kin, ks);
}
void launch_bulk_rows(const uint64_t* keys, uint64_t k, uint64_t* start, uint64_t* end, uint32_t n, uint32_t* deg,
                      int ks, hipStream_t s) {
  if (!n) return;
  if (k) k_bulk_bounds<<<grid_for(k), kTpb, 0, s>>>(keys, k, start, end, ks);
  k_bulk_deg<<<grid_for(n), kTpb, 0, s>>>(start, end, n, deg);
}
void launch_bulk_place(const uint64_t* keys, const uint32_t* wts, uint64_t k, const uint64_t* start, CsrRef c,
                       int64_t* rowsum, const uint32_t* lab_or_null, i64a* dein, int ks, hipStream_t s) {
  if (k) k_bulk_place<<<grid_for(k), kTpb, 0, s>>>(keys, wts, k, start, c, rowsum, lab_or_null, dein, ks);
}
void launch_hub_entries(const uint32_t* dout, const uint32_t* din_or_null, uint32_t n, uint32_t lim, u64a* total,
                        hipStream_t s) {
  if (n) {
    const unsigned g = grid_for(n) < kItemBlocks ? grid_for(n) : kItemBlocks;
    k_hub_entries<<<g, kTpb, 0, s>>>(dout, din_or_null, n, lim, total);
  }
}
void launch_bulk_mark(uint32_t n, CsrRef out, CsrRef in, const uint32_t* lab0, const int64_t* Kout, const int64_t* Kin,
                      SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, hipStream_t s) {
  if (n) k_bulk_mark<<<grid_for(n), kTpb, 0, s>>>(n, out, in, lab0, Kout, Kin, touched, tko, tki, seeds0);
}
void launch_bulk_totals(uint32_t n, const uint32_t* lab0, const int64_t* kout, const int64_t* kin_or_null, int64_t* Kout,
                        int64_t* Kin_or_null, hipStream_t s) {
  if (n) k_bulk_totals<<<grid_for(n), kTpb, 0, s>>>(n, lab0, kout, kin_or_null, Kout, Kin_or_null);
}
void launch_degrees_up(uint32_t n, const uint8_t* alive, const uint32_t* par, const int64_t* kout, const int64_t* kin,
                       int64_t* kout_up, int64_t* kin_up_or_null, hipStream_t s) {
  if (n) k_degrees_up<<<grid_for(n), kTpb, 0, s>>>(n, alive, par, kout, kin, kout_up, kin_up_or_null);
}
void launch_count_members(uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* stamp, uint32_t ep,
                          u64a* count, hipStream_t s) {
  if (n) k_count_members<<<grid_for(n) < 2048u ? grid_for(n) : 2048u, kTpb, 0, s>>>(n, alive, key, stamp, ep, count);
}
void launch_refresh_scalars(CsrRef out, CsrRef in, uint32_t n, const int64_t* kout, const int64_t* kin, SetRef seeds,
                            i64a* ein, u64a* skk_lo, i64a* skk_hi, hipStream_t s) {
  if (n) k_refresh_scalars<<<grid_waves(n) < 4096u ? grid_waves(n) : 4096u, kTpb, 0, s>>>(out, in, n, kout, kin, seeds,
                                                                                           ein, skk_lo, skk_hi);
}
void launch_sum_u32(const uint32_t* a, uint32_t n, u64a* total, hipStream_t s) {
  if (n) k_sum_u32<<<grid_for(n) < 1024u ? grid_for(n) : 1024u, kTpb, 0, s>>>(a, n, total);
}
void launch_recount_degrees(CsrRef c, uint32_t n, int64_t* deg_out, hipStream_t s) {
  if (n) k_recount_degrees<<<grid_waves(n), kTpb, 0, s>>>(c, n, deg_out);
}

}  // namespace ldl
