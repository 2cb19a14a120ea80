// Host-side launchers of the LD-Leiden HIP kernels (definitions in kernels_*.hip, prims.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldl {

typedef unsigned long long u64a;
typedef long long i64a;

// SplitMix64's output function (Steele, Lea and Flood, 2014) of a 64-bit state: the
// counter-based hash of the randomised refinement (keys on the host, priorities on the device).
__host__ __device__ __forceinline__ uint64_t splitmix64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// draw priority of target y for vertex u under an iteration key (odd, so never 0)
__device__ __forceinline__ uint32_t draw_priority(uint64_t key, uint32_t u, uint32_t y) {
  return (uint32_t)(splitmix64_out(splitmix64_out(key ^ u) ^ y) >> 32) | 1u;
}

// A stamped set over ids [0, n): x is a member iff stamp[x] == epoch; members are appended to
// `list` and counted in *count.
struct SetRef {
  uint32_t* stamp;
  uint32_t* list;
  uint32_t* count;
  uint32_t epoch;
};

// Dynamic CSR (one orientation of one level): row u holds deg[u] entries at off[u] within a
// pool with room for cap[u].  Weights are u32 at level 0 and i64 above.
struct CsrRef {
  uint64_t* off;
  uint32_t* deg;
  uint32_t* cap;
  uint32_t* nbr;
  void* w;
  int wide;  // 0: uint32 weights, 1: int64 weights
};

// Everything the local-move and refinement kernels read for one level.
struct MoveView {
  CsrRef out, in;            // in.off == nullptr for undirected graphs
  const uint32_t* lab;       // P^r
  const uint32_t* par;       // pi_r (refinement)
  const uint2* lp;           // (P^r, pi_r) of every node packed in one word (refinement)
  const uint8_t* alive;
  const int64_t* kout;       // level-r degrees
  const int64_t* kin;
  const int64_t* Kout;       // community totals (move) or refined totals (refinement)
  const int64_t* Kin;
  const uint32_t* rsize;     // refined community sizes (refinement)
  int64_t qm;                // q * m
  int64_t p;                 // gamma numerator
  int directed;
  int empty_target;          // move: also offer the empty community labelled v (variant)
  uint64_t rkey;             // refinement: key of the iteration's random draw (0: best gain)
  uint32_t lim[5];           // degree-bin limits (entries per vertex), see kBinCap
};

struct CandBuf {
  uint32_t* v;
  uint32_t* a;
  uint32_t* b;
  uint64_t* glo;
  int64_t* ghi;
  uint32_t* count;
};

// Bucket pool of the hub bin, cap entries each: the distinct (key, weight) pairs of every chunk
// of a hub's entries, at the start of the chunk's own stretch (ekey, ew), and the same pairs
// scattered into per-hub hash partitions (bkey, bw).
struct HubPool {
  uint32_t* ekey;
  int64_t* ew;
  uint32_t* bkey;
  int64_t* bw;
  uint64_t cap;         // entries
  u64a* top;            // device word: entries the last launch needed
  uint32_t* over_count; // device flags: bit 0 pool too small, bit 1 more hubs than the bound,
                        // bit 2 a partition had more distinct keys than its LDS table holds
};

struct MoveStats {  // per-launch counters (null: not counted)
  u64a* entries;
  u64a* distinct;
  u64a* vertices;
  u64a* cands;
  u64a* maxhi;      // max of the high 64 bits of emitted gains (gains are positive)
};

// a device-resident list: base + *start, *count items
struct BinRef {
  const uint32_t* base;
  const uint32_t* start;
  const uint32_t* count;
};

constexpr int kNumBins = 6;
// Degree bins: a vertex with T > 0 entries goes to the first bin b < kNumBins - 1 with
// T <= lim[b], else to the hub path (bin kNumBins - 1).  Bin b's kernel accepts at most
// kBinCap[b] entries, so 0 <= lim[0] <= ... <= lim[4] with lim[b] <= kBinCap[b]; the limits only
// decide which kernel evaluates a vertex, never the result.  kBinLimit are the defaults: bin 3 is
// empty, so vertices with 129..2048 entries go to the 256-lane workgroup kernel (measured as fast
// as or faster than one wavefront per vertex for 129..512 entries on R-MAT batch updates).
constexpr uint32_t kBinCap[kNumBins - 1] = {8, 32, 128, 512, 2048};
constexpr uint32_t kBinLimit[kNumBins - 1] = {8, 32, 128, 128, 2048};
// statistics category of a candidate kernel: 2 kNumBins refine + kNumBins wide + bin
constexpr int kNumCats = 4 * kNumBins;

// ---------------------------------------------------------------- sets and generic helpers
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s);
void launch_fill_i64(int64_t* p, int64_t v, uint64_t n, hipStream_t s);
void launch_iota(uint32_t* p, uint64_t n, hipStream_t s);
void launch_copy_i64(int64_t* dst, const int64_t* src, uint64_t n, hipStream_t s);
// set.add(x) for every x in list[0..count)
void launch_set_add_list(SetRef set, const uint32_t* list, uint32_t count, hipStream_t s);
// set.add(key[x]) for every x in list[0..count) (optionally only alive x).  The list launchers
// below take an optional countp: the length is then read on the device (count is its bound).
void launch_set_add_mapped(SetRef set, const uint32_t* list, uint32_t count, const uint32_t* key,
                           const uint8_t* alive_or_null, hipStream_t s, const uint32_t* countp = nullptr);
// set.add(u) for every alive u < n with mark[key[u]] == mark_epoch
// plain-store marking (stamp[x] = ep, no list): members of marked keys, listed vertices and
// their neighbours, accepted movers and their neighbours; a later select builds the list
void launch_mark_members(uint32_t* stamp, uint32_t ep, uint32_t n, const uint8_t* alive, const uint32_t* key,
                         const uint32_t* mark, uint32_t mark_ep, hipStream_t s);
void launch_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, const uint32_t* na,
                                uint32_t na_max, CandBuf cand, CsrRef out, CsrRef in, int directed, hipStream_t s);
void launch_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t nr, const uint32_t* par,
                         const uint32_t* oldpar, hipStream_t s, const uint32_t* countp = nullptr);
// degree binning without global atomics: per-block histograms, then a fill whose blocks
// derive their output positions from the histograms
constexpr unsigned kBinBlocks = 256;
// (the count kernel also clears zero_words[0..nzero), the counters of the pass that follows)
void launch_bin_count(const MoveView& mv, const uint32_t* list, const uint32_t* count, int refine, uint32_t* hist,
                      uint32_t* zero_words, uint32_t nzero, hipStream_t s);
void launch_bin_fill(const MoveView& mv, const uint32_t* list, const uint32_t* count, int refine, const uint32_t* hist,
                     uint32_t* out, uint32_t* bin_start, uint32_t* bin_count, hipStream_t s);
// wavefront items over a node list (count on the device, at most `bound` nodes): node i has
// out.deg + in.deg entries (in only when in.off is set), split into items of kItem entries;
// icnt/ioff hold bound + 1 words, of which words 0..count are written (ioff[count] is the item
// total); zero_a / zero_b (optional, bound + 1 words) are cleared at 0..count; csum holds
// kItemScanBlocks words of chunk sums
constexpr uint32_t kItem = 512;
constexpr unsigned kItemBlocks = 2048;
constexpr unsigned kItemScanBlocks = 1024;
// (node i = list[idx[i]] when idx is given)
void launch_items(const uint32_t* list, const uint32_t* idx, const uint32_t* count, uint32_t bound, CsrRef out,
                  CsrRef in, uint64_t* icnt, uint64_t* ioff, uint64_t* csum, uint64_t* zero_a, uint64_t* zero_b,
                  hipStream_t s);
// stamp[x] = ep for every listed node and every neighbour over its items
// (with ustamp / uep, the stamps of the listed set, and bound = n: a list of at least n/4 nodes
// is pulled instead -- alive nodes that are listed or have a listed neighbour -- same set)
void launch_mark_items(uint32_t* stamp, uint32_t ep, const uint32_t* list, const uint32_t* count, uint32_t bound,
                       const uint64_t* ioff, CsrRef out, CsrRef in, hipStream_t s, const uint32_t* ustamp = nullptr,
                       uint32_t uep = 0, const uint8_t* alive = nullptr);
// subtract-add tuples over items: per-node counts (added into zeroed counts), then tuples at
// toffs (the exclusive prefix of counts) with a zeroed per-node cursor; seeds marked by
// plain stores (seed_stamp may be null when not repairing)
// po[x] = (par[x], cstamp[x] == cep ? oldpar[x] : par[x]) for x < n
void launch_pack_parents(uint32_t n, const uint32_t* par, const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep,
                         uint2* po, hipStream_t s);
// (repair: a neighbour x changed parent iff po[x].x != po[x].y; otherwise po is unused)
void launch_tuples_count(const uint32_t* list, const uint32_t* count, uint32_t bound, const uint64_t* ioff, CsrRef out,
                         CsrRef in, const uint2* po, int repair, u64a* counts, hipStream_t s);
// (repair with tkeys == nullptr: only the seeds are marked, no tuple is written)
void launch_tuples_gen(const uint32_t* list, const uint32_t* count, uint32_t bound, const uint64_t* ioff, CsrRef out,
                       CsrRef in, const uint32_t* par, const uint2* po, int repair, const uint64_t* toffs, u64a* cur,
                       uint64_t* tkeys, int64_t* tvals, uint32_t* seed_stamp, uint32_t seed_ep, int ks, hipStream_t s);

// ---------------------------------------------------------------- dynamic CSR
// Records sorted by key = row << ks | col (ks = bits of a vertex id) with deltas; zero deltas
// are ignored.
// row lookup of sorted records split over (segment, record chunk, row slice) items: slot of
// every record (or -1).  Segments (first record of each row, ascending) come from
// prim_select_heads.
int launch_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo, const uint32_t* nseg_ptr,
                       uint64_t* seg_hi, uint64_t* items, uint64_t* item_off, uint64_t* items_big,
                       uint64_t* item_off_big, int64_t* slot_out, void** tmp, size_t* tmp_bytes, int ks,
                       hipStream_t s);
// in-place row update (record types into rtype, hole scratch of k words; optional row delta
// sums added to deg_arr); rows that outgrow their capacity are listed for launch_seg_move,
// which takes new regions from the pool (bit 0 of *overflow when full: grow, launch again)
void launch_seg_update(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                       const uint64_t* seg_hi, const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* rtype,
                       uint64_t* hole, int64_t* deg_arr, uint32_t* rowdel, uint32_t* rowins, uint32_t* move_list,
                       uint32_t* move_count, int ks, hipStream_t s);
void launch_seg_move(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                     const uint64_t* seg_hi, const uint8_t* rtype, const uint32_t* rowdel, const uint32_t* rowins,
                     uint32_t* move_list, const uint32_t* move_count, u64a* pool_top, uint64_t pool_cap,
                     uint32_t* overflow, int tight, int ks, hipStream_t s);
void launch_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot, uint64_t k,
                            const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                            int directed, int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm,
                            int ks, hipStream_t s);
// new_cap[u] = deg[u] + slack, for a pool rebuild
// (tight: exactly deg[u], no slack)
void launch_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n, int tight, hipStream_t s);
void launch_csr_move_rows(CsrRef from, CsrRef to, const uint64_t* new_off, const uint32_t* new_cap, uint32_t n,
                          hipStream_t s);
void launch_csr_entries(CsrRef c, uint32_t n, uint64_t* out_keys, int64_t* out_w, u64a* counter, hipStream_t s);

// ---------------------------------------------------------------- batch ingest
// kinds: 0 insert (u,v,w), 1 delete (u,v), 2 change (u,v,w)
void launch_ingest_records(const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                           uint64_t nc, uint32_t n, int directed, uint64_t* keys, uint32_t* idx, uint32_t* err,
                           int ks, hipStream_t s);
void launch_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed, uint64_t* ekeys,
                           int64_t* edelta, u64a* count, int ks, hipStream_t s);
// touched communities of the level-0 entries (old totals recorded), seeds at level 0
void launch_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                        const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, int ks, hipStream_t s);
void launch_ingest_totals(const uint64_t* ekeys, const int64_t* edelta, uint64_t k, const uint32_t* lab0,
                          int64_t* Kout, int64_t* Kin_or_null, i64a* dein, int ks, hipStream_t s);
void launch_dskk(const uint32_t* touched, const uint32_t* nt, uint32_t nt_max, const int64_t* Kout, const int64_t* Kin,
                 const int64_t* tko, const int64_t* tki, u64a* lo, i64a* hi, hipStream_t s);
// ---- bulk load: an insert-only batch into a level-0 graph that has never held an entry
// insert records (key, weight); bad ids or zero weights set err bit 0
void launch_bulk_records(const uint32_t* ins, uint64_t k, uint32_t n, int directed, uint64_t* keys, uint32_t* wts,
                         uint32_t* err, int ks, hipStream_t s);
// sorted records: duplicate flag (err bit 1), unsigned matrix sum into *dm
void launch_bulk_check(const uint64_t* keys, const uint32_t* wts, uint64_t k, int directed, uint32_t* err, u64a* dm,
                       int ks, hipStream_t s);
// undirected: (u, v, w) and (v, u, w) for u != v appended at *count (2k entries of room)
void launch_bulk_mirror(const uint64_t* keys, const uint32_t* wts, uint64_t k, uint64_t* ekeys, uint32_t* ew,
                        u64a* count, int ks, hipStream_t s);
// directed in-rows: column counts into deg (zero at launch), then every record scattered to its
// column's row (cursor: n zeroed words) with its weight added to kin
void launch_bulk_count_cols(const uint64_t* keys, uint64_t k, uint32_t* deg, int ks, hipStream_t s);
void launch_bulk_scatter_in(const uint64_t* keys, const uint32_t* wts, uint64_t k, CsrRef in, uint32_t* cursor,
                            int64_t* kin, int ks, hipStream_t s);
// row bounds of a sorted entry list (start and end: n zeroed words each) and row degrees
void launch_bulk_rows(const uint64_t* keys, uint64_t k, uint64_t* start, uint64_t* end, uint32_t n, uint32_t* deg,
                      int ks, hipStream_t s);
// entries into their slots (rows laid out for their degrees); row weight sums added to rowsum,
// intra-community weight into *dein
void launch_bulk_place(const uint64_t* keys, const uint32_t* wts, uint64_t k, const uint64_t* start, CsrRef c,
                       int64_t* rowsum, const uint32_t* lab_or_null, i64a* dein, int ks, hipStream_t s);
// *total += entries (out + in) of the vertices with more than lim entries (*total zero at launch)
void launch_hub_entries(const uint32_t* dout, const uint32_t* din_or_null, uint32_t n, uint32_t lim, u64a* total,
                        hipStream_t s);
void launch_bulk_mark(uint32_t n, CsrRef out, CsrRef in, const uint32_t* lab0, const int64_t* Kout, const int64_t* Kin,
                      SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, hipStream_t s);
// Kout[lab0[x]] += kout[x] (and Kin with kin) for degrees that were zero before the load
void launch_bulk_totals(uint32_t n, const uint32_t* lab0, const int64_t* kout, const int64_t* kin_or_null, int64_t* Kout,
                        int64_t* Kin_or_null, hipStream_t s);
// cascade: (x,y) <- (par[x], par[y]); keys rebuilt; both endpoints seeded
void launch_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                        uint64_t* keys, int64_t* vals, SetRef seeds, int ks, hipStream_t s);
// list = ids x < n with stamp[x] == ep (ascending within 4096-id chunks), count into *count
void launch_select_stamp(const uint32_t* stamp, uint32_t ep, uint32_t n, uint32_t* list, uint32_t* count,
                         hipStream_t s);
void launch_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey, int ks, hipStream_t s);
// kout[row] += d for every record (row, col, d); kin[col] += d as well when kin_or_null is given
void launch_record_degrees(const uint64_t* keys, const int64_t* vals, uint64_t k, int64_t* kout, int64_t* kin_or_null,
                           int ks, hipStream_t s);
void launch_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k, int ks, hipStream_t s);

// ---------------------------------------------------------------- local move / refinement
// candidate kernels of degree bins 0..kNumBins-2 over a device-resident bin list
void launch_best(const MoveView& mv, int bin, BinRef br, uint32_t max_count, int refine, CandBuf cand, MoveStats st,
                 hipStream_t s, hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr);
// hub bin, device driven: per-hub entry counts, chunk items and hash partitions are prefix-summed
// over `bound` + 1 entries (bound >= number of hubs); hubs whose entries do not fit the pool are
// skipped and flagged.  Work arrays hold bound + 1 entries, partition arrays cap / 16 + bound + 1.
struct U64x3 {
  uint64_t x, y, z;
};
struct HubWork {
  U64x3* cnt;      // per hub: entries, chunk items, partitions (bound + 1 entries)
  U64x3* off;      // their exclusive prefix
  int64_t* own;    // weight towards the own community, per hub
  uint32_t* icnt;     // per chunk item: distinct pairs it left in the pool
  uint32_t* pcount;   // per partition: entries counted (zero between launches)
  uint32_t* pcur;     // per partition: scatter cursor (zero between launches)
  uint64_t* poff;     // per partition: first bucket entry
  uint32_t* pcnt;     // per partition: bucket entries
  int64_t* phi;    // partial bests, one per partition
  uint64_t* plo;
  uint32_t* pid;
  int* pvalid;
  int pshift;      // partitions per hub: ceil(T 2^pshift / kPartEntries), at most ceil(T / 16)
  uint32_t tslots; // LDS table slots of a partition (power of two <= kPartSlots)
};
constexpr uint32_t kPartEntries = 2048;   // target entries per partition (pshift 0)
constexpr uint32_t kPartSlots = 4096;     // LDS table slots of a partition
constexpr int kPartShiftMax = 6;
int launch_hub(const MoveView& mv, BinRef br, uint32_t bound, int refine, HubPool hub, HubWork hw, CandBuf cand,
               MoveStats st, void** tmp, size_t* tmp_bytes, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b);

// ---------------------------------------------------------------- decouple (exact greedy filter)
// first live candidate leaving / entering each community (per-community words, size n)
struct LfFirst {
  u64a* hi;
  u64a* lo;
  uint32_t* v;
};
constexpr unsigned kLfBlocks = 1024;
// The whole filter in one workgroup when there are at most kLfSmall candidates (count read on the
// device): accepted candidate indices in acc[0..*nacc), *nlive = 0.  With more candidates it does
// nothing but set *nacc = *nlive = 0 (the caller then runs the rounds below).
constexpr uint32_t kLfSmall = 1024;
void launch_lf_small(CandBuf cand, uint32_t* acc, uint32_t* nacc, uint32_t* nlive, hipStream_t s);
// live = 0..K-1 with K read on the device (at most bound), flags cleared, *nlive = K, *nacc = 0
void launch_lf_init(const uint32_t* K, uint32_t bound, uint32_t* live, uint8_t* flag, uint32_t* nlive, uint32_t* nacc,
                    hipStream_t s);
// one round over the live list (count on the device): accepted candidates are appended to
// acc_list, survivors to live2 (its count is reset by the round)
void launch_lf_round(const uint32_t* live, const uint32_t* nl, uint32_t bound, CandBuf cand, LfFirst E, LfFirst A,
                     uint32_t* accE, uint32_t* accA, uint32_t ep, uint8_t* flag, uint32_t* acc_list,
                     uint32_t* acc_count, uint32_t* live2, uint32_t* live2_count, hipStream_t s);

// ---------------------------------------------------------------- commit / rollback / expand
// na: device count of accepted candidates (acc list), na_max an upper bound for the grid
void launch_commit_mark(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* mov_stamp,
                        uint32_t mov_ep, uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin, SetRef touched,
                        int64_t* tko, int64_t* tki, hipStream_t s);
void launch_commit_apply(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* lab,
                         const int64_t* kout, const int64_t* kin, int64_t* Kout, int64_t* Kin_or_null, int forward,
                         hipStream_t s);
// big: room for na_max mover ids, *nbig zero at launch (movers with long rows are listed there
// and split over the grid)
void launch_commit_dein(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, CsrRef out, CsrRef in,
                        int directed, const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep,
                        const uint32_t* oldlab, uint32_t* big, uint32_t* nbig, i64a* dein, hipStream_t s);
void launch_mark_acc_comms(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* stamp,
                           uint32_t ep, hipStream_t s);
void launch_set_add_acc_v(SetRef set, const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand,
                          hipStream_t s);

// ---------------------------------------------------------------- refinement bookkeeping
void launch_ref_init_top(uint32_t n, const uint8_t* alive, const int64_t* kout, const int64_t* kin, int64_t* Krout,
                         int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s);
void launch_ref_reset(const uint32_t* R, uint32_t nr, uint32_t* par, uint32_t* oldpar, const int64_t* kout,
                      const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, int phase,
                      hipStream_t s, const uint32_t* countp = nullptr);
// forward: singletons join their targets; otherwise the same moves are undone
void launch_ref_commit(const uint32_t* acc, const uint32_t* na, uint32_t na_max, CandBuf cand, uint32_t* par,
                       uint2* lp, const int64_t* kout, const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null,
                       uint32_t* rsize, int forward, hipStream_t s);
// lp[u] = (lab[u], par[u]) for u < n
void launch_pack_lab_par(uint32_t n, const uint32_t* lab, const uint32_t* par, uint2* lp, hipStream_t s);
// out = src[0], src[stride], ... below *count (count on the device, at most bound); *out_count set
void launch_stride_sample(const uint32_t* src, const uint32_t* count, uint32_t bound, uint32_t stride, uint32_t* out,
                          uint32_t* out_count, hipStream_t s);
// SPExpand over wavefront items of the movers (node i = movers[idx[i]], count on the device;
// items from launch_items with the same list): plain-store marks into Rcur and Rset, oldpar of
// new Rset members = themselves; the lists are built later by select
void launch_spexpand(const uint32_t* movers, const uint32_t* idx, const uint32_t* count, uint32_t bound,
                     const uint64_t* ioff, CsrRef out, CsrRef in, const uint2* lp, const uint32_t* rsize,
                     uint32_t* rcur_stamp, uint32_t rcur_ep, uint32_t* rset_stamp, uint32_t rset_ep, uint32_t* oldpar,
                     hipStream_t s);

// ---------------------------------------------------------------- aggregate repair
// materialise: every entry of every alive node (list = alive nodes); repair: entries of C
void launch_live_update(const uint32_t* cand, uint32_t k, const uint32_t* rsize_below, uint8_t* alive,
                        uint32_t* par_or_null, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                        SetRef revived, hipStream_t s, const uint32_t* countp = nullptr);
void launch_live_prop(const uint32_t* died, uint32_t nd, const uint32_t* revived, uint32_t nr,
                      const uint32_t* par, uint32_t* rsize, SetRef cand, hipStream_t s);
void launch_label_up(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint8_t* alive_up,
                     const uint32_t* lab, uint32_t* lab_up, hipStream_t s);
void launch_alive_list(uint32_t n, const uint8_t* alive, SetRef set, hipStream_t s);
void launch_materialise_nodes(uint32_t n, const uint32_t* rsize, uint8_t* alive_up, const uint32_t* lab,
                              uint32_t* lab_up, uint32_t* par_up_or_null, hipStream_t s);
void launch_label_refresh(uint32_t n, const uint8_t* alive, const uint32_t* par, const uint32_t* lab_up,
                          uint32_t* lab, SetRef seeds, hipStream_t s);
void launch_recount_degrees(CsrRef c, uint32_t n, int64_t* deg_out, hipStream_t s);
// *total += sum of a[0..n)
void launch_sum_u32(const uint32_t* a, uint32_t n, u64a* total, hipStream_t s);
// *count += alive nodes u < n with stamp[key[u]] == ep
void launch_count_members(uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* stamp, uint32_t ep,
                          u64a* count, hipStream_t s);
// seeds (stamps only) = nodes with an out- or in-entry; *ein += self-loop weights; sum kout kin
// added exactly into (skk_lo, skk_hi)
void launch_refresh_scalars(CsrRef out, CsrRef in, uint32_t n, const int64_t* kout, const int64_t* kin, SetRef seeds,
                            i64a* ein, u64a* skk_lo, i64a* skk_hi, hipStream_t s);
// kout_up[par[u]] += kout[u] (kin likewise when kin_up_or_null is set) over alive u < n
void launch_degrees_up(uint32_t n, const uint8_t* alive, const uint32_t* par, const int64_t* kout, const int64_t* kin,
                       int64_t* kout_up, int64_t* kin_up_or_null, hipStream_t s);

// ---------------------------------------------------------------- library primitives (hipCUB)
// Temporary storage of the primitives comes from this allocator when one is set for the calling
// thread (null: hipMalloc / hipFree); prim_free_tmp releases it the same way.
struct PrimAlloc {
  void* (*alloc)(void* ctx, size_t bytes);
  void (*free)(void* ctx, void* p, size_t bytes);
  void* ctx;
};
void prim_set_allocator(const PrimAlloc* a);
void prim_free_tmp(void* tmp, size_t bytes);
// temp storage is grown on demand through *tmp / *tmp_bytes (device memory owned by caller)
int prim_sort_pairs_u64_u32_db(void** tmp, size_t* tmp_bytes, uint64_t* k0, uint64_t* k1, uint32_t* v0, uint32_t* v1,
                               uint64_t n, int begin_bit, int end_bit, int* sel, hipStream_t s);
int prim_sort_pairs_u64_u32(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                            uint32_t* vout, uint64_t n, int begin_bit, int end_bit, hipStream_t s);
int prim_sort_pairs_u64_i64(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const int64_t* vin,
                            int64_t* vout, uint64_t n, int begin_bit, int end_bit, hipStream_t s);
int prim_reduce_by_key(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const int64_t* vin,
                       int64_t* vout, u64a* nruns, uint64_t n, hipStream_t s);
int prim_exclusive_sum_u64(void** tmp, size_t* tmp_bytes, const uint64_t* in, uint64_t* out, uint64_t n,
                           hipStream_t s);
// ids i < n with stamp[i] == ep, in increasing order, count written to *d_count
int prim_select_stamp(void** tmp, size_t* tmp_bytes, const uint32_t* stamp, uint32_t ep, uint32_t n, uint32_t* out,
                      uint32_t* d_count, hipStream_t s);
// first index of every run of equal rows (key >> ks) in sorted keys, ascending; count to *d_count
int prim_select_heads(void** tmp, size_t* tmp_bytes, const uint64_t* keys, uint64_t k, int ks, uint64_t* out,
                      uint32_t* d_count, hipStream_t s);
int prim_exclusive_sum_u64x3(void** tmp, size_t* tmp_bytes, const U64x3* in, U64x3* out, uint64_t n, hipStream_t s);
int prim_exclusive_sum_u32(void** tmp, size_t* tmp_bytes, const uint32_t* in, uint32_t* out, uint64_t n,
                           hipStream_t s);
int prim_max_u64(void** tmp, size_t* tmp_bytes, const uint64_t* in, u64a* out, uint64_t n, hipStream_t s);

}  // namespace ldl
