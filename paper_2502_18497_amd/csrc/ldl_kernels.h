// Host-side launchers of the LD-Leiden HIP kernels (definitions in kernels_*.hip, prims.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldl {

typedef unsigned long long u64a;
typedef long long i64a;

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
  const uint8_t* alive;
  const int64_t* kout;       // level-r degrees
  const int64_t* kin;
  const int64_t* Kout;       // community totals (move) or refined totals (refinement)
  const int64_t* Kin;
  const uint32_t* rsize;     // refined community sizes (refinement)
  int64_t qm;                // q * m
  int64_t p;                 // gamma numerator
  int directed;
};

struct CandBuf {
  uint32_t* v;
  uint32_t* a;
  uint32_t* b;
  uint64_t* glo;
  int64_t* ghi;
  uint32_t* count;
};

struct HubPool {
  uint32_t* keys;
  u64a* vals;
  u64a* top;           // device bump counter (slots)
  uint64_t cap;        // slots
  uint32_t* over;      // overflow list
  uint32_t* over_count;
};

struct MoveStats {  // per-launch counters (null: not counted)
  u64a* entries;
  u64a* distinct;
  u64a* vertices;
  u64a* cands;
};

constexpr int kNumBins = 5;
constexpr uint32_t kHubScanSlots = 8192;   // table slots evaluated per hub scan workgroup
// degree bins: total entries T in (0,8], (8,32], (32,128], (128,2048], (2048, inf)
constexpr uint32_t kBinLimit[kNumBins - 1] = {8, 32, 128, 2048};

// ---------------------------------------------------------------- sets and generic helpers
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s);
void launch_fill_i64(int64_t* p, int64_t v, uint64_t n, hipStream_t s);
void launch_iota(uint32_t* p, uint64_t n, hipStream_t s);
void launch_copy_i64(int64_t* dst, const int64_t* src, uint64_t n, hipStream_t s);
// set.add(x) for every x in list[0..count)
void launch_set_add_list(SetRef set, const uint32_t* list, uint32_t count, hipStream_t s);
// set.add(key[x]) for every x in list[0..count) (optionally only alive x)
void launch_set_add_mapped(SetRef set, const uint32_t* list, uint32_t count, const uint32_t* key,
                           const uint8_t* alive_or_null, hipStream_t s);
// set.add(u) for every alive u < n with mark[key[u]] == mark_epoch
void launch_members(SetRef set, uint32_t n, const uint8_t* alive, const uint32_t* key, const uint32_t* mark,
                    uint32_t mark_epoch, hipStream_t s);
// plain-store marking (stamp[x] = ep, no list): members of marked keys, listed vertices and
// their neighbours, accepted movers and their neighbours; a later select builds the list
void launch_mark_members(uint32_t* stamp, uint32_t ep, uint32_t n, const uint8_t* alive, const uint32_t* key,
                         const uint32_t* mark, uint32_t mark_ep, hipStream_t s);
void launch_mark_neighbours(uint32_t* stamp, uint32_t ep, const uint32_t* list, uint32_t count, CsrRef out, CsrRef in,
                            int directed, hipStream_t s);
void launch_mark_neighbours_acc(uint32_t* stamp, uint32_t ep, const uint32_t* acc, uint32_t na, CandBuf cand,
                                CsrRef out, CsrRef in, int directed, hipStream_t s);
void launch_mark_changed(uint32_t* stamp, uint32_t ep, const uint32_t* rset, uint32_t nr, const uint32_t* par,
                         const uint32_t* oldpar, hipStream_t s);
// degree binning without global atomics: per-block histograms, scan, fill
constexpr unsigned kBinBlocks = 1024;
void launch_bin_count(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, uint32_t* hist,
                      hipStream_t s);
void launch_bin_fill(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, const uint32_t* offs,
                     uint32_t* out, uint32_t* bin_start, uint32_t* bin_count, hipStream_t s);
// aggregation tuples at precomputed per-node offsets (no global atomics)
void launch_tuple_counts(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* cstamp,
                         uint32_t cep, int repair, uint64_t* counts, hipStream_t s);
void launch_tuples_at(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* par,
                      const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep, int repair, const uint64_t* offs,
                      uint64_t* tkeys, int64_t* tvals, SetRef seeds_or_null, hipStream_t s);
// set.add(u) for u in list and every neighbour of u
void launch_neighbours(SetRef set, const uint32_t* list, uint32_t count, CsrRef out, CsrRef in, int directed,
                       hipStream_t s);

// ---------------------------------------------------------------- dynamic CSR
// Records sorted by key = row << 32 | col with deltas; zero deltas are ignored.
void launch_csr_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, uint8_t* insflag,
                     uint32_t* rowdel, uint32_t* rowins, SetRef dirty, hipStream_t s);
// row segments of sorted keys (first record index per row) and the segment-wise row lookup
void launch_segments(const uint64_t* keys, uint64_t k, uint64_t* seg_lo, uint32_t* nseg, hipStream_t s);
void launch_seg_find(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                     const uint32_t* nseg_ptr, uint32_t nseg_max, int64_t* slot_out, uint8_t* insflag,
                     uint32_t* rowdel, uint32_t* rowins, SetRef dirty, int apply, hipStream_t s);
// row lookup of sorted records split over (segment, record chunk, row slice) items: slot of
// every record (or -1); then the per-segment apply (optionally adding row delta sums to deg)
void launch_seg_lookup(CsrRef c, const uint64_t* keys, uint64_t k, const uint64_t* seg_lo, const uint32_t* nseg_ptr,
                       uint64_t* seg_hi, uint64_t* items, uint64_t* item_off, int64_t* slot_out, void** tmp,
                       size_t* tmp_bytes, hipStream_t s);
void launch_seg_apply(CsrRef c, const uint64_t* keys, const int64_t* delta, uint64_t k, const uint64_t* seg_lo,
                      const uint64_t* seg_hi, const uint32_t* nseg_ptr, const int64_t* slot, uint8_t* insflag,
                      uint32_t* rowdel, uint32_t* rowins, int64_t* deg_arr, uint32_t* dirty_list, uint32_t* dirty_count,
                      hipStream_t s);
void launch_ingest_validate(CsrRef out0, const uint64_t* keys, const uint32_t* idx, const int64_t* slot, uint64_t k,
                            const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                            int directed, int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm,
                            hipStream_t s);
void launch_csr_plan(CsrRef c, const uint32_t* dirty, uint32_t nd, const uint32_t* rowdel, const uint32_t* rowins,
                     uint64_t* plan_off, uint32_t* plan_cap, u64a* pool_top, uint64_t pool_cap, uint32_t* overflow,
                     hipStream_t s);
void launch_csr_rewrite(CsrRef c, const uint32_t* dirty, uint32_t nd, uint32_t* rowdel, uint32_t* rowins,
                        const uint64_t* plan_off, const uint32_t* plan_cap, const uint64_t* keys, const int64_t* delta,
                        const uint8_t* insflag, uint64_t k, hipStream_t s);
void launch_csr_degrees(int64_t* kout, int64_t* kin_or_null, const uint64_t* keys, const int64_t* delta, uint64_t k,
                        hipStream_t s);
// new_cap[u] = deg[u] + slack, for a pool rebuild
void launch_csr_newcap(const uint32_t* deg, uint32_t* newcap, uint64_t* newcap64, uint32_t n, hipStream_t s);
void launch_csr_move_rows(CsrRef from, CsrRef to, const uint64_t* new_off, const uint32_t* new_cap, uint32_t n,
                          hipStream_t s);
void launch_csr_entries(CsrRef c, uint32_t n, uint64_t* out_keys, int64_t* out_w, u64a* counter, hipStream_t s);

// ---------------------------------------------------------------- batch ingest
// kinds: 0 insert (u,v,w), 1 delete (u,v), 2 change (u,v,w)
void launch_ingest_records(const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                           uint64_t nc, uint32_t n, int directed, uint64_t* keys, uint32_t* idx, uint32_t* err,
                           hipStream_t s);
void launch_ingest_check(CsrRef out0, const uint64_t* keys, const uint32_t* idx, uint64_t k, const uint32_t* ins,
                         uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg, int directed,
                         int64_t* delta, uint32_t* err, uint32_t* first_bad, i64a* dm, hipStream_t s);
void launch_ingest_entries(const uint64_t* keys, const int64_t* delta, uint64_t k, int directed, uint64_t* ekeys,
                           int64_t* edelta, u64a* count, hipStream_t s);
// touched communities of the level-0 entries (old totals recorded), seeds at level 0
void launch_ingest_mark(const uint64_t* ekeys, uint64_t k, const uint32_t* lab0, const int64_t* Kout,
                        const int64_t* Kin, SetRef touched, int64_t* tko, int64_t* tki, SetRef seeds0, hipStream_t s);
void launch_ingest_totals(const uint64_t* ekeys, const int64_t* edelta, uint64_t k, const uint32_t* lab0,
                          int64_t* Kout, int64_t* Kin_or_null, i64a* dein, hipStream_t s);
void launch_dskk(const uint32_t* touched, uint32_t nt, const int64_t* Kout, const int64_t* Kin,
                 const int64_t* tko, const int64_t* tki, u64a* lo, i64a* hi, hipStream_t s);
// cascade: (x,y) <- (par[x], par[y]); keys rebuilt; both endpoints seeded
void launch_cascade_map(uint32_t* ex, uint32_t* ey, const int64_t* ed, uint64_t k, const uint32_t* par,
                        uint64_t* keys, int64_t* vals, SetRef seeds, hipStream_t s);
void launch_split_keys(const uint64_t* keys, uint64_t k, uint32_t* ex, uint32_t* ey, hipStream_t s);
void launch_transpose_keys(const uint64_t* keys, uint64_t* tkeys, uint64_t k, hipStream_t s);

// ---------------------------------------------------------------- local move / refinement
void launch_bin(const MoveView& mv, const uint32_t* list, uint32_t count, int refine, uint32_t* const* bins,
                uint32_t* bin_counts, hipStream_t s);
// one launch per bin; bin index b in [0, kNumBins); hub bin may need re-launches on overflow
void launch_best(const MoveView& mv, int bin, const uint32_t* list, uint32_t count, int refine, CandBuf cand,
                 HubPool hub, MoveStats st, hipStream_t s);

// hubs split over workgroups: table sizes, then per group of hubs [i0, i0+ng) whose tables
// span [base0, base0+span) of the pool: clear, insert, scan into partial bests, final reduce
void launch_hub_prep(const MoveView& mv, const uint32_t* list, uint32_t h, uint64_t* hsize, u64a* maxT,
                     hipStream_t s);
void launch_hub_group(const MoveView& mv, const uint32_t* list, uint32_t i0, uint32_t ng, const uint64_t* hoff,
                      uint64_t base0, uint64_t span, uint64_t maxT, int refine, HubPool hub, int64_t* own,
                      uint32_t max_parts, int64_t* phi, uint64_t* plo, uint32_t* pid, int* pvalid, CandBuf cand,
                      MoveStats st, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b);

// ---------------------------------------------------------------- decouple (exact greedy filter)
void launch_rank_from_order(const uint32_t* order, uint32_t k, uint32_t* rank, hipStream_t s);
void launch_gather_u64(const uint64_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst, int invert,
                       hipStream_t s);
void launch_gather_u32_as_u64(const uint32_t* src, const uint32_t* idx, uint32_t k, uint64_t* dst, hipStream_t s);
void launch_lf_reset(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, uint32_t* minE,
                     uint32_t* minA, hipStream_t s);
void launch_lf_min(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* rank,
                   uint32_t* minE, uint32_t* minA, hipStream_t s);
void launch_lf_accept(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* rank,
                      const uint32_t* minE, const uint32_t* minA, uint32_t* accE, uint32_t* accA, uint32_t ep,
                      uint8_t* flag, uint32_t* acc_list, uint32_t* acc_count, hipStream_t s);
void launch_lf_reject(const uint32_t* live, uint32_t nl, const uint32_t* a, const uint32_t* b, const uint32_t* accE,
                      const uint32_t* accA, uint32_t ep, const uint8_t* flag, uint32_t* live2, uint32_t* live2_count,
                      hipStream_t s);

// ---------------------------------------------------------------- commit / rollback / expand
void launch_commit_mark(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* mov_stamp, uint32_t mov_ep,
                        uint32_t* oldlab, const int64_t* Kout, const int64_t* Kin, SetRef touched, int64_t* tko,
                        int64_t* tki, hipStream_t s);
void launch_commit_apply(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* lab, const int64_t* kout,
                         const int64_t* kin, int64_t* Kout, int64_t* Kin_or_null, int forward, hipStream_t s);
void launch_commit_dein(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                        const uint32_t* lab, const uint32_t* mov_stamp, uint32_t mov_ep, const uint32_t* oldlab,
                        i64a* dein, hipStream_t s);
void launch_mark_acc_comms(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* stamp, uint32_t ep,
                           hipStream_t s);
void launch_set_add_acc_v(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand, hipStream_t s);
void launch_neighbours_acc(SetRef set, const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in,
                           int directed, hipStream_t s);

// ---------------------------------------------------------------- refinement bookkeeping
void launch_ref_init_top(uint32_t n, const uint8_t* alive, const int64_t* kout, const int64_t* kin, int64_t* Krout,
                         int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s);
void launch_ref_reset(const uint32_t* R, uint32_t nr, uint32_t* par, uint32_t* oldpar, const int64_t* kout,
                      const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, int phase,
                      hipStream_t s);
void launch_ref_commit(const uint32_t* acc, uint32_t na, CandBuf cand, uint32_t* par, const int64_t* kout,
                       const int64_t* kin, int64_t* Krout, int64_t* Krin_or_null, uint32_t* rsize, hipStream_t s);
void launch_spexpand(const uint32_t* acc, uint32_t na, CandBuf cand, CsrRef out, CsrRef in, int directed,
                     const uint32_t* lab, const uint32_t* par, const uint32_t* rsize, SetRef rcur, SetRef rset,
                     uint32_t* oldpar, hipStream_t s);

// ---------------------------------------------------------------- aggregate repair
void launch_changed(const uint32_t* rset, uint32_t nr, const uint32_t* par, const uint32_t* oldpar, SetRef C,
                    hipStream_t s);
void launch_tuple_count(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, u64a* total,
                        hipStream_t s);
// materialise: every entry of every alive node (list = alive nodes); repair: entries of C
void launch_tuples(const uint32_t* list, uint32_t k, CsrRef out, CsrRef in, int directed, const uint32_t* par,
                   const uint32_t* oldpar, const uint32_t* cstamp, uint32_t cep, int repair, uint64_t* tkeys,
                   int64_t* tvals, u64a* tcount, uint64_t tcap, SetRef seeds_or_null, hipStream_t s);
void launch_live_update(const uint32_t* cand, uint32_t k, const uint32_t* rsize_below, uint8_t* alive,
                        uint32_t* par_or_null, uint32_t* lab, const uint32_t* lab_below, SetRef died,
                        SetRef revived, hipStream_t s);
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

// ---------------------------------------------------------------- library primitives (hipCUB)
// temp storage is grown on demand through *tmp / *tmp_bytes (device memory owned by caller)
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
int prim_exclusive_sum_u32(void** tmp, size_t* tmp_bytes, const uint32_t* in, uint32_t* out, uint64_t n,
                           hipStream_t s);
int prim_max_u64(void** tmp, size_t* tmp_bytes, const uint64_t* in, u64a* out, uint64_t n, hipStream_t s);

}  // namespace ldl
