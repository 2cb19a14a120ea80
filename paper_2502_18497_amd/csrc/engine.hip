// Host engine of the LD-Leiden batch update (Algorithm 1) and the C ABI of include/ldl.h.
//
// Device state per level r = 0..L (node ids share [0, n) at every level, Sec. III-A):
//   dynamic CSR (out; in as well for directed graphs), alive flags, degrees kout/kin, labels
//   P^r, parents pi_r and refined-community sizes (r < L).  Community totals Kout/Kin are one
//   level-invariant table.  The host keeps m, Ein and sum Kout*Kin exactly and reads back the
//   small counters that decide Algorithm 1's data-dependent control flow.
//
// Readings of the paper's open points (also stated in the oracle):
//   * gains are compared exactly as integers; candidates need gain > 0; ties go to the
//     lowest community id; candidates are ordered by gain, then vertex id (Sec. III-E)
//   * every iteration is round-synchronous: candidates see the state at its start
//   * seeds of level r: changed entry endpoints and their ancestors; the frontier is the
//     seeds plus all members of their communities; Expand adds movers, their neighbours and
//     all members of the source and target communities
//   * TouchedRefined: refined communities of the level's seeds and movers, reset to
//     singletons; only singletons move during refinement, to adjacent refined communities
//     carrying the same move label
//   * a level is materialised from scratch (Eq. 3) the first time it is reached; afterwards
//     it is repaired by subtract-add tuples and the tuple deltas cascade to every level above
//   * moves at level r >= 1 are pushed down by relabelling P^s(u) = P^{s+1}(pi_s(u)); the
//     relabelled nodes seed the next outer pass
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ldl.h"
#include "ldl_check.h"
#include "ldl_kernels.h"

namespace ldl {

typedef __int128 i128;


struct DeviceError {
  hipError_t e;
};
struct NoMem {};

static void hcheck(hipError_t e) {
  if (e != hipSuccess) throw DeviceError{e};
}

// Recount sums of ldl_check_invariants_noalloc, for callers that cannot allocate device memory:
// 512 bytes that every device the library runs on holds until the process ends.  Host code never
// uses this name as an address: each device's copy is reached through the address that
// hipGetSymbolAddress returned for it (noalloc_scratch below).
constexpr int kNoAllocWords = 64;
static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];
static_assert(sizeof(InvScratch) <= kNoAllocWords * sizeof(unsigned long long), "recount sums fit the scratch");

// Device address of `scratch` on the current device, looked up once per device (with that
// device current) and kept.
static void* noalloc_scratch(int device) {
  static std::mutex mu;
  static void* addr[256] = {};
  if (device < 0 || device >= 256) throw DeviceError{hipErrorInvalidDevice};
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) throw DeviceError{e == hipSuccess ? hipErrorUnknown : e};
    addr[device] = p;
  }
  return addr[device];
}


// Device-side counters and accumulators, mirrored into pinned host memory on demand.
// Counters written by one candidate pass (cleared together before it).
struct PassScal {
  u64a st_entries[kNumBins], st_distinct[kNumBins], st_vertices[kNumBins], st_cands[kNumBins];
  u64a maxhi;       // max high word of the candidates' gains
  u64a hub_need;    // bucket-pool entries the hub passes needed
  uint32_t ncand;
  uint32_t hub_over;
  // commit of the iteration: exact changes of Ein and sum Kout*Kin, touched communities
  i64a cdein;
  u64a cdskk_lo;
  i64a cdskk_hi;
  uint32_t ntouch;
  uint32_t nbig;    // movers of the commit listed for the split Ein pass
};
static_assert(sizeof(PassScal) % 4 == 0, "PassScal is cleared as 32-bit words");
struct Scal {
  uint32_t counts[64];
  uint32_t bins[8];
  uint32_t bin_start[8];
  uint32_t nacc, nacc2, nlive[2], err, first_bad, nseg, nmove, overflow;   // nmove, overflow adjacent
  u64a pool_top[2 * 17];
  i64a dm, dein;
  u64a dskk_lo;
  i64a dskk_hi;
  u64a tcount, tneed, nruns, ecount, nnz;
  PassScal ps;
};

enum SetId {
  S_D0 = 0,  // 0..16 seed sets per level
  S_U = 17, S_U2, S_S, S_MOVED, S_RSET, S_RCUR, S_C, S_TOUCH, S_COMM, S_REFM, S_MOV, S_LVC, S_DIED,
  S_REV, S_DIED2, S_REV2, S_TMP, S_NSETS
};

struct HSet {
  uint32_t* stamp = nullptr;
  uint32_t* list = nullptr;
  uint32_t epoch = 0;
  int ci = 0;
};

struct Csr {
  CsrRef ref{};
  uint64_t pool_cap = 0;
  int slot = 0;  // index of its pool-top counter
};

struct Level {
  Csr out, in;
  uint8_t* alive = nullptr;
  int64_t* kout = nullptr;
  int64_t* kin = nullptr;  // == kout for undirected graphs
  uint32_t* lab = nullptr;
  uint32_t* par = nullptr;
  uint32_t* rsize = nullptr;
};

struct TraceRec {
  int64_t v[8];
};

struct Engine {
  // configuration
  int directed = 0;
  int64_t gp = 1, gq = 1;
  int N = 2, L = 4, M = 5;
  int64_t an = 1, ad = 1000, bn = 1, bd = 100;
  int64_t rn = 0, rd = 1;   // adaptive refresh threshold (0: never)
  int empty_target = 0;     // BestMove may also target the empty community labelled by the vertex
  uint64_t scratch_limit = 0;   // free the growable scratch after a call that leaves more (0: keep)
  int refine_random = 0;        // BestRef draws among improving targets (seeded)
  uint64_t refine_seed = 0;
  uint64_t batches = 0;         // batches accepted so far (creation's is batch 0)
  uint64_t cur_batch = 0;       // index of the batch being applied
  uint64_t cur_rkey = 0;        // key of the current refinement iteration's draw (0: none)
  int device = 0;
  int profile = 0;
  int test_flags = 0;   // see ldl_config
  hipStream_t st = nullptr;
  bool own_stream = false;
  InvScratch* static_sums = nullptr;   // this device's copy of `scratch` (allocation-free recount)
  uint32_t n = 0;
  int id_bits = 32;     // bits of a vertex id: keys row << 32 | col need 2 * id_bits bits
  bool broken = false;
  bool mutating = false;   // the current call has passed validation and started changing state

  // exact scalars (host)
  int64_t m = 0, Ein = 0;
  i128 SKK = 0;
  int top = 0;
  int pass_idx = 0;

  std::vector<Level> lv;
  int64_t* Kout = nullptr;
  int64_t* Kin = nullptr;

  Scal* ds = nullptr;
  Scal* hs = nullptr;
  HSet sets[S_NSETS];
  bool set_has_list[S_NSETS];
  bool set_selected[S_NSETS];   // list and count always rebuilt by a select

  // scratch (size n unless noted)
  uint32_t *oldlab = nullptr, *oldpar = nullptr, *rowdel = nullptr, *rowins = nullptr;
  uint32_t* bigmov = nullptr;   // movers with long rows, for the split Ein pass of a commit
  uint2* lpk = nullptr;   // (label, parent) of the level being refined, packed for one gather
  // Deferred aggregate records per level (entry deltas not yet applied to that level's CSR; the
  // level's degrees already include them).  See defer() and flush_to().
  struct PendBuf {
    uint64_t* keys = nullptr;
    int64_t* vals = nullptr;
    uint64_t count = 0, cap = 0;
  };
  std::vector<PendBuf> pend;
  // rebuild_flag[s]: level s's matrix is rebuilt from level s-1 by Eq. 3 before it is next read,
  // instead of applying its deferred records (set when a repair would sort more tuples than a
  // rebuild, or more than one chunk); its degrees stay exact meanwhile
  std::vector<uint8_t> rebuild_flag;
  // Tuples are sorted in chunks of at most this many (radix-sort and tuple buffers are sized by
  // it); test flag 128 makes the chunks tiny so that every path through them is exercised.
  static constexpr uint64_t kTupleChunk = 1ull << 28;
  uint64_t tuple_chunk() const { return (test_flags & 128) ? 4096 : kTupleChunk; }
  static constexpr int kChunkSlot = 60;   // ds->counts word holding a chunk's list length
  uint32_t lim[2][kNumBins - 1];   // degree-bin limits for 32-bit (level 0) and 64-bit weights
  uint32_t *accE = nullptr, *accA = nullptr;
  LfFirst lfE{}, lfA{};
  uint32_t *lf_la = nullptr, *lf_lb = nullptr;
  int lf_ca = 0;                 // index of lf_la's count in ds->nlive
  uint32_t acc_epoch = 0;
  uint8_t* lfflag = nullptr;
  uint32_t *liveA = nullptr, *liveB = nullptr, *acc = nullptr, *entry = nullptr;
  int64_t *tko = nullptr, *tki = nullptr;
  uint32_t* bins[kNumBins] = {};
  uint32_t* binbuf = nullptr;
  uint32_t* bhist = nullptr;
  uint64_t *tcounts = nullptr, *toffs = nullptr, *tcur = nullptr, *it_cnt = nullptr, *it_off = nullptr;
  uint64_t* it_csum = nullptr;   // chunk sums of the item scan
  HubWork hw{};
  uint64_t part_cap = 0;
  uint64_t hw_cap = 0;   // entries of hw.cnt / hw.off / hw.own
  CandBuf cand{};
  HubPool hub{};
  // growable record buffers
  uint64_t rec_cap = 0;
  uint64_t *rkey0 = nullptr, *rkey1 = nullptr;
  uint32_t *ridx0 = nullptr, *ridx1 = nullptr;
  int64_t* rdelta = nullptr;
  uint64_t ent_cap = 0;
  uint64_t *ekey0 = nullptr, *ekey1 = nullptr;
  int64_t *edel0 = nullptr, *edel1 = nullptr;
  uint32_t *ex = nullptr, *ey = nullptr;
  uint8_t* insflag = nullptr;     // record types of the row update
  uint64_t* holebuf = nullptr;
  uint32_t* movelist = nullptr;
  uint64_t* seg_lo = nullptr;
  uint64_t *seg_hi = nullptr, *items = nullptr, *item_off = nullptr, *items_big = nullptr, *item_off_big = nullptr;
  int64_t* slotbuf = nullptr;
  int64_t* rslot = nullptr;
  uint64_t ins_cap = 0;
  uint64_t tup_cap = 0;
  uint64_t *tk0 = nullptr, *tk1 = nullptr, *tk2 = nullptr;
  int64_t *tv0 = nullptr, *tv1 = nullptr, *tv2 = nullptr;
  uint32_t *tx = nullptr, *ty = nullptr;
  void* cub_tmp = nullptr;
  size_t cub_bytes = 0;
  // a host batch's staging: pinned host words and device words, grown on demand and kept, so a
  // call allocates (and frees) nothing in the steady state
  uint32_t* stage_h = nullptr;
  uint32_t* stage_d = nullptr;
  uint64_t stage_hcap = 0, stage_dcap = 0;
  hipEvent_t call_t0 = nullptr, call_t1 = nullptr;   // brackets of a call (its total_ms)
  static constexpr uint64_t kPinnedStageMax = 1ull << 26;   // words staged through pinned memory
  // device memory: hipMalloc / hipFree, or the caller's allocator hook (ldl_config.alloc/free)
  ldl_alloc_fn halloc = nullptr;
  ldl_free_fn hfree = nullptr;
  void* hctx = nullptr;
  PrimAlloc palloc{};   // the same source for the library primitives' temporary storage
  std::vector<std::pair<void*, uint64_t>> owned;
  // device bytes held now, at the start of the current call and at its peak; the growth of the
  // last batch calls (the serving loop's admission reads it through ldl_memory)
  uint64_t held = 0, call_start = 0, call_peak = 0;
  uint64_t growth_hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t growth_next = 0, calls_done = 0;
  void call_begin() { call_start = call_peak = held; }
  void call_end() {
    if (calls_done++ == 0) return;   // creation's own allocations are the state, not scratch growth
    growth_hist[growth_next++ % 8] = call_peak - call_start;
  }
  uint64_t recent_growth() const {
    uint64_t g = 0;
    for (uint64_t x : growth_hist) g = std::max(g, x);
    return g;
  }

  // statistics / trace
  ldl_batch_stats stats{};
  bool tracing = false;
  std::vector<TraceRec> trace;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  struct Pending {
    int bin;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;

  // ------------------------------------------------------------------ memory helpers
  void* raw_alloc(uint64_t bytes) {
    if (bytes == 0) bytes = 1;
    void* p = nullptr;
    if (halloc) {
      p = halloc(hctx, bytes, device, (void*)st);
      if (!p) throw NoMem{};
    } else {
      const hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        throw NoMem{};
      }
      hcheck(e);
    }
    held += bytes;
    call_peak = std::max(call_peak, held);
    return p;
  }
  void raw_free(void* p, uint64_t bytes) {
    if (!p) return;
    held -= std::min(held, bytes);
    if (hfree) hfree(hctx, p, bytes, device, (void*)st);
    else (void)hipFree(p);
  }
  static void* prim_alloc_cb(void* ctx, size_t bytes) {
    try {
      return ((Engine*)ctx)->raw_alloc(bytes);
    } catch (...) {
      return nullptr;
    }
  }
  static void prim_free_cb(void* ctx, void* p, size_t bytes) { ((Engine*)ctx)->raw_free(p, bytes); }
  template <typename T>
  T* alloc(uint64_t count) {
    const uint64_t bytes = (count ? count : 1) * sizeof(T);
    T* p = (T*)raw_alloc(bytes);
    owned.push_back(std::make_pair((void*)p, bytes));
    return p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find_if(owned.begin(), owned.end(), [&](const std::pair<void*, uint64_t>& o) { return o.first == p; });
    if (it == owned.end()) return;
    const uint64_t bytes = it->second;
    owned.erase(it);
    raw_free(p, bytes);
  }
  template <typename T>
  void regrow(T*& p, uint64_t count) {
    release((void*)p);
    p = alloc<T>(count);
  }

  ~Engine() {
    if (st) (void)hipStreamSynchronize(st);
    for (auto& o : owned) raw_free(o.first, o.second);
    if (hs) (void)hipHostFree(hs);
    if (stage_h) (void)hipHostFree(stage_h);
    if (call_t0) (void)hipEventDestroy(call_t0);
    if (call_t1) (void)hipEventDestroy(call_t1);
    raw_free(cub_tmp, cub_bytes);   // allocated through the same source (palloc)
    for (auto& e : ev_pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    if (own_stream && st) (void)hipStreamDestroy(st);
  }

  // ------------------------------------------------------------------ sets
  SetRef ref(int id) {
    HSet& s = sets[id];
    return SetRef{s.stamp, set_has_list[id] ? s.list : nullptr, &ds->counts[s.ci], s.epoch};
  }
  // empty a set: a new epoch, and a zero count for sets whose kernels append to the list
  void begin(int id) {
    HSet& s = sets[id];
    if (++s.epoch == 0) {
      hcheck(hipMemsetAsync(s.stamp, 0, sizeof(uint32_t) * (uint64_t)n, st));
      s.epoch = 1;
    }
    if (set_has_list[id] && !set_selected[id]) hcheck(hipMemsetAsync(&ds->counts[s.ci], 0, sizeof(uint32_t), st));
  }
  // a new epoch only (the caller counts the members elsewhere)
  void begin_epoch(int id) {
    HSet& s = sets[id];
    if (++s.epoch == 0) {
      hcheck(hipMemsetAsync(s.stamp, 0, sizeof(uint32_t) * (uint64_t)n, st));
      s.epoch = 1;
    }
  }
  uint32_t count(int id) const { return hs->counts[sets[id].ci]; }
  void sync_read() {
    hcheck(hipMemcpyAsync(hs, ds, sizeof(Scal), hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    stats.host_syncs++;
  }
  template <typename T>
  void zero(T* field) {
    hcheck(hipMemsetAsync(field, 0, sizeof(T), st));
  }

  i128 qnum() const { return (i128)gq * m * Ein - (i128)gp * SKK; }

  // list of a marked set: ids with stamp == epoch (list order carries no meaning), count into the
  // set's counter
  void select_set(int id) {
    HSet& s = sets[id];
    launch_select_stamp(s.stamp, s.epoch, n, s.list, &ds->counts[s.ci], st);
  }

  // per-node tuple counts over the list of set `sid` (k nodes) and their exclusive prefix
  // (toffs); returns the tuple total and grows the tuple buffers
  uint64_t tuple_offsets(int sid, uint32_t k, CsrRef out, CsrRef in, const uint2* po, int repair, bool grow = true) {
    return tuple_offsets_at(sets[sid].list, &ds->counts[sets[sid].ci], k, out, in, po, repair, grow);
  }
  // the same over list[0..k) with its length in the device word cnt; grow = false leaves the
  // tuple buffers as they are (the caller decides how the tuples are produced)
  uint64_t tuple_offsets_at(const uint32_t* list, const uint32_t* cnt, uint32_t k, CsrRef out, CsrRef in,
                            const uint2* po, int repair, bool grow) {
    if (k == 0) return 0;
    launch_items(list, nullptr, cnt, k, out, in, it_cnt, it_off, it_csum, tcounts, tcur, st);
    launch_tuples_count(list, cnt, k, it_off, out, in, po, repair, (u64a*)tcounts, st);
    cub(prim_exclusive_sum_u64(&cub_tmp, &cub_bytes, tcounts, toffs, (uint64_t)k + 1, st));
    uint64_t T = 0;
    hcheck(hipMemcpyAsync(&T, toffs + k, 8, hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    if (grow) ensure_tuples(T + 16);
    return T;
  }

  // ------------------------------------------------------------------ setup
  void init(const ldl_config& c, uint32_t n_) {
    directed = c.directed != 0;
    gp = c.gamma_num; gq = c.gamma_den;
    N = c.N; L = c.L; M = c.M;
    an = c.alpha_num; ad = c.alpha_den; bn = c.beta_num; bd = c.beta_den;
    rn = c.refresh_num; rd = c.refresh_den;
    empty_target = c.empty_target;
    scratch_limit = c.scratch_limit;
    refine_random = c.refine_random;
    refine_seed = c.refine_seed;
    halloc = c.alloc;
    hfree = c.free;
    hctx = c.alloc_ctx;
    if (halloc) {
      palloc = PrimAlloc{&Engine::prim_alloc_cb, &Engine::prim_free_cb, this};
      prim_set_allocator(&palloc);   // for the rest of this call (the entry point resets it)
    }
    device = c.device;
    profile = c.profile;
    test_flags = c.test_flags;
    n = n_;
    id_bits = 1;
    while (id_bits < 32 && (1ull << id_bits) < (uint64_t)n) ++id_bits;
    hcheck(hipSetDevice(device));
    static_sums = (InvScratch*)noalloc_scratch(device);
    if (c.stream) {
      st = (hipStream_t)c.stream;
    } else {
      hcheck(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      own_stream = true;
    }
    ds = alloc<Scal>(1);
    hcheck(hipMemsetAsync(ds, 0, sizeof(Scal), st));
    void* hp = nullptr;
    hcheck(hipHostMalloc(&hp, sizeof(Scal), hipHostMallocDefault));
    hs = (Scal*)hp;
    std::memset(hs, 0, sizeof(Scal));
    for (int i = 0; i < S_NSETS; ++i) {
      set_has_list[i] = !(i == S_COMM || i == S_REFM || i == S_MOV);
      set_selected[i] = i == S_U || i == S_U2 || i == S_S || i == S_RCUR || i == S_RSET || i == S_C;
      if (i <= 16 && i > L) continue;
      sets[i].stamp = alloc<uint32_t>(n);
      hcheck(hipMemsetAsync(sets[i].stamp, 0, sizeof(uint32_t) * (uint64_t)n, st));
      if (set_has_list[i]) sets[i].list = alloc<uint32_t>(n);
      sets[i].ci = i;
      sets[i].epoch = 0;
    }
    for (int i = 0; i < S_NSETS; ++i)
      if (sets[i].stamp) begin(i);   // epoch 1: stamps start at 0, so every set starts empty
    hcheck(hipMemsetAsync(ds->counts, 0, sizeof(ds->counts), st));
    lv.resize(L + 1);
    pend.resize(L + 1);
    rebuild_flag.assign(L + 2, 0);
    for (int r = 0; r <= L; ++r) {
      Level& V = lv[r];
      V.alive = alloc<uint8_t>(n);
      V.kout = alloc<int64_t>(n);
      V.kin = directed ? alloc<int64_t>(n) : V.kout;
      V.lab = alloc<uint32_t>(n);
      launch_fill_u8(V.alive, r == 0 ? 1 : 0, n, st);
      launch_fill_i64(V.kout, 0, n, st);
      if (directed) launch_fill_i64(V.kin, 0, n, st);
      launch_iota(V.lab, n, st);
      if (r < L) {
        V.par = alloc<uint32_t>(n);
        V.rsize = alloc<uint32_t>(n);
        launch_iota(V.par, n, st);
        launch_fill_u32(V.rsize, 0, n, st);
      }
      V.out.slot = 2 * r;
      V.in.slot = 2 * r + 1;
      csr_init(V.out, r > 0);
      if (directed) csr_init(V.in, r > 0);
    }
    Kout = alloc<int64_t>(n);
    Kin = directed ? alloc<int64_t>(n) : Kout;
    launch_fill_i64(Kout, 0, n, st);
    if (directed) launch_fill_i64(Kin, 0, n, st);
    oldlab = alloc<uint32_t>(n);
    lpk = alloc<uint2>(n);
    for (int w = 0; w < 2; ++w)
      for (int b = 0; b < kNumBins - 1; ++b) lim[w][b] = kBinLimit[b];
    std::memset(lf_lastK, 0xFF, sizeof(lf_lastK));
    std::memset(lf_first, 0xFF, sizeof(lf_first));
    oldpar = alloc<uint32_t>(n);
    bigmov = alloc<uint32_t>(n);
    rowdel = alloc<uint32_t>(n);
    rowins = alloc<uint32_t>(n);
    lfE = LfFirst{alloc<u64a>(n), alloc<u64a>(n), alloc<uint32_t>(n)};
    lfA = LfFirst{alloc<u64a>(n), alloc<u64a>(n), alloc<uint32_t>(n)};
    for (LfFirst* f : {&lfE, &lfA}) {   // empty: the decoupling rounds keep them so
      hcheck(hipMemsetAsync(f->hi, 0, 8ull * n, st));
      hcheck(hipMemsetAsync(f->lo, 0, 8ull * n, st));
      hcheck(hipMemsetAsync(f->v, 0xFF, 4ull * n, st));
    }
    accE = alloc<uint32_t>(n);
    accA = alloc<uint32_t>(n);
    launch_fill_u32(accE, 0, n, st);
    launch_fill_u32(accA, 0, n, st);
    lfflag = alloc<uint8_t>(n);
    liveA = alloc<uint32_t>(n);
    liveB = alloc<uint32_t>(n);
    acc = alloc<uint32_t>(n);
    entry = alloc<uint32_t>(n);
    tko = alloc<int64_t>(n);
    tki = alloc<int64_t>(n);
    for (int b = 0; b < kNumBins; ++b) bins[b] = nullptr;
    binbuf = alloc<uint32_t>(n);
    bhist = alloc<uint32_t>(kNumBins * kBinBlocks + 1);
    hcheck(hipMemsetAsync(bhist, 0, 4ull * (kNumBins * kBinBlocks + 1), st));
    tcounts = alloc<uint64_t>((uint64_t)n + 1);
    toffs = alloc<uint64_t>((uint64_t)n + 1);
    hcheck(hipMemsetAsync(tcounts, 0, 8ull * ((uint64_t)n + 1), st));
    tcur = alloc<uint64_t>((uint64_t)n + 1);
    it_cnt = alloc<uint64_t>((uint64_t)n + 1);
    it_off = alloc<uint64_t>((uint64_t)n + 1);
    it_csum = alloc<uint64_t>(kItemScanBlocks);
    cand.v = alloc<uint32_t>(n);
    cand.a = alloc<uint32_t>(n);
    cand.b = alloc<uint32_t>(n);
    cand.glo = alloc<uint64_t>(n);
    cand.ghi = alloc<int64_t>(n);
    cand.count = &ds->ps.ncand;
    hub.top = &ds->ps.hub_need;
    hub.over_count = &ds->ps.hub_over;
    hw.pshift = 0;
    hw.tslots = (test_flags & 16) ? 64u : kPartSlots;
    hub_pool((test_flags & 2) ? 0 : std::min<uint64_t>(4ull * n, 1ull << 26));
    hcheck(hipStreamSynchronize(st));
  }

  // (re)allocate the hub bucket pool for at least `entries` entries and its partition arrays
  // (partition counts and cursors start at zero; the hub kernels return them to zero)
  void hub_pool(uint64_t entries) {
    uint64_t hc = (test_flags & 2) ? 256 : 1ull << 16;
    if (hc < entries) hc = (entries + entries / 8 + 0xFFFF) & ~0xFFFFull;
    release(hub.ekey);
    release(hub.ew);
    release(hub.bkey);
    release(hub.bw);
    hub.ekey = nullptr;
    hub.ew = nullptr;
    hub.bkey = nullptr;
    hub.bw = nullptr;
    hub.ekey = alloc<uint32_t>(hc);
    hub.ew = alloc<int64_t>(hc);
    hub.bkey = alloc<uint32_t>(hc);
    hub.bw = alloc<int64_t>(hc);
    hub.cap = hc;
  }
  // per-hub work arrays for at most `bound` hubs and partition arrays for the pool's entries (a
  // hub of T entries has ceil(T 2^pshift / kPartEntries) partitions, at most one per 16 entries);
  // partition counts and cursors start at zero and the hub kernels return them to zero
  void hub_work(uint32_t bound) {
    const uint64_t per = std::min<uint64_t>((hub.cap << hw.pshift) / kPartEntries, hub.cap / 16);
    const uint64_t parts = per + (uint64_t)bound + 2;
    if ((uint64_t)bound + 1 <= hw_cap && parts <= part_cap) return;
    hcheck(hipStreamSynchronize(st));   // queued hub passes may still use the arrays
    if ((uint64_t)bound + 1 > hw_cap) {
      const uint64_t c = std::min<uint64_t>((uint64_t)n + 1, (uint64_t)bound + 1 + bound / 4);
      regrow(hw.cnt, c); regrow(hw.off, c); regrow(hw.own, c);
      hw_cap = c;
    }
    if (parts > part_cap) {
      regrow(hw.phi, parts); regrow(hw.plo, parts); regrow(hw.pid, parts); regrow(hw.pvalid, parts);
      regrow(hw.pcount, parts); regrow(hw.pcur, parts); regrow(hw.poff, parts); regrow(hw.pcnt, parts);
      regrow(hw.icnt, parts);   // chunk items: at most one per kPartEntries entries, so fewer than partitions
      hcheck(hipMemsetAsync(hw.pcount, 0, 4ull * parts, st));
      hcheck(hipMemsetAsync(hw.pcur, 0, 4ull * parts, st));
      part_cap = parts;
    }
  }

  // upper bound on the number of hub vertices (more than kBinLimit[kNumBins - 2] entries) of level r
  uint32_t hub_bound(int r) const {
    const Level& V = lv[r];
    const uint64_t ent = V.out.pool_cap + (directed ? V.in.pool_cap : 0);
    const uint64_t b = ent / ((uint64_t)lim[V.out.ref.wide][kNumBins - 2] + 1) + 1;
    return (uint32_t)std::min<uint64_t>(b, n);
  }

  void csr_init(Csr& c, bool wide) {
    c.ref.off = alloc<uint64_t>(n);
    c.ref.deg = alloc<uint32_t>(n);
    c.ref.cap = alloc<uint32_t>(n);
    hcheck(hipMemsetAsync(c.ref.off, 0, 8ull * n, st));
    hcheck(hipMemsetAsync(c.ref.deg, 0, 4ull * n, st));
    hcheck(hipMemsetAsync(c.ref.cap, 0, 4ull * n, st));
    c.ref.wide = wide ? 1 : 0;
    c.ref.nbr = nullptr;
    c.ref.w = nullptr;
    c.pool_cap = 0;
  }

  // ------------------------------------------------------------------ growable buffers
  void ensure_records(uint64_t k) {
    if (k <= rec_cap) return;
    uint64_t c = std::max<uint64_t>(k, rec_cap * 2);
    regrow(rkey0, c); regrow(rkey1, c); regrow(ridx0, c); regrow(ridx1, c); regrow(rdelta, c); regrow(rslot, c);
    rec_cap = c;
  }
  void ensure_entries(uint64_t k) {
    if (k <= ent_cap) return;
    uint64_t c = std::max<uint64_t>(k, ent_cap * 2);
    regrow(ekey0, c); regrow(ekey1, c); regrow(edel0, c); regrow(edel1, c); regrow(ex, c); regrow(ey, c);
    ent_cap = c;
  }
  void ensure_insflag(uint64_t k) {
    if (k <= ins_cap) return;
    uint64_t c = std::max<uint64_t>(k, ins_cap * 2);
    regrow(insflag, c);
    regrow(holebuf, c);
    regrow(movelist, c);
    regrow(seg_lo, c);
    regrow(seg_hi, c);
    regrow(items, c + 1);
    regrow(item_off, c + 1);
    regrow(items_big, c + 1);
    regrow(item_off_big, c + 1);
    regrow(slotbuf, c);
    ins_cap = c;
  }
  void ensure_tuples(uint64_t k) {
    if (k <= tup_cap) return;
    uint64_t c = std::max<uint64_t>(k, tup_cap + tup_cap / 2);
    regrow(tk0, c); regrow(tk1, c); regrow(tk2, c); regrow(tv0, c); regrow(tv1, c); regrow(tv2, c);
    regrow(tx, c); regrow(ty, c);
    tup_cap = c;
  }
  // Free the growable scratch (aggregation tuples, reduced records, sorted entries, row-update
  // buffers, the library primitives' temporary storage); the next call that needs them allocates
  // them again at its own size.  The state is untouched.
  uint64_t scratch_bytes() const {
    return tup_cap * 56 + rec_cap * 40 + ent_cap * 40 + ins_cap * 69 + cub_bytes + 4 * stage_dcap;
  }
  // device words holding a host batch of `words` words (copied through pinned host memory)
  uint32_t* stage_batch(const uint32_t* ins, uint64_t ni, const uint32_t* del, uint64_t nd, const uint32_t* chg,
                        uint64_t nc) {
    const uint64_t words = 3 * ni + 2 * nd + 3 * nc;
    if (words == 0) return nullptr;
    if (words > stage_dcap) {
      release(stage_d);
      stage_d = nullptr;
      stage_dcap = 0;
      const uint64_t c = std::max<uint64_t>(words, 1ull << 16);
      stage_d = alloc<uint32_t>(c);
      stage_dcap = c;
    }
    if (words > kPinnedStageMax) {   // a large batch (a graph's first) is copied from its own pages
      if (ni) hcheck(hipMemcpyAsync(stage_d, ins, 12 * ni, hipMemcpyHostToDevice, st));
      if (nd) hcheck(hipMemcpyAsync(stage_d + 3 * ni, del, 8 * nd, hipMemcpyHostToDevice, st));
      if (nc) hcheck(hipMemcpyAsync(stage_d + 3 * ni + 2 * nd, chg, 12 * nc, hipMemcpyHostToDevice, st));
      return stage_d;
    }
    if (words > stage_hcap) {
      if (stage_h) hcheck(hipHostFree(stage_h));
      stage_h = nullptr;
      stage_hcap = 0;
      const uint64_t c = std::max<uint64_t>(words, 1ull << 16);
      if (hipHostMalloc((void**)&stage_h, 4 * c, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        stage_h = nullptr;
        throw NoMem{};
      }
      stage_hcap = c;
    }
    // the previous call's copy out of stage_h ended with that call (its stream was synchronised)
    if (ni) std::memcpy(stage_h, ins, 12 * ni);
    if (nd) std::memcpy(stage_h + 3 * ni, del, 8 * nd);
    if (nc) std::memcpy(stage_h + 3 * ni + 2 * nd, chg, 12 * nc);
    hcheck(hipMemcpyAsync(stage_d, stage_h, 4 * words, hipMemcpyHostToDevice, st));
    return stage_d;
  }
  void release_scratch() {
    hcheck(hipStreamSynchronize(st));
    for (void** p : {(void**)&tk0, (void**)&tk1, (void**)&tk2, (void**)&tv0, (void**)&tv1, (void**)&tv2,
                     (void**)&tx, (void**)&ty, (void**)&rkey0, (void**)&rkey1, (void**)&ridx0, (void**)&ridx1,
                     (void**)&rdelta, (void**)&rslot, (void**)&ekey0, (void**)&ekey1, (void**)&edel0,
                     (void**)&edel1, (void**)&ex, (void**)&ey, (void**)&insflag, (void**)&holebuf,
                     (void**)&movelist, (void**)&seg_lo, (void**)&seg_hi, (void**)&items, (void**)&item_off,
                     (void**)&items_big, (void**)&item_off_big, (void**)&slotbuf}) {
      release(*p);
      *p = nullptr;
    }
    tup_cap = rec_cap = ent_cap = ins_cap = 0;
    release(stage_d);
    stage_d = nullptr;
    stage_dcap = 0;
    if (stage_h) hcheck(hipHostFree(stage_h));
    stage_h = nullptr;
    stage_hcap = 0;
    prim_free_tmp(cub_tmp, cub_bytes);
    cub_tmp = nullptr;
    cub_bytes = 0;
  }
  void cub(int rc) {
    if (rc == -2) throw NoMem{};
    if (rc != 0) throw DeviceError{hipErrorUnknown};
  }

  // ------------------------------------------------------------------ dynamic CSR
  // Rebuild the pool of c with per-row slack and room for `extra` more slots (plus a share of
  // 2^-room_shift of the total for rows that move later).
  void csr_grow(Csr& c, uint64_t extra, int room_shift = 1) {
    uint32_t* newcap = alloc<uint32_t>(n);
    uint64_t* newcap64 = alloc<uint64_t>(n);
    uint64_t* newoff = alloc<uint64_t>(n);
    const int tight = (test_flags & 4) ? 1 : 0;
    launch_csr_newcap(c.ref.deg, newcap, newcap64, n, tight, st);
    cub(prim_exclusive_sum_u64(&cub_tmp, &cub_bytes, newcap64, newoff, n, st));
    uint64_t last_off = 0, last_cap = 0;
    hcheck(hipMemcpyAsync(&last_off, newoff + (n - 1), 8, hipMemcpyDeviceToHost, st));
    hcheck(hipMemcpyAsync(&last_cap, newcap64 + (n - 1), 8, hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    const uint64_t used = last_off + last_cap;
    uint64_t cap = tight ? used + extra : used + extra + ((used + extra) >> room_shift) + 1024;
    CsrRef to = c.ref;
    to.nbr = alloc<uint32_t>(cap);
    to.w = c.ref.wide ? (void*)alloc<int64_t>(cap) : (void*)alloc<uint32_t>(cap);
    if (c.ref.nbr) launch_csr_move_rows(c.ref, to, newoff, newcap, n, st);
    else {
      hcheck(hipMemcpyAsync(c.ref.off, newoff, 8ull * n, hipMemcpyDeviceToDevice, st));
      hcheck(hipMemcpyAsync(c.ref.cap, newcap, 4ull * n, hipMemcpyDeviceToDevice, st));
    }
    hcheck(hipStreamSynchronize(st));
    release(c.ref.nbr);
    release(c.ref.w);
    c.ref.nbr = to.nbr;
    c.ref.w = to.w;
    c.pool_cap = cap;
    hcheck(hipMemcpyAsync(&ds->pool_top[c.slot], &used, 8, hipMemcpyHostToDevice, st));
    hcheck(hipStreamSynchronize(st));
    release(newcap);
    release(newcap64);
    release(newoff);
  }

  // Apply sorted records (key = row << id_bits | col, distinct keys) to one orientation; when
  // deg_arr is given, each row's delta sum is added to it.  Rows are updated in place; rows
  // that outgrow their capacity move to new pool regions (the pool grows when full).
  void csr_apply(Csr& c, const uint64_t* keys, const int64_t* delta, uint64_t k, int64_t* deg_arr) {
    if (k == 0) return;
    if (!c.ref.nbr) csr_grow(c, k + 4ull * n);
    ensure_insflag(k);
    cub(prim_select_heads(&cub_tmp, &cub_bytes, keys, k, id_bits, seg_lo, &ds->nseg, st));
    cub(launch_seg_lookup(c.ref, keys, k, seg_lo, &ds->nseg, seg_hi, items, item_off, items_big, item_off_big,
                          slotbuf, &cub_tmp, &cub_bytes, id_bits, st));
    hcheck(hipMemsetAsync(&ds->nmove, 0, 2 * sizeof(uint32_t), st));   // nmove, overflow
    launch_seg_update(c.ref, keys, delta, k, seg_lo, seg_hi, &ds->nseg, slotbuf, insflag, holebuf, deg_arr, rowdel,
                      rowins, movelist, &ds->nmove, id_bits, st);
    launch_seg_move(c.ref, keys, delta, k, seg_lo, seg_hi, insflag, rowdel, rowins, movelist, &ds->nmove,
                    &ds->pool_top[c.slot], c.pool_cap, &ds->overflow, (test_flags & 4) ? 1 : 0, id_bits, st);
    sync_read();
    for (int attempt = 0; hs->overflow; ++attempt) {
      if (attempt > 6) throw NoMem{};
      csr_grow(c, 2 * k + (c.pool_cap / 4 << attempt));   // the extra room doubles per failed attempt
      zero(&ds->overflow);
      launch_seg_move(c.ref, keys, delta, k, seg_lo, seg_hi, insflag, rowdel, rowins, movelist, &ds->nmove,
                      &ds->pool_top[c.slot], c.pool_cap, &ds->overflow, (test_flags & 4) ? 1 : 0, id_bits, st);
      sync_read();
    }
  }

  // Apply reduced records to level s (out, and in via a transposed sort when directed).
  void apply_records(int s, const uint64_t* keys, const int64_t* vals, uint64_t k, bool degrees) {
    if (k == 0) return;
    Level& V = lv[s];
    csr_apply(V.out, keys, vals, k, degrees ? V.kout : nullptr);
    if (directed) {
      // scratch tk1/tk2/tv2 must not alias the caller's keys/vals
      if (k > tup_cap || keys == tk1 || keys == tk2 || vals == tv2) throw DeviceError{hipErrorInvalidValue};
      launch_transpose_keys(keys, tk2, k, id_bits, st);
      cub(prim_sort_pairs_u64_i64(&cub_tmp, &cub_bytes, tk2, tk1, vals, tv2, k, 0, 2 * id_bits, st));
      // tk1 and tv2 now hold the transposed records in (col, row) order
      csr_apply(V.in, tk1, tv2, k, degrees ? V.kin : nullptr);
    }
  }

  // sort (keys, vals) of length k and reduce equal keys; result in (tk2, tv2) with *runs
  uint64_t sort_reduce(uint64_t* keys, int64_t* vals, uint64_t k, uint64_t* okeys, int64_t* ovals) {
    if (k == 0) return 0;
    cub(prim_sort_pairs_u64_i64(&cub_tmp, &cub_bytes, keys, tk1, vals, tv1, k, 0, 2 * id_bits, st));
    cub(prim_reduce_by_key(&cub_tmp, &cub_bytes, tk1, okeys, tv1, ovals, &ds->nruns, k, st));
    sync_read();
    return hs->nruns;
  }

  // ------------------------------------------------------------------ deferred aggregate records
  // Entry deltas for an aggregate level s >= 1 (from the batch's level-0 changes and from the
  // subtract-add tuples of aggregate repair) are appended to pend[s] and applied to the CSR of
  // level s in one sort, reduce and row update right before level s is processed (and for every
  // level before the call returns); the reduced deltas then cascade to level s+1 through pi_s
  // the same way.  Integer sums commute, so the CSRs are exactly those of applying every delta at
  // once.  Nothing reads the CSR of level s before that point, and pi_s does not change before it
  // (only refinement of level s changes pi_s).  The degrees of level s, which refinement of level
  // s-1 reads as refined-community totals, are updated when a delta is deferred.
  void pend_reserve(int s, uint64_t extra) {
    PendBuf& p = pend[s];
    if (p.count + extra <= p.cap) return;
    const uint64_t c = std::max<uint64_t>(p.count + extra, p.cap + p.cap / 2);
    uint64_t* nk = alloc<uint64_t>(c);
    int64_t* nv = alloc<int64_t>(c);
    if (p.count) {
      hcheck(hipMemcpyAsync(nk, p.keys, 8 * p.count, hipMemcpyDeviceToDevice, st));
      hcheck(hipMemcpyAsync(nv, p.vals, 8 * p.count, hipMemcpyDeviceToDevice, st));
    }
    hcheck(hipStreamSynchronize(st));
    release(p.keys);
    release(p.vals);
    p.keys = nk;
    p.vals = nv;
    p.cap = c;
  }
  void defer(int s, const uint64_t* keys, const int64_t* vals, uint64_t k, bool degrees) {
    if (k == 0) return;
    if (degrees) launch_record_degrees(keys, vals, k, lv[s].kout, directed ? lv[s].kin : nullptr, id_bits, st);
    if (!rebuild_flag[s] && pend[s].count + k > tuple_chunk()) rebuild_flag[s] = 1;
    if (rebuild_flag[s]) {   // the rebuild supersedes the records (the degrees are exact already)
      pend[s].count = 0;
      return;
    }
    pend_reserve(s, k);
    PendBuf& p = pend[s];
    hcheck(hipMemcpyAsync(p.keys + p.count, keys, 8 * k, hipMemcpyDeviceToDevice, st));
    hcheck(hipMemcpyAsync(p.vals + p.count, vals, 8 * k, hipMemcpyDeviceToDevice, st));
    p.count += k;
  }
  // apply the deferred records of levels 1..s (in order: each cascades into the next)
  void flush_to(int s) {
    for (int t = 1; t <= s && t <= top; ++t) {
      PendBuf& p = pend[t];
      if (rebuild_flag[t]) {
        p.count = 0;
        rebuild_flag[t] = 0;
        build_level(t - 1);
        stats.agg_rebuilds++;
        if (t + 1 <= top) {
          // the change of W_t reaches the level above through a rebuild as well; its degrees
          // (row sums, read as refined-community totals) are recounted from this level's now
          Level& U = lv[t + 1];
          launch_fill_i64(U.kout, 0, n, st);
          if (directed) launch_fill_i64(U.kin, 0, n, st);
          launch_degrees_up(n, lv[t].alive, lv[t].par, lv[t].kout, lv[t].kin, U.kout, directed ? U.kin : nullptr, st);
          rebuild_flag[t + 1] = 1;
        }
        continue;
      }
      const uint64_t k = p.count;
      if (!k) continue;
      p.count = 0;
      ensure_tuples(k + 16);
      const uint64_t R = sort_reduce(p.keys, p.vals, k, tk2, tv2);
      stats.agg_records += R;
      if (R == 0) continue;
      hcheck(hipMemcpyAsync(tk0, tk2, 8 * R, hipMemcpyDeviceToDevice, st));
      hcheck(hipMemcpyAsync(tv0, tv2, 8 * R, hipMemcpyDeviceToDevice, st));
      apply_records(t, tk0, tv0, R, false);   // degrees were updated when deferred
      if (t + 1 <= top) {
        launch_split_keys(tk0, R, tx, ty, id_bits, st);
        SetRef none{};
        launch_cascade_map(tx, ty, tv0, R, lv[t].par, tk2, tv2, none, id_bits, st);
        defer(t + 1, tk2, tv2, R, true);
      }
    }
  }

  // ------------------------------------------------------------------ bulk load
  // An insert-only batch into a graph without entries and without aggregate levels (the first
  // batch: static Leiden at creation, Sec. IV-E) lays its rows out directly from the sorted
  // records: a ping-pong sort and a placement pass, with no lookup or row-update buffers; the
  // in-rows of a directed graph are filled by scattering the same records.  A graph of k edges
  // needs 24 bytes per edge of transient memory during the sort and 12 afterwards (undirected
  // graphs: 12 per mirrored entry more) beside its adjacency.  The resulting matrix, degrees, totals and seeds are those of
  // the general path; rows hold their entries in column order, with the same per-row slack.
  bool bulk_eligible(uint64_t nd, uint64_t nc) const {
    return nd == 0 && nc == 0 && top == 0 && m == 0 && !(test_flags & 32);   // m == 0: no entry at all
  }
  struct Transient {   // device buffers released when the bulk load returns or throws
    Engine* e;
    std::vector<void*> ps;
    template <typename T>
    T* get(uint64_t count) {
      T* p = e->alloc<T>(count);
      ps.push_back((void*)p);
      return p;
    }
    void drop(void* p) {   // release early (after the stream has drained)
      hcheck(hipStreamSynchronize(e->st));
      e->release(p);
      ps.erase(std::find(ps.begin(), ps.end(), p));
    }
    ~Transient() {
      for (void* p : ps) e->release(p);
    }
  };
  void bulk_drop_pool(Csr& c) {   // a pool whose rows are all empty: laid out anew
    hcheck(hipStreamSynchronize(st));
    release(c.ref.nbr);
    release(c.ref.w);
    c.ref.nbr = nullptr;
    c.ref.w = nullptr;
    c.pool_cap = 0;
  }
  // rows of c (level 0, no entry) from a sorted entry list
  void bulk_rows(Csr& c, const uint64_t* keys, const uint32_t* wts, uint64_t E, int64_t* rowsum,
                 const uint32_t* lab_or_null) {
    if (c.ref.nbr) bulk_drop_pool(c);
    uint64_t* start = tcounts;   // n + 1 words each; no aggregation pass is running
    uint64_t* end = toffs;
    hcheck(hipMemsetAsync(start, 0, 8ull * n, st));
    hcheck(hipMemsetAsync(end, 0, 8ull * n, st));
    launch_bulk_rows(keys, E, start, end, n, c.ref.deg, id_bits, st);
    csr_grow(c, 0, 3);
    launch_bulk_place(keys, wts, E, start, c.ref, rowsum, lab_or_null, &ds->dein, id_bits, st);
    hcheck(hipMemsetAsync(tcounts, 0, 8ull * ((uint64_t)n + 1), st));   // kept zero between passes
  }
  int bulk_ingest(const uint32_t* dins, uint64_t K) {
    Transient t{this, {}};
    uint64_t* k0 = t.get<uint64_t>(K);
    uint64_t* k1 = t.get<uint64_t>(K);
    uint32_t* v0 = t.get<uint32_t>(K);
    uint32_t* v1 = t.get<uint32_t>(K);
    zero(&ds->err);
    zero(&ds->dm);
    zero(&ds->dein);
    launch_bulk_records(dins, K, n, directed, k0, v0, &ds->err, id_bits, st);
    int sel = 0;
    cub(prim_sort_pairs_u64_u32_db(&cub_tmp, &cub_bytes, k0, k1, v0, v1, K, 0, 2 * id_bits, &sel, st));
    uint64_t* keys = sel ? k1 : k0;   // sorted records and their weights
    uint32_t* wts = sel ? v1 : v0;
    uint64_t* kfree = sel ? k0 : k1;  // the other halves of the ping-pong pairs
    uint32_t* vfree = sel ? v0 : v1;
    launch_bulk_check(keys, wts, K, directed, &ds->err, (u64a*)&ds->dm, id_bits, st);
    sync_read();
    if (hs->err & 1u) return LDL_EINVAL;
    if (hs->err & 2u) return LDL_EDUP;
    const uint64_t dm = (uint64_t)hs->dm;   // unsigned sum of the batch's weights
    if (dm >= ((uint64_t)1 << 40) || m + (int64_t)dm >= ((int64_t)1 << 40)) return LDL_EOVERFLOW;
    mutating = true;
    Level& V0 = lv[0];
    t.drop(kfree);   // the ping-pong halves are not needed any more
    t.drop(vfree);
    if (directed) {
      bulk_rows(V0.out, keys, wts, K, V0.kout, V0.lab);
      // in-rows: column counts, the layout, then every record scattered to its column's row
      // (entry order inside a row carries no meaning)
      launch_bulk_count_cols(keys, K, V0.in.ref.deg, id_bits, st);
      if (V0.in.ref.nbr) bulk_drop_pool(V0.in);
      csr_grow(V0.in, 0, 3);
      uint32_t* cursor = t.get<uint32_t>(n);
      hcheck(hipMemsetAsync(cursor, 0, 4ull * n, st));
      launch_bulk_scatter_in(keys, wts, K, V0.in.ref, cursor, V0.kin, id_bits, st);
    } else {
      zero(&ds->ecount);
      uint64_t* e0 = t.get<uint64_t>(2 * K);
      uint32_t* w0 = t.get<uint32_t>(2 * K);
      launch_bulk_mirror(keys, wts, K, e0, w0, &ds->ecount, id_bits, st);
      sync_read();
      const uint64_t E = hs->ecount;
      t.drop(keys);
      t.drop(wts);
      uint64_t* e1 = t.get<uint64_t>(E);
      uint32_t* w1 = t.get<uint32_t>(E);
      int sel2 = 0;
      cub(prim_sort_pairs_u64_u32_db(&cub_tmp, &cub_bytes, e0, e1, w0, w1, E, 0, 2 * id_bits, &sel2, st));
      bulk_rows(V0.out, sel2 ? e1 : e0, sel2 ? w1 : w0, E, V0.kout, V0.lab);
    }
    // statistic repair and level-0 seeds (Algorithm 1, batch ingest)
    const CsrRef in = directed ? V0.in.ref : CsrRef{};
    begin(S_TOUCH);
    launch_bulk_mark(n, V0.out.ref, in, V0.lab, Kout, Kin, ref(S_TOUCH), tko, tki, ref(S_D0), st);
    launch_bulk_totals(n, V0.lab, V0.kout, directed ? V0.kin : nullptr, Kout, directed ? Kin : nullptr, st);
    zero(&ds->dskk_lo);
    zero(&ds->dskk_hi);
    launch_dskk(sets[S_TOUCH].list, &ds->counts[sets[S_TOUCH].ci], n, Kout, Kin, tko, tki, &ds->dskk_lo,
                &ds->dskk_hi, st);
    sync_read();
    stats.updates = K;
    m += (int64_t)dm;
    Ein += hs->dein;
    SKK += ((i128)hs->dskk_hi << 64) | (i128)hs->dskk_lo;
    return LDL_OK;
  }

  // ------------------------------------------------------------------ batch ingest
  // Returns LDL_OK or a validation error (state untouched).
  int ingest(const uint32_t* dins, uint64_t ni, const uint32_t* ddel, uint64_t nd, const uint32_t* dchg,
             uint64_t nc) {
    const uint64_t K = ni + nd + nc;
    if (K == 0) return LDL_OK;
    if (bulk_eligible(nd, nc)) {
      const int rc = bulk_ingest(dins, ni);
      if (rc == LDL_OK && !(test_flags & 2)) {
        // the first search scans every vertex: size the hub bucket pool for level 0's hubs now
        // (after the load's transient buffers are gone) instead of growing it in a redo
        zero(&ds->tneed);
        launch_hub_entries(lv[0].out.ref.deg, directed ? lv[0].in.ref.deg : nullptr, n, lim[0][kNumBins - 2],
                           &ds->tneed, st);
        sync_read();
        if (hs->tneed > hub.cap) hub_pool(hs->tneed);
      }
      return rc;
    }
    ensure_records(K);
    ensure_entries(2 * K);
    ensure_tuples(2 * K);
    zero(&ds->err);
    hcheck(hipMemsetAsync(&ds->first_bad, 0xFF, 4, st));
    zero(&ds->dm);
    launch_ingest_records(dins, ni, ddel, nd, dchg, nc, n, directed, rkey0, ridx0, &ds->err, id_bits, st);
    cub(prim_sort_pairs_u64_u32(&cub_tmp, &cub_bytes, rkey0, rkey1, ridx0, ridx1, K, 0, 2 * id_bits, st));
    sync_read();
    if (hs->err & 1u) return LDL_EINVAL;
    Level& V0 = lv[0];
    if (!V0.out.ref.nbr) csr_grow(V0.out, 2 * K + 4ull * n);
    ensure_insflag(K);
    cub(prim_select_heads(&cub_tmp, &cub_bytes, rkey1, K, id_bits, seg_lo, &ds->nseg, st));
    cub(launch_seg_lookup(V0.out.ref, rkey1, K, seg_lo, &ds->nseg, seg_hi, items, item_off, items_big, item_off_big,
                          rslot, &cub_tmp, &cub_bytes, id_bits, st));
    launch_ingest_validate(V0.out.ref, rkey1, ridx1, rslot, K, dins, ni, ddel, nd, dchg, directed, rdelta, &ds->err,
                           &ds->first_bad, &ds->dm, id_bits, st);
    sync_read();
    if (hs->err & 2u) return LDL_EDUP;
    if (hs->err & 12u) return hs->first_bad < ni ? LDL_EOVERFLOW : LDL_ENOEDGE;
    if (m + hs->dm >= ((int64_t)1 << 40)) return LDL_EOVERFLOW;
    mutating = true;
    const int64_t dm = hs->dm;
    // matrix entries of the net changes
    zero(&ds->ecount);
    launch_ingest_entries(rkey1, rdelta, K, directed, ekey0, edel0, &ds->ecount, id_bits, st);
    sync_read();
    const uint64_t E = hs->ecount;
    if (E == 0) return LDL_OK;
    cub(prim_sort_pairs_u64_i64(&cub_tmp, &cub_bytes, ekey0, ekey1, edel0, edel1, E, 0, 2 * id_bits, st));
    stats.updates = K;
    // statistic repair and level-0 seeds (Algorithm 1, batch ingest)
    begin(S_TOUCH);
    launch_ingest_mark(ekey1, E, V0.lab, Kout, Kin, ref(S_TOUCH), tko, tki, ref(S_D0), id_bits, st);
    zero(&ds->dein);
    zero(&ds->dskk_lo);
    zero(&ds->dskk_hi);
    launch_ingest_totals(ekey1, edel1, E, V0.lab, Kout, directed ? Kin : nullptr, &ds->dein, id_bits, st);
    launch_dskk(sets[S_TOUCH].list, &ds->counts[sets[S_TOUCH].ci], (uint32_t)std::min<uint64_t>(2 * E, n), Kout, Kin,
                tko, tki, &ds->dskk_lo, &ds->dskk_hi, st);
    apply_records(0, ekey1, edel1, E, true);
    sync_read();
    m += dm;
    Ein += hs->dein;
    SKK += ((i128)hs->dskk_hi << 64) | (i128)hs->dskk_lo;
    // the entry deltas go to level 1 (deferred; they reach higher levels when level 1 is
    // flushed); their ancestors at every existing level are seeds
    if (top >= 1) {
      launch_split_keys(ekey1, E, ex, ey, id_bits, st);
      for (int s = 1; s <= top; ++s) {
        launch_cascade_map(ex, ey, edel1, E, lv[s - 1].par, tk0, tv0, ref(S_D0 + s), id_bits, st);
        if (s == 1) defer(1, tk0, tv0, E, true);
      }
    }
    return LDL_OK;
  }

  // ------------------------------------------------------------------ candidates
  MoveView view(int r, int refine) {
    Level& V = lv[r];
    MoveView mv{};
    mv.out = V.out.ref;
    mv.in = directed ? V.in.ref : CsrRef{};
    mv.lab = V.lab;
    mv.par = V.par;
    mv.lp = refine ? lpk : nullptr;
    mv.alive = V.alive;
    mv.kout = V.kout;
    mv.kin = V.kin;
    if (refine) {
      mv.Kout = lv[r + 1].kout;
      mv.Kin = lv[r + 1].kin;
    } else {
      mv.Kout = Kout;
      mv.Kin = Kin;
    }
    mv.rsize = V.rsize;
    mv.qm = gq * m;
    mv.p = gp;
    mv.directed = directed;
    mv.empty_target = refine ? 0 : empty_target;
    mv.rkey = refine ? cur_rkey : 0;
    for (int b = 0; b < kNumBins - 1; ++b) mv.lim[b] = lim[V.out.ref.wide][b];
    return mv;
  }

  std::pair<hipEvent_t, hipEvent_t> next_events() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t a, b;
      hcheck(hipEventCreate(&a));
      hcheck(hipEventCreate(&b));
      ev_pool.push_back(std::make_pair(a, b));
    }
    return ev_pool[ev_used++];
  }

  // BestMove_r / BestRef_r over the list of set `sid` (its count stays on the device):
  // candidates in `cand`, their count in ds->ps.ncand.  With profiling, every candidate
  // kernel is bracketed by HIP events on its stream; its algorithmic bytes follow from the
  // counters it accumulates, read back by best_finish.
  void best_launch(int r, int sid, int refine) {
    MoveView mv = view(r, refine);
    const uint32_t* list = sets[sid].list;
    const uint32_t* cnt = &ds->counts[sets[sid].ci];
    const int cat0 = 2 * kNumBins * refine + kNumBins * lv[r].out.ref.wide;
    const uint32_t hb = hub_bound(r);
    if (hb) hub_work(hb);   // grows (rarely) before the search is queued, outside its timing
    std::pair<hipEvent_t, hipEvent_t> whole{};
    if (profile) {
      whole = next_events();
      hcheck(hipEventRecord(whole.first, st));
    }
    launch_bin_count(mv, list, cnt, refine, bhist, (uint32_t*)&ds->ps, sizeof(PassScal) / 4, st);
    launch_bin_fill(mv, list, cnt, refine, bhist, binbuf, ds->bin_start, ds->bins, st);
    for (int b = 0; b < kNumBins; ++b) {
      if (b == kNumBins - 1 && hb == 0) break;
      if (b < kNumBins - 1 && mv.lim[b] == (b ? mv.lim[b - 1] : 0u)) continue;   // no entry count maps here
      MoveStats ms{&ds->ps.st_entries[b], &ds->ps.st_distinct[b], &ds->ps.st_vertices[b], &ds->ps.st_cands[b],
                   &ds->ps.maxhi};
      BinRef br{binbuf, &ds->bin_start[b], &ds->bins[b]};
      std::pair<hipEvent_t, hipEvent_t> ev{};
      if (profile) ev = next_events();
      if (b < kNumBins - 1) {
        // with profiling, the events are attached to the kernel's dispatch
        // the grid is sized for n vertices (test flag 64: for one, i.e. a single workgroup)
        launch_best(mv, b, br, (test_flags & 64) ? 1u : n, refine, cand, ms, st, profile ? ev.first : nullptr,
                    profile ? ev.second : nullptr);
      } else {
        // hubs: the events time the keys pass, which reads the entries and their labels
        cub(launch_hub(mv, br, hb, refine, hub, hw, cand, ms, &cub_tmp, &cub_bytes, st, profile ? ev.first : nullptr,
                       profile ? ev.second : nullptr));
      }
      if (profile) pending.push_back(Pending{cat0 + b, ev.first, ev.second, 0.0});
    }
    if (profile) {
      hcheck(hipEventRecord(whole.second, st));
      pending.push_back(Pending{-1, whole.first, whole.second, 0.0});
    }
  }

  // After a synchronisation: false when the hub pool was too small (it has been grown and the
  // pass must be redone; profiling records of the pass are dropped).  Otherwise the scanned
  // count, the candidate count and the pass statistics.
  bool best_finish(int r, int sid, int refine, size_t first_pending, uint32_t& scanned, uint32_t& K) {
    const PassScal& ps = hs->ps;
    if (ps.hub_over & 2u) throw DeviceError{hipErrorUnknown};
    if (ps.hub_over & 1u) {
      hub_pool(ps.hub_need);
      pending.resize(first_pending);
      return false;
    }
    if (ps.hub_over & 4u) {   // a hash partition outgrew its LDS table: more partitions per hub
      if (hw.pshift >= kPartShiftMax) throw DeviceError{hipErrorUnknown};
      hw.pshift++;
      pending.resize(first_pending);
      return false;
    }
    scanned = hs->counts[sets[sid].ci];
    K = ps.ncand;
    if (ps.maxhi > stats.max_gain_hi) stats.max_gain_hi = ps.maxhi;
    // algorithmic bytes: per vertex its list id, offsets and degrees, label, degrees and the
    // totals of its own community; per entry neighbour id, weight and neighbour label (plus
    // the parent in refinement); per distinct community its totals; per candidate 28 bytes.
    // The hub insert kernel reads per vertex its id, offsets, degrees and label, and the entries.
    const int wide = lv[r].out.ref.wide;
    const int cat0 = 2 * kNumBins * refine + kNumBins * wide;
    const double wb = wide ? 8.0 : 4.0;
    const double dirf = directed ? 2.0 : 1.0;
    const double per_v = 4 + 12 * dirf + 4 + 8 * dirf + (refine ? 0 : 8 * dirf);
    const double per_e = 4 + wb + 4 + (refine ? 4 : 0);
    const double per_d = 8 * dirf;
    for (int b = 0; b < kNumBins; ++b) {
      stats.scanned_vertices += ps.st_vertices[b];
      stats.scanned_entries += ps.st_entries[b];
      stats.distinct_comms += ps.st_distinct[b];
      stats.bin_entries[cat0 + b] += ps.st_entries[b];
      if (profile) {
        const double bytes = b < kNumBins - 1
                                 ? per_v * ps.st_vertices[b] + per_e * ps.st_entries[b] +
                                       per_d * ps.st_distinct[b] + 28.0 * ps.st_cands[b]
                                 : (4 + 12 * dirf + 4) * ps.st_vertices[b] + per_e * ps.st_entries[b];
        for (size_t i = first_pending; i < pending.size(); ++i)
          if (pending[i].bin == cat0 + b) pending[i].bytes = bytes;
      }
    }
    stats.candidates += K;
    return true;
  }

  // ---- exact greedy filter over the candidates (Sec. III-E), count read on the device:
  // accepted candidate indices are appended to `acc`, their count in ds->nacc
  static constexpr int kLfRounds = 4;   // rounds launched before the host looks
  int lf_rounds() const { return (test_flags & 1) ? 1 : kLfRounds; }
  // Which filter to queue before the candidate count is known.  For the first iteration of a
  // level's move or refinement phase: the one-workgroup filter if the same pass, level and phase
  // of the previous batch started with at most half of what it holds, else the rounds.  For a
  // later iteration: the one-workgroup filter unless the previous iteration had far more
  // candidates than it holds (candidate counts fall fast after the first iteration).  A wrong
  // guess costs one more synchronisation, never a different result.
  uint32_t lf_lastK[17][2];       // ~0u: the phase's first iteration is next
  uint32_t lf_first[4][17][2];    // first iteration's count per pass (the last slot: later passes)
  uint32_t& lf_first_of(int r, int refine) { return lf_first[pass_idx < 4 ? pass_idx : 3][r][refine]; }
  bool lf_small_predicted(int r, int refine) {
    if (test_flags & 1) return false;
    if (test_flags & 8) return true;
    if (lf_lastK[r][refine] == ~0u) return lf_first_of(r, refine) <= kLfSmall / 2;
    return lf_lastK[r][refine] <= 16 * kLfSmall;
  }
  void decouple_start() {
    if (++acc_epoch == 0) {
      launch_fill_u32(accE, 0, n, st);
      launch_fill_u32(accA, 0, n, st);
      acc_epoch = 1;
    }
    launch_lf_init(&ds->ps.ncand, n, liveA, lfflag, &ds->nlive[0], &ds->nacc, st);
    lf_la = liveA;
    lf_lb = liveB;
    lf_ca = 0;
    decouple_rounds(lf_rounds());
  }
  void decouple_rounds(int rounds) {
    for (int k = 0; k < rounds; ++k) {
      launch_lf_round(lf_la, &ds->nlive[lf_ca], n, cand, lfE, lfA, accE, accA, acc_epoch, lfflag, acc, &ds->nacc,
                      lf_lb, &ds->nlive[1 - lf_ca], st);
      std::swap(lf_la, lf_lb);
      lf_ca = 1 - lf_ca;
      stats.lf_rounds++;
    }
  }
  // after a synchronisation: finish the filter when candidates are still live; returns the
  // index where the newly accepted candidates start (the total is then in hs->nacc)
  // `committed` false: none of the accepted moves has been committed yet (returns 0)
  uint32_t decouple_finish(bool committed = true) {
    const uint32_t na1 = committed ? hs->nacc : 0;
    uint32_t known = hs->nlive[lf_ca];
    while (known) {
      decouple_rounds(lf_rounds());
      sync_read();
      const uint32_t nl = hs->nlive[lf_ca];
      if (nl >= known) throw DeviceError{hipErrorUnknown};   // every round accepts a candidate
      known = nl;
    }
    return na1;
  }

  // the iterations after `iter` of a phase whose next set is empty: each would scan nothing,
  // accept nothing and pass no stop, so they are recorded (as the paper's loop runs them) but
  // not launched
  void record_empty(int r, int phase, int iter) {
    for (int j = iter + 1; j <= M; ++j) record(r, phase, j, 0, 0, 0, 0);
  }
  static constexpr uint32_t kProbeEmpty = 2048;
  void record(int r, int phase, int iter, uint64_t nscan, uint64_t ncand, uint64_t nacc, i128 dq) {
    if (!tracing) return;
    TraceRec t;
    t.v[0] = pass_idx; t.v[1] = r; t.v[2] = phase; t.v[3] = iter;
    t.v[4] = (int64_t)nscan; t.v[5] = (int64_t)ncand; t.v[6] = (int64_t)nacc; t.v[7] = (int64_t)(uint64_t)dq;
    trace.push_back(t);
  }

  // ------------------------------------------------------------------ move commit
  // commit the accepted moves acc[0..*nap) (count on the device): labels and totals, and the
  // exact change of Ein and of sum Kout*Kin into ds->dein / ds->dskk_{lo,hi}
  void commit_launch(int r, const uint32_t* accp, const uint32_t* nap) {
    Level& V = lv[r];
    begin_epoch(S_TOUCH);   // its count for the commit is ps.ntouch, cleared with the pass counters
    begin(S_MOV);
    SetRef touched{sets[S_TOUCH].stamp, sets[S_TOUCH].list, &ds->ps.ntouch, sets[S_TOUCH].epoch};
    launch_commit_mark(accp, nap, n, cand, sets[S_MOV].stamp, sets[S_MOV].epoch, oldlab, Kout, Kin, touched, tko,
                       tki, st);
    launch_commit_apply(accp, nap, n, cand, V.lab, V.kout, V.kin, Kout, directed ? Kin : nullptr, 1, st);
    launch_commit_dein(accp, nap, n, cand, V.out.ref, directed ? V.in.ref : V.out.ref, directed, V.lab,
                       sets[S_MOV].stamp, sets[S_MOV].epoch, oldlab, bigmov, &ds->ps.nbig, &ds->ps.cdein, st);
    launch_dskk(sets[S_TOUCH].list, &ds->ps.ntouch, n, Kout, Kin, tko, tki, &ds->ps.cdskk_lo, &ds->ps.cdskk_hi, st);
  }
  i128 read_dskk() const { return ((i128)hs->ps.cdskk_hi << 64) | (i128)hs->ps.cdskk_lo; }

  // One speculative local-move (refine = 0) or refinement (refine = 1) iteration over set sid:
  // candidates, decoupling rounds and the commit are queued together and read back by one
  // synchronisation.  A hub-pool overflow undoes the commit and redoes the iteration; live
  // candidates after the first rounds are finished and committed as a second phase (the
  // changes of Ein and sum Kout*Kin add up over the phases).
  void iterate(int r, int sid, int refine, uint32_t& scanned, uint32_t& K, uint32_t& na, int64_t& dein, i128& dskk) {
    Level& V = lv[r];
    Level* H = refine ? &lv[r + 1] : nullptr;
    int64_t* Krin = (refine && directed) ? H->kin : nullptr;
    auto commit = [&](const uint32_t* accp, const uint32_t* nap, int forward) {
      if (refine)
        launch_ref_commit(accp, nap, n, cand, V.par, lpk, V.kout, V.kin, H->kout, Krin, V.rsize, forward, st);
      else if (forward) commit_launch(r, accp, nap);
      else launch_commit_apply(accp, nap, n, cand, V.lab, V.kout, V.kin, Kout, directed ? Kin : nullptr, 0, st);
    };
    bool small = false;
    for (int attempt = 0;; ++attempt) {
      const size_t fp = pending.size();
      best_launch(r, sid, refine);
      small = lf_small_predicted(r, refine);
      if (small) {
        launch_lf_small(cand, acc, &ds->nacc, &ds->nlive[0], st);
        lf_ca = 0;
        stats.lf_rounds++;
      } else {
        decouple_start();
      }
      commit(acc, &ds->nacc, 1);
      sync_read();
      if (best_finish(r, sid, refine, fp, scanned, K)) break;
      commit(acc, &ds->nacc, 0);   // undo: the candidate set was incomplete
      if (attempt > 2 + kPartShiftMax) throw NoMem{};
    }
    if (lf_lastK[r][refine] == ~0u) lf_first_of(r, refine) = K;
    lf_lastK[r][refine] = K;
    dein = refine ? 0 : hs->ps.cdein;
    dskk = refine ? 0 : read_dskk();
    const bool missed = small && K > kLfSmall;   // the filter has not run, nothing is committed
    if (missed) {
      decouple_start();
      sync_read();
    }
    const uint32_t na1 = decouple_finish(!missed);
    na = hs->nacc;
    if (na > na1) {
      hcheck(hipMemsetD32Async((hipDeviceptr_t)&ds->nacc2, (int)(na - na1), 1, st));
      hcheck(hipMemsetAsync(&ds->ps.cdein, 0, 32, st));   // cdein, cdskk_lo/hi, ntouch, nbig
      commit(acc + na1, &ds->nacc2, 1);
      sync_read();
      if (!refine) {
        dein += hs->ps.cdein;
        dskk += read_dskk();
      }
    }
  }

  // ------------------------------------------------------------------ one level
  void process_level(int r) {
    Level& V = lv[r];
    stats.levels_processed++;
    // the seed count was read by the caller's synchronisation; flushing does not change the seeds
    const uint32_t E0 = count(S_D0 + r);
    flush_to(r);   // level r's CSR receives its deferred records (and passes them upwards)
    hcheck(hipMemcpyAsync(entry, sets[S_D0 + r].list, 4ull * E0, hipMemcpyDeviceToDevice, st));
    begin(S_D0 + r);
    // frontier: alive seeds and all members of their communities
    begin(S_COMM);
    launch_set_add_mapped(ref(S_COMM), entry, E0, V.lab, V.alive, st);
    begin(S_U);
    launch_mark_members(sets[S_U].stamp, sets[S_U].epoch, n, V.alive, V.lab, sets[S_COMM].stamp, sets[S_COMM].epoch,
                        st);
    select_set(S_U);
    const i128 Q0 = qnum();
    begin(S_MOVED);
    lf_lastK[r][0] = lf_lastK[r][1] = ~0u;   // each phase's first iteration: predicted from the last batch
    CsrRef in = directed ? V.in.ref : V.out.ref;
    for (int j = 1; j <= M; ++j) {
      stats.move_iters++;
      // scan set: the frontier and its neighbours (counts stay on the device)
      begin(S_S);
      const CsrRef in_or_none = directed ? V.in.ref : CsrRef{};
      launch_items(sets[S_U].list, nullptr, &ds->counts[sets[S_U].ci], n, V.out.ref, in_or_none, it_cnt, it_off,
                   it_csum, nullptr, nullptr, st);
      launch_mark_items(sets[S_S].stamp, sets[S_S].epoch, sets[S_U].list, &ds->counts[sets[S_U].ci], n, it_off,
                        V.out.ref, in_or_none, st, sets[S_U].stamp, sets[S_U].epoch, V.alive);
      select_set(S_S);
      uint32_t nS = 0, K = 0, na = 0;
      int64_t dein = 0;
      i128 dskk = 0;
      iterate(r, S_S, 0, nS, K, na, dein, dskk);
      const i128 dq = (i128)gq * m * dein - (i128)gp * dskk;
      record(r, 0, j, nS, K, na, dq);
      const uint32_t* nap = &ds->nacc;
      if (dq < 0) {  // negative batch gain: undo every accepted move of the iteration
        launch_commit_apply(acc, nap, na, cand, V.lab, V.kout, V.kin, Kout, directed ? Kin : nullptr, 0, st);
        stats.rollbacks++;
        break;
      }
      Ein += dein;
      SKK += dskk;
      stats.accepted += na;
      launch_set_add_acc_v(ref(S_MOVED), acc, nap, na, cand, st);
      if ((i128)ad * dq < (i128)an * Q0) break;            // alpha stop of the move loop
      if ((i128)bd * na < (i128)bn * nS) break;           // beta stop of the move loop
      if (j == M) break;                                  // the next frontier would not be used
      if (nS == 0) {   // empty scan set: every later iteration is empty too and changes nothing
        record_empty(r, 0, j);
        break;
      }
      // Expand_r: movers, their neighbours, members of the touched communities
      begin(S_U2);
      if (na) {
        begin(S_COMM);
        launch_mark_acc_comms(acc, nap, na, cand, sets[S_COMM].stamp, sets[S_COMM].epoch, st);
        launch_mark_members(sets[S_U2].stamp, sets[S_U2].epoch, n, V.alive, V.lab, sets[S_COMM].stamp,
                            sets[S_COMM].epoch, st);
        launch_mark_neighbours_acc(sets[S_U2].stamp, sets[S_U2].epoch, acc, nap, na, cand, V.out.ref, in, directed,
                                   st);
        select_set(S_U2);
      } else {
        zero(&ds->counts[sets[S_U2].ci]);
      }
      std::swap(sets[S_U], sets[S_U2]);
    }
    // the movers' count is final after the move phase: the synchronisations of refinement and
    // aggregation have read it; without refinement (r == L) one is needed here
    if (r < L) refine(r, E0);
    else sync_read();
    if (r >= 1 && count(S_MOVED) > 0) label_refresh(r);
  }

  // ------------------------------------------------------------------ refinement
  void refine(int r, uint32_t E0) {
    Level& V = lv[r];
    Level& H = lv[r + 1];
    int64_t* Krin = directed ? H.kin : nullptr;
    if (r == top) launch_ref_init_top(n, V.alive, V.kout, V.kin, H.kout, Krin, V.rsize, st);
    // the list lengths below stay on the device (no host synchronisation before the iterations)
    const uint32_t* nMoved = &ds->counts[sets[S_MOVED].ci];
    begin(S_REFM);
    launch_set_add_mapped(ref(S_REFM), entry, E0, V.par, nullptr, st);
    launch_set_add_mapped(ref(S_REFM), sets[S_MOVED].list, n, V.par, nullptr, st, nMoved);
    begin(S_RSET);
    launch_mark_members(sets[S_RSET].stamp, sets[S_RSET].epoch, n, V.alive, V.par, sets[S_REFM].stamp,
                        sets[S_REFM].epoch, st);
    select_set(S_RSET);
    const uint32_t* nR0 = &ds->counts[sets[S_RSET].ci];
    launch_ref_reset(sets[S_RSET].list, n, V.par, oldpar, V.kout, V.kin, H.kout, Krin, V.rsize, 0, st, nR0);
    launch_ref_reset(sets[S_RSET].list, n, V.par, oldpar, V.kout, V.kin, H.kout, Krin, V.rsize, 1, st, nR0);
    launch_pack_lab_par(n, V.lab, V.par, lpk, st);   // refinement commits keep it current
    int cur = S_RSET;          // the set whose list this iteration scans
    bool rset_grew = false;    // SPExpand marked new members: rebuild the Rset list at the end
    CsrRef in = directed ? V.in.ref : V.out.ref;
    for (int j = 1; j <= M; ++j) {
      stats.refine_iters++;
      // the draw's key: SplitMix64's first output of the seed chained with the batch, the pass,
      // then level and iteration in one word
      cur_rkey = refine_random
                     ? splitmix64_out(splitmix64_out(splitmix64_out(splitmix64_out(refine_seed + 0x9E3779B97F4A7C15ull) ^
                                                                    cur_batch) ^
                                                     (uint64_t)pass_idx) ^
                                      (((uint64_t)r << 32) | (uint64_t)j)) |
                           1ull
                     : 0;
      uint32_t Rc = 0, K = 0, na = 0;
      int64_t dein_unused = 0;
      i128 dskk_unused = 0;
      iterate(r, cur, 1, Rc, K, na, dein_unused, dskk_unused);
      const uint32_t* nap = &ds->nacc;
      stats.refine_moves += na;
      record(r, 1, j, Rc, K, na, 0);
      if ((i128)bd * na < (i128)bn * Rc) break;            // beta stop of the refinement loop
      if (Rc == 0) {   // an empty set stays empty: the later iterations change nothing
        record_empty(r, 1, j);
        break;
      }
      begin(S_RCUR);
      const CsrRef in_or_none = directed ? V.in.ref : CsrRef{};
      launch_items(cand.v, acc, nap, na, V.out.ref, in_or_none, it_cnt, it_off, it_csum, nullptr, nullptr, st);
      launch_spexpand(cand.v, acc, nap, na, it_off, V.out.ref, in_or_none, lpk, V.rsize, sets[S_RCUR].stamp,
                      sets[S_RCUR].epoch, sets[S_RSET].stamp, sets[S_RSET].epoch, oldpar, st);
      select_set(S_RCUR);
      rset_grew = rset_grew || na > 0;
      cur = S_RCUR;
      if (j < M && na <= kProbeEmpty) {   // few movers often leave the next set empty: look first
        sync_read();
        if (count(S_RCUR) == 0) {
          record_empty(r, 1, j);
          break;
        }
      }
    }
    if (rset_grew) select_set(S_RSET);
    if (r == top) materialise(r);
    else aggregate(r, E0);
  }

  // ------------------------------------------------------------------ aggregate repair
  void aggregate(int r, uint32_t E0) {
    Level& V = lv[r];
    Level& H = lv[r + 1];
    begin(S_C);
    launch_mark_changed(sets[S_C].stamp, sets[S_C].epoch, sets[S_RSET].list, n, V.par, oldpar, st,
                        &ds->counts[sets[S_RSET].ci]);
    select_set(S_C);
    sync_read();
    const uint32_t nC = count(S_C), nRset = count(S_RSET), nMoved = count(S_MOVED);
    CsrRef in = directed ? V.in.ref : V.out.ref;
    const int Dn = S_D0 + r + 1;
    // both parents of every node in one word for the tuple kernels (lpk's storage is free here:
    // refinement of this level has finished)
    uint2* po = lpk;
    launch_pack_parents(n, V.par, oldpar, sets[S_C].stamp, sets[S_C].epoch, po, st);
    const uint64_t T = tuple_offsets(S_C, nC, V.out.ref, in, po, 1, false);
    // Repair by subtract-add tuples, or -- when they would outnumber the tuples of building level
    // r+1 from scratch (Eq. 3 over every out-entry of level r), or exceed a chunk -- rebuild level
    // r+1 before it is next read; both give the same matrix (Eq. 3), so only the cost differs.
    // The rebuild still marks every seed the tuples' endpoints would.
    bool rebuild_up = rebuild_flag[r + 1] != 0;
    if (!rebuild_up && T > tuple_chunk()) rebuild_up = true;
    if (!rebuild_up && T > (1u << 16)) rebuild_up = T > level_out_entries(r);
    if (rebuild_up) {
      if (nC)
        launch_tuples_gen(sets[S_C].list, &ds->counts[sets[S_C].ci], nC, it_off, V.out.ref, in, V.par, po, 1, toffs,
                          (u64a*)tcur, nullptr, nullptr, sets[Dn].stamp, sets[Dn].epoch, id_bits, st);
      rebuild_flag[r + 1] = 1;
      pend[r + 1].count = 0;
    } else {
      // the tuples are written straight into the deferred records of level r+1
      pend_reserve(r + 1, T);
      PendBuf& pn = pend[r + 1];
      if (nC)
        launch_tuples_gen(sets[S_C].list, &ds->counts[sets[S_C].ci], nC, it_off, V.out.ref, in, V.par, po, 1, toffs,
                          (u64a*)tcur, pn.keys + pn.count, pn.vals + pn.count, sets[Dn].stamp, sets[Dn].epoch,
                          id_bits, st);
      pn.count += T;
    }
    // NextFrontier: parents of seeds, movers and refined nodes; old parents of changed nodes
    launch_set_add_mapped(ref(Dn), entry, E0, V.par, nullptr, st);
    launch_set_add_mapped(ref(Dn), sets[S_MOVED].list, nMoved, V.par, nullptr, st);
    launch_set_add_mapped(ref(Dn), sets[S_RSET].list, nRset, V.par, nullptr, st);
    launch_set_add_mapped(ref(Dn), sets[S_C].list, nC, oldpar, nullptr, st);
    select_set(Dn);   // the tuple kernel marked seeds without listing them
    // liveness of level r+1 and revival / death chains above it
    begin(S_LVC);
    launch_set_add_mapped(ref(S_LVC), sets[S_RSET].list, nRset, oldpar, nullptr, st);
    launch_set_add_mapped(ref(S_LVC), sets[S_RSET].list, nRset, V.par, nullptr, st);
    begin(S_DIED);
    begin(S_REV);
    launch_live_update(sets[S_LVC].list, n, V.rsize, H.alive, r + 1 < L ? H.par : nullptr, H.lab, V.lab,
                       ref(S_DIED), ref(S_REV), st, &ds->counts[sets[S_LVC].ci]);
    launch_label_up(sets[S_RSET].list, nRset, V.par, H.alive, V.lab, H.lab, st);
    int died = S_DIED, rev = S_REV, died2 = S_DIED2, rev2 = S_REV2;
    for (int s = r + 2; s <= top; ++s) {
      sync_read();
      const uint32_t nd = count(died), nrv = count(rev);
      if (nd + nrv == 0) break;
      begin(S_LVC);
      launch_live_prop(sets[died].list, nd, sets[rev].list, nrv, lv[s - 1].par, lv[s - 1].rsize, ref(S_LVC), st);
      begin(died2);
      begin(rev2);
      launch_live_update(sets[S_LVC].list, n, lv[s - 1].rsize, lv[s].alive, s < L ? lv[s].par : nullptr, lv[s].lab,
                         lv[s - 1].lab, ref(died2), ref(rev2), st, &ds->counts[sets[S_LVC].ci]);
      std::swap(died, died2);
      std::swap(rev, rev2);
    }
    // the subtract-add tuples wait in pend[r+1] (level r+1's degrees are already exact: the
    // refinement commits maintain them as refined-community totals)
    stats.agg_tuples += T;
  }

  // first visit of level r+1: Eq. 3 from scratch
  void materialise(int r) {
    Level& V = lv[r];
    Level& H = lv[r + 1];
    launch_materialise_nodes(n, V.rsize, H.alive, V.lab, H.lab, r + 1 < L ? H.par : nullptr, st);
    build_level(r);
    top = r + 1;
    launch_alive_list(n, H.alive, ref(S_D0 + r + 1), st);
  }

  // out-entries of level r (the tuples of building level r+1 from scratch)
  uint64_t level_out_entries(int r) {
    zero(&ds->nnz);
    launch_sum_u32(lv[r].out.ref.deg, n, &ds->nnz, st);
    uint64_t k = 0;
    hcheck(hipMemcpyAsync(&k, &ds->nnz, 8, hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    stats.host_syncs++;
    return k;
  }

  // every row of c empty and its pool released (the next row update lays the pool out anew)
  void drop_csr(Csr& c) {
    hcheck(hipStreamSynchronize(st));
    release(c.ref.nbr);
    release(c.ref.w);
    c.ref.nbr = nullptr;
    c.ref.w = nullptr;
    c.pool_cap = 0;
    hcheck(hipMemsetAsync(c.ref.off, 0, 8ull * n, st));
    hcheck(hipMemsetAsync(c.ref.deg, 0, 4ull * n, st));
    hcheck(hipMemsetAsync(c.ref.cap, 0, 4ull * n, st));
  }

  // W_{r+1} = Eq. 3 of (W_r, pi_r) from scratch into level r+1's emptied rows: the (pi(u), pi(v),
  // w) tuples of every out-entry of an alive level-r node, in chunks of whole nodes with at most
  // tuple_chunk() tuples each (one node with more forms its own chunk), each chunk sorted,
  // reduced and added to the rows (sums over chunks commute).  Level r+1's degrees are exact
  // already and are not touched.
  void build_level(int r) {
    Level& V = lv[r];
    Level& H = lv[r + 1];
    drop_csr(H.out);
    if (directed) drop_csr(H.in);
    begin(S_TMP);
    launch_alive_list(n, V.alive, ref(S_TMP), st);
    sync_read();
    const uint32_t na = count(S_TMP);
    if (na == 0) return;
    const uint32_t* list = sets[S_TMP].list;
    const uint64_t C = tuple_chunk();
    const uint64_t T = tuple_offsets_at(list, &ds->counts[sets[S_TMP].ci], na, V.out.ref, CsrRef{}, nullptr, 0, false);
    std::vector<uint64_t> offs;
    if (T > C) {
      offs.resize((size_t)na + 1);
      hcheck(hipMemcpyAsync(offs.data(), toffs, 8ull * ((uint64_t)na + 1), hipMemcpyDeviceToHost, st));
      hcheck(hipStreamSynchronize(st));
    }
    uint32_t* cntp = &ds->counts[kChunkSlot];
    for (uint32_t i0 = 0; i0 < na;) {
      uint32_t i1 = na;
      uint64_t Tc = T;
      const uint32_t* sub = list + i0;
      const uint32_t* subcnt = &ds->counts[sets[S_TMP].ci];
      if (T > C) {
        // the longest run of nodes from i0 whose tuples fit a chunk (at least one node)
        const uint64_t limit = offs[i0] + C;
        i1 = (uint32_t)(std::upper_bound(offs.begin() + i0 + 1, offs.end(), limit) - offs.begin()) - 1;
        if (i1 <= i0) i1 = i0 + 1;
        hcheck(hipMemsetD32Async((hipDeviceptr_t)cntp, (int)(i1 - i0), 1, st));
        subcnt = cntp;
        Tc = tuple_offsets_at(sub, subcnt, i1 - i0, V.out.ref, CsrRef{}, nullptr, 0, false);
      }
      ensure_tuples(Tc + 16);
      if (Tc) {
        launch_tuples_gen(sub, subcnt, i1 - i0, it_off, V.out.ref, CsrRef{}, V.par, nullptr, 0, toffs, (u64a*)tcur,
                          tk0, tv0, nullptr, 0, id_bits, st);
        const uint64_t R = sort_reduce(tk0, tv0, Tc, tk2, tv2);
        hcheck(hipMemcpyAsync(tk0, tk2, 8 * R, hipMemcpyDeviceToDevice, st));
        hcheck(hipMemcpyAsync(tv0, tv2, 8 * R, hipMemcpyDeviceToDevice, st));
        apply_records(r + 1, tk0, tv0, R, false);
      }
      i0 = i1;
    }
  }

  void label_refresh(int r) {
    for (int s = r - 1; s >= 0; --s)
      launch_label_refresh(n, lv[s].alive, lv[s].par, lv[s + 1].lab, lv[s].lab, ref(S_D0 + s), st);
  }

  // ------------------------------------------------------------------ Algorithm 1
  // Adaptive refresh (a variant, off unless rn > 0): the size of the level-0 frontier A^0 (alive
  // seeds and every alive member of their communities); when it reaches rn/rd of n, locality no
  // longer holds (Sec. IV-F, Sec. V) and the batch reoptimises from scratch.
  void maybe_refresh() {
    if (rn <= 0) return;
    Level& V0 = lv[0];
    begin(S_COMM);
    launch_set_add_mapped(ref(S_COMM), sets[S_D0].list, n, V0.lab, V0.alive, st, &ds->counts[sets[S_D0].ci]);
    zero(&ds->tcount);
    launch_count_members(n, V0.alive, V0.lab, sets[S_COMM].stamp, sets[S_COMM].epoch, &ds->tcount, st);
    sync_read();
    const uint64_t a0 = hs->tcount;
    stats.frontier0 = a0;
    if ((i128)rd * a0 < (i128)rn * n) return;
    record(0, 2, 0, a0, 0, 0, 0);
    stats.refreshes = 1;
    refresh_state();
  }
  // The state static Leiden starts from on the current graph: singleton labels and parents at
  // level 0, no aggregate level, totals equal to the degrees, Ein the self-loops, and every node
  // with an entry a seed (the state ldl_create reaches before its passes).
  void refresh_state() {
    Level& V0 = lv[0];
    launch_iota(V0.lab, n, st);
    if (L > 0) {
      launch_iota(V0.par, n, st);
      launch_fill_u32(V0.rsize, 0, n, st);
    }
    for (int r = 1; r <= top; ++r) {
      Level& V = lv[r];
      launch_fill_u8(V.alive, 0, n, st);
      launch_iota(V.lab, n, st);
      launch_fill_i64(V.kout, 0, n, st);
      if (directed) launch_fill_i64(V.kin, 0, n, st);
      if (r < L) {
        launch_iota(V.par, n, st);
        launch_fill_u32(V.rsize, 0, n, st);
      }
      drop_csr(V.out);
      if (directed) drop_csr(V.in);
      pend[r].count = 0;
      rebuild_flag[r] = 0;
    }
    for (int r = 0; r <= L; ++r) begin(S_D0 + r);
    top = 0;
    launch_copy_i64(Kout, V0.kout, n, st);
    if (directed) launch_copy_i64(Kin, V0.kin, n, st);
    zero(&ds->dein);
    zero(&ds->dskk_lo);
    zero(&ds->dskk_hi);
    launch_refresh_scalars(V0.out.ref, directed ? V0.in.ref : CsrRef{}, n, V0.kout, V0.kin, ref(S_D0), &ds->dein,
                           &ds->dskk_lo, &ds->dskk_hi, st);
    select_set(S_D0);
    sync_read();
    Ein = hs->dein;
    SKK = ((i128)hs->dskk_hi << 64) | (i128)hs->dskk_lo;
  }

  int apply(const uint32_t* dins, uint64_t ni, const uint32_t* ddel, uint64_t nd, const uint32_t* dchg, uint64_t nc) {
    const int rc = ingest(dins, ni, ddel, nd, dchg, nc);
    if (rc != LDL_OK) return rc;
    cur_batch = batches++;   // the batch is accepted
    maybe_refresh();
    for (int i = 1; i <= N; ++i) {
      pass_idx = i;
      const i128 Qp = qnum();
      bool any = false;
      for (int r = 0; r <= top && r <= L; ++r) {
        sync_read();
        if (count(S_D0 + r) == 0) continue;
        any = true;
        process_level(r);
      }
      sync_read();
      bool all_empty = true;
      for (int r = 0; r <= L; ++r)
        if (count(S_D0 + r)) all_empty = false;
      if (!any || all_empty) break;
      if ((i128)ad * (qnum() - Qp) < (i128)an * Qp) break;  // alpha stop of the passes
    }
    flush_to(top);
    for (int r = 0; r <= L; ++r) begin(S_D0 + r);
    hcheck(hipStreamSynchronize(st));
    mutating = false;
    return LDL_OK;
  }

  // ------------------------------------------------------------------ degree-bin autotuner
  // The bin limits decide which kernel evaluates a vertex, never what it computes, so any valid
  // choice gives the same candidates.  The tuner times the move-phase candidate search over all
  // alive nodes of a level and over a 1/64 stride sample of them (the small frontiers of batch
  // updates), and runs one round of coordinate descent over the five limits.
  static bool valid_limits(const uint32_t* l) {
    for (int b = 0; b < kNumBins - 1; ++b)
      if (l[b] > kBinCap[b] || (b && l[b] < l[b - 1])) return false;
    return true;
  }
  // median time in ms of `reps` candidate searches (move mode) at level r over the list of set sid
  double time_search(int r, int sid, int reps, hipEvent_t a, hipEvent_t b) {
    std::vector<float> t;
    for (int k = 0; k < reps; ++k) {
      for (int attempt = 0;; ++attempt) {
        hcheck(hipEventRecord(a, st));
        best_launch(r, sid, 0);
        hcheck(hipEventRecord(b, st));
        sync_read();
        uint32_t sc = 0, K = 0;
        if (best_finish(r, sid, 0, pending.size(), sc, K)) break;
        if (attempt > 2 + kPartShiftMax) throw NoMem{};
      }
      float ms = 0;
      hcheck(hipEventElapsedTime(&ms, a, b));
      t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
  }
  void autotune(ldl_tune_report* rep) {
    static const uint32_t opts[kNumBins - 1][4] = {{0, 4, 8, 8}, {16, 24, 32, 32}, {64, 96, 128, 128},
                                                    {128, 256, 384, 512}, {1024, 2048, 2048, 2048}};
    const int saved_profile = profile;
    profile = 0;
    hipEvent_t a = nullptr, b = nullptr;
    hcheck(hipEventCreate(&a));
    hcheck(hipEventCreate(&b));
    ldl_tune_report out{};
    for (int w = 0; w < 2; ++w) {
      for (int k = 0; k < kNumBins - 1; ++k) out.limit[w][k] = lim[w][k];
      const int r = w;   // level 0 holds the 32-bit weights, level 1 the 64-bit ones
      if (r > top) continue;
      begin(S_TMP);
      launch_alive_list(n, lv[r].alive, ref(S_TMP), st);
      sync_read();
      const uint32_t na = count(S_TMP);
      if (na == 0) continue;
      launch_stride_sample(sets[S_TMP].list, &ds->counts[sets[S_TMP].ci], n, 64, sets[S_REV2].list,
                           &ds->counts[sets[S_REV2].ci], st);
      auto cost = [&]() { return time_search(r, S_TMP, 3, a, b) + time_search(r, S_REV2, 3, a, b); };
      double best = cost();
      out.ms_before[w] = best;
      for (int k = 0; k < kNumBins - 1; ++k) {
        const uint32_t keep = lim[w][k];
        uint32_t best_v = keep;
        for (int o = 0; o < 4; ++o) {
          const uint32_t v = opts[k][o];
          if (v == keep || (o && v == opts[k][o - 1])) continue;
          lim[w][k] = v;
          if (!valid_limits(lim[w])) continue;
          const double c = cost();
          out.trials++;
          if (c < best) {
            best = c;
            best_v = v;
          }
        }
        lim[w][k] = best_v;
      }
      out.ms_after[w] = best;
      for (int k = 0; k < kNumBins - 1; ++k) out.limit[w][k] = lim[w][k];
    }
    begin(S_TMP);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    profile = saved_profile;
    stats = ldl_batch_stats{};
    pending.clear();
    ev_used = 0;
    if (rep) *rep = out;
  }

  void finish_profile() {
    if (!profile) return;
    hcheck(hipStreamSynchronize(st));
    for (const Pending& p : pending) {
      float ms = 0;
      hcheck(hipEventElapsedTime(&ms, p.a, p.b));
      if (p.bin < 0) {   // a whole candidate search
        stats.search_ms += ms;
        continue;
      }
      stats.bin_ms[p.bin] += ms;
      stats.bin_bytes[p.bin] += p.bytes;
      stats.bin_launches[p.bin] += 1;
      stats.bm_ms += ms;
      stats.bm_bytes += p.bytes;
      stats.bm_launches += 1;
    }
    ev_used = 0;
    pending.clear();
  }

  // ------------------------------------------------------------------ invariant recount
  // Device recount of the invariants (I1-I3, I5, I6 and the transpose / symmetry of the stored
  // matrices) with the scratch words at sc: one row pass per CSR and one node pass per level,
  // then a comparison of the sums on the host.
  void check_invariants(InvScratch* sc, ldl_invariant_report* rep) {
    ldl_invariant_report out{};
    out.level = -1;
    auto fail = [&](uint32_t bits, int r) {
      if (!bits) return;
      out.failed |= bits;
      if (out.level < 0) out.level = r;
    };
    uint64_t prev_w = 0, prev_a1 = 0, prev_a2 = 0;   // parent-mapped sums of the level below
    for (int r = 0; r <= top; ++r) {
      Level& V = lv[r];
      const bool up = r < top;
      launch_inv_clear(sc, st);
      launch_inv_rows(V.out.ref, n, V.alive, V.kout, up ? V.par : nullptr, r == 0 ? V.lab : nullptr, 0, sc, st);
      if (directed) launch_inv_rows(V.in.ref, n, V.alive, V.kin, nullptr, nullptr, 1, sc, st);
      launch_inv_nodes(n, V.alive, V.lab, up ? V.par : nullptr, up ? V.rsize : nullptr, V.kout, V.kin,
                       up ? lv[r + 1].alive : nullptr, up ? lv[r + 1].lab : nullptr, r == 0 ? Kout : nullptr,
                       r == 0 ? Kin : nullptr, sc, st);
      InvScratch h;
      hcheck(hipMemcpyAsync(&h, sc, sizeof(InvScratch), hipMemcpyDeviceToHost, st));
      hcheck(hipStreamSynchronize(st));
      uint32_t bits = 0;
      if (h.flags & kInvDegrees) bits |= LDL_INV_DEGREES;
      if (h.flags & kInvAggregate) bits |= LDL_INV_AGGREGATE;
      if (h.flags & kInvLabels) bits |= LDL_INV_LABELS;
      if (h.flags & kInvRoots) bits |= LDL_INV_ROOTS;
      if (h.flags & kInvRange) bits |= LDL_INV_RANGE;
      // the in-rows hold the transpose of the out-rows (directed); an undirected matrix is symmetric
      const bool tr_ok = directed ? (h.out[0] == h.in[0] && h.out[1] == h.in[1] && h.out[2] == h.in[2] &&
                                     h.out[3] == h.in[3])
                                  : (h.out[2] == h.out[4] && h.out[3] == h.out[5]);
      if (!tr_ok) bits |= LDL_INV_TRANSPOSE;
      // Eq. 3: this level's matrix is the grouped sum of the level below under its parents
      if (r >= 1 && !(h.out[1] == prev_w && h.out[2] == prev_a1 && h.out[3] == prev_a2)) bits |= LDL_INV_AGGREGATE;
      if (up) {
        prev_w = h.out[1];
        prev_a1 = h.out[6];
        prev_a2 = h.out[7];
        if (h.node[0] != h.node[1]) bits |= LDL_INV_AGGREGATE;   // refined sizes count the children
      }
      if (r == 0) {
        const i128 skk = ((i128)(int64_t)h.skk_hi << 64) | (i128)h.node[kInvNodeWords];
        const bool tot_ok = (int64_t)h.out[1] == m && (int64_t)h.out[8] == Ein && h.node[2] == h.node[4] &&
                            h.node[3] == h.node[5] && (int64_t)h.node[6] == m && (int64_t)h.node[7] == m && skk == SKK;
        if (!tot_ok) bits |= LDL_INV_TOTALS;
      }
      fail(bits, r);
      out.entries += h.out[0] + (directed ? h.in[0] : 0);
    }
    if (rep) *rep = out;
  }

  // ------------------------------------------------------------------ export
  void export_entries(int r, std::vector<uint64_t>& keys, std::vector<int64_t>& w) {
    Level& V = lv[r];
    zero(&ds->ecount);
    sync_read();
    uint64_t nnz = nnz_of(r);
    keys.assign(nnz, 0);
    w.assign(nnz, 0);
    if (nnz == 0 || !V.out.ref.nbr) return;
    ensure_tuples(nnz);
    zero(&ds->ecount);
    launch_csr_entries(V.out.ref, n, tk0, tv0, &ds->ecount, st);
    hcheck(hipMemcpyAsync(keys.data(), tk0, 8 * nnz, hipMemcpyDeviceToHost, st));
    hcheck(hipMemcpyAsync(w.data(), tv0, 8 * nnz, hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    std::vector<std::pair<uint64_t, int64_t>> kv(nnz);
    for (uint64_t i = 0; i < nnz; ++i) kv[i] = std::make_pair(keys[i], w[i]);
    std::sort(kv.begin(), kv.end());
    for (uint64_t i = 0; i < nnz; ++i) { keys[i] = kv[i].first; w[i] = kv[i].second; }
  }
  // ------------------------------------------------------------------ state blob
  // Layout (little-endian): StateHeader, community totals Kout[n] (and Kin[n] when directed),
  // then per level r = 0..top: alive u8[n], lab u32[n], (r < L) par u32[n] and rsize u32[n],
  // kout i64[n], (directed) kin i64[n], deg u32[n] (out-rows), nnz u64, then the row-major
  // entries: columns u32[nnz] (ascending within a row) and weights (u32 at level 0, i64 above).
  struct StateHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int32_t cfg[14];   // directed, gamma p, q, N, L, M, alpha num, den, beta num, den, refresh num, den,
                       // variants (1 empty target, 2 randomised refinement), refinement seed
    uint32_t n;
    int32_t top;
    int64_t m, ein, skk_hi;
    uint64_t skk_lo;
    uint64_t batches;   // batches accepted so far (the randomised refinement's counter)
    uint32_t lim[2][5];
    uint64_t total_bytes;
  };
  static constexpr uint32_t kStateVersion = 3;
  uint64_t level_node_bytes(int r) const {
    return (uint64_t)n * (1 + 4 + (r < L ? 8 : 0) + 8 + (directed ? 8 : 0) + 4) + 8;
  }
  uint64_t state_bytes(std::vector<uint64_t>& nnz) {
    nnz.assign(top + 1, 0);
    uint64_t b = sizeof(StateHeader) + 8ull * n * (directed ? 2 : 1);
    for (int r = 0; r <= top; ++r) {
      nnz[r] = nnz_of(r);
      b += level_node_bytes(r) + nnz[r] * (4 + (r == 0 ? 4 : 8));
    }
    return b;
  }
  void export_state(uint8_t* out, uint64_t bytes) {
    uint8_t* p = out;
    auto put = [&](const void* src, uint64_t k) {
      std::memcpy(p, src, k);
      p += k;
    };
    auto put_dev = [&](const void* dsrc, uint64_t k) {
      hcheck(hipMemcpyAsync(p, dsrc, k, hipMemcpyDeviceToHost, st));
      hcheck(hipStreamSynchronize(st));
      p += k;
    };
    StateHeader hd{};
    std::memcpy(hd.magic, "LDLSTATE", 8);
    hd.version = kStateVersion;
    hd.header_bytes = sizeof(StateHeader);
    const int32_t c14[14] = {directed, (int32_t)gp, (int32_t)gq, N, L, M, (int32_t)an, (int32_t)ad, (int32_t)bn,
                             (int32_t)bd, (int32_t)rn, (int32_t)rd, empty_target | (refine_random << 1),
                             (int32_t)(uint32_t)refine_seed};
    std::memcpy(hd.cfg, c14, sizeof(c14));
    hd.batches = batches;
    hd.n = n;
    hd.top = top;
    hd.m = m;
    hd.ein = Ein;
    hd.skk_hi = (int64_t)(SKK >> 64);
    hd.skk_lo = (uint64_t)SKK;
    std::memcpy(hd.lim, lim, sizeof(hd.lim));
    hd.total_bytes = bytes;
    put(&hd, sizeof hd);
    put_dev(Kout, 8ull * n);
    if (directed) put_dev(Kin, 8ull * n);
    for (int r = 0; r <= top; ++r) {
      Level& V = lv[r];
      put_dev(V.alive, n);
      put_dev(V.lab, 4ull * n);
      if (r < L) {
        put_dev(V.par, 4ull * n);
        put_dev(V.rsize, 4ull * n);
      }
      put_dev(V.kout, 8ull * n);
      if (directed) put_dev(V.kin, 8ull * n);
      std::vector<uint64_t> keys;
      std::vector<int64_t> w;
      export_entries(r, keys, w);   // sorted by (row, column)
      std::vector<uint32_t> deg(n, 0);
      for (uint64_t k : keys) deg[k >> 32]++;
      put(deg.data(), 4ull * n);
      const uint64_t nnz = keys.size();
      put(&nnz, 8);
      for (uint64_t k : keys) {
        const uint32_t c = (uint32_t)k;
        put(&c, 4);
      }
      if (r == 0) {
        for (int64_t x : w) {
          const uint32_t v = (uint32_t)x;
          put(&v, 4);
        }
      } else {
        put(w.data(), 8 * nnz);
      }
    }
    if ((uint64_t)(p - out) != bytes) throw DeviceError{hipErrorUnknown};
  }
  // Restore a state written by export_state into this freshly initialised engine (same n and
  // parameters).  The caller has checked the header and the blob's size.
  int import_state(const uint8_t* blob, uint64_t bytes) {
    const StateHeader& hd = *(const StateHeader*)blob;
    const uint8_t* p = blob + sizeof(StateHeader);
    const uint8_t* end = blob + bytes;
    auto take = [&](uint64_t k) -> const uint8_t* {
      if ((uint64_t)(end - p) < k) return nullptr;
      const uint8_t* q = p;
      p += k;
      return q;
    };
    if (hd.top < 0 || hd.top > L) return LDL_EINVAL;
    if (hd.m < 0 || hd.m >= ((int64_t)1 << 40)) return LDL_EINVAL;
    for (int w = 0; w < 2; ++w)
      if (!valid_limits(hd.lim[w])) return LDL_EINVAL;
    // validate the whole blob on the host before any device state is written
    struct LevelPtrs {
      const uint8_t *alive, *lab, *par, *rsize, *kout, *kin, *deg, *cols, *w;
      uint64_t nnz;
    };
    const uint8_t* kout_t = take(8ull * n);
    const uint8_t* kin_t = directed ? take(8ull * n) : kout_t;
    if (!kout_t || !kin_t) return LDL_EINVAL;
    std::vector<LevelPtrs> lp(hd.top + 1);
    for (int r = 0; r <= hd.top; ++r) {
      LevelPtrs& q = lp[r];
      q.alive = take(n);
      q.lab = take(4ull * n);
      q.par = r < L ? take(4ull * n) : nullptr;
      q.rsize = r < L ? take(4ull * n) : nullptr;
      q.kout = take(8ull * n);
      q.kin = directed ? take(8ull * n) : q.kout;
      q.deg = take(4ull * n);
      const uint8_t* nz = take(8);
      if (!q.alive || !q.lab || (r < L && (!q.par || !q.rsize)) || !q.kout || !q.kin || !q.deg || !nz)
        return LDL_EINVAL;
      std::memcpy(&q.nnz, nz, 8);
      if (q.nnz >= (1ull << 31)) return LDL_EINVAL;   // restored through the row-update path
      q.cols = take(4 * q.nnz);
      q.w = take((r == 0 ? 4 : 8) * q.nnz);
      if (!q.cols || !q.w) return LDL_EINVAL;
      const uint32_t* lab = (const uint32_t*)q.lab;
      const uint32_t* deg = (const uint32_t*)q.deg;
      const uint32_t* cols = (const uint32_t*)q.cols;
      uint64_t sum = 0;
      for (uint32_t u = 0; u < n; ++u) {
        if (lab[u] >= n || (q.par && ((const uint32_t*)q.par)[u] >= n)) return LDL_EINVAL;
        sum += deg[u];
      }
      if (sum != q.nnz) return LDL_EINVAL;
      uint64_t k = 0;
      for (uint32_t u = 0; u < n; ++u)
        for (uint32_t i = 0; i < deg[u]; ++i, ++k) {
          if (cols[k] >= n || (i && cols[k] <= cols[k - 1])) return LDL_EINVAL;   // ascending, distinct
          const int64_t w = r == 0 ? (int64_t)((const uint32_t*)q.w)[k] : ((const int64_t*)q.w)[k];
          if (w <= 0) return LDL_EINVAL;
        }
    }
    if (p != end) return LDL_EINVAL;
    mutating = true;
    hcheck(hipMemcpyAsync(Kout, kout_t, 8ull * n, hipMemcpyHostToDevice, st));
    if (directed) hcheck(hipMemcpyAsync(Kin, kin_t, 8ull * n, hipMemcpyHostToDevice, st));
    top = hd.top;
    for (int r = 0; r <= top; ++r) {
      const LevelPtrs& q = lp[r];
      Level& V = lv[r];
      hcheck(hipMemcpyAsync(V.alive, q.alive, n, hipMemcpyHostToDevice, st));
      hcheck(hipMemcpyAsync(V.lab, q.lab, 4ull * n, hipMemcpyHostToDevice, st));
      if (r < L) {
        hcheck(hipMemcpyAsync(V.par, q.par, 4ull * n, hipMemcpyHostToDevice, st));
        hcheck(hipMemcpyAsync(V.rsize, q.rsize, 4ull * n, hipMemcpyHostToDevice, st));
      }
      if (q.nnz) {   // rows through the general row-update path (the degrees are restored below)
        std::vector<uint64_t> keys(q.nnz);
        std::vector<int64_t> w(q.nnz);
        const uint32_t* deg = (const uint32_t*)q.deg;
        const uint32_t* cols = (const uint32_t*)q.cols;
        uint64_t k = 0;
        for (uint32_t u = 0; u < n; ++u)
          for (uint32_t i = 0; i < deg[u]; ++i, ++k) {
            keys[k] = ((uint64_t)u << id_bits) | cols[k];
            w[k] = r == 0 ? (int64_t)((const uint32_t*)q.w)[k] : ((const int64_t*)q.w)[k];
          }
        ensure_tuples(q.nnz + 16);
        hcheck(hipMemcpyAsync(tk0, keys.data(), 8 * q.nnz, hipMemcpyHostToDevice, st));
        hcheck(hipMemcpyAsync(tv0, w.data(), 8 * q.nnz, hipMemcpyHostToDevice, st));
        apply_records(r, tk0, tv0, q.nnz, false);
        hcheck(hipStreamSynchronize(st));
      }
      hcheck(hipMemcpyAsync(V.kout, q.kout, 8ull * n, hipMemcpyHostToDevice, st));
      if (directed) hcheck(hipMemcpyAsync(V.kin, q.kin, 8ull * n, hipMemcpyHostToDevice, st));
      hcheck(hipStreamSynchronize(st));
    }
    m = hd.m;
    Ein = hd.ein;
    SKK = ((i128)hd.skk_hi << 64) | (i128)hd.skk_lo;
    batches = hd.batches;
    std::memcpy(lim, hd.lim, sizeof(lim));
    mutating = false;
    return LDL_OK;
  }

  uint64_t nnz_of(int r) {
    std::vector<uint32_t> deg(n);
    hcheck(hipMemcpyAsync(deg.data(), lv[r].out.ref.deg, 4ull * n, hipMemcpyDeviceToHost, st));
    hcheck(hipStreamSynchronize(st));
    uint64_t s = 0;
    for (uint32_t d : deg) s += d;
    return s;
  }
};

}  // namespace ldl

// ====================================================================== C ABI

struct ldl_handle {
  ldl::Engine* e;
};

namespace {

// A device error poisons the handle; so does running out of memory once the batch has started
// changing the state (the batch can then be neither finished nor undone).
int guard_err(ldl_handle* h, int code) {
  if (h && (code == LDL_EDEVICE || (code == LDL_ENOMEM && h->e->mutating))) h->e->broken = true;
  return code;
}

// the handle's allocator serves the library primitives' temporary storage during the call
struct PrimAllocScope {
  explicit PrimAllocScope(ldl_handle* h) { ldl::prim_set_allocator(h && h->e->halloc ? &h->e->palloc : nullptr); }
  ~PrimAllocScope() { ldl::prim_set_allocator(nullptr); }
};

template <typename F>
int run_guarded(ldl_handle* h, F&& f) {
  PrimAllocScope scope(h);
  try {
    return f();
  } catch (const ldl::NoMem&) {
    return guard_err(h, LDL_ENOMEM);
  } catch (const ldl::DeviceError&) {
    return guard_err(h, LDL_EDEVICE);
  } catch (const std::bad_alloc&) {
    return guard_err(h, LDL_ENOMEM);
  }
}

bool cfg_ok(const ldl_config& c) {
  auto in16 = [](int32_t x, int32_t lo) { return x >= lo && x < 65536; };
  return in16(c.gamma_num, 1) && in16(c.gamma_den, 1) && c.N >= 1 && c.M >= 1 && c.L >= 0 && c.L <= 16 &&
         in16(c.alpha_num, 0) && in16(c.alpha_den, 1) && in16(c.beta_num, 0) && in16(c.beta_den, 1) &&
         in16(c.refresh_num, 0) && in16(c.refresh_den, 1) && (c.directed == 0 || c.directed == 1) &&
         (c.empty_target == 0 || c.empty_target == 1) && (c.refine_random == 0 || c.refine_random == 1) &&
         ((c.alloc == nullptr) == (c.free == nullptr));
}

int apply_common(ldl_handle* h, const ldl_edge* ins, uint64_t ni, const ldl_pair* del, uint64_t nd,
                 const ldl_edge* chg, uint64_t nc, ldl_batch_stats* stats, bool on_device) {
  if (!h) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  if ((ni && !ins) || (nd && !del) || (nc && !chg)) return LDL_EINVAL;
  const bool bulk = h->e->bulk_eligible(nd, nc);   // laid out from 64-bit-count sorts
  if (ni + nd + nc >= (1ull << (bulk ? 32 : (h->e->directed ? 31 : 30)))) return LDL_EINVAL;
  h->e->mutating = false;
  return run_guarded(h, [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    e.stats = ldl_batch_stats{};
    e.call_begin();
    if (!e.call_t0) ldl::hcheck(hipEventCreate(&e.call_t0));
    if (!e.call_t1) ldl::hcheck(hipEventCreate(&e.call_t1));
    ldl::hcheck(hipEventRecord(e.call_t0, e.st));
    const uint32_t *di = (const uint32_t*)ins, *dd = (const uint32_t*)del, *dc = (const uint32_t*)chg;
    if (!on_device) {
      const uint32_t* staged = e.stage_batch(di, ni, dd, nd, dc, nc);
      di = staged;
      dd = staged ? staged + 3 * ni : nullptr;
      dc = staged ? staged + 3 * ni + 2 * nd : nullptr;
    }
    int rc;
    try {
      rc = e.apply(di, ni, dd, nd, dc, nc);
    } catch (...) {
      (void)hipStreamSynchronize(e.st);   // the staged copy may still be reading stage_h
      throw;
    }
    ldl::hcheck(hipEventRecord(e.call_t1, e.st));
    ldl::hcheck(hipEventSynchronize(e.call_t1));
    float ms = 0;
    ldl::hcheck(hipEventElapsedTime(&ms, e.call_t0, e.call_t1));
    ldl::hcheck(hipStreamSynchronize(e.st));
    e.finish_profile();
    e.call_end();
    if (e.scratch_limit && e.scratch_bytes() > e.scratch_limit) e.release_scratch();
    e.stats.total_ms = ms;
    if (stats) *stats = e.stats;
    return rc;
  });
}

}  // namespace

extern "C" {

void ldl_default_config(ldl_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->directed = 0;
  c->gamma_num = 1; c->gamma_den = 1;
  c->N = 2; c->L = 4; c->M = 5;
  c->alpha_num = 1; c->alpha_den = 1000;
  c->beta_num = 1; c->beta_den = 100;
  c->device = 0;
  c->stream = nullptr;
  c->profile = 0;
  c->refresh_num = 0;
  c->refresh_den = 1;
  c->alloc = nullptr;
  c->free = nullptr;
  c->alloc_ctx = nullptr;
  c->empty_target = 0;
  c->scratch_limit = 0;
  c->refine_random = 0;
  c->refine_seed = 0;
}

int ldl_create(const ldl_config* cfg, uint32_t n, const ldl_edge* edges, uint64_t n_edges, ldl_handle** out) {
  if (!out) return LDL_EINVAL;
  *out = nullptr;
  ldl_config c;
  ldl_default_config(&c);
  if (cfg) c = *cfg;
  if (n == 0 || !cfg_ok(c) || (n_edges && !edges)) return LDL_EINVAL;
  ldl_handle* h = new (std::nothrow) ldl_handle;
  if (!h) return LDL_ENOMEM;
  h->e = new (std::nothrow) ldl::Engine();
  if (!h->e) {
    delete h;
    return LDL_ENOMEM;
  }
  int rc = run_guarded(h, [&]() -> int {
    h->e->init(c, n);
    return LDL_OK;
  });
  if (rc == LDL_OK) rc = apply_common(h, edges, n_edges, nullptr, 0, nullptr, 0, nullptr, false);
  // static Leiden's scratch is sized for the whole graph; batches regrow what they need
  if (rc == LDL_OK) rc = ldl_release_scratch(h);
  if (rc != LDL_OK) {
    delete h->e;
    delete h;
    return rc;
  }
  *out = h;
  return LDL_OK;
}

int ldl_release_scratch(ldl_handle* h) {
  if (!h) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(h, [&]() -> int {
    ldl::hcheck(hipSetDevice(h->e->device));
    h->e->release_scratch();
    return LDL_OK;
  });
}

int ldl_apply_batch(ldl_handle* h, const ldl_edge* ins, uint64_t n_ins, const ldl_pair* del, uint64_t n_del,
                    const ldl_edge* chg, uint64_t n_chg, ldl_batch_stats* stats) {
  return apply_common(h, ins, n_ins, del, n_del, chg, n_chg, stats, false);
}

int ldl_apply_batch_device(ldl_handle* h, const ldl_edge* d_ins, uint64_t n_ins, const ldl_pair* d_del,
                           uint64_t n_del, const ldl_edge* d_chg, uint64_t n_chg, ldl_batch_stats* stats) {
  return apply_common(h, d_ins, n_ins, d_del, n_del, d_chg, n_chg, stats, true);
}

int ldl_get_partition(const ldl_handle* h, uint32_t* labels, uint64_t n) {
  if (!h || !labels || n != h->e->n) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    ldl::hcheck(hipMemcpyAsync(labels, e.lv[0].lab, 4ull * e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipStreamSynchronize(e.st));
    return LDL_OK;
  });
}

int ldl_modularity_exact(const ldl_handle* h, int64_t* num_hi, uint64_t* num_lo, int64_t* den_hi,
                         uint64_t* den_lo) {
  if (!h || !num_hi || !num_lo || !den_hi || !den_lo) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  const ldl::Engine& e = *h->e;
  const ldl::i128 num = e.qnum();
  const ldl::i128 den = (ldl::i128)e.gq * e.m * e.m;
  *num_hi = (int64_t)(num >> 64);
  *num_lo = (uint64_t)num;
  *den_hi = (int64_t)(den >> 64);
  *den_lo = (uint64_t)den;
  return LDL_OK;
}

int ldl_modularity(const ldl_handle* h, double* q) {
  if (!h || !q) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  const ldl::Engine& e = *h->e;
  if (e.m == 0) {
    *q = 0.0;
    return LDL_OK;
  }
  *q = (double)e.qnum() / ((double)e.gq * (double)e.m * (double)e.m);
  return LDL_OK;
}

void ldl_destroy(ldl_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->e->device);
  delete h->e;
  delete h;
}

int ldl_export_scalars(const ldl_handle* h, int32_t* top, int64_t* m, int64_t* ein, int64_t* skk_hi,
                       uint64_t* skk_lo) {
  if (!h || !top || !m || !ein || !skk_hi || !skk_lo) return LDL_EINVAL;
  const ldl::Engine& e = *h->e;
  *top = e.top;
  *m = e.m;
  *ein = e.Ein;
  *skk_hi = (int64_t)(e.SKK >> 64);
  *skk_lo = (uint64_t)e.SKK;
  return LDL_OK;
}

int ldl_export_totals(const ldl_handle* h, int64_t* kout, int64_t* kin) {
  if (!h || !kout || !kin) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    ldl::hcheck(hipMemcpyAsync(kout, e.Kout, 8ull * e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipMemcpyAsync(kin, e.Kin, 8ull * e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipStreamSynchronize(e.st));
    return LDL_OK;
  });
}

int ldl_export_level(const ldl_handle* h, int32_t r, uint8_t* alive, uint32_t* lab, uint32_t* par, int64_t* kout,
                     int64_t* kin) {
  if (!h || !alive || !lab || !par || !kout || !kin) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  if (r < 0 || r > h->e->top) return LDL_EINVAL;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    ldl::Level& V = e.lv[r];
    ldl::hcheck(hipMemcpyAsync(alive, V.alive, e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipMemcpyAsync(lab, V.lab, 4ull * e.n, hipMemcpyDeviceToHost, e.st));
    if (V.par) ldl::hcheck(hipMemcpyAsync(par, V.par, 4ull * e.n, hipMemcpyDeviceToHost, e.st));
    else std::memset(par, 0, 4ull * e.n);
    ldl::hcheck(hipMemcpyAsync(kout, V.kout, 8ull * e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipMemcpyAsync(kin, V.kin, 8ull * e.n, hipMemcpyDeviceToHost, e.st));
    ldl::hcheck(hipStreamSynchronize(e.st));
    return LDL_OK;
  });
}

uint64_t ldl_level_nnz(const ldl_handle* h, int32_t r) {
  if (!h || h->e->broken || r < 0 || r > h->e->top) return 0;
  uint64_t v = 0;
  int rc = run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    v = h->e->nnz_of(r);
    return LDL_OK;
  });
  return rc == LDL_OK ? v : 0;
}

int ldl_export_entries(const ldl_handle* h, int32_t r, uint32_t* rows, uint32_t* cols, int64_t* w) {
  if (!h || !rows || !cols || !w) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  if (r < 0 || r > h->e->top) return LDL_EINVAL;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    std::vector<uint64_t> keys;
    std::vector<int64_t> ws;
    h->e->export_entries(r, keys, ws);
    for (size_t i = 0; i < keys.size(); ++i) {
      rows[i] = (uint32_t)(keys[i] >> 32);
      cols[i] = (uint32_t)keys[i];
      w[i] = ws[i];
    }
    return LDL_OK;
  });
}

int ldl_get_partition_device(const ldl_handle* h, uint32_t* d_labels, uint64_t n) {
  if (!h || !d_labels || n != h->e->n) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    ldl::hcheck(hipMemcpyAsync(d_labels, e.lv[0].lab, 4ull * e.n, hipMemcpyDeviceToDevice, e.st));
    ldl::hcheck(hipStreamSynchronize(e.st));
    return LDL_OK;
  });
}

int ldl_export_state(const ldl_handle* h, void* blob, uint64_t capacity, uint64_t* size) {
  if (!h || !size) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    std::vector<uint64_t> nnz;
    const uint64_t bytes = e.state_bytes(nnz);
    *size = bytes;
    if (!blob) return LDL_OK;
    if (capacity < bytes) return LDL_EINVAL;
    e.export_state((uint8_t*)blob, bytes);
    return LDL_OK;
  });
}

int ldl_import_state(const ldl_config* cfg, const void* blob, uint64_t size, ldl_handle** out) {
  if (!out) return LDL_EINVAL;
  *out = nullptr;
  using Hd = ldl::Engine::StateHeader;
  if (!blob || size < sizeof(Hd)) return LDL_EINVAL;
  Hd hd;
  std::memcpy(&hd, blob, sizeof(Hd));
  if (std::memcmp(hd.magic, "LDLSTATE", 8) != 0 || hd.version != ldl::Engine::kStateVersion ||
      hd.header_bytes != sizeof(Hd) || hd.total_bytes != size || hd.n == 0)
    return LDL_EINVAL;
  ldl_config c;
  ldl_default_config(&c);
  if (cfg) c = *cfg;   // device, stream, profile and test flags from the caller
  c.directed = hd.cfg[0];
  c.gamma_num = hd.cfg[1]; c.gamma_den = hd.cfg[2];
  c.N = hd.cfg[3]; c.L = hd.cfg[4]; c.M = hd.cfg[5];
  c.alpha_num = hd.cfg[6]; c.alpha_den = hd.cfg[7];
  c.beta_num = hd.cfg[8]; c.beta_den = hd.cfg[9];
  c.refresh_num = hd.cfg[10]; c.refresh_den = hd.cfg[11];
  if (hd.cfg[12] & ~3) return LDL_EINVAL;
  c.empty_target = hd.cfg[12] & 1;
  c.refine_random = (hd.cfg[12] >> 1) & 1;
  c.refine_seed = (uint32_t)hd.cfg[13];
  if (!cfg_ok(c)) return LDL_EINVAL;
  ldl_handle* h = new (std::nothrow) ldl_handle;
  if (!h) return LDL_ENOMEM;
  h->e = new (std::nothrow) ldl::Engine();
  if (!h->e) {
    delete h;
    return LDL_ENOMEM;
  }
  int rc = run_guarded(h, [&]() -> int {
    h->e->init(c, hd.n);
    const int r = h->e->import_state((const uint8_t*)blob, size);
    if (r == LDL_OK) h->e->release_scratch();
    return r;
  });
  if (rc != LDL_OK) {
    delete h->e;
    delete h;
    return rc;
  }
  *out = h;
  return LDL_OK;
}

int ldl_check_invariants(const ldl_handle* h, ldl_invariant_report* report) {
  if (!h || !report) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    ldl::InvScratch* sc = e.alloc<ldl::InvScratch>(1);   // the recount's sums, freed on return
    try {
      e.check_invariants(sc, report);
    } catch (...) {
      e.release(sc);
      throw;
    }
    e.release(sc);
    return LDL_OK;
  });
}

int ldl_check_invariants_noalloc(const ldl_handle* h, ldl_invariant_report* report) {
  if (!h || !report) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(const_cast<ldl_handle*>(h), [&]() -> int {
    ldl::Engine& e = *h->e;
    ldl::hcheck(hipSetDevice(e.device));
    e.check_invariants(e.static_sums, report);   // the device's static sums; no allocation
    return LDL_OK;
  });
}

int ldl_memory(const ldl_handle* h, uint64_t* held_bytes, uint64_t* recent_growth_bytes) {
  if (!h || !held_bytes || !recent_growth_bytes) return LDL_EINVAL;
  *held_bytes = h->e->held + (h->e->halloc ? 0 : h->e->cub_bytes);   // with the hook, held counts it
  *recent_growth_bytes = h->e->recent_growth();
  return LDL_OK;
}

int ldl_set_trace(ldl_handle* h, int32_t on) {
  if (!h) return LDL_EINVAL;
  h->e->tracing = on != 0;
  h->e->trace.clear();
  return LDL_OK;
}

uint64_t ldl_trace_len(const ldl_handle* h) { return h ? h->e->trace.size() : 0; }

int ldl_trace(const ldl_handle* h, int64_t* out) {
  if (!h || !out) return LDL_EINVAL;
  for (size_t i = 0; i < h->e->trace.size(); ++i) std::memcpy(out + 8 * i, h->e->trace[i].v, 64);
  return LDL_OK;
}

int ldl_get_bins(const ldl_handle* h, uint32_t limits[2][5]) {
  if (!h || !limits) return LDL_EINVAL;
  for (int w = 0; w < 2; ++w)
    for (int b = 0; b < 5; ++b) limits[w][b] = h->e->lim[w][b];
  return LDL_OK;
}

int ldl_set_bins(ldl_handle* h, const uint32_t limits[2][5]) {
  if (!h || !limits) return LDL_EINVAL;
  if (!ldl::Engine::valid_limits(limits[0]) || !ldl::Engine::valid_limits(limits[1])) return LDL_EINVAL;
  for (int w = 0; w < 2; ++w)
    for (int b = 0; b < 5; ++b) h->e->lim[w][b] = limits[w][b];
  return LDL_OK;
}

int ldl_autotune(ldl_handle* h, ldl_tune_report* report) {
  if (!h) return LDL_EINVAL;
  if (h->e->broken) return LDL_EBROKEN;
  return run_guarded(h, [&]() -> int {
    ldl::hcheck(hipSetDevice(h->e->device));
    h->e->autotune(report);
    return LDL_OK;
  });
}

const char* ldl_strerror(int code) {
  switch (code) {
    case LDL_OK: return "LDL_OK";
    case LDL_EINVAL: return "LDL_EINVAL";
    case LDL_EDUP: return "LDL_EDUP";
    case LDL_ENOEDGE: return "LDL_ENOEDGE";
    case LDL_EOVERFLOW: return "LDL_EOVERFLOW";
    case LDL_ENOMEM: return "LDL_ENOMEM";
    case LDL_EDEVICE: return "LDL_EDEVICE";
    case LDL_EBROKEN: return "LDL_EBROKEN";
    default: return "LDL_UNKNOWN";
  }
}

const char* ldl_version(void) { return "ldl 0.1.0 (gfx950)"; }

}  // extern "C"
