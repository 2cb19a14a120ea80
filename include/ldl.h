/*
 * ldl.h -- C ABI of the MI355X (gfx950) LD-Leiden library.
 *
 * LD-Leiden maintains a modularity partition of a weighted directed or undirected graph
 * under batches of edge insertions, deletions and weight changes (paper Sec. II, problem
 * statement).  Each batch runs the paper's Algorithm 1 (Sec. III-C) on the GPU: batch
 * apply and statistic repair, frontier-restricted local moves with the decoupling filter
 * (Sec. III-D, III-E), restricted refinement, and subtract-add repair of the aggregate
 * hierarchy (Sec. III-F, Eq. 3).
 *
 * Arithmetic is exact: weights are integers, gains are compared as integers (the modularity
 * change scaled by q*m^2 for resolution gamma = p/q; half of that for undirected graphs), ties
 * go to the lowest community id and every stage is round-synchronous, so results are
 * deterministic and independent of launch shapes.
 *
 * Conventions for every call:
 *   - Return value: LDL_OK (0) or a negative LDL_E* code.  Batches are atomic: validation and
 *     the allocations that depend on the batch size finish before the state changes, so on
 *     LDL_EINVAL, LDL_EDUP, LDL_ENOEDGE, LDL_EOVERFLOW and on LDL_ENOMEM from those
 *     allocations the graph and partition are unchanged.  After LDL_EDEVICE, or LDL_ENOMEM
 *     once the update has started (a pool that cannot grow), the handle is poisoned and every
 *     later call returns LDL_EBROKEN.
 *   - A batch holds fewer than 2^31 updates (2^30 for undirected graphs), else LDL_EINVAL; an
 *     insert-only batch into a graph without entries and without aggregate levels (the first
 *     batch, as at creation) may hold up to 2^32 - 1.
 *   - Vertices are 0..n-1 (n fixed at creation).  Undirected pairs are unordered.
 *   - Input arrays are owned by the caller and only read during the call; the handle owns
 *     all device memory it allocates.  A handle is not thread-safe; distinct handles may be
 *     used from different threads.
 *   - All calls are synchronous with respect to the handle's stream.
 */
#ifndef LDL_H
#define LDL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDL_OK 0
#define LDL_EINVAL (-1)    /* null pointer, n == 0, id >= n, zero weight, bad config       */
#define LDL_EDUP (-2)      /* a vertex pair appears twice in one batch                      */
#define LDL_ENOEDGE (-3)   /* deletion or change of an absent edge                          */
#define LDL_EOVERFLOW (-4) /* an edge weight would exceed 2^32-1, or m would reach 2^40    */
#define LDL_ENOMEM (-5)    /* device allocation failed                                      */
#define LDL_EDEVICE (-6)   /* a HIP runtime error; the handle is poisoned                   */
#define LDL_EBROKEN (-7)   /* the handle was poisoned by an earlier device error            */

typedef struct ldl_handle ldl_handle;

/* An edge (u, v) with integer weight w >= 1. */
typedef struct ldl_edge {
  uint32_t u, v, w;
} ldl_edge;

/* A vertex pair (u, v). */
typedef struct ldl_pair {
  uint32_t u, v;
} ldl_pair;

/*
 * Parameters (paper Table I; defaults from the parameter study, Sec. IV-D):
 *   directed            0: undirected (W symmetric), 1: directed
 *   gamma_num/den       resolution gamma = num/den of Eq. 1, both in [1, 65535]; default 1/1
 *   N                   outer passes (>= 1); default 2
 *   L                   top hierarchy level index, levels 0..L (0..16); default 4
 *   M                   move / refinement iterations per level (>= 1); default 5
 *   alpha_num/den       gain threshold alpha (Algorithm 1's move and pass stops); default 1/1000
 *   beta_num/den        moved-fraction threshold beta (move and refinement stops); default 1/100
 *   device              HIP device ordinal
 *   stream              hipStream_t to run on, or NULL for the handle's own stream
 *   profile             nonzero: time the local-move kernels with HIP events (see stats)
 *   refresh_num/den     adaptive refresh threshold rho (a variant, off by default: 0/1).  When a
 *                       batch's level-0 frontier (InitFrontier: its alive seeds and every alive
 *                       member of their communities) holds at least rho n vertices, locality no
 *                       longer holds (Sec. IV-F, Sec. V) and the batch reoptimises from scratch:
 *                       hierarchy and partition are discarded and static Leiden runs on the
 *                       current graph (the state ldl_create would reach for the current edges).
 *                       num in [0, 65535], den in [1, 65535]
 *   alloc/free/alloc_ctx device allocator hook (see ldl_alloc_fn); NULL for hipMalloc / hipFree.
 *                       One of the two set without the other is LDL_EINVAL.
 *   empty_target        0 or 1 (a variant, off by default).  The paper's BestMove considers the
 *                       communities adjacent to v only (Sec. III-C).  With 1 it also considers an
 *                       empty community, as the Louvain and Leiden move phases do: the community
 *                       labelled v itself, offered when v does not carry label v and that
 *                       community's totals Kout, Kin are zero (so no weight leads to it and the
 *                       gain of Eq. 2 is that of an empty target).  It is one more candidate in the
 *                       comparison (larger exact gain, equal gains to the lower id); refinement
 *                       is unchanged.
 *   refine_random       0 or 1 (a variant, off by default).  The paper's BestRef, like BestMove,
 *   refine_seed         takes the target of largest gain (Algorithm 1).  With 1 the target is
 *                       drawn at random among the refined communities of strictly positive gain,
 *                       as the Leiden refinement of Traag et al. draws among improving ones; here
 *                       uniformly (the large-temperature limit of its exp(gain / theta) weights,
 *                       which keeps the choice exact).  Every such target y of node u gets the
 *                       priority high32(mix(mix(key ^ u) ^ y)) | 1, where mix is SplitMix64's
 *                       output function and key = mix(mix(mix(mix(seed + 0x9E3779B97F4A7C15) ^
 *                       batch) ^ pass) ^ (level << 32 | iteration)) | 1, with batch the number of
 *                       batches the handle accepted before this one (creation's is 0); the highest
 *                       priority wins (equal priorities: the larger gain, then the lower id).
 *                       The seed and the batch count travel in ldl_export_state's blob.
 *   scratch_limit       bytes of growable scratch (see ldl_release_scratch) a handle may keep
 *                       between calls: a call that leaves more frees it before returning (0, the
 *                       default: keep it for the next call).  For many resident graphs whose
 *                       occasional large batches would otherwise each keep their peak scratch.
 *   test_flags          0 in production.  Bits that drive rarely taken internal paths, with
 *                       results unchanged: 1 = one decoupling round between host checks (second
 *                       commit phase), 2 = minimal hub bucket pool (overflow and redo of an
 *                       iteration), 4 = no spare adjacency capacity (row moves, pool growth),
 *                       8 = always queue the one-workgroup decoupling filter first (iterations
 *                       with more candidates than it holds run the filter after the host check),
 *                       16 = 64-slot LDS tables for the hub partitions (partition overflow, redo of
 *                       the iteration with more partitions per hub), 32 = no bulk load (the first
 *                       insert-only batch of a graph goes through the general lookup and row-update
 *                       path instead of being laid out directly from its sorted records), 64 = every
 *                       candidate kernel of the degree bins runs as one workgroup (each workgroup
 *                       and wavefront walks many vertices through its software pipeline),
 *                       128 = aggregation tuples sorted in chunks of 4,096, and every repair of
 *                       more than 4,096 tuples done as a rebuild of the level above from scratch
 */
/* Device-memory allocator hook (for example a caching allocator such as PyTorch's): alloc returns
 * `bytes` of device memory on `device` for use on `stream` (the handle's stream), or NULL when it
 * cannot; free releases a pointer alloc returned, with the same size, device and stream.  ctx is
 * passed through.  Both are called only from the thread that calls into the handle. */
typedef void* (*ldl_alloc_fn)(void* ctx, uint64_t bytes, int32_t device, void* stream);
typedef void (*ldl_free_fn)(void* ctx, void* ptr, uint64_t bytes, int32_t device, void* stream);

typedef struct ldl_config {
  int32_t directed;
  int32_t gamma_num, gamma_den;
  int32_t N, L, M;
  int32_t alpha_num, alpha_den;
  int32_t beta_num, beta_den;
  int32_t device;
  void* stream;
  int32_t profile;
  int32_t test_flags;
  int32_t refresh_num, refresh_den;
  ldl_alloc_fn alloc;   /* both set: every device allocation of the handle goes through them; */
  ldl_free_fn free;     /* both NULL: hipMalloc / hipFree                                      */
  void* alloc_ctx;
  int32_t empty_target;
  uint64_t scratch_limit;
  int32_t refine_random;
  uint32_t refine_seed;
} ldl_config;

/* Per-call statistics (all counts summed over the call). */
typedef struct ldl_batch_stats {
  uint64_t updates;           /* input updates that changed a weight                      */
  uint64_t levels_processed;  /* process-level invocations over all passes                */
  uint64_t move_iters;        /* move iterations launched (not those over an empty set)   */
  uint64_t refine_iters;      /* refinement iterations launched (idem)                    */
  uint64_t scanned_vertices;  /* vertices evaluated by the local-move kernels             */
  uint64_t scanned_entries;   /* adjacency entries read by the local-move kernels         */
  uint64_t distinct_comms;    /* (vertex, neighbour community) pairs evaluated            */
  uint64_t candidates;        /* candidates with positive gain                            */
  uint64_t accepted;          /* moves accepted by the decoupling filter                  */
  uint64_t rollbacks;         /* move mini-batches rolled back (negative batch gain)      */
  uint64_t refine_moves;      /* accepted refinement moves                                */
  uint64_t agg_tuples;        /* aggregate-repair tuples emitted                          */
  uint64_t bm_launches;       /* local-move kernel launches (profile != 0)                */
  double bm_ms;               /* summed local-move kernel time in ms (profile != 0)       */
  double bm_bytes;            /* algorithmic bytes of those kernels (profile != 0)        */
  double total_ms;            /* wall time of the call measured with HIP events           */
  /* per candidate kernel k = 12*refine + 6*wide + bin, where bin is the degree bin of the
   * scanned vertices (entries per vertex in (0,8], (8,32], (32,128], (128,512], (512,2048],
   * above), wide = 1 for the int64 weights of aggregate levels and refine = 1 for BestRef:
   * launches, kernel time (HIP events around each launch, profile != 0), algorithmic bytes
   * (profile != 0) and adjacency entries read */
  uint64_t bin_launches[24];
  double bin_ms[24];
  double bin_bytes[24];
  uint64_t bin_entries[24];
  uint64_t lf_rounds;         /* decoupling rounds launched                               */
  uint64_t host_syncs;        /* stream synchronisations (host reads of device counters)  */
  uint64_t agg_records;       /* reduced records applied to levels above 0                */
  double search_ms;           /* summed time of whole candidate searches: binning, every bin's
                                 kernel and the hub path's passes and final reduction
                                 (HIP events, profile != 0)                                  */
  uint64_t max_gain_hi;       /* largest high 64-bit word of any candidate's exact 128-bit gain
                                 (nonzero once a gain reaches 2^64)                          */
  uint64_t agg_rebuilds;      /* aggregate levels rebuilt from scratch by Eq. 3 instead of
                                 repaired by subtract-add tuples (same matrix, lower cost)    */
  uint64_t refreshes;         /* 1 when the batch switched to full reoptimisation (refresh)   */
  uint64_t frontier0;         /* level-0 frontier size checked against the refresh threshold
                                 (0 when refresh is off)                                      */
} ldl_batch_stats;

/* Fill *cfg with the defaults listed above (undirected, device 0, own stream). */
void ldl_default_config(ldl_config* cfg);

/*
 * Create a handle for n vertices and the initial edge set (host array, n_edges entries,
 * insertion semantics; a repeated pair is LDL_EDUP).  Runs static Leiden, i.e. the batch
 * update applied to the all-singleton state (Sec. IV-E: batch 0 initialises the full snapshot).
 * cfg may be NULL for the defaults.  On success *out receives the handle.
 */
int ldl_create(const ldl_config* cfg, uint32_t n, const ldl_edge* edges, uint64_t n_edges,
               ldl_handle** out);

/*
 * Apply one batch (host arrays; any count may be 0) and run Algorithm 1:
 *   ins[i]: w_new = w_old + w (creates the edge when absent)
 *   del[i]: removes the edge (absent edge: LDL_ENOEDGE)
 *   chg[i]: sets the weight to w >= 1 (absent edge: LDL_ENOEDGE)
 * A pair may appear at most once across the three lists.  stats may be NULL.
 */
int ldl_apply_batch(ldl_handle* h, const ldl_edge* ins, uint64_t n_ins, const ldl_pair* del,
                    uint64_t n_del, const ldl_edge* chg, uint64_t n_chg, ldl_batch_stats* stats);

/* As ldl_apply_batch, with the three arrays in device memory of the handle's device.  They are read
 * on the handle's stream (ldl_config.stream, or its own), which waits for no other stream: work that
 * writes them on another stream must have completed before the call. */
int ldl_apply_batch_device(ldl_handle* h, const ldl_edge* d_ins, uint64_t n_ins, const ldl_pair* d_del,
                           uint64_t n_del, const ldl_edge* d_chg, uint64_t n_chg, ldl_batch_stats* stats);

/* Copy the level-0 partition (community id of each vertex, ids in [0, n)) into the caller's
 * host array of length n (n must equal the handle's vertex count). */
int ldl_get_partition(const ldl_handle* h, uint32_t* labels, uint64_t n);

/* Eq. 1 for the current partition in FP64: Qnum / (q m^2), with Qnum exact (0 when m == 0). */
int ldl_modularity(const ldl_handle* h, double* q);

/* Exact numerator q*m*Ein - p*sum_c Kout_c Kin_c as a signed 128-bit value (hi, lo) and the
 * denominator q*m^2 likewise; Q = num / den. */
int ldl_modularity_exact(const ldl_handle* h, int64_t* num_hi, uint64_t* num_lo, int64_t* den_hi,
                         uint64_t* den_lo);

/* Free the handle's growable scratch: aggregation tuples, reduced records, sorted entries,
 * row-update buffers, the sort and scan primitives' temporary storage and the staging buffers of
 * host batches (pinned host and device memory), all of which a batch call grows to its own size
 * and keeps for the next call.  The next call that needs them
 * allocates them again; the state and every later result are unchanged.  ldl_create and
 * ldl_import_state end with it (static Leiden's scratch is sized for the whole graph), so a
 * resident handle holds its state plus what its batches use.  LDL_EINVAL for NULL. */
int ldl_release_scratch(ldl_handle* h);

/* Release every device resource of the handle.  NULL is ignored. */
void ldl_destroy(ldl_handle* h);

/*
 * State export for checking (host arrays sized by the caller):
 *   ldl_export_scalars: top level index, m, Ein, sum Kout*Kin (hi, lo)
 *   ldl_export_totals:  community totals Kout, Kin (length n each)
 *   ldl_export_level:   node arrays of level r (alive u8, label u32, parent u32, kout, kin i64)
 *   ldl_level_nnz:      number of stored matrix entries of level r (returns 0 on error)
 *   ldl_export_entries: those entries as (row, col, weight) arrays of length nnz, row-major
 */
int ldl_export_scalars(const ldl_handle* h, int32_t* top, int64_t* m, int64_t* ein, int64_t* skk_hi,
                       uint64_t* skk_lo);
int ldl_export_totals(const ldl_handle* h, int64_t* kout, int64_t* kin);
int ldl_export_level(const ldl_handle* h, int32_t r, uint8_t* alive, uint32_t* lab, uint32_t* par,
                     int64_t* kout, int64_t* kin);
uint64_t ldl_level_nnz(const ldl_handle* h, int32_t r);
int ldl_export_entries(const ldl_handle* h, int32_t r, uint32_t* rows, uint32_t* cols, int64_t* w);

/* Copy the level-0 partition (as ldl_get_partition) into device memory of the handle's device
 * (d_labels: n u32 words, caller-owned).  The copy has completed when the call returns. */
int ldl_get_partition_device(const ldl_handle* h, uint32_t* d_labels, uint64_t n);

/*
 * Checkpoint of the whole state (paper Sec. III-A: the hierarchy H = (G^0..G^L) with its parent
 * maps, level labels and cached community totals, plus the exact m, Ein and sum Kout*Kin of
 * Eq. 1) as an opaque, versioned blob in host memory.  ldl_export_state writes the blob size to
 * *size; with blob == NULL it only reports the size, with capacity < size it returns LDL_EINVAL
 * and writes nothing.  Equal states give equal blobs.  ldl_import_state creates a new handle from
 * a blob (cfg supplies device, stream, profile and test flags, or NULL for the defaults; the
 * method parameters come from the blob); a handle continued from the import behaves exactly like
 * the exported one.  A blob that is truncated, of another version, or holds an id >= n, a zero or
 * negative weight, or a level with 2^31 or more entries is LDL_EINVAL (the blob is only checked
 * for consistency of its layout; ldl_check_invariants recounts the method's invariants).
 */
int ldl_export_state(const ldl_handle* h, void* blob, uint64_t capacity, uint64_t* size);
int ldl_import_state(const ldl_config* cfg, const void* blob, uint64_t size, ldl_handle** out);

/*
 * Device-side recount of the state's invariants, reading every stored entry once per
 * orientation and every node once per level:
 *   LDL_INV_DEGREES    kout/kin are the row/column sums of each level's matrix (positive weights,
 *                      entries only between alive nodes, dead nodes have zero degrees)
 *   LDL_INV_TRANSPOSE  the in-rows of a directed level hold the transpose of its out-rows; an
 *                      undirected level's matrix is symmetric
 *   LDL_INV_AGGREGATE  Eq. 3 (Sec. III-F): W_{r+1}(x,y) = sum of W_r(u,v) over pi_r(u) = x,
 *                      pi_r(v) = y, and a level-(r+1) node is alive iff it has an alive child
 *   LDL_INV_LABELS     labels nest: P^r(u) = P^{r+1}(pi_r(u)) (Sec. III-A)
 *   LDL_INV_ROOTS      an alive refined community x contains its root node x at level r
 *   LDL_INV_TOTALS     m, Ein and the community totals Kout/Kin recounted from the level-0 matrix
 *                      and P^0, and sum Kout*Kin exactly (the terms of Eq. 1)
 *   LDL_INV_RANGE      a neighbour id or label outside [0, n)
 * Degrees, labels, roots, liveness, m, Ein and sum Kout*Kin are compared exactly; the matrix
 * comparisons (aggregation, transpose) and the per-community totals compare weighted 64-bit
 * fingerprints (sums of w * h(key) for two fixed odd hash functions), which always differ when a
 * single entry differs.  report->failed is the mask of failed checks (0: all hold), report->level
 * the lowest level where one failed (-1: none), report->entries the matrix entries read.  The
 * call allocates its small block of recount sums on the device and frees it before returning.
 */
#define LDL_INV_DEGREES 1u
#define LDL_INV_TRANSPOSE 2u
#define LDL_INV_AGGREGATE 4u
#define LDL_INV_LABELS 8u
#define LDL_INV_ROOTS 16u
#define LDL_INV_TOTALS 32u
#define LDL_INV_RANGE 64u
typedef struct ldl_invariant_report {
  uint32_t failed;
  int32_t level;
  uint64_t entries;
} ldl_invariant_report;
int ldl_check_invariants(const ldl_handle* h, ldl_invariant_report* report);

/*
 * ldl_check_invariants for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same recount and the same
 * report, with its sums in a 512-byte block of static device memory that each device holds for
 * the life of the process (its address is looked up once per device when a handle is created on
 * it).  It calls no allocating routine.  There is no size limit (the kernels loop over any n and
 * any number of entries with a fixed grid).  Every call on one device shares that device's block
 * and clears it first: calls that overlap on one device (different handles on different host
 * threads or streams) race and may report wrong results.
 */
int ldl_check_invariants_noalloc(const ldl_handle* h, ldl_invariant_report* report);

/* Device memory of the handle: *held_bytes it holds now (state and the scratch it keeps between
 * calls), *recent_growth_bytes the largest amount one of its last 8 batch calls allocated beyond
 * what it held when the call began (creation not counted).  Read by the serving loop's
 * admission; a handle must not be in use by another thread during the call. */
int ldl_memory(const ldl_handle* h, uint64_t* held_bytes, uint64_t* recent_growth_bytes);

/* Per-iteration trace (8 int64 per record: pass, level, phase 0 move / 1 refine, iteration,
 * scanned vertices, candidates, accepted, low 64 bits of the exact batch gain). */
int ldl_set_trace(ldl_handle* h, int32_t on);
uint64_t ldl_trace_len(const ldl_handle* h);
int ldl_trace(const ldl_handle* h, int64_t* out);

/*
 * Multi-graph batched mode.  bs[i] is applied to hs[i]; entries that name the same handle are
 * applied in index order, one at a time, and entries of different handles run concurrently on
 * up to `workers` host threads, each handle on its own HIP stream (workers == 0: one per
 * distinct handle, at most 64).  The result of every handle is identical to applying its
 * batches alone with ldl_apply_batch.  Arrays are host memory owned by the caller.  status[i]
 * (nullable) receives each entry's return code, stats[i] (nullable) its statistics; the call
 * returns LDL_OK if every entry succeeded, else the first failing code in index order.
 */
typedef struct ldl_batch {
  const ldl_edge* ins;
  uint64_t n_ins;
  const ldl_pair* del;
  uint64_t n_del;
  const ldl_edge* chg;
  uint64_t n_chg;
} ldl_batch;

int ldl_apply_batches(ldl_handle* const* hs, const ldl_batch* bs, uint32_t count, uint32_t workers, int* status,
                      ldl_batch_stats* stats);

/*
 * Serving loop over resident graphs.  A server owns `workers` host threads.  ldl_server_submit
 * copies a batch for handle h into a request and returns its ticket; requests of one handle
 * run in submission order, back to back on the worker that holds the handle; requests of
 * different handles overlap on the device.  A request is admitted only while the estimated
 * device-memory footprint of all running requests stays within `mem_budget_bytes` (a request
 * larger than the budget runs alone); a request's footprint is the larger of a linear estimate in
 * its update count (1 MiB + 256 B per update) and the most its handle's recent batch calls have
 * allocated (ldl_memory), taken when it is admitted.  ldl_server_wait blocks until the ticket completes and
 * returns its code, statistics and latency (submission to completion, milliseconds); a ticket can
 * be waited on once (a second or concurrent wait on it returns LDL_EINVAL).  A handle
 * must not be used outside the server while it has queued requests.
 */
typedef struct ldl_server ldl_server;

int ldl_server_create(uint32_t workers, uint64_t mem_budget_bytes, ldl_server** out);
int ldl_server_submit(ldl_server* s, ldl_handle* h, const ldl_edge* ins, uint64_t n_ins, const ldl_pair* del,
                      uint64_t n_del, const ldl_edge* chg, uint64_t n_chg, uint64_t* ticket);
int ldl_server_wait(ldl_server* s, uint64_t ticket, int* status, ldl_batch_stats* stats, double* latency_ms);
/* Block until every submitted request has completed. */
int ldl_server_drain(ldl_server* s);
/* Drain, stop the workers and free the server (handles stay valid). NULL is ignored. */
void ldl_server_destroy(ldl_server* s);

/*
 * Degree bins of the candidate search (the per-vertex neighbour-community accumulation and argmax
 * of Sec. III-D; the bins are an implementation choice, not part of the method).  A vertex with T
 * adjacency entries (out + in) is evaluated by the kernel of the first bin b with T <= limit[b],
 * or by the multi-workgroup hub path when T exceeds limit[4].  Bin b's kernel holds at most
 * {8, 32, 128, 512, 2048}[b] entries, so a valid set has limit[b] <= that cap and
 * limit[0] <= limit[1] <= ... <= limit[4]; equal neighbours leave a bin empty.  Row 0 applies to
 * level 0 (32-bit weights), row 1 to the aggregate levels (64-bit weights).  Every valid set gives
 * bit-identical results; only the speed differs.  Defaults: {8, 32, 128, 128, 2048} for both (bin 3
 * empty: vertices with 129..2048 entries go to the 256-lane workgroup kernel).
 * ldl_set_bins returns LDL_EINVAL for an invalid set (limits unchanged).
 */
int ldl_get_bins(const ldl_handle* h, uint32_t limits[2][5]);
int ldl_set_bins(ldl_handle* h, const uint32_t limits[2][5]);

/*
 * Autotuner of the degree bins: on the handle's current graph, times the move-phase candidate
 * search over every alive node of level 0 (and of level 1 when it exists) plus a 1/64 stride
 * sample of them (the small frontiers of batch updates), runs one round of coordinate descent over
 * the five limits of each row and keeps the fastest set.  Read-only for the graph and partition.
 * report (nullable) receives the chosen limits and the cost (full + sample, ms) before and after.
 */
typedef struct ldl_tune_report {
  uint32_t limit[2][5];
  double ms_before[2];
  double ms_after[2];
  uint32_t trials;
} ldl_tune_report;

int ldl_autotune(ldl_handle* h, ldl_tune_report* report);

/* Human-readable name of an LDL_* code. */
const char* ldl_strerror(int code);

/* Library version string. */
const char* ldl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LDL_H */
