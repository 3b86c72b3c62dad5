/*
 * lcc.h -- C-ABI of the MI355X LambdaCC multilevel clustering library (pLouvain / Louvain+, pLeiden).
 *
 * The library clusters an undirected graph by maximising the LambdaCC objective (Eq. 1 of the paper):
 *
 *     lambdaCC(C) = sum over clusters C_i of sum over ordered pairs u != v in C_i of w(u,v) - lambda w(u) w(v)
 *
 * with the synchronous multilevel methods of the paper: Louvain / Louvain+ (Alg. 1, local move Alg. 2 with
 * the afterburner filter Alg. 3, contraction Alg. 4) and pLeiden (Alg. 5, spanning-tree refinement Alg. 6,
 * alternate local move Sec. V-A).  Modularity (w(v) = weighted degree, lambda = gamma / sum_v w(v)) and the
 * Constant Potts Model (w(v) = 1) are special cases (Sec. II-A).
 *
 * All arithmetic is exact: integer weights, 64-bit sums, scores compared as exact integers.  Results are
 * deterministic and independent of scheduling.
 *
 * Every entry point returns an lcc_status; on a negative status no output buffer is written and
 * lcc_last_error() (thread-local) describes the failure.  No C++ exception crosses this boundary.
 * Every step of a clustering call runs on the GPU; there is no CPU fallback.  lcc_objective, which scores given
 * labels of a host graph (no clustering), is the one host-side computation.
 */
#ifndef LCC_H
#define LCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LCC_OK = 0,
  LCC_ERR_INVALID = -1,       /* malformed arguments or CSR structure (offsets, index range, options) */
  LCC_ERR_NOT_SYMMETRIC = -2, /* some edge (u,v) has no reverse (v,u) of equal weight */
  LCC_ERR_SELF_LOOP = -3,     /* some row v contains v */
  LCC_ERR_UNSORTED = -4,      /* a row is not strictly ascending (duplicates count as unsorted) */
  LCC_ERR_WEIGHT = -5,        /* an edge weight <= 0 or a given vertex weight < 0 */
  LCC_ERR_LAMBDA = -6,        /* lambda outside [0, 1] or undefined (zero denominator / zero total weight) */
  LCC_ERR_OVERFLOW = -7,      /* exactness bound violated: total edge weight >= 2^32, a given vertex weight
                                 >= 2^31, or q * W_E + p * W^2 >= 2^62 for lambda = p / q in lowest terms
                                 (modularity: 2 W^2 < 2^62, i.e. W below about 1.5e9) */
  LCC_ERR_OOM = -8,           /* the allocator returned NULL */
  LCC_ERR_DEVICE = -9,        /* a HIP runtime call failed */
  LCC_ERR_BUSY = -10,         /* server: admission refused (footprint exceeds the free budget) */
  LCC_ERR_NOT_FOUND = -11     /* server: unknown ticket */
} lcc_status;

/* Method variants.  LCC_PLOUVAIN is the paper's pLouvain (Louvain+ with the uncoarsening local move,
 * Alg. 1 line 12); LCC_LOUVAIN omits the uncoarsening local move; LCC_PLEIDEN is Alg. 5; LCC_PLEIDEN_PLUS
 * adds the uncoarsening local move to pLeiden (Sec. VI-A). */
typedef enum { LCC_LOUVAIN = 0, LCC_PLOUVAIN = 1, LCC_PLEIDEN = 2, LCC_PLEIDEN_PLUS = 3 } lcc_variant;

/* Vertex weights w(v): given by the caller, the weighted degree (modularity), or 1 (CPM). */
typedef enum { LCC_VW_GIVEN = 0, LCC_VW_WEIGHTED_DEGREE = 1, LCC_VW_UNIT = 2 } lcc_vw_mode;

/* Where the graph arrays and labels_out live. */
typedef enum { LCC_MEM_HOST = 0, LCC_MEM_DEVICE = 1 } lcc_mem;

/* Undirected graph in symmetric CSR (Sec. IV: both (u,v) and (v,u) are stored).  Row v lists the neighbours
 * of v strictly ascending, without v itself.  Borrowed for the duration of a call.
 *   n            vertices, 0 <= n < 2^31
 *   nnz          stored (directed) entries = offsets[n], 0 <= nnz < 2^31
 *   offsets      n+1 entries, int32 (offsets_bits = 32) or int64 (offsets_bits = 64), offsets[0] = 0
 *   indices      nnz int32 neighbour ids
 *   edge_w       nnz int32 weights > 0, symmetric; NULL means every weight is 1
 *   vertex_w     n int64 weights >= 0, read only when vw_mode = LCC_VW_GIVEN
 *   mem          all arrays of this graph are host (LCC_MEM_HOST) or device (LCC_MEM_DEVICE) pointers */
typedef struct {
  int64_t n;
  int64_t nnz;
  const void* offsets;
  int32_t offsets_bits;
  const int32_t* indices;
  const int32_t* edge_w;
  const int64_t* vertex_w;
  lcc_vw_mode vw_mode;
  lcc_mem mem;
} lcc_graph;

/* lambda = num / den, or num / (den * W) when over_total_weight != 0, W = sum of the vertex weights.
 * Modularity with resolution gamma = a / b: vw_mode = LCC_VW_WEIGHTED_DEGREE, {a, b, 1}.  CPM 1/20: {1, 20, 0}. */
typedef struct {
  uint64_t num;
  uint64_t den;
  int32_t over_total_weight;
} lcc_lambda;

/* Trace sink (optional): records of 8 int64 {kind, level, phase, pass, a, b, c, d}:
 *   kind 1  local-move pass:     a = candidates |L|, b = kept moves |M|, c = objective numerator after the pass
 *   kind 2  level summary:       pass = 0, a = n_l, b = nnz_l, c = clusters after the local move, d = numerator
 *   kind 3  alternate local move: a = non-node-optimal vertices, b = committed prefix, c = numerator after
 *   kind 4  refinement:          a = refined clusters, b = refinement call index, c = |U|, d = tree members
 * phase 0 = coarsening, 1 = uncoarsening.  Numerators are level-local (constant offsets between levels). */
typedef struct {
  int64_t* records;  /* host array of 8 * capacity int64 */
  int64_t capacity;
  int64_t count;     /* set by the call: number of records produced (may exceed capacity) */
} lcc_trace;

/* Result-affecting options (lcc_default_options fills the paper's settings, Sec. VI-C):
 *   pass_limit 6; temperature phi = 3/4 for passes 1-4 and 1/4 for passes 5-6 (phase k covers the passes
 *   <= phi_until[k]); afterburner tie window epsilon = 1/10 on the objective change (Sec. IV-A);
 *   seed for the refinement's random choices; max_levels 64 (a guard; hitting it sets LCC_FLAG_LEVEL_CAP);
 *   validate != 0 checks the CSR on the device before clustering. */
typedef struct {
  int32_t pass_limit;
  int32_t n_phi;
  uint32_t phi_num[8], phi_den[8], phi_until[8];
  uint32_t eps_num, eps_den;
  uint64_t seed;
  int32_t max_levels;
  int32_t validate;
  lcc_trace* trace;
  int32_t symmetry;  /* LCC_SYM_*: the local move's symmetry breaking (default LCC_SYM_AFTERBURNER) */
  int32_t reserved;  /* 0 */
} lcc_options;

/* Symmetry breaking of the local move (Sec. IV-A); the other two are the ablations of Table 2:
 *   LCC_SYM_AFTERBURNER  the afterburner filter, Alg. 3
 *   LCC_SYM_NONE         no symmetry breaking: every candidate moves
 *   LCC_SYM_MLH          minimum label heuristic in odd passes (a candidate moves only to a cluster of lower id
 *                        than its current one, or to a new singleton); every candidate moves in even passes
 * The paper pairs both ablations with phi = 0 (phi_num = 0 in every phase). */
enum { LCC_SYM_AFTERBURNER = 0, LCC_SYM_NONE = 1, LCC_SYM_MLH = 2 };

enum { LCC_FLAG_LEVEL_CAP = 1, LCC_FLAG_REFINE_NO_PROGRESS = 2 };

/* Result of a clustering.  objective = lambdaCC (Eq. 1) as FP64; the exact value is obj_num / obj_den with
 * obj_num a signed 128-bit integer split into (obj_num_hi, obj_num_lo).  modularity is the Newman-Girvan
 * modularity (with the requested resolution) when vw_mode = LCC_VW_WEIGHTED_DEGREE and lambda is over the
 * total weight, NaN otherwise. */
typedef struct {
  int64_t num_clusters;
  double objective;
  double modularity;
  int64_t obj_num_hi;
  uint64_t obj_num_lo;
  uint64_t obj_den;
  int32_t levels;
  uint32_t flags;
} lcc_result;

/* Device-memory allocator used for every device buffer the library needs (stream-ordered on the call's
 * stream is not required: buffers are freed only after the stream is synchronised).  NULL functions select
 * hipMalloc / hipFree. */
typedef void* (*lcc_alloc_fn)(size_t bytes, void* user);
typedef void (*lcc_free_fn)(void* ptr, void* user);

typedef struct lcc_ctx lcc_ctx;
typedef struct lcc_server lcc_server;

/* Create a context on HIP device `device`.  The context owns its scratch workspace (grown on demand through
 * the allocator, released by lcc_destroy).  A context runs one call at a time. */
lcc_status lcc_create(int device, lcc_alloc_fn alloc, lcc_free_fn free_fn, void* user, lcc_ctx** out);
lcc_status lcc_destroy(lcc_ctx* ctx);

/* Fill *opts with the paper's settings (see lcc_options). */
void lcc_default_options(lcc_options* opts);

/* Device bytes one lcc_cluster call on a graph of n vertices and nnz entries holds at most (workspace +
 * coarse levels) when its coarsening is geometric: every coarse level of pLouvain+ is kept for the
 * uncoarsening, so a coarsening that removes few vertices per level holds more (the call then grows its
 * level pool through the allocator); Louvain, pLeiden and pLeiden+ hold at most two levels at a time.  Used
 * for admission control (the server also counts what its slots actually hold). */
lcc_status lcc_workspace_bytes(int64_t n, int64_t nnz, lcc_variant variant, size_t* bytes);

/* Cluster one graph (Alg. 1 or Alg. 5 with the setup of Sec. II).  labels_out: n int32, in the same memory
 * space as the graph, receives compact labels 0..c-1 numbered in ascending order of the cluster's
 * top-level id.  stream: hipStream_t (NULL = the default stream); the call returns after the stream has
 * completed its work.  opts NULL = lcc_default_options. */
lcc_status lcc_cluster(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                       const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res);

/* Size in bytes of the device array that lcc_cluster_noalloc works in (one per device, per process). */
#define LCC_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* lcc_cluster for callers that cannot allocate device memory (serving loops, harnesses that forbid it).
 * Arguments, results, ownership and errors are those of lcc_cluster, with these differences:
 *   - every device buffer of the call (workspace and coarse levels) is carved from a static device array of
 *     LCC_NOALLOC_SCRATCH_BYTES that each device holds from the library's load until the process ends; the
 *     call makes no device allocation (no hipMalloc, no hipFree, no use of the context's allocator) and leaves
 *     the context's own workspace as it was;
 *   - limit: the graph is accepted iff lcc_workspace_bytes(n, nnz, variant) <= LCC_NOALLOC_SCRATCH_BYTES,
 *     else LCC_ERR_INVALID is returned before any device work; LCC_ERR_OOM if the coarse levels of a run
 *     outgrow the array (nothing is written then);
 *   - all calls on one device share its array: the library serialises them (a call holds the array until
 *     its stream has completed).  The array keeps the last call's contents; each call clears what must start
 *     at zero;
 *   - the call synchronises its stream (as lcc_cluster does), so it cannot be captured into a HIP graph;
 *     kernel timing (lcc_profile_enable) does not apply to it. */
lcc_status lcc_cluster_noalloc(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                               const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res);

/* lcc_cluster with the iteration inputs of the paper (Sec. II-B, Sec. IV-D), each optional (NULL = none),
 * n int32 in the same memory space as the graph, borrowed for the call:
 *   init_labels  labels in [0, n) (LCC_ERR_INVALID otherwise).  pLeiden / pLeiden+ start from this clustering
 *                (Alg. 5's C_in: feeding a result back iterates pLeiden); Louvain / Louvain+ start the level-0
 *                local move from it instead of singletons (the iteration the Leiden authors describe)
 *   constraint   any int32 labels; Louvain / Louvain+ only and not together with init_labels
 *                (LCC_ERR_INVALID otherwise).  The coarsening local moves only join clusters of neighbours
 *                with the vertex's own constraint label, so every coarse vertex lies inside one constraint
 *                cluster; the uncoarsening local moves are free.  Feeding a Louvain+ result back as the
 *                constraint is the paper's new Louvain+ iteration. */
lcc_status lcc_cluster_ex(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                          const lcc_options* opts, void* stream, const int32_t* init_labels,
                          const int32_t* constraint, int32_t* labels_out, lcc_result* res);

/* Cluster `count` independent graphs (each with its own lambda, vertex-weight mode and variant) in one call.
 * Results are identical to `count` separate lcc_cluster calls.  labels_out[i] and res[i] as for lcc_cluster.
 * When every graph uses a variant of one family -- LCC_LOUVAIN / LCC_PLOUVAIN, or LCC_PLEIDEN / LCC_PLEIDEN_PLUS --
 * and opts->trace is NULL, the graphs are processed together (host graphs are first copied to the device): their
 * CSRs are concatenated into one union graph and every kernel launch of a level covers all graphs still
 * coarsening (Alg. 1 or Alg. 5 applied to the union, with each graph's own lambda, objective, best-so-far
 * state, alternate local move, refinement stream, no-progress retries and level count), provided the union
 * has fewer than 2^31 - 1 vertices and 2^31 - 1 entries.  Otherwise the graphs run one after another.
 * The workspace is sized for the union (sum of n, sum of nnz).  On a failure the status of the first problem
 * found is returned and no result is written; in the fused form structural faults of any graph (CSR layout,
 * symmetry, weights) are reported before lambda and bound problems, which are checked per graph in order. */
lcc_status lcc_cluster_batch(lcc_ctx* ctx, const lcc_graph* gs, const lcc_lambda* lambdas,
                             const lcc_variant* variants, int64_t count, const lcc_options* opts, void* stream,
                             int32_t* const* labels_out, lcc_result* res);

/* Exact objective (Eq. 1) of a given clustering of a host graph (g->mem = LCC_MEM_HOST), evaluated on the host
 * in 128-bit integers: labels are n int32 in [0, n) (host memory).  The graph passes the same checks as for
 * clustering (offsets, index range, self-loops, sorted rows, weights, symmetry, in that order, then the labels
 * and lambda).  Its exactness domain is wider than the clustering calls': q W_E + p W^2 < 2^126 (lambda = p / q
 * in lowest terms, W = sum of the vertex weights < 2^63, W_E = sum of the stored edge weights), else
 * LCC_ERR_OVERFLOW.  res: num_clusters = distinct labels, obj_num / obj_den = lambdaCC exactly (Sec. II,
 * Eq. 1 over ordered pairs), objective and modularity in FP64 as for lcc_cluster, levels = 1, flags = 0.
 * A device graph is refused (LCC_ERR_INVALID); use lcc_objective_device. */
lcc_status lcc_objective(const lcc_graph* g, lcc_lambda lambda, const int32_t* labels, lcc_result* res);

/* The same evaluation on the device for a graph in either memory (a host graph and its labels are copied to the
 * device first), queued on `stream` of the context's device; the clustering calls' exactness bound applies
 * (LCC_ERR_OVERFLOW as for lcc_cluster).  Returns when the result is on the host. */
lcc_status lcc_objective_device(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, const int32_t* labels,
                                void* stream, lcc_result* res);

/* Launch tuning of a context.  Every setting gives bit-identical results; only the work decomposition
 * changes.  bucket_max[k] is the largest row degree put in degree bucket k (0-3: groups of 4/8/16/32 lanes,
 * 4: a wavefront with a 256-slot LDS hash, 5 and 6: workgroups with 2048- and 8192-slot LDS hashes, 6's rows
 * above 4096 on workgroups with a 16384-slot hash; rows above bucket_max[6] go to the hub path of 2048-edge
 * chunks).  The default bounds are {4, 8, 16, 32, 128, 1024, 8192}; a bucket's kernels serve rows up to
 * {4, 8, 16, 32, 128, 1024, 8192}, so a tuning may set the bounds anywhere up to these capacities
 * (non-decreasing in k, >= 0); equal neighbouring bounds leave a bucket empty.  grid_cap (64..65536, default 2048) bounds the
 * workgroups of the persistent per-vertex launches.  hash_shift (0..2, default 0) sizes the LDS hash of a row
 * of degree d in buckets 4-6 at 2^hash_shift times the smallest power of two >= 2 d slots (a lower load
 * factor, fewer probe collisions), capped at the bucket's table.  lcc_set_tuning returns LCC_ERR_INVALID for a setting
 * outside these limits and leaves the context unchanged; the tuning applies to later calls on the context
 * (and to the execution slots of servers created afterwards). */
typedef struct {
  int64_t bucket_max[7];
  int32_t grid_cap;
  int32_t hash_shift;
} lcc_tuning;

void lcc_default_tuning(lcc_tuning* t);
lcc_status lcc_set_tuning(lcc_ctx* ctx, const lcc_tuning* t);
lcc_status lcc_get_tuning(lcc_ctx* ctx, lcc_tuning* t);

/* Autotuner: times a fixed list of candidate tunings (three grid caps with the current bounds, then bucket
 * layouts that move rows to larger-capacity buckets with the best cap, then hash_shift 0, 1 and 2 with the best
 * layout) on the given graphs, `trials` timed
 * runs each after one warm-up run (the fastest run counts), and keeps the fastest tuning on the context.
 * Each run is one lcc_cluster_batch call over the graphs (lcc_cluster when count == 1) on `stream`; graphs,
 * lambdas, variants and opts are as for lcc_cluster_batch, and labels are written to scratch the tuner owns.
 * *best receives the chosen tuning and *best_ms (may be NULL) its time per run.  On a failing run its status
 * is returned and the context keeps the tuning it had. */
lcc_status lcc_autotune(lcc_ctx* ctx, const lcc_graph* gs, const lcc_lambda* lambdas, const lcc_variant* variants,
                        int64_t count, const lcc_options* opts, void* stream, int32_t trials, lcc_tuning* best,
                        double* best_ms);

/* Continuous-batching server over one context (its device and allocator).  The server runs 4 execution
 * slots (one per hardware queue HIP gives a process by default; the environment variable LCC_SERVER_SLOTS,
 * 1-16, overrides it), each with its own context and HIP stream, so admitted jobs run concurrently on the
 * GPU.  A free slot admits the oldest queued job whose footprint (lcc_workspace_bytes) fits the unreserved
 * part of hbm_budget (a job passed over 4 times blocks further overtaking); if that job is a request of at most
 * 2^22 entries, the slot also takes the other queued such requests of its family (Louvain / Louvain+, or pLeiden
 * / pLeiden+) with the same options (up to 256 requests, 2^25 entries) and runs them as one fused
 * lcc_cluster_batch call.  Results are
 * identical to plain lcc_cluster calls.
 * Device memory: every slot allocates through ctx's allocator, and the bytes the slots hold (workspaces and
 * coarse levels, also while idle) plus the footprints reserved for running jobs never exceed hbm_budget.  An
 * idle slot keeps its workspace for the next job unless it holds more than hbm_budget / slots or a queued
 * job needs the memory.  A job whose coarse levels outgrow its footprint while other jobs hold memory is
 * refused the extra memory and rerun alone, once every other slot is idle and empty; it fails with
 * LCC_ERR_OOM only if it does not fit hbm_budget even then.
 *   lcc_server_create  hbm_budget > 0 bytes; the server keeps ctx's device and allocator (ctx must outlive it)
 *   lcc_submit         copies the graph (host or device memory) before returning and queues the job; returns
 *                      LCC_ERR_BUSY when the job's footprint alone exceeds hbm_budget; *ticket identifies it
 *   lcc_poll           *done = 0 while the job runs; once finished, *done = 1, labels_out (n int32, host
 *                      memory, may be NULL) and *res are written, the job's status is returned and the ticket
 *                      is released (LCC_ERR_NOT_FOUND afterwards)
 *   lcc_server_destroy waits for running jobs; queued jobs are dropped.  Thread-safe: submit and poll may be
 *                      called from any threads. */
lcc_status lcc_server_create(lcc_ctx* ctx, size_t hbm_budget, lcc_server** out);
lcc_status lcc_submit(lcc_server* s, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                      const lcc_options* opts, uint64_t* ticket);
lcc_status lcc_poll(lcc_server* s, uint64_t ticket, int* done, int32_t* labels_out, lcc_result* res);
lcc_status lcc_server_destroy(lcc_server* s);

/* Kernel timing (diagnostics, for measuring kernels against the memory roofline).  While a family bit is
 * set, the launches of that kernel family in lcc_cluster calls on the context are bracketed by HIP events on
 * the call's stream; their durations and algorithmic bytes (what the method must move: per edge and per
 * vertex of the launch, plus one cluster-weight read per enumerated (vertex, cluster) pair) are added to a
 * per-family tally.  Families (bit = index): 0-7 enumeration + argmax of local-move passes for degree
 * buckets 0-7, 8 the first (singleton) pass, 9 reserved.  lcc_profile_read copies up to `capacity` tallies
 * (in family order) and sets *count to the number of families; reset != 0 clears them. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;
} lcc_kernel_stat;
lcc_status lcc_profile_enable(lcc_ctx* ctx, uint64_t family_mask);
lcc_status lcc_profile_read(lcc_ctx* ctx, lcc_kernel_stat* stats, int32_t capacity, int32_t* count, int32_t reset);

const char* lcc_status_string(lcc_status st);
const char* lcc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LCC_H */
