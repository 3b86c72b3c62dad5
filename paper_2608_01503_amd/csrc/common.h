// Internal header of the MI355X LambdaCC library: device helpers, control-block layout and the host-side
// launchers each translation unit exports to the driver.  Not part of the public C-ABI (include/lcc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

namespace lcc {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int NBUCKET = 8;
constexpr int MAX_PASSES = 32;
// Per-workgroup counter partials.  Thousands of workgroups each adding a partial to one global address
// serialise on that address (about 12 ns per atomic on MI355X, so 4096 workgroups cost about 50 us); workgroup
// b adds instead into stripe b mod NSTRIPE of the counter (stripes 128 bytes apart), and one workgroup later
// adds the stripes of each counter into its destination and clears them (a fold kernel, or the prologue of
// the next single-workgroup bookkeeping kernel of the local move).
constexpr int NSTRIPE = 1024;
constexpr int STRIPE_W = 16;  // int64 slots per stripe, one per counter id
enum : int {
  CT_NCAND = 0,  // candidates of a pass
  CT_OWN = 1,    // sum of own-cluster weights
  CT_PAIRS = 2,  // CT_PAIRS + bucket: enumerated (vertex, other cluster) pairs
  CT_NM = 10,    // kept moves
  CT_SQ = 11,    // change of the sum of squared cluster weights
  CT_INT = 12,   // internal edge weight
  CT_COUNT = 13
};
constexpr int32_t D_NONE = -1;   // no destination
constexpr int32_t D_EMPTY = -2;  // destination = a new singleton cluster

// Degree buckets (upper bounds, inclusive).  Buckets 0-3 are handled by sub-wave groups of 4/8/16/32 lanes
// (one neighbour per lane), 4-5 by one wavefront per vertex, 6-7 by one workgroup per vertex.  The local-move
// kernels aggregate neighbour clusters with register shuffles (0-3), an LDS hash (4-6) or a global-memory
// hash inside the edge arena (7).  BUCKET_CAP holds the largest row each of buckets 0-6 can serve (the lane
// count of its group, half the slots of its LDS hash); a tuning may set lower bounds, never higher ones, and
// every setting gives the same results.
constexpr int64_t BUCKET_CAP[NBUCKET - 1] = {4, 8, 16, 32, 128, 1024, 8192};
// default bounds: every row up to 8192 entries is aggregated in LDS (bucket 6's rows above B6_SPLIT take the
// 16384-slot table), longer ones in the hub chunks
constexpr int64_t BUCKET_DEFAULT[NBUCKET - 1] = {4, 8, 16, 32, 128, 1024, 8192};
constexpr int LDS_SLOTS_B4 = 256;
constexpr int LDS_SLOTS_B5 = 2048;
constexpr int LDS_SLOTS_B6 = 8192;    // bucket 6 rows up to 4096 (512 threads)
constexpr int LDS_SLOTS_B6X = 16384;  // bucket 6 rows 4097-8192 (1024 threads, 128 KB of LDS)
constexpr int64_t B6_SPLIT = LDS_SLOTS_B6 / 2;  // bucket 6 rows above this take the 16384-slot table

struct BucketBounds {
  int64_t max[NBUCKET - 1];  // upper degree bound of buckets 0..6; bucket 7 takes the rest
};

__host__ __device__ inline int bucket_of(int64_t d, const BucketBounds& bb) {
  int b = 0;
  while (b < NBUCKET - 1 && d > bb.max[b]) ++b;
  return b;
}

// splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014)
__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
// MurmurHash3 32-bit finaliser (Appleby): a bijection on 32-bit words
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6BU;
  h ^= h >> 13;
  h *= 0xC2B2AE35U;
  return h ^ (h >> 16);
}
// t-th output (t = 0, 1, ...) of the splitmix64 generator seeded with `seed`
__host__ __device__ __forceinline__ uint64_t seed_stream(uint64_t seed, uint64_t t) {
  return fmix64(seed + (t + 1) * 0x9E3779B97F4A7C15ULL);
}

// Statistics of one LocalMovePasses call, written by the device.  State k = clustering after k passes.
struct LMSlot {
  int64_t nL[MAX_PASSES + 1];   // candidates of pass i
  int64_t nM[MAX_PASSES + 1];   // kept moves of pass i
  int64_t I[MAX_PASSES + 1];    // ordered internal edge weight of state k
  int64_t SW2[MAX_PASSES + 1];  // sum over clusters of W_c^2 for state k
  int32_t skip[MAX_PASSES + 2]; // pass i repeats pass i-1 exactly (no move, same temperature)
  int32_t copy;                 // current best-so-far decision: copy C -> C_out
  int32_t pad;
  int64_t n_empty;              // movers to a new singleton in the current pass
  int64_t Nbest;                // objective numerator of C_out
  int64_t N0;                   // objective numerator of the starting clustering
  int64_t nlab;                 // distinct labels of the clustering the driver ranked after the call
};

// Scalars shared by the driver and the kernels.
struct Ctrl {
  uint32_t err_bits;            // validation errors (ERR_* bits)
  uint32_t pad0;
  int64_t bucket_count[NBUCKET];
  int64_t bucket_off[NBUCKET + 1];
  int64_t bucket_cursor[NBUCKET];
  int64_t bucket6_hi;           // rows of bucket 6 longer than B6_SPLIT (placed at the end of its list)
  int64_t bucket6_cursor_hi;
  uint64_t sum_we;              // total edge weight W_E
  uint64_t sum_w;               // total vertex weight W
  uint64_t sum_w2;              // sum of w(v)^2
  int64_t count0, count1, count2, count3;  // scratch counters (clusters, entries, ...)
  int64_t obj_I;                // objective kernel: internal weight
  int64_t obj_SW2;              // objective kernel: sum of squared cluster weights
  int64_t lmalt_k, lmalt_best_k;
  int64_t refine_U, refine_m;
  int64_t lmalt_best;
  int64_t bucket_edges[NBUCKET];  // sum of degrees per bucket (level being prepared)
  int64_t enum_bytes[NBUCKET];    // algorithmic bytes of the enumeration launches, per bucket (accumulated)
  int64_t nlab;                   // distinct labels of the clustering the driver ranked last
};

enum : uint32_t {
  ERRB_INVALID = 1u << 0,
  ERRB_SELF_LOOP = 1u << 1,
  ERRB_UNSORTED = 1u << 2,
  ERRB_WEIGHT = 1u << 3,
  ERRB_NOT_SYMMETRIC = 1u << 4,
  ERRB_VW_TOO_BIG = 1u << 5,
  ERRB_INTERNAL = 1u << 6,  // an internal invariant failed (reported as LCC_ERR_DEVICE)
};

// A level graph on the device.  off int64[n+1], idx int32[nnz], w int32[nnz], vw int64[n].
struct DevGraph {
  int64_t n = 0, nnz = 0;
  const int64_t* off = nullptr;
  const int32_t* idx = nullptr;
  const int32_t* w = nullptr;
  const int64_t* vw = nullptr;
};

// Vertex lists of the degree buckets of one level (all buckets in one array, bucket b at [off[b], off[b+1])).
struct Buckets {
  const int32_t* list = nullptr;
  int32_t grid_cap = 2048;  // workgroups of the persistent per-vertex launches (a result-neutral tuning)
  int64_t hub_deg = 4096;   // rows longer than this are in the hub bucket (its lower bound, exclusive)
  int64_t count6_hi = 0;    // the last count6_hi rows of bucket 6's list are longer than B6_SPLIT
  int32_t hash_shift = 0;   // LDS hash of a row of degree d: pow2ceil(2 d) << hash_shift slots, capped (a tuning)
  int64_t count[NBUCKET] = {};
  int64_t off[NBUCKET + 1] = {};
  // hub (last bucket) vertices are processed in fixed-size edge chunks: chunk range of hub k is
  // [hub_chunk_off[k], hub_chunk_off[k+1]); per-chunk partial results and per-hub accumulators:
  int64_t edges[NBUCKET] = {};
  const int32_t* hub_chunk_off = nullptr;
  int64_t hub_chunks = 0;
  int64_t* hub_ps = nullptr;
  int32_t* hub_pc = nullptr;
  int64_t* hub_pown = nullptr;
  int64_t* hub_acc = nullptr;
  int64_t* stripes = nullptr;  // NSTRIPE * STRIPE_W counter partials, all zero between folds
};

// Scoring parameters of a level: lambda = p / q; phi = phi_a / phi_b; tie window threshold on |delta_u -
// delta_v| (see lm.hip).
struct Score {
  int64_t p, q;
  int64_t tie;
};

// Several independent graphs can be clustered together as one union level: their vertex ranges are
// concatenated (graph k owns ids [vbase[k], vbase[k+1]) at every level) and no edge joins two graphs.  Each
// graph keeps its own lambda and tie window, and every id-dependent choice (the afterburner's hash order) uses
// the graph-local id, so each graph's result equals the result of clustering it alone.
// ScoreSrc gives the kernels the scoring parameters of a vertex: `s` for every vertex of a single graph, or
// tab[gid[v]] in a union.  ownv (union only) receives each vertex's weight to its own cluster.  cons (optional)
// is a constraint clustering of the level's vertices: a vertex only considers the clusters of neighbours with
// its own constraint label (the coarsening of the constrained Louvain+ iteration).
struct ScoreSrc {
  Score s{};
  const Score* tab = nullptr;
  const int32_t* gid = nullptr;
  const int32_t* vbase = nullptr;
  int64_t* ownv = nullptr;
  const int32_t* cons = nullptr;
  __device__ __forceinline__ Score at(int32_t v) const { return tab ? tab[gid[v]] : s; }
  __device__ __forceinline__ int32_t base(int32_t v) const { return tab ? vbase[gid[v]] : 0; }
  __device__ __forceinline__ int32_t con(int32_t v) const { return cons ? cons[v] : 0; }
};

// Per-graph state of a union local move (device arrays; G graphs).
struct SegLM {
  int32_t G = 0;
  const Score* score = nullptr;     // [G]
  const int32_t* gid = nullptr;     // per vertex of the level
  const int32_t* vbase = nullptr;   // [G + 1]
  const int64_t* sumw2 = nullptr;   // [G] sum of w(v)^2 over the graph's vertices at this level
  int64_t* I = nullptr;             // [(MAX_PASSES + 1) * G] internal weight of state k of graph g
  int64_t* SW2 = nullptr;           // [(MAX_PASSES + 1) * G]
  int64_t* Nbest = nullptr;         // [G]
  int64_t* N0 = nullptr;            // [G]
  int32_t* copy = nullptr;          // [G] C_out <- C for this graph after the current best-so-far check
  int64_t* ownv = nullptr;          // per vertex scratch
};


// Block-level aggregation of (key -> int64 sum) in an LDS open-addressing table: many threads adding to the
// same cluster id (a popular destination, a giant cluster) meet in LDS, and the tile is flushed to global
// memory with one atomic per distinct key.  The caller guarantees fewer than SLOTS distinct keys per tile
// and brackets add() with __syncthreads() after clear() and before flush().
template <int SLOTS>
struct LdsAgg {
  int32_t* keys;
  unsigned long long* vals;
  __device__ __forceinline__ void clear() {
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) { keys[s] = -1; vals[s] = 0; }
  }
  // returns 1 when k took a new slot
  __device__ __forceinline__ int add(int32_t k, int64_t v) {
    uint32_t h = ((uint32_t)k * 2654435761u) & (SLOTS - 1);
    for (int probe = 0; probe < SLOTS; ++probe) {
      int32_t prev = atomicCAS(&keys[h], -1, k);
      if (prev == -1 || prev == k) { atomicAdd(&vals[h], (unsigned long long)v); return prev == -1; }
      h = (h + 1) & (SLOTS - 1);
    }
    return 0;
  }
  __device__ __forceinline__ void flush(int64_t* out) {
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
      int32_t k = keys[s];
      if (k >= 0 && vals[s]) atomicAdd((unsigned long long*)&out[k], vals[s]);
    }
  }
  // flush, returning this thread's share of the change of the sum of squares of out: each atomic returns the
  // value it added to, so the shares of all flushes add up to the exact change (sum of (old + v)^2 - old^2)
  __device__ __forceinline__ int64_t flush_sq(int64_t* out) {
    uint64_t d = 0;  // modulo 2^64: the shares of all threads add up to a value that fits
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
      int32_t k = keys[s];
      if (k >= 0 && vals[s]) {
        const int64_t v = (int64_t)vals[s];
        const int64_t old = (int64_t)atomicAdd((unsigned long long*)&out[k], vals[s]);
        d += (uint64_t)(2 * old * v + v * v);
      }
    }
    return (int64_t)d;
  }
};

// Packed per-vertex local-move state read by the afterburner: cluster, destination (D_NONE when v is not a
// candidate), delta.  16 bytes, one load per neighbour.
struct alignas(16) VState {
  int32_t c;
  int32_t d;
  int64_t delta;
};

// Optional kernel timing (diagnostics): launch sites bracket instrumented launches with prof_begin/prof_end;
// both are no-ops unless the calling thread's context has profiling enabled for that family.  bytes = the
// launch's algorithmic bytes known on the host; device-counted parts are added by the driver.
enum ProfFamily : int {
  PF_ENUM_B0 = 0,  // ..PF_ENUM_B0 + 7: enumeration + argmax of local-move passes, per degree bucket
  PF_SINGLE = 8,   // first (singleton) local-move pass, all buckets
  PF_AFTERBURNER = 9,
  PF_COUNT = 10
};
void prof_begin(int family, hipStream_t st);
void prof_end(int family, double bytes, hipStream_t st);

// ---------------------------------------------------------------------------------------------------------
// Host-side launchers (all asynchronous on `st`)
// ---------------------------------------------------------------------------------------------------------

// prim.hip
size_t scan_temp_bytes(int64_t n);
// out[i] = sum_{j<i} in[j] for i in [0, n], out[n] = total.  If `cond` is not null the kernels do nothing
// when *cond == 0.
void scan_u8_i32(const uint8_t* in, int32_t* out, int64_t n, void* temp, const int64_t* cond, hipStream_t st);
void scan_i32_i32(const int32_t* in, int32_t* out, int64_t n, void* temp, hipStream_t st);
void scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st);
void scan_i64_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st);
void scan_u32_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t st);
void scan_u32_i64(const uint32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st);
// LSD radix sort of (key, val) pairs over the 8-bit digits starting at the given bit shifts (ascending);
// stable.  Ping-pongs between (k0, v0) and (k1, v1); returns 0 if the result is in (k0, v0), 1 otherwise.
size_t radix_temp_bytes(int64_t m);
int radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t m, const int* shifts,
                     int npass, void* temp, hipStream_t st);
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void store_count(const int32_t* src, int64_t* dst, hipStream_t st);  // *dst = *src on the device
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st);
void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st);
void zero_bytes(void* p, size_t bytes, hipStream_t st);  // a fill kernel, safe inside captured graphs
void iota_i32(int32_t* p, int64_t n, hipStream_t st);
void copy_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t st);
void offsets32_to_64(const int32_t* in, int64_t* out, int64_t n1, hipStream_t st);

// lm.hip: setup, buckets, local move, objective
void launch_validate_offsets(const int64_t* off, int64_t n, int64_t nnz, Ctrl* ctrl, hipStream_t st);
// Union levels: vw_mode per graph (gmode[gid[v]]) when gmode is not null; rowsum (if not null) receives
// every vertex's weighted degree.
// The exact symmetry check: by search (search = true; the balance lands in ctrl->count0 and must be 0), or by
// transposition (k0 set: nnz (key, value) pairs twice for the sort's ping-pong and radix_temp_bytes(nnz) of
// temp), or none.
struct SymBuffers {
  bool search = false;
  uint64_t* k0 = nullptr;  // transposition (k0 set): nnz / 2 pairs in each of (k0, v0) and (k1, v1)
  uint32_t* v0 = nullptr;
  uint64_t* k1 = nullptr;
  uint32_t* v1 = nullptr;
  void* temp = nullptr;       // the sort's scratch
  int32_t* lo = nullptr;      // n: entries of each row towards lower ids
  int64_t* lbase = nullptr;   // n + 1: their exclusive scan
  void* scan_temp = nullptr;
};
// Graphs (of a union: its largest graph) up to this many entries are checked by search: the rows a search
// visits stay in cache.  So are graphs of at most SYM_SEARCH_MAX_AVG_DEG entries per row (half an entry per
// row searches, one short row each, against four sort passes over every entry).  Others by transposition.
constexpr int64_t SYM_SEARCH_MAX_NNZ = (int64_t)1 << 23;
constexpr int64_t SYM_SEARCH_MAX_AVG_DEG = 8;
void launch_validate_rows(const DevGraph& g, const Buckets& b, int vw_mode, const int64_t* vw_given,
                          int64_t* vw_out, Ctrl* ctrl, hipStream_t st, const SymBuffers& sb,
                          const int32_t* gid = nullptr, const int8_t* gmode = nullptr, int64_t* rowsum = nullptr);
// Degree buckets of the vertices of a level; with gid/gact only the vertices whose graph has gact set.
void launch_buckets(const int64_t* off, int64_t n, int32_t* list, Ctrl* ctrl, const BucketBounds& bb, hipStream_t st,
                    const int32_t* gid = nullptr, const uint8_t* gact = nullptr);
// out[k] = sum of x[i] (or x[i]^2) over i in [vbase[k], vbase[k+1]), k < G
void launch_seg_sum(const int64_t* x, int square, const int32_t* vbase, int64_t G, int64_t* out, hipStream_t st);
// per-vertex internal weight (sum of w(u,v) over neighbours in v's cluster) into out[v]
void launch_internal_per_vertex(const DevGraph& g, const Buckets& b, const int32_t* C, int64_t* out,
                                hipStream_t st);
// chunk offsets of the hubs (n7 entries of the last bucket): chunk_off[n7+1] via cnt[n7] scratch
void launch_hub_chunks(const int32_t* hubs, int64_t n7, const int64_t* off, int32_t* cnt, int32_t* chunk_off,
                       void* temp, hipStream_t st);
constexpr int64_t HUB_CHUNK_EDGES = 2048;
void launch_vertex_sums(const int64_t* vw, int64_t n, Ctrl* ctrl, hipStream_t st);

// Device arrays whose entries carry a 32-bit tag instead of being cleared before each use: the free-id marks
// of the local move and the status words of single-pass scans.  `last` (host) is the last tag handed out;
// all arrays start at zero (no tag) and are cleared again when the tags run out.
struct Tagged {
  uint32_t last = 0;
  uint32_t* held = nullptr;              // per cluster id: the tag of the last pass that saw it held
  int64_t held_cap = 0;
  unsigned long long* status = nullptr;  // per scan tile: tag << 32 | inclusive << 31 | value
  int64_t status_cap = 0;
  uint32_t* ticket = nullptr;            // tile counter of single-pass scans, 0 between launches
};
uint32_t next_tag(Tagged& t, hipStream_t st);
// k consecutive tags in out[0..k); when fewer than k remain, the tagged words are cleared first (on st)
void next_tags(Tagged& t, int k, uint32_t* out, hipStream_t st);

// Single-pass exclusive scan by decoupled look-back.  Tiles of LB_TILE items are drawn from a ticket counter
// in launch order, so a tile waits only for tiles that a running workgroup already holds.  A tile publishes
// its own total first, then walks back over its predecessors' words (64 per step, one per lane) until it
// meets an inclusive prefix, and publishes its own inclusive prefix.  Values are below 2^31.
constexpr int LB_ITEMS = 8;
constexpr int LB_TILE = BLOCK * LB_ITEMS;  // 2048

__device__ __forceinline__ unsigned long long lb_word(uint32_t tag, bool inclusive, uint32_t v) {
  return ((unsigned long long)tag << 32) | ((unsigned long long)inclusive << 31) | (unsigned long long)v;
}

// Next tile of this workgroup.  Each workgroup stops at its first ticket past the last tile, so a launch
// draws tiles + gridDim.x tickets; the workgroup that draws the last one returns the counter to 0.
__device__ __forceinline__ uint32_t lb_next(uint32_t* ticket, uint32_t draws, uint32_t* sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(ticket, 1u);
    if (t == draws - 1) atomicExch(ticket, 0u);
    *sh = t;
  }
  __syncthreads();
  return *sh;
}

// Exclusive scan of one value per thread over the block (BLOCK threads); *total = block sum.
__device__ __forceinline__ uint32_t lb_block_excl(uint32_t x, uint32_t* total, uint32_t* wsum) {
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += y;
  }
  if (lane == WAVE - 1) wsum[wv] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < BLOCK / WAVE; ++k) {
    const uint32_t s = wsum[k];
    if (k < wv) before += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

// Exclusive prefix of tile t whose own total is agg (called by every thread of the block).
__device__ __forceinline__ uint32_t lb_prefix(unsigned long long* status, uint32_t t, uint32_t tag, uint32_t agg,
                                              uint32_t* sh) {
  if (threadIdx.x < WAVE) {
    const int lane = threadIdx.x;
    uint32_t excl = 0;
    if (lane == 0)
      __hip_atomic_store(&status[t], lb_word(tag, t == 0, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t > 0) {
      int64_t j = (int64_t)t - 1 - lane;  // lane k reads tile t-1-k
      for (;;) {
        unsigned long long s = lb_word(tag, true, 0);  // before tile 0: an inclusive prefix of 0
        if (j >= 0) {
          do {
            s = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } while ((uint32_t)(s >> 32) != tag);
        }
        const unsigned long long pm = __ballot((s >> 31) & 1ull);
        uint32_t val = (uint32_t)s & 0x7FFFFFFFu;
        if (pm && lane > __ffsll((long long)pm) - 1) val = 0;  // beyond the nearest inclusive prefix
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) val += __shfl_xor(val, o, WAVE);
        excl += val;
        if (pm) break;
        j -= WAVE;
      }
      if (lane == 0)
        __hip_atomic_store(&status[t], lb_word(tag, true, excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) *sh = excl;
  }
  __syncthreads();
  return *sh;
}

struct LMBuffers {
  int32_t* C;      // current clustering (labels in [0, n))
  int32_t* Cout;   // best-so-far clustering
  int64_t* W;      // cluster weights, indexed by cluster id
  VState* vs;      // packed (C, D, delta)
  uint8_t* keep;   // afterburner verdict
  uint8_t* empty;  // kept movers to a new singleton
  int32_t* scan_a; // n+1
  int32_t* scan_b; // n+1
  int32_t* freelist;
  uint32_t* arena; // 2 * nnz (key, value) slots for the global-memory hash
  void* scan_temp;
  int64_t* enum_bytes;  // per-bucket algorithmic bytes of the enumeration launches (diagnostics), or null
  Tagged* tg;      // free-id marks and single-pass scan state
};

struct LMParams {
  Score sc;
  SegLM seg;       // union of several graphs when seg.G > 0 (sc unused then)
  const int32_t* cons = nullptr;  // constraint clustering of the level's vertices (or null)
  int symmetry = 0;                // 0 afterburner (Alg. 3), 1 none, 2 minimum label heuristic in odd passes
  int pass_limit;
  uint32_t phi_num[MAX_PASSES + 1], phi_den[MAX_PASSES + 1];  // per pass (1-based)
  int64_t sum_w2;  // sum of w(v)^2 of the level
};

// Runs LocalMovePasses (Alg. 2) on level graph g from the clustering in bufs.C (`singleton` = C is the
// identity).  Leaves C_out in bufs.Cout.  Statistics in *slot.
void local_move(const DevGraph& g, const Buckets& b, const LMParams& prm, bool singleton, LMBuffers& bufs,
                LMSlot* slot, Ctrl* ctrl, hipStream_t st);
// Destinations without the temperature rule (candidate iff the move strictly improves): used by
// LocalMoveAlt.  Fills bufs.vs and bufs.keep (keep = non-node-optimal).
void launch_destinations_strict(const DevGraph& g, const Buckets& b, const ScoreSrc& ss, LMBuffers& bufs,
                                LMSlot* slot, hipStream_t st);
void launch_cluster_weights(const int32_t* C, const int64_t* vw, int64_t n, int64_t* W, hipStream_t st);
// Exact objective pieces of clustering C: ctrl->obj_I and ctrl->obj_SW2 (W must hold C's cluster weights).
void launch_objective(const DevGraph& g, const Buckets& b, const int32_t* C, const int64_t* W,
                      Ctrl* ctrl, hipStream_t st);
// sg: a union of graphs (free ids per graph), or empty
void launch_apply_and_empty(const DevGraph& g, const Buckets& b, LMBuffers& bufs, const SegLM& sg, LMSlot* slot,
                            hipStream_t st);

// contract.hip
// used flags of labels -> rank (compact map) : rank[c] for c in [0, n), count at rank[n].
// With gid/gact (a union of graphs) only the labels of the graphs with gact set count; map is -1 elsewhere.
void launch_label_rank(const int32_t* labels, int64_t n, uint8_t* used, int32_t* rank, void* temp,
                       hipStream_t st, const int32_t* gid = nullptr, const uint8_t* gact = nullptr);
void launch_map_labels(const int32_t* labels, const int32_t* rank, int64_t n, int32_t* map, hipStream_t st,
                       const int32_t* gid = nullptr, const uint8_t* gact = nullptr);
// union: graph of every coarse vertex (cgid[map[v]] = gid[v]); every graph's first id after a compaction by
// rank (vbase_c[k] = rank[vbase[k]], k <= G)
void launch_coarse_gid(const int32_t* map, const int32_t* gid, int64_t n, int32_t* cgid, hipStream_t st);
void launch_rebase(const int32_t* rank, const int32_t* vbase, int64_t G, int32_t* vbase_c, hipStream_t st);
void launch_coarse_vw(const int32_t* map, const int64_t* vw, int64_t n, int64_t* cvw, hipStream_t st);
void launch_cross_count(const DevGraph& g, const Buckets& b, const int32_t* map, int32_t* cnt,
                        hipStream_t st);
void launch_cross_emit(const DevGraph& g, const Buckets& b, const int32_t* map, int64_t* cursor,
                       uint64_t* keys, uint32_t* vals, hipStream_t st);
void launch_heads(const uint64_t* keys, int64_t m, uint8_t* head, hipStream_t st);
// coarse CSR from sorted (x << 32 | y) keys: uid = exclusive scan of run heads; pref = exclusive scan of the
// values (m + 1); hstart/ux scratch of nnz_c + 1 entries.
void launch_coarse_write(const uint64_t* keys, const uint32_t* vals, const uint8_t* head, const int32_t* uid,
                         int64_t m, int64_t nnzc, int64_t nc, int64_t* pref, int32_t* hstart, int32_t* ux,
                         int32_t* cidx, int32_t* cw, int64_t* coff, void* temp, hipStream_t st);
// fine_C[v] = coarse_C[map[v]] where map[v] >= 0; in a union (gid set) rebased from graph gid[v]'s coarse id
// range (vbase_c) to its fine id range (vbase_f)
void launch_project(const int32_t* coarse_C, const int32_t* map, int64_t n, int32_t* fine_C, hipStream_t st,
                    const int32_t* gid = nullptr, const int32_t* vbase_f = nullptr,
                    const int32_t* vbase_c = nullptr);
// Cc[map[v]] = rankB[B[v]] where map[v] >= 0.  In a union (gid set): the graph-local rank, rebased from graph
// gid[v]'s fine id range (vbase_f) to its coarse one (vbase_c); for a graph with keep[k] set (its coarse level
// repeats the fine one) B[v] itself, rebased.
void launch_downsample(const int32_t* B, const int32_t* rankB, const int32_t* map, int64_t n, int32_t* Cc,
                       hipStream_t st, const int32_t* gid = nullptr, const int32_t* vbase_f = nullptr,
                       const int32_t* vbase_c = nullptr, const uint8_t* keep = nullptr);

// refine.hip: pLeidenR (Alg. 6)
struct RefineBuffers {
  int64_t* WB; int64_t* aB; int64_t* aX; uint8_t* inU; int32_t* H; int32_t* par; int32_t* root;
  uint8_t* flip; uint8_t* has_child; int32_t* tsz; uint8_t* member;
  int32_t* tree_sz;  // n + 1: per root, its tree's size when it has 2 or more members
  uint64_t* k0; uint32_t* v0; uint64_t* k1; uint32_t* v1;
  int64_t* pw; int64_t* pc; int64_t* tmp64a; int64_t* tmp64b; int32_t* pos_of; int32_t* fail;
  void* scan_temp;
};
// Throws the library's device error (LCC_ERR_DEVICE with the HIP message) when e is not hipSuccess.
void device_check(hipError_t e, const char* what);

// segsort.hip: grouped placement and segmented sorting.
// out[grp[i]] += cnt[i] over items with grp[i] >= 0.
void launch_group_sum(const int32_t* grp, const int32_t* cnt, int64_t n, int64_t* out, hipStream_t st);
// pos[i] = the start of cnt[i] (1 when cnt is null) positions of item i inside segment grp[i], for items with
// grp[i] >= 0 (and mask[i] set when mask is given); segment s starts at start[s]; cursor: nseg scratch.
void launch_group_place(const int32_t* grp, const int32_t* cnt, const uint8_t* mask, int64_t n, const int64_t* start,
                        int64_t nseg, unsigned long long* cursor, int64_t* pos, hipStream_t st);
// (kout, vout) = (kin, vin) with the m items of every segment [off[s], off[s+1]) sorted by key.  Every key of
// segment s is below every key of segment s + 1, and keys inside a segment differ only in their low
// `low_bits` bits, so the whole output is sorted.  (kin, vin) are clobbered (the second buffer of the long
// segments' passes); m < 2^32.  take() hands out stream-ordered scratch.
void segsort_pairs(uint64_t* kin, uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t m, const int64_t* off,
                   int64_t nseg, int low_bits, void* scan_temp, const std::function<void*(size_t)>& take,
                   hipStream_t st);

// What the refinement of a vertex depends on besides the graph: the scoring parameters, the random stream s_t
// of the refinement call and the vertex id that enters the hashes.  For one graph these are `s`, `st` and v;
// in a union of graphs (gid set) they are those of the vertex's own graph, with graph-local ids, so every graph
// is refined exactly as alone, and graphs with act[k] == 0 are left unrefined (none of their vertices is in U).
struct RefSrc {
  Score s{};
  uint64_t st = 0;
  const int32_t* gid = nullptr;
  const int32_t* vbase = nullptr;
  const Score* tab = nullptr;     // [G]
  const uint64_t* stt = nullptr;  // [G]
  const uint8_t* act = nullptr;   // [G]
  __device__ __forceinline__ Score sc(int32_t v) const { return gid ? tab[gid[v]] : s; }
  __device__ __forceinline__ uint64_t seed(int32_t v) const { return gid ? stt[gid[v]] : st; }
  __device__ __forceinline__ uint32_t fseed(int32_t v) const { return (uint32_t)(seed(v) >> 32); }
  __device__ __forceinline__ uint32_t loc(int32_t v) const {
    return gid ? (uint32_t)(v - vbase[gid[v]]) : (uint32_t)v;
  }
  __device__ __forceinline__ bool on(int32_t v) const { return !act || act[gid[v]]; }
};

void refine(const DevGraph& g, const Buckets& b, const RefSrc& rs, const int32_t* B, int32_t* R, RefineBuffers& rb,
            Ctrl* ctrl, const std::function<void*(size_t)>& take, hipStream_t st);

// lmalt.hip: LocalMoveAlt (Sec. V-A)
// A union of graphs: only the graphs with act[k] set take the move, each with its own scoring parameters, its
// own committed prefix (best_k[k], device) and its own free ids (sg).
struct AltSeg {
  ScoreSrc ss;
  const uint8_t* act = nullptr;  // [G]
  int64_t* best_k = nullptr;     // [G]
  SegLM sg;
};
// Returns false (nothing done) when the mover count is 2^30 or more.  seg: a union of graphs (null: one graph).
bool lmalt(const DevGraph& g, const Buckets& b, const Score& sc, LMBuffers& bufs, LMSlot* slot, Ctrl* ctrl,
           int32_t* list, int64_t* gain, const std::function<void*(size_t)>& take, hipStream_t st,
           const AltSeg* seg = nullptr);

}  // namespace lcc
