// Host driver and C-ABI of the MI355X LambdaCC library (include/lcc.h).
//
// A context owns a workspace carved once per graph size (per-vertex state, degree buckets, the edge arena
// shared by the hub hash tables, the contraction sort and the refinement sort) and a pool from which the
// coarse level graphs are bump-allocated (reset at the end of every call, kept for the next).  All work of a
// call is queued on the caller's stream; the host synchronises only where a size decides the next launch
// (bucket counts, cluster counts, coarse entry counts) -- a handful of times per level.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lcc.h"
#include "common.h"

using namespace lcc;

namespace {

thread_local std::string g_last_error;

struct Fail {
  lcc_status st;
};

[[noreturn]] void fail(lcc_status st, const std::string& msg) {
  g_last_error = msg;
  throw Fail{st};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(LCC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
constexpr int NSLOT = 4 * 1024 + 16;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    size_t bytes = align_up((size_t)std::max<int64_t>(count, 1) * sizeof(T));
    T* p = base ? (T*)(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

// Workspace buffers of one context, sized for a level-0 graph of n vertices and nnz entries.
struct WS {
  Ctrl* ctrl;
  LMSlot* slots;
  int64_t* in_off; int32_t* in_idx; int32_t* in_w; int64_t* in_vwg; int32_t* in_labels;
  int64_t* vw0;
  int32_t *C, *Cout, *scan_a, *scan_b, *freelist;
  int64_t* W;
  VState* vs;
  uint8_t *keep, *empty, *used;
  int32_t *rank, *cnt, *list0, *hub_cnt, *hub_off0;
  int64_t* pos;
  int64_t* hub_ps; int32_t* hub_pc; int64_t* hub_pown; int64_t* hub_acc;
  uint64_t *k0, *k1; uint32_t *v0, *v1;
  uint8_t* head; int32_t* uid; int32_t* ux;
  int64_t *WB, *aB, *aX, *pw, *pc, *t64a, *t64b, *alt_gain;
  uint8_t *inU, *flip, *has_child, *member;
  int32_t *H, *par, *root, *tsz, *pos_of, *fail, *tree_sz, *alt_list;
  int32_t* gid0;  // union of graphs: graph of every level-0 vertex
  int64_t *seg0, *seg1;  // contraction: entries per coarse row (then the rows' cursors) and the rows' starts
  Tagged tg;      // free-id marks and single-pass scan state (zeroed when the workspace is allocated)
  int64_t* stripes;  // per-workgroup counter partials (zeroed when the workspace is allocated)
  void* scan_temp;
};

size_t carve(WS& w, char* base, int64_t n, int64_t nnz) {
  Carver c{base};
  const int64_t M = std::max(n, nnz);
  const int64_t nch = nnz / HUB_CHUNK_EDGES + n + 1;
  w.ctrl = c.take<Ctrl>(1);
  w.slots = c.take<LMSlot>(NSLOT);
  w.in_off = c.take<int64_t>(n + 1);
  w.in_idx = c.take<int32_t>(nnz);
  w.in_w = c.take<int32_t>(nnz);
  w.in_vwg = c.take<int64_t>(n);
  w.in_labels = c.take<int32_t>(n);
  w.vw0 = c.take<int64_t>(n);
  w.C = c.take<int32_t>(n); w.Cout = c.take<int32_t>(n);
  w.scan_a = c.take<int32_t>(n + 1); w.scan_b = c.take<int32_t>(n + 1); w.freelist = c.take<int32_t>(n);
  w.W = c.take<int64_t>(n);
  w.vs = c.take<VState>(n);
  w.keep = c.take<uint8_t>(n); w.empty = c.take<uint8_t>(n); w.used = c.take<uint8_t>(n);
  w.rank = c.take<int32_t>(n + 1); w.cnt = c.take<int32_t>(n); w.list0 = c.take<int32_t>(n);
  w.hub_cnt = c.take<int32_t>(n); w.hub_off0 = c.take<int32_t>(n + 1);
  w.pos = c.take<int64_t>(n + 1);
  w.hub_ps = c.take<int64_t>(nch); w.hub_pc = c.take<int32_t>(nch); w.hub_pown = c.take<int64_t>(nch);
  w.hub_acc = c.take<int64_t>(n);
  // k0 and k1 are adjacent: together they also hold the hub hash tables (2 nnz slots of 8 bytes)
  w.k0 = c.take<uint64_t>(M + 1); w.k1 = c.take<uint64_t>(M + 1);
  w.v0 = c.take<uint32_t>(M + 1); w.v1 = c.take<uint32_t>(M + 1);
  w.head = c.take<uint8_t>(M); w.uid = c.take<int32_t>(M + 1); w.ux = c.take<int32_t>(M + 1);
  w.WB = c.take<int64_t>(n); w.aB = c.take<int64_t>(n); w.aX = c.take<int64_t>(n);
  w.pw = c.take<int64_t>(n + 1); w.pc = c.take<int64_t>(n + 1);
  w.t64a = c.take<int64_t>(n); w.t64b = c.take<int64_t>(n); w.alt_gain = c.take<int64_t>(n);
  w.inU = c.take<uint8_t>(n); w.flip = c.take<uint8_t>(n); w.has_child = c.take<uint8_t>(n);
  w.member = c.take<uint8_t>(n);
  w.H = c.take<int32_t>(n); w.par = c.take<int32_t>(n); w.root = c.take<int32_t>(n); w.tsz = c.take<int32_t>(n);
  w.pos_of = c.take<int32_t>(n); w.fail = c.take<int32_t>(n); w.tree_sz = c.take<int32_t>(n + 1);
  w.alt_list = c.take<int32_t>(n);
  w.gid0 = c.take<int32_t>(n);
  w.seg0 = c.take<int64_t>(n + 1); w.seg1 = c.take<int64_t>(n + 1);
  w.tg = Tagged{};
  w.tg.held = c.take<uint32_t>(n); w.tg.held_cap = n;
  w.tg.status_cap = (M + 1) / LB_TILE + 2;
  w.tg.status = c.take<unsigned long long>(w.tg.status_cap);
  w.tg.ticket = c.take<uint32_t>(1);
  w.stripes = c.take<int64_t>((int64_t)NSTRIPE * STRIPE_W);
  w.scan_temp = c.take<char>((int64_t)scan_temp_bytes(M + 1));
  return c.off;
}

// Level graphs: bump allocation from chunks of the caller's allocator, reset per call.
struct Pool {
  struct Chunk { char* p; size_t cap; };
  std::vector<Chunk> chunks;
  size_t cur = 0, off = 0;
};

// Footprint of the coarse levels (a generous geometric bound; the pool grows if a graph needs more).
size_t level_bytes(int64_t n, int64_t nnz) {
  return align_up((size_t)(n + 1) * 8) + align_up((size_t)nnz * 8) + align_up((size_t)n * 8) +
         4 * align_up((size_t)n * 4) + align_up((size_t)(n + 2) * 4);
}

// Scratch of lcc_cluster_noalloc: a fixed device array that holds that entry point's workspace and level pool,
// for callers that cannot allocate device memory.  Every device the library runs on holds its own copy until
// the process ends.  Host code never uses the array's name as an address (it is a host-side stand-in): the
// device address comes from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t NOALLOC_BYTES = (size_t)LCC_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[NOALLOC_BYTES];

struct ScratchDev {
  std::mutex setup_mu;     // guards ptr / err / done
  std::mutex call_mu;      // one no-allocation call at a time on the device: they share its array
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
  bool done = false;
};
constexpr int MAX_DEVICES = 64;
ScratchDev g_scratch[MAX_DEVICES];

// Device address of `scratch` on `device` (which must be current); taken at the first request per device.
void* scratch_address(int device, hipError_t* err) {
  ScratchDev& s = g_scratch[device];
  std::lock_guard<std::mutex> lk(s.setup_mu);
  if (!s.done) {
    void* p = nullptr;
    s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.ptr = s.err == hipSuccess ? p : nullptr;
    s.done = true;
  }
  *err = s.err;
  return s.ptr;
}

// No-allocation mode of a context: the workspace and the level pool are bump-allocated from the device's
// scratch array instead of the context's allocator.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  size_t ws_end = 0;
};

}  // namespace

static lcc_tuning initial_tuning() {
  lcc_tuning t{};
  for (int k = 0; k < NBUCKET - 1; ++k) t.bucket_max[k] = BUCKET_DEFAULT[k];
  t.grid_cap = 2048;
  return t;
}

struct lcc_ctx {
  int device = 0;
  lcc_tuning tune = initial_tuning();  // result-neutral launch tuning
  BucketBounds bounds() const {
    BucketBounds b;
    for (int k = 0; k < NBUCKET - 1; ++k) b.max[k] = tune.bucket_max[k];
    return b;
  }
  lcc_alloc_fn alloc = nullptr;
  lcc_free_fn freef = nullptr;
  void* user = nullptr;
  char* ws_base = nullptr;
  size_t ws_bytes = 0;
  int64_t ws_n = -1, ws_nnz = -1;
  WS w{};
  Pool pool;
  Arena* arena = nullptr;       // set for the duration of a no-allocation call
  Ctrl* h_ctrl = nullptr;       // pinned mirror
  LMSlot* h_slots = nullptr;    // pinned mirror
  std::mutex mu;
  // kernel timing (diagnostics)
  uint64_t prof_mask = 0;
  struct ProfRec { int fam; hipEvent_t a, b; double bytes; };
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> prof_recs;
  hipEvent_t prof_open[PF_COUNT] = {};
  int64_t prof_launches[PF_COUNT] = {};
  double prof_ms[PF_COUNT] = {};
  double prof_bytes[PF_COUNT] = {};
  hipEvent_t event() {
    if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (alloc) p = alloc(bytes, user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) fail(LCC_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (freef) freef(p, user);
    else (void)hipFree(p);
  }
  // The context's own work is drained when a call returns (every call ends with a stream synchronisation), so
  // growing the workspace waits for nothing but the new workspace's initialisation on the call's stream: no
  // device-wide synchronisation that would also wait for other contexts' streams.
  void ensure_ws(int64_t n, int64_t nnz, hipStream_t st) {
    if (arena) {  // carved from the scratch array for exactly this graph (the caller checked the size)
      WS tmp{};
      const size_t need = carve(tmp, nullptr, n, nnz);
      if (need > arena->cap) fail(LCC_ERR_INVALID, "graph exceeds the no-allocation scratch");
      w = WS{};
      carve(w, arena->base, n, nnz);
      ws_base = arena->base;
      ws_bytes = need;
      ws_n = n;
      ws_nnz = nnz;
      arena->ws_end = arena->off = align_up(need);
      return;
    }
    if (n <= ws_n && nnz <= ws_nnz) return;
    int64_t nn = std::max(n, ws_n), ne = std::max(nnz, ws_nnz);
    WS tmp{};
    size_t need = carve(tmp, nullptr, nn, ne);
    if (ws_base) { dfree(ws_base); ws_base = nullptr; }
    // until the new workspace is in place the context has none: a failed allocation must not leave the sizes
    // of the freed one behind for the next call
    ws_n = ws_nnz = -1;
    ws_bytes = 0;
    w = WS{};
    ws_base = (char*)dalloc(need);
    ws_bytes = need;
    carve(w, ws_base, nn, ne);
    hip_check(hipMemsetAsync(w.tg.held, 0, (size_t)w.tg.held_cap * sizeof(uint32_t), st), "workspace");
    hip_check(hipMemsetAsync(w.tg.status, 0, (size_t)w.tg.status_cap * sizeof(unsigned long long), st), "workspace");
    hip_check(hipMemsetAsync(w.tg.ticket, 0, sizeof(uint32_t), st), "workspace");
    hip_check(hipMemsetAsync(w.stripes, 0, (size_t)NSTRIPE * STRIPE_W * sizeof(int64_t), st), "workspace");
    hip_check(hipStreamSynchronize(st), "workspace");
    // tags are result-neutral; LCC_TAG_BASE starts their sequence elsewhere (tests use it to reach the
    // wrap-around, which otherwise takes billions of passes)
    if (const char* tb = getenv("LCC_TAG_BASE")) w.tg.last = (uint32_t)strtoul(tb, nullptr, 10);
    ws_n = nn;
    ws_nnz = ne;
  }
  void* pool_take(size_t bytes) {
    bytes = align_up(bytes);
    if (arena) {
      if (bytes > arena->cap - arena->off)
        fail(LCC_ERR_OOM, "no-allocation scratch of " + std::to_string(arena->cap) + " bytes exhausted by the coarse levels");
      void* p = arena->base + arena->off;
      arena->off += bytes;
      return p;
    }
    while (pool.cur < pool.chunks.size()) {
      auto& c = pool.chunks[pool.cur];
      if (pool.off + bytes <= c.cap) {
        void* p = c.p + pool.off;
        pool.off += bytes;
        return p;
      }
      ++pool.cur;
      pool.off = 0;
    }
    // chunks of one input-sized level: two hold the coarse levels of a geometric coarsening, the bound that
    // lcc_workspace_bytes reports
    size_t cap = std::max(bytes, level_bytes(ws_n, ws_nnz));
    pool.chunks.push_back({(char*)dalloc(cap), cap});
    pool.cur = pool.chunks.size() - 1;
    pool.off = bytes;
    return pool.chunks.back().p;
  }
  void pool_reset() {
    if (arena) { arena->off = arena->ws_end; return; }
    pool.cur = 0;
    pool.off = 0;
  }
  // scratch taken after a mark is handed out again after the release (the stream must be done with it)
  std::pair<size_t, size_t> pool_mark() const {
    if (arena) return {0, arena->off};
    return {pool.cur, pool.off};
  }
  void pool_release(std::pair<size_t, size_t> m) {
    if (arena) { arena->off = m.second; return; }
    pool.cur = m.first;
    pool.off = m.second;
  }
};

thread_local lcc_ctx* g_prof_ctx = nullptr;  // context whose call runs on this thread, when profiling

namespace lcc {
void prof_begin(int family, hipStream_t st) {
  lcc_ctx* c = g_prof_ctx;
  if (!c || !((c->prof_mask >> family) & 1)) return;
  hipEvent_t e = c->event();
  if (!e) return;
  (void)hipEventRecord(e, st);
  c->prof_open[family] = e;
}
void prof_end(int family, double bytes, hipStream_t st) {
  lcc_ctx* c = g_prof_ctx;
  if (!c || !((c->prof_mask >> family) & 1) || !c->prof_open[family]) return;
  hipEvent_t e = c->event();
  if (!e) return;
  (void)hipEventRecord(e, st);
  c->prof_recs.push_back({family, c->prof_open[family], e, bytes});
  c->prof_open[family] = nullptr;
}
void device_check(hipError_t e, const char* what) { hip_check(e, what); }
}  // namespace lcc

namespace {

const char* const PROF_NAMES[PF_COUNT] = {"enum_b0", "enum_b1", "enum_b2", "enum_b3", "enum_b4", "enum_b5",
                                          "enum_b6", "enum_b7", "single", "afterburner"};

// After the call's stream has completed: fold the recorded launches into the context's tallies.
void prof_resolve(lcc_ctx* c, const Ctrl* h) {
  for (auto& r : c->prof_recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_launches[r.fam] += 1;
      c->prof_ms[r.fam] += ms;
      c->prof_bytes[r.fam] += r.bytes;
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_recs.clear();
  // the enumeration launches count their algorithmic bytes on the device; buckets 0-2 share one launch
  // (family 0)
  for (int k = 0; k < NBUCKET; ++k) {
    const int f = PF_ENUM_B0 + (k < 3 ? 0 : k);
    if ((c->prof_mask >> f) & 1) c->prof_bytes[f] += (double)h->enum_bytes[k];
  }
}

template <typename T>
T* take(lcc_ctx* ctx, int64_t count) {
  return (T*)ctx->pool_take((size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

struct Level {
  DevGraph g;
  Buckets b;
  int32_t* map = nullptr;  // fine vertex -> coarse vertex of the next level
  int32_t* C = nullptr;    // clustering of this level
  int64_t sum_w2 = 0;
  // union of graphs: graph of every vertex, first vertex of every graph (device and host), per-graph sum w^2
  int32_t* gid = nullptr;
  int32_t* vbase = nullptr;
  std::vector<int32_t> hvb;
  int64_t* sumw2g = nullptr;
  // constraint clustering of the level's vertices (constrained Louvain+ coarsening), or null
  int32_t* B = nullptr;
};

__global__ void k_reset_level_counters(Ctrl* c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int b = 0; b < NBUCKET; ++b) { c->bucket_count[b] = 0; c->bucket_cursor[b] = 0; c->bucket_edges[b] = 0; }
  c->count3 = 0;
  c->bucket6_hi = 0;
  c->sum_w = 0;
  c->sum_w2 = 0;
}

__global__ void k_ones(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 1;
}

__global__ void k_labels_in_range(const int32_t* lab, int64_t n, Ctrl* c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (lab[i] < 0 || lab[i] >= n) atomicOr(&c->err_bits, ERRB_INVALID);
}

unsigned grid1(int64_t n) {
  int64_t g = (n + BLOCK - 1) / BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

struct Run {
  lcc_ctx* ctx;
  hipStream_t st;
  WS& w;
  lcc_options o;
  Score sc{};
  int64_t p = 0, q = 1;
  std::vector<Level> lv;
  std::vector<int64_t> trace;   // 8 int64 per record
  int nslot = 0;
  uint32_t flags = 0;
  uint64_t W = 0;
  uint64_t refine_calls = 0;
  // union of G graphs (G > 0): per-graph scoring parameters and local-move statistics on the device
  int64_t G = 0;
  Score* d_score = nullptr;
  int64_t *gI = nullptr, *gSW2 = nullptr, *gNbest = nullptr, *gN0 = nullptr;
  int32_t* gcopy = nullptr;
  uint8_t* gact = nullptr;
  int32_t* gtmp = nullptr;
  // Variants without an uncoarsening local move (Louvain, pLeiden) need a coarse level's graph only until the
  // next level is built: the coarse graphs then alternate between two buffers sized for the input, so the
  // memory does not grow with the number of levels.  The maps and clusterings of every level stay.
  bool pingpong = false;
  char* ppbuf[2] = {nullptr, nullptr};
  size_t ppcap = 0, ppoff = 0;
  int ppcur = 0;

  Run(lcc_ctx* c, hipStream_t s) : ctx(c), st(s), w(c->w) {}

  void use_pingpong(int64_t n, int64_t nnz) {
    pingpong = true;
    ppcap = align_up((size_t)(n + 1) * 8) + align_up((size_t)std::max<int64_t>(n, 1) * 8) +
            2 * align_up((size_t)std::max<int64_t>(nnz, 1) * 4) + align_up((size_t)std::max<int64_t>(n, 1) * 4) +
            align_up((size_t)(n + 1) * 4);
  }
  void level_begin(int l) {
    if (!pingpong) return;
    ppcur = l & 1;
    if (!ppbuf[ppcur]) ppbuf[ppcur] = (char*)ctx->pool_take(ppcap);
    ppoff = 0;
  }
  // storage of a coarse level's graph arrays
  template <typename T>
  T* level_take(int64_t count) {
    if (!pingpong) return take<T>(ctx, count);
    size_t b = align_up((size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (ppoff + b > ppcap) fail(LCC_ERR_DEVICE, "internal: coarse level exceeds its buffer");
    T* p = (T*)(ppbuf[ppcur] + ppoff);
    ppoff += b;
    return p;
  }

  void sync(const char* what) {
    hip_check(hipGetLastError(), what);
    hip_check(hipStreamSynchronize(st), what);
  }
  void read_ctrl(const char* what) {
    hip_check(hipMemcpyAsync(ctx->h_ctrl, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st), what);
    sync(what);
  }
  void rec(int64_t kind, int64_t level, int64_t phase, int64_t pass, int64_t a, int64_t b, int64_t c,
           int64_t d) {
    int64_t r[8] = {kind, level, phase, pass, a, b, c, d};
    trace.insert(trace.end(), r, r + 8);
  }

  // degree buckets of a level + hub chunk offsets + vertex weight sums.  In a union, `act` restricts the
  // buckets to the graphs with act set and `into` receives them instead of L.b.
  void prepare(Level& L, int32_t* list, int32_t* hub_off, const uint8_t* act = nullptr, Buckets* into = nullptr) {
    const int64_t n = L.g.n;
    k_reset_level_counters<<<1, 1, 0, st>>>(w.ctrl);
    launch_buckets(L.g.off, n, list, w.ctrl, ctx->bounds(), st, G ? L.gid : nullptr, act);
    if (!into) launch_vertex_sums(L.g.vw, n, w.ctrl, st);
    if (G && !into) {
      L.sumw2g = take<int64_t>(ctx, G);
      launch_seg_sum(L.g.vw, 1, L.vbase, G, L.sumw2g, st);
    }
    read_ctrl("buckets");
    Buckets& b = into ? *into : L.b;
    b.list = list;
    for (int k = 0; k < NBUCKET; ++k) {
      b.count[k] = ctx->h_ctrl->bucket_count[k];
      b.off[k] = ctx->h_ctrl->bucket_off[k];
      b.edges[k] = ctx->h_ctrl->bucket_edges[k];
    }
    b.off[NBUCKET] = ctx->h_ctrl->bucket_off[NBUCKET];
    b.hub_chunks = ctx->h_ctrl->count3;
    b.hub_chunk_off = hub_off;
    b.hub_ps = w.hub_ps; b.hub_pc = w.hub_pc; b.hub_pown = w.hub_pown; b.hub_acc = w.hub_acc; b.stripes = w.stripes;
    b.grid_cap = ctx->tune.grid_cap;
    b.hub_deg = ctx->tune.bucket_max[NBUCKET - 2];
    b.hash_shift = ctx->tune.hash_shift;
    b.count6_hi = ctx->h_ctrl->bucket6_hi;
    if (!into) L.sum_w2 = (int64_t)ctx->h_ctrl->sum_w2;
    if (b.count[NBUCKET - 1]) launch_hub_chunks(list + b.off[NBUCKET - 1], b.count[NBUCKET - 1], L.g.off, w.hub_cnt, hub_off, w.scan_temp, st);
  }

  LMBuffers bufs() {
    LMBuffers B{};
    B.C = w.C; B.Cout = w.Cout; B.W = w.W; B.vs = w.vs; B.keep = w.keep; B.empty = w.empty;
    B.scan_a = w.scan_a; B.scan_b = w.scan_b; B.freelist = w.freelist; B.arena = (uint32_t*)w.k0;
    B.scan_temp = w.scan_temp;
    B.enum_bytes = &w.ctrl->enum_bytes[0];
    B.tg = &w.tg;
    return B;
  }

  LMParams lm_params(const Level& L, bool constrained = false) {
    LMParams P{};
    P.sc = sc;
    P.cons = constrained ? L.B : nullptr;
    P.pass_limit = o.pass_limit;
    for (int i = 1; i <= o.pass_limit; ++i) {
      int k = 0;
      while (k < o.n_phi - 1 && (uint32_t)i > o.phi_until[k]) ++k;
      P.phi_num[i] = o.phi_num[k];
      P.phi_den[i] = o.phi_den[k];
    }
    P.sum_w2 = L.sum_w2;
    P.symmetry = o.symmetry;
    if (G) {
      SegLM& q = P.seg;
      q.G = (int32_t)G;
      q.score = d_score;
      q.gid = L.gid;
      q.vbase = L.vbase;
      q.sumw2 = L.sumw2g;
      q.I = gI;
      q.SW2 = gSW2;
      q.Nbest = gNbest;
      q.N0 = gN0;
      q.copy = gcopy;
      q.ownv = w.t64a;
    }
    return P;
  }

  // LocalMovePasses on level l from L.C (or singletons); result in L.C.  Returns the slot used.
  int local_move_level(int l, bool singleton, int phase, const Buckets* only = nullptr) {
    Level& L = lv[l];
    if (nslot >= NSLOT) fail(LCC_ERR_INVALID, "too many local-move calls");
    int s = nslot++;
    rec(-1, l, phase, 0, s, 0, 0, 0);  // marker: the pass records of slot s go here
    LMBuffers B = bufs();
    if (!singleton) copy_i32(w.C, L.C, L.g.n, st);
    local_move(L.g, only ? *only : L.b, lm_params(L, phase == 0), singleton, B, w.slots + s, w.ctrl, st);
    copy_i32(L.C, w.Cout, L.g.n, st);
    return s;
  }

  LMSlot read_slot(int s) {
    hip_check(hipMemcpyAsync(ctx->h_slots + s, w.slots + s, sizeof(LMSlot), hipMemcpyDeviceToHost, st), "slot");
    sync("slot");
    return ctx->h_slots[s];
  }

  // w.rank = the label rank of `labels`; their count is stored on the device at *dst (a field of a slot or of
  // the control block), so it comes back with the next read of that block: no copy or synchronisation of its own
  void rank_labels(const int32_t* labels, int64_t n, int64_t* dst) {
    launch_label_rank(labels, n, w.used, w.rank, w.scan_temp, st);
    store_count(w.rank + n, dst, st);
  }

  int64_t count_labels(const int32_t* labels, int64_t n) {
    launch_label_rank(labels, n, w.used, w.rank, w.scan_temp, st);
    int32_t nc = 0;
    hip_check(hipMemcpyAsync(&nc, w.rank + n, sizeof(int32_t), hipMemcpyDeviceToHost, st), "count");
    sync("count");
    return nc;
  }

  // Union: number of distinct labels of every graph of level L (labels of graph k lie in its own id range).
  // With nb / n0: also every graph's best and starting objective of the last local move (one synchronisation).
  std::vector<int64_t> count_labels_seg(const int32_t* labels, const Level& L, std::vector<int64_t>* nb = nullptr,
                                        std::vector<int64_t>* n0 = nullptr) {
    launch_label_rank(labels, L.g.n, w.used, w.rank, w.scan_temp, st);
    launch_rebase(w.rank, L.vbase, G, gtmp, st);
    std::vector<int32_t> h((size_t)G + 1);
    hip_check(hipMemcpyAsync(h.data(), gtmp, (size_t)(G + 1) * 4, hipMemcpyDeviceToHost, st), "counts");
    if (nb) {
      nb->resize((size_t)G);
      hip_check(hipMemcpyAsync(nb->data(), gNbest, (size_t)G * 8, hipMemcpyDeviceToHost, st), "best");
    }
    if (n0) {
      n0->resize((size_t)G);
      hip_check(hipMemcpyAsync(n0->data(), gN0, (size_t)G * 8, hipMemcpyDeviceToHost, st), "start");
    }
    sync("counts");
    std::vector<int64_t> nc((size_t)G);
    for (int64_t k = 0; k < G; ++k) nc[k] = h[k + 1] - h[k];
    return nc;
  }

  // Contract level l by `labels` (rank already in w.rank, nc clusters) into a new level l+1.  In a union only
  // the graphs with gact set go on (the rank is recomputed over their labels; nc is derived here).
  void contract(int l, const int32_t* labels, int64_t nc, const uint8_t* gact = nullptr) {
    Level& L = lv[l];
    const int64_t n = L.g.n;
    Level N;
    if (G) {
      launch_label_rank(labels, n, w.used, w.rank, w.scan_temp, st, L.gid, gact);
      N.vbase = take<int32_t>(ctx, G + 1);
      launch_rebase(w.rank, L.vbase, G, N.vbase, st);
      N.hvb.resize((size_t)G + 1);
      hip_check(hipMemcpyAsync(N.hvb.data(), N.vbase, (size_t)(G + 1) * 4, hipMemcpyDeviceToHost, st), "vbase");
      sync("vbase");
      nc = N.hvb[G];
    }
    L.map = take<int32_t>(ctx, n);
    launch_map_labels(labels, w.rank, n, L.map, st, G ? L.gid : nullptr, gact);
    if (G) {
      N.gid = take<int32_t>(ctx, nc);
      launch_coarse_gid(L.map, L.gid, n, N.gid, st);
    }
    if (L.B) {  // a coarse vertex lies inside one constraint cluster: it inherits that cluster
      N.B = take<int32_t>(ctx, nc);
      launch_coarse_gid(L.map, L.B, n, N.B, st);
    }
    level_begin(l + 1);
    int64_t* coff = level_take<int64_t>(nc + 1);
    int64_t* cvw = level_take<int64_t>(nc);
    fill_i64(cvw, 0, nc, st);
    launch_coarse_vw(L.map, L.g.vw, n, cvw, st);
    // cross entries per fine vertex and per coarse row; row x's entries take the range [xoff[x], xoff[x+1])
    // and every fine vertex claims its share of its row's range
    launch_cross_count(L.g, L.b, L.map, w.cnt, st);
    int64_t* ecnt = w.seg0;
    int64_t* xoff = w.seg1;
    fill_i64(ecnt, 0, nc, st);
    launch_group_sum(L.map, w.cnt, n, ecnt, st);
    scan_i64_i64(ecnt, xoff, nc, w.scan_temp, st);
    int64_t E = 0;
    hip_check(hipMemcpyAsync(&E, xoff + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st), "entries");
    sync("entries");
    int64_t nnzc = 0;
    int32_t* cidx;
    int32_t* cw;
    if (E > 0) {
      launch_group_place(L.map, w.cnt, nullptr, n, xoff, nc, (unsigned long long*)ecnt, w.pos, st);
      launch_cross_emit(L.g, L.b, L.map, w.pos, w.k0, w.v0, st);
      // each row sorted by neighbour: the whole array is then in (x, y) order
      int ybits = 1;
      while (((int64_t)1 << ybits) < nc) ++ybits;
      {
        const auto mk = ctx->pool_mark();
        segsort_pairs(w.k0, w.v0, w.k1, w.v1, E, xoff, nc, ybits, w.scan_temp,
                      [&](size_t by) { return ctx->pool_take(by); }, st);
        ctx->pool_release(mk);
      }
      const uint64_t* ks = w.k1;
      const uint32_t* vs = w.v1;
      int64_t* pref = (int64_t*)w.k0;  // the input key buffer is free
      int32_t* hstart = (int32_t*)w.v0;
      launch_heads(ks, E, w.head, st);
      scan_u8_i32(w.head, w.uid, E, w.scan_temp, nullptr, st);
      int32_t nz = 0;
      hip_check(hipMemcpyAsync(&nz, w.uid + E, sizeof(int32_t), hipMemcpyDeviceToHost, st), "coarse nnz");
      sync("coarse nnz");
      nnzc = nz;
      cidx = level_take<int32_t>(nnzc);
      cw = level_take<int32_t>(nnzc);
      launch_coarse_write(ks, vs, w.head, w.uid, E, nnzc, nc, pref, hstart, w.ux, cidx, cw, coff, w.scan_temp, st);
    } else {
      cidx = level_take<int32_t>(1);
      cw = level_take<int32_t>(1);
      fill_i64(coff, 0, nc + 1, st);
    }
    N.g.n = nc;
    N.g.nnz = nnzc;
    N.g.off = coff;
    N.g.idx = cidx;
    N.g.w = cw;
    N.g.vw = cvw;
    N.C = take<int32_t>(ctx, nc);
    lv.push_back(N);
    Level& NL = lv.back();
    prepare(NL, level_take<int32_t>(nc), level_take<int32_t>(nc + 1));
  }

  // ---------------------------------------------------------------------------------------------------
  // Alg. 1: Louvain / Louvain+
  // ---------------------------------------------------------------------------------------------------
  // init (optional): the level-0 local move starts from it instead of singletons.  A constraint in lv[0].B
  // confines the coarsening local moves; the uncoarsening ones are free (the iteration of Sec. IV-D).
  int louvain(bool plus, const int32_t* init = nullptr) {
    int l = 0;
    if (init) copy_i32(lv[0].C, init, lv[0].g.n, st);
    for (;;) {
      int s = local_move_level(l, !(l == 0 && init), 0);
      Level& L = lv[l];
      rank_labels(L.C, L.g.n, &w.slots[s].nlab);
      LMSlot S = read_slot(s);
      const int64_t nc = S.nlab;
      rec(2, l, 0, 0, L.g.n, L.g.nnz, nc, S.Nbest);
      if (nc == L.g.n) break;
      if (l + 1 >= o.max_levels) { flags |= LCC_FLAG_LEVEL_CAP; break; }
      contract(l, lv[l].C, nc);
      ++l;
    }
    int top = l;
    for (int k = top - 1; k >= 0; --k) {
      Level& L = lv[k];
      launch_project(lv[k + 1].C, L.map, L.g.n, L.C, st);
      if (plus) {
        int s = local_move_level(k, false, 1);
        rank_labels(L.C, L.g.n, &w.slots[s].nlab);
        LMSlot S = read_slot(s);
        const int64_t nc = S.nlab;
        rec(2, k, 1, 0, L.g.n, L.g.nnz, nc, S.Nbest);
      }
    }
    return top;
  }

  // ---------------------------------------------------------------------------------------------------
  // Alg. 1 on a union of graphs: every graph follows its own level sequence.  A graph whose local move leaves
  // as many clusters as vertices (or that reaches the level cap) stops coarsening at that level (top[k]) and
  // is left out of every coarser level; on the way back, level l's uncoarsening local move covers only the
  // graphs with top[k] > l and plus[k].
  // ---------------------------------------------------------------------------------------------------
  int louvain_seg(const std::vector<uint8_t>& plus, std::vector<int>& top, std::vector<uint32_t>& gflags) {
    std::vector<uint8_t> cont((size_t)G);
    for (int64_t k = 0; k < G; ++k) cont[k] = lv[0].hvb[k + 1] > lv[0].hvb[k];
    int l = 0;
    for (;;) {
      local_move_level(l, true, 0);
      Level& L = lv[l];
      std::vector<int64_t> nc = count_labels_seg(L.C, L);
      bool any = false;
      for (int64_t k = 0; k < G; ++k) {
        if (!cont[k]) continue;
        const int64_t nk = L.hvb[k + 1] - L.hvb[k];
        if (nc[k] == nk) {
          top[k] = l;
          cont[k] = 0;
        } else if (l + 1 >= o.max_levels) {
          top[k] = l;
          gflags[k] |= LCC_FLAG_LEVEL_CAP;
          cont[k] = 0;
        } else {
          any = true;
        }
      }
      if (!any) break;
      hip_check(hipMemcpyAsync(gact, cont.data(), (size_t)G, hipMemcpyHostToDevice, st), "active graphs");
      contract(l, L.C, 0, gact);
      ++l;
    }
    const int T = l;
    std::vector<uint8_t> act((size_t)G);
    for (int k = T - 1; k >= 0; --k) {
      Level& L = lv[k];
      launch_project(lv[k + 1].C, L.map, L.g.n, L.C, st, L.gid, L.vbase, lv[k + 1].vbase);
      bool any = false;
      for (int64_t g = 0; g < G; ++g) {
        act[g] = top[g] > k && plus[g];
        any = any || act[g];
      }
      if (!any) continue;
      hip_check(hipMemcpyAsync(gact, act.data(), (size_t)G, hipMemcpyHostToDevice, st), "active graphs");
      Buckets only;
      prepare(L, take<int32_t>(ctx, L.g.n), take<int32_t>(ctx, L.g.n + 1), gact, &only);
      local_move_level(k, false, 1, &only);
    }
    return T;
  }

  // ---------------------------------------------------------------------------------------------------
  // Alg. 5: pLeiden / pLeiden+
  // ---------------------------------------------------------------------------------------------------
  RefineBuffers rbufs() {
    RefineBuffers r{};
    r.WB = w.WB; r.aB = w.aB; r.aX = w.aX; r.inU = w.inU; r.H = w.H; r.par = w.par; r.root = w.root;
    r.flip = w.flip; r.has_child = w.has_child; r.tsz = w.tsz; r.member = w.member; r.tree_sz = w.tree_sz;
    r.k0 = w.k0; r.v0 = w.v0; r.k1 = w.k1; r.v1 = w.v1;
    r.pw = w.pw; r.pc = w.pc; r.tmp64a = w.t64a; r.tmp64b = w.t64b; r.pos_of = w.pos_of; r.fail = w.fail;
    r.scan_temp = w.scan_temp;
    return r;
  }

  int leiden(bool plus, const int32_t* init) {
    int l = 0;
    int noprog = 0;
    if (init) copy_i32(lv[0].C, init, lv[0].g.n, st);
    bool singleton = init == nullptr;
    for (;;) {
      Level& L = lv[l];
      const int64_t n = L.g.n;
      int s = local_move_level(l, singleton, 0);
      singleton = false;
      rank_labels(L.C, n, &w.slots[s].nlab);  // the count of C_l, unless the alternate move below changes it
      LMSlot S = read_slot(s);
      int64_t nc = S.nlab;
      int64_t N = S.Nbest;
      if (S.Nbest == S.N0) {
        // C_l unchanged by the local move: the alternate local move (Sec. V-A) from C_l
        LMBuffers B = bufs();
        copy_i32(w.C, L.C, n, st);
        launch_cluster_weights(w.C, L.g.vw, n, w.W, st);
        if (nslot >= NSLOT) fail(LCC_ERR_INVALID, "too many local-move calls");
        int s2 = nslot++;
        const auto mark = ctx->pool_mark();  // the alternate move's scratch is released below
        if (!lmalt(L.g, L.b, sc, B, w.slots + s2, w.ctrl, w.alt_list, w.alt_gain,
                   [this](size_t bytes) { return ctx->pool_take(bytes); }, st))
          fail(LCC_ERR_INVALID, "alternate local move with 2^30 or more movers is not supported");
        copy_i32(L.C, w.C, n, st);
        launch_cluster_weights(w.C, L.g.vw, n, w.W, st);
        launch_objective(L.g, L.b, w.C, w.W, w.ctrl, st);
        rank_labels(L.C, n, &w.ctrl->nlab);
        read_ctrl("lmalt");  // the stream is done with the scratch
        nc = ctx->h_ctrl->nlab;
        ctx->pool_release(mark);
        N = q * ctx->h_ctrl->obj_I - p * (ctx->h_ctrl->obj_SW2 - L.sum_w2);
        rec(3, l, 0, 0, ctx->h_ctrl->lmalt_k, ctx->h_ctrl->lmalt_best_k, N, 0);
      }
      rec(2, l, 0, 0, n, L.g.nnz, nc, N);
      if (nc == n) break;
      if (l + 1 >= o.max_levels) { flags |= LCC_FLAG_LEVEL_CAP; break; }
      // refinement R of B = C_l; compaction of B for the downsampled clustering
      int32_t* R = w.in_labels;
      RefineBuffers rb = rbufs();
      {
        const auto mk = ctx->pool_mark();  // the refinement's sort scratch is released right after
        RefSrc rs;
        rs.s = sc;
        rs.st = seed_stream(o.seed, refine_calls);
        refine(L.g, L.b, rs, L.C, R, rb, w.ctrl, [&](size_t by) { return ctx->pool_take(by); }, st);
        ctx->pool_release(mk);
      }
      rank_labels(R, n, &w.ctrl->nlab);
      read_ctrl("refine");
      const int64_t nR = ctx->h_ctrl->nlab;
      if (ctx->h_ctrl->err_bits & ERRB_INTERNAL) fail(LCC_ERR_DEVICE, "refinement produced a parent cycle");
      rec(4, l, 0, 0, nR, (int64_t)refine_calls, ctx->h_ctrl->refine_U, ctx->h_ctrl->refine_m);
      ++refine_calls;
      if (nR == n) {
        if (++noprog >= 3) { flags |= LCC_FLAG_REFINE_NO_PROGRESS; break; }
        continue;  // the same level again with the next refinement seed
      }
      noprog = 0;
      contract(l, R, nR);
      // Downsample: C_{l+1}[x] = compact(C_l)[C_l[v]] for any v in x
      Level& L2 = lv[l];
      launch_label_rank(L2.C, n, w.used, w.rank, w.scan_temp, st);  // w.rank = compaction of C_l
      launch_downsample(L2.C, w.rank, L2.map, n, lv[l + 1].C, st);
      ++l;
    }
    int top = l;
    for (int k = top - 1; k >= 0; --k) {
      Level& L = lv[k];
      launch_project(lv[k + 1].C, L.map, L.g.n, L.C, st);
      if (plus) {
        int s = local_move_level(k, false, 1);
        rank_labels(L.C, L.g.n, &w.slots[s].nlab);
        LMSlot S = read_slot(s);
        const int64_t nc = S.nlab;
        rec(2, k, 1, 0, L.g.n, L.g.nnz, nc, S.Nbest);
      }
    }
    return top;
  }

  // ---------------------------------------------------------------------------------------------------
  // Alg. 5 on a union of graphs.  Every graph follows its own sequence: the alternate local move where its
  // local move left C_l unchanged, its own refinement stream (s_t with t = its own refinement count) and
  // termination.  A graph whose refinement makes no progress repeats its level: its part of the next union
  // level is the same graph (the contraction by singletons is the identity) and starts from the same C_l; that
  // union level is not one of its own levels.  On the way back (pLeiden+), union level l's local move covers the
  // graphs with top[k] > l whose level l -> l+1 was a real contraction.
  // ---------------------------------------------------------------------------------------------------
  int leiden_seg(const std::vector<uint8_t>& plus, std::vector<int>& top, std::vector<int>& levels,
                 std::vector<uint32_t>& gflags) {
    std::vector<uint8_t> cont((size_t)G), alt((size_t)G), rep((size_t)G);
    std::vector<int> own((size_t)G, 0), noprog((size_t)G, 0);  // the graph's own level; no-progress retries
    std::vector<uint64_t> calls((size_t)G, 0), hst((size_t)G);
    std::vector<std::vector<uint8_t>> repeated;  // repeated[l][k]: union level l -> l+1 repeats graph k's level
    for (int64_t k = 0; k < G; ++k) cont[k] = lv[0].hvb[k + 1] > lv[0].hvb[k];
    uint64_t* d_st = take<uint64_t>(ctx, G);
    uint8_t* d_alt = take<uint8_t>(ctx, G);
    uint8_t* d_rep = take<uint8_t>(ctx, G);
    int64_t* d_bestk = take<int64_t>(ctx, G);
    int l = 0;
    for (;;) {
      const int64_t n = lv[l].g.n;
      local_move_level(l, l == 0, 0);
      std::vector<int64_t> nb, n0;
      std::vector<int64_t> nc = count_labels_seg(lv[l].C, lv[l], &nb, &n0);
      // C_l unchanged by the local move: the alternate local move (Sec. V-A), for those graphs together
      bool any_alt = false;
      for (int64_t k = 0; k < G; ++k) {
        alt[k] = cont[k] && nb[k] == n0[k];
        any_alt = any_alt || alt[k];
      }
      if (any_alt) {
        Level& L = lv[l];
        hip_check(hipMemcpyAsync(d_alt, alt.data(), (size_t)G, hipMemcpyHostToDevice, st), "alternate graphs");
        LMBuffers B = bufs();
        copy_i32(w.C, L.C, n, st);
        launch_cluster_weights(w.C, L.g.vw, n, w.W, st);
        if (nslot >= NSLOT) fail(LCC_ERR_INVALID, "too many local-move calls");
        int s2 = nslot++;
        AltSeg as;
        as.ss.tab = d_score; as.ss.gid = L.gid; as.ss.vbase = L.vbase;
        as.act = d_alt;
        as.best_k = d_bestk;
        as.sg = lm_params(L).seg;
        const auto mark = ctx->pool_mark();
        if (!lmalt(L.g, L.b, sc, B, w.slots + s2, w.ctrl, w.alt_list, w.alt_gain,
                   [this](size_t bytes) { return ctx->pool_take(bytes); }, st, &as))
          fail(LCC_ERR_INVALID, "alternate local move with 2^30 or more movers is not supported");
        copy_i32(L.C, w.C, n, st);
        nc = count_labels_seg(L.C, L);  // the stream is done with the scratch
        ctx->pool_release(mark);
      }
      bool any = false;
      for (int64_t k = 0; k < G; ++k) {
        if (!cont[k]) continue;
        const int64_t nk = lv[l].hvb[k + 1] - lv[l].hvb[k];
        if (nc[k] == nk) {
          top[k] = l; cont[k] = 0;
        } else if (own[k] + 1 >= o.max_levels) {
          top[k] = l; gflags[k] |= LCC_FLAG_LEVEL_CAP; cont[k] = 0;
        } else {
          any = true;
        }
      }
      if (!any) break;
      // refinement of the continuing graphs, each with its own stream
      for (int64_t k = 0; k < G; ++k) hst[k] = seed_stream(o.seed, calls[k]);
      hip_check(hipMemcpyAsync(d_st, hst.data(), (size_t)G * 8, hipMemcpyHostToDevice, st), "streams");
      hip_check(hipMemcpyAsync(gact, cont.data(), (size_t)G, hipMemcpyHostToDevice, st), "active graphs");
      int32_t* R = w.in_labels;
      {
        Level& L = lv[l];
        RefineBuffers rb = rbufs();
        RefSrc rs;
        rs.gid = L.gid; rs.vbase = L.vbase; rs.tab = d_score; rs.stt = d_st; rs.act = gact;
        const auto mk = ctx->pool_mark();
        refine(L.g, L.b, rs, L.C, R, rb, w.ctrl, [&](size_t by) { return ctx->pool_take(by); }, st);
        ctx->pool_release(mk);
      }
      // the control block comes back with the counts' synchronisation
      hip_check(hipMemcpyAsync(ctx->h_ctrl, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "refine");
      std::vector<int64_t> nR = count_labels_seg(R, lv[l]);
      if (ctx->h_ctrl->err_bits & ERRB_INTERNAL) fail(LCC_ERR_DEVICE, "refinement produced a parent cycle");
      any = false;
      for (int64_t k = 0; k < G; ++k) {
        rep[k] = 0;
        if (!cont[k]) continue;
        ++calls[k];
        const int64_t nk = lv[l].hvb[k + 1] - lv[l].hvb[k];
        if (nR[k] == nk) {
          if (++noprog[k] >= 3) {
            gflags[k] |= LCC_FLAG_REFINE_NO_PROGRESS; top[k] = l; cont[k] = 0;
            continue;
          }
          rep[k] = 1;  // the same level again with the next refinement stream
        } else {
          noprog[k] = 0;
        }
        any = true;
      }
      if (!any) break;
      hip_check(hipMemcpyAsync(gact, cont.data(), (size_t)G, hipMemcpyHostToDevice, st), "active graphs");
      hip_check(hipMemcpyAsync(d_rep, rep.data(), (size_t)G, hipMemcpyHostToDevice, st), "repeated graphs");
      if (lv.size() + 1 > lv.capacity()) fail(LCC_ERR_INVALID, "internal: too many union levels");
      contract(l, R, 0, gact);
      // Downsample: C_{l+1}[x] = graph-local compact(C_l)[C_l[v]] for any v in x; a repeated graph keeps C_l
      Level& L2 = lv[l];
      launch_label_rank(L2.C, n, w.used, w.rank, w.scan_temp, st, L2.gid, gact);
      launch_downsample(L2.C, w.rank, L2.map, n, lv[l + 1].C, st, L2.gid, L2.vbase, lv[l + 1].vbase, d_rep);
      for (int64_t k = 0; k < G; ++k)
        if (cont[k] && !rep[k]) ++own[k];
      repeated.push_back(rep);
      ++l;
    }
    const int T = l;
    for (int64_t k = 0; k < G; ++k) levels[k] = own[k] + 1;
    std::vector<uint8_t> act((size_t)G);
    for (int j = T - 1; j >= 0; --j) {
      Level& L = lv[j];
      launch_project(lv[j + 1].C, L.map, L.g.n, L.C, st, L.gid, L.vbase, lv[j + 1].vbase);
      bool any = false;
      for (int64_t k = 0; k < G; ++k) {
        act[k] = top[k] > j && plus[k] && !repeated[(size_t)j][k];
        any = any || act[k];
      }
      if (!any) continue;
      hip_check(hipMemcpyAsync(gact, act.data(), (size_t)G, hipMemcpyHostToDevice, st), "active graphs");
      Buckets only;
      prepare(L, take<int32_t>(ctx, L.g.n), take<int32_t>(ctx, L.g.n + 1), gact, &only);
      local_move_level(j, false, 1, &only);
    }
    return T;
  }

  void emit_pass_records() {
    // local-move pass records are read back in one copy at the end
    if (!nslot) return;
    hip_check(hipMemcpyAsync(ctx->h_slots, w.slots, sizeof(LMSlot) * nslot, hipMemcpyDeviceToHost, st), "slots");
    sync("slots");
  }
};

void default_opts(lcc_options* o) {
  memset(o, 0, sizeof(*o));
  o->pass_limit = 6;
  o->n_phi = 2;
  o->phi_num[0] = 3; o->phi_den[0] = 4; o->phi_until[0] = 4;
  o->phi_num[1] = 1; o->phi_den[1] = 4; o->phi_until[1] = 6;
  o->eps_num = 1; o->eps_den = 10;
  o->seed = 1;
  o->max_levels = 64;
  o->validate = 1;
  o->trace = nullptr;
}

void check_opts(const lcc_options& o) {
  if (o.pass_limit < 0 || o.pass_limit > MAX_PASSES) fail(LCC_ERR_INVALID, "pass_limit outside [0, 32]");
  if (o.n_phi < 1 || o.n_phi > 8) fail(LCC_ERR_INVALID, "n_phi outside [1, 8]");
  for (int k = 0; k < o.n_phi; ++k)
    if (o.phi_den[k] == 0 || o.phi_num[k] > o.phi_den[k]) fail(LCC_ERR_INVALID, "temperature phi outside [0, 1]");
  if (o.eps_den == 0) fail(LCC_ERR_INVALID, "eps_den = 0");
  if (o.max_levels <= 0 || o.max_levels > 1024) fail(LCC_ERR_INVALID, "max_levels outside [1, 1024]");
  if (o.symmetry < LCC_SYM_AFTERBURNER || o.symmetry > LCC_SYM_MLH) fail(LCC_ERR_INVALID, "unknown symmetry mode");
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) { uint64_t t = a % b; a = b; b = t; }
  return a;
}

// Setup (Sec. II): copy or adopt the input, validate it on the device, derive vertex weights, W, W_E,
// lambda = p / q in lowest terms and the exactness bound.  Fills lv[0].
void setup(Run& R, const lcc_graph* g, lcc_lambda lam, const int32_t* init_labels) {
  lcc_ctx* ctx = R.ctx;
  WS& w = R.w;
  hipStream_t st = R.st;
  const int64_t n = g->n, nnz = g->nnz;
  Level L0;
  L0.g.n = n;
  L0.g.nnz = nnz;
  const bool host = g->mem == LCC_MEM_HOST;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (bytes) hip_check(hipMemcpyAsync(dst, src, bytes, host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st), "input copy");
  };
  // offsets
  if (g->offsets_bits == 64 && !host) {
    L0.g.off = (const int64_t*)g->offsets;
  } else if (g->offsets_bits == 64) {
    cp(w.in_off, g->offsets, (size_t)(n + 1) * 8);
    L0.g.off = w.in_off;
  } else {
    int32_t* tmp = (int32_t*)w.k0;  // staging for 32-bit offsets
    cp(tmp, g->offsets, (size_t)(n + 1) * 4);
    offsets32_to_64(tmp, w.in_off, n + 1, st);
    L0.g.off = w.in_off;
  }
  if (host) { cp(w.in_idx, g->indices, (size_t)nnz * 4); L0.g.idx = w.in_idx; }
  else L0.g.idx = g->indices;
  if (!g->edge_w) {
    k_ones<<<grid1(nnz), BLOCK, 0, st>>>(w.in_w, nnz);
    L0.g.w = w.in_w;
  } else if (host) {
    cp(w.in_w, g->edge_w, (size_t)nnz * 4);
    L0.g.w = w.in_w;
  } else {
    L0.g.w = g->edge_w;
  }
  const int64_t* vwg = nullptr;
  if (g->vw_mode == LCC_VW_GIVEN) {
    if (host) { cp(w.in_vwg, g->vertex_w, (size_t)n * 8); vwg = w.in_vwg; }
    else vwg = g->vertex_w;
  }
  L0.g.vw = w.vw0;
  L0.C = take<int32_t>(ctx, n);
  zero_bytes(w.ctrl, sizeof(Ctrl), st);
  // offsets
  launch_validate_offsets(L0.g.off, n, nnz, w.ctrl, st);
  R.read_ctrl("validate offsets");
  if (ctx->h_ctrl->err_bits & ERRB_INVALID) fail(LCC_ERR_INVALID, "CSR offsets are not a valid row partition");
  R.lv.push_back(L0);
  Level& L = R.lv[0];
  // buckets need only the offsets; vertex weights are derived by the row pass below
  {
    // prepare() reads vertex sums, which are not derived yet: buckets first, sums after the row pass
    k_reset_level_counters<<<1, 1, 0, st>>>(w.ctrl);
    launch_buckets(L.g.off, n, w.list0, w.ctrl, ctx->bounds(), st);
    R.read_ctrl("buckets");
    Buckets& b = L.b;
    b.list = w.list0;
    for (int k = 0; k < NBUCKET; ++k) {
      b.count[k] = ctx->h_ctrl->bucket_count[k];
      b.off[k] = ctx->h_ctrl->bucket_off[k];
      b.edges[k] = ctx->h_ctrl->bucket_edges[k];
    }
    b.off[NBUCKET] = ctx->h_ctrl->bucket_off[NBUCKET];
    b.hub_chunks = ctx->h_ctrl->count3;
    b.hub_chunk_off = w.hub_off0;
    b.hub_ps = w.hub_ps; b.hub_pc = w.hub_pc; b.hub_pown = w.hub_pown; b.hub_acc = w.hub_acc; b.stripes = w.stripes;
    b.grid_cap = ctx->tune.grid_cap;
    b.hub_deg = ctx->tune.bucket_max[NBUCKET - 2];
    b.hash_shift = ctx->tune.hash_shift;
    b.count6_hi = ctx->h_ctrl->bucket6_hi;
    if (b.count[NBUCKET - 1])
      launch_hub_chunks(w.list0 + b.off[NBUCKET - 1], b.count[NBUCKET - 1], L.g.off, w.hub_cnt, w.hub_off0, w.scan_temp, st);
  }
  const auto sym_mark = ctx->pool_mark();  // the symmetry check's sort scratch is released below
  SymBuffers sb;
  if (R.o.validate && (nnz <= SYM_SEARCH_MAX_NNZ || nnz <= SYM_SEARCH_MAX_AVG_DEG * n)) {
    sb.search = true;
  } else if (R.o.validate) {
    sb.k0 = w.k0; sb.v0 = w.v0; sb.k1 = w.k1; sb.v1 = w.v1;
    sb.lo = w.cnt; sb.lbase = w.seg0; sb.scan_temp = w.scan_temp;
    sb.temp = ctx->pool_take(radix_temp_bytes(nnz));
  }
  launch_validate_rows(L.g, L.b, (int)g->vw_mode, vwg, w.vw0, w.ctrl, st, sb);
  launch_vertex_sums(w.vw0, n, w.ctrl, st);
  if (init_labels) k_labels_in_range<<<grid1(n), BLOCK, 0, st>>>(init_labels, n, w.ctrl);
  R.read_ctrl("validate rows");
  ctx->pool_release(sym_mark);
  const Ctrl& c = *ctx->h_ctrl;
  uint32_t e = c.err_bits;
  if (!R.o.validate) e &= ERRB_INVALID | ERRB_VW_TOO_BIG;  // structural faults that would break the kernels
  if (e & ERRB_INVALID) fail(LCC_ERR_INVALID, "neighbour index out of range (or initial label outside [0, n))");
  if (e & ERRB_SELF_LOOP) fail(LCC_ERR_SELF_LOOP, "a row contains its own vertex");
  if (e & ERRB_UNSORTED) fail(LCC_ERR_UNSORTED, "a row is not strictly ascending");
  if (e & ERRB_WEIGHT) fail(LCC_ERR_WEIGHT, "an edge weight <= 0 or a vertex weight < 0");
  if ((e & ERRB_NOT_SYMMETRIC) || (sb.search && c.count0 != 0)) fail(LCC_ERR_NOT_SYMMETRIC, "the graph is not symmetric");
  if (c.sum_we >= ((uint64_t)1 << 32)) fail(LCC_ERR_OVERFLOW, "total edge weight >= 2^32");
  if (e & ERRB_VW_TOO_BIG) fail(LCC_ERR_OVERFLOW, "a vertex weight >= 2^31");
  L.sum_w2 = (int64_t)c.sum_w2;
  R.W = c.sum_w;
  const unsigned __int128 W = c.sum_w, WE = c.sum_we;
  if (lam.den == 0) fail(LCC_ERR_LAMBDA, "lambda denominator is zero");
  unsigned __int128 P = lam.num, Q = (unsigned __int128)lam.den * (lam.over_total_weight ? W : 1);
  if (Q == 0 || P > Q) fail(LCC_ERR_LAMBDA, "lambda outside [0, 1] or undefined");
  if (Q >> 64) fail(LCC_ERR_OVERFLOW, "lambda denominator >= 2^64");
  uint64_t p = (uint64_t)P, q = (uint64_t)Q;
  if (p == 0) q = 1;
  else { uint64_t d = gcd64(p, q); p /= d; q /= d; }
  if ((unsigned __int128)q * WE + (unsigned __int128)p * W * W >= ((unsigned __int128)1 << 62))
    fail(LCC_ERR_OVERFLOW, "q W_E + p W^2 >= 2^62");
  R.p = (int64_t)p;
  R.q = (int64_t)q;
  R.sc.p = R.p;
  R.sc.q = R.q;
  // tie window: |delta_u - delta_v| <= floor((eps_num q - 1) / (2 eps_den)), at least 0
  __int128 num = (__int128)R.o.eps_num * q - 1;
  __int128 den = 2 * (__int128)R.o.eps_den;
  __int128 t = num >= 0 ? num / den : -1;
  R.sc.tie = t < 0 ? 0 : (int64_t)t;
}

// Scoring parameters of one graph (lambda = p / q in lowest terms, tie window), or a failure status.
lcc_status graph_score(lcc_lambda lam, unsigned __int128 W, unsigned __int128 WE, const lcc_options& o, Score* out,
                       const char** why) {
  if (WE >= ((unsigned __int128)1 << 32)) { *why = "total edge weight >= 2^32"; return LCC_ERR_OVERFLOW; }
  if (lam.den == 0) { *why = "lambda denominator is zero"; return LCC_ERR_LAMBDA; }
  unsigned __int128 P = lam.num, Q = (unsigned __int128)lam.den * (lam.over_total_weight ? W : 1);
  if (Q == 0 || P > Q) { *why = "lambda outside [0, 1] or undefined"; return LCC_ERR_LAMBDA; }
  if (Q >> 64) { *why = "lambda denominator >= 2^64"; return LCC_ERR_OVERFLOW; }
  uint64_t p = (uint64_t)P, q = (uint64_t)Q;
  if (p == 0) q = 1;
  else { uint64_t d = gcd64(p, q); p /= d; q /= d; }
  if ((unsigned __int128)q * WE + (unsigned __int128)p * W * W >= ((unsigned __int128)1 << 62)) {
    *why = "q W_E + p W^2 >= 2^62";
    return LCC_ERR_OVERFLOW;
  }
  out->p = (int64_t)p;
  out->q = (int64_t)q;
  __int128 num = (__int128)o.eps_num * q - 1;
  __int128 den = 2 * (__int128)o.eps_den;
  __int128 t = num >= 0 ? num / den : -1;
  out->tie = t < 0 ? 0 : (int64_t)t;
  return LCC_OK;
}

void fill_result(lcc_result* res, int64_t nc, __int128 N, int64_t p, int64_t q, int64_t sum_w2, uint64_t W,
                 bool modularity, int levels, uint32_t flags) {
  res->num_clusters = nc;
  res->obj_num_hi = (int64_t)(N >> 64);
  res->obj_num_lo = (uint64_t)N;
  res->obj_den = (uint64_t)q;
  res->objective = (double)N / (double)q;
  if (modularity && W > 0) {
    __int128 num = N - (__int128)p * sum_w2;
    res->modularity = (double)num / ((double)q * (double)W);
  } else {
    res->modularity = NAN;
  }
  res->levels = levels;
  res->flags = flags;
}

void check_graph_args(const lcc_graph* g) {
  if (!g) fail(LCC_ERR_INVALID, "graph is NULL");
  if (g->n < 0 || g->n > 2147483647LL) fail(LCC_ERR_INVALID, "n outside [0, 2^31)");
  // entry positions of the contraction (run starts, coarse entry ids) are 32-bit
  if (g->nnz < 0 || g->nnz > 2147483647LL) fail(LCC_ERR_INVALID, "nnz outside [0, 2^31)");
  if (g->offsets_bits != 32 && g->offsets_bits != 64) fail(LCC_ERR_INVALID, "offsets_bits must be 32 or 64");
  if (!g->offsets) fail(LCC_ERR_INVALID, "offsets is NULL");
  if (g->nnz > 0 && !g->indices) fail(LCC_ERR_INVALID, "indices is NULL");
  if (g->vw_mode != LCC_VW_GIVEN && g->vw_mode != LCC_VW_WEIGHTED_DEGREE && g->vw_mode != LCC_VW_UNIT)
    fail(LCC_ERR_INVALID, "unknown vertex-weight mode");
  if (g->vw_mode == LCC_VW_GIVEN && !g->vertex_w && g->n > 0) fail(LCC_ERR_INVALID, "vertex_w is NULL");
  if (g->mem != LCC_MEM_HOST && g->mem != LCC_MEM_DEVICE) fail(LCC_ERR_INVALID, "unknown memory kind");
}

// Footprint bound of one call (workspace + coarse levels), the admission figure of lcc_workspace_bytes.
// Louvain and pLouvain+ keep coarse levels in pool chunks of one input-sized level: two hold a geometric
// coarsening (pLouvain+ keeps every level, so a slow coarsening holds more).  pLeiden and pLeiden+ keep two
// alternating level buffers plus the refinement's and the alternate move's transient scratch: three chunks.
size_t call_bytes(int64_t n, int64_t nnz, lcc_variant variant) {
  WS tmp{};
  const size_t levels = (variant == LCC_PLEIDEN || variant == LCC_PLEIDEN_PLUS) ? 3 : 2;
  return carve(tmp, nullptr, n, nnz) + levels * level_bytes(n, nnz);
}

// Puts a context into no-allocation mode for one call and restores its own workspace afterwards.
struct ArenaSwap {
  lcc_ctx* c;
  bool on = false;
  WS w{};
  char* base = nullptr;
  size_t bytes = 0;
  int64_t n = -1, nnz = -1;
  void engage(Arena* a) {
    w = c->w; base = c->ws_base; bytes = c->ws_bytes; n = c->ws_n; nnz = c->ws_nnz;
    c->arena = a;
    on = true;
  }
  ~ArenaSwap() {
    if (!on) return;
    c->arena = nullptr;
    c->w = w; c->ws_base = base; c->ws_bytes = bytes; c->ws_n = n; c->ws_nnz = nnz;
  }
};

lcc_status cluster_impl(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lam, lcc_variant variant,
                        const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res,
                        const int32_t* init_labels, const int32_t* constraint = nullptr, bool noalloc = false) {
  if (!ctx) fail(LCC_ERR_INVALID, "context is NULL");
  check_graph_args(g);
  if (!res) fail(LCC_ERR_INVALID, "result is NULL");
  if (g->n > 0 && !labels_out) fail(LCC_ERR_INVALID, "labels_out is NULL");
  if (variant < LCC_LOUVAIN || variant > LCC_PLEIDEN_PLUS) fail(LCC_ERR_INVALID, "unknown variant");
  if (constraint && (init_labels || variant == LCC_PLEIDEN || variant == LCC_PLEIDEN_PLUS))
    fail(LCC_ERR_INVALID, "a constraint clustering applies to Louvain variants without initial labels");
  std::unique_lock<std::mutex> call_lock;  // no-allocation calls on one device share its scratch array
  if (noalloc) {
    const size_t need = call_bytes(g->n, g->nnz, variant);
    if (need > NOALLOC_BYTES)
      fail(LCC_ERR_INVALID, "graph too large for the no-allocation scratch: lcc_workspace_bytes = " +
                                std::to_string(need) + " > " + std::to_string(NOALLOC_BYTES));
    if (ctx->device >= MAX_DEVICES) fail(LCC_ERR_INVALID, "no-allocation scratch: device index beyond 63");
    call_lock = std::unique_lock<std::mutex>(g_scratch[ctx->device].call_mu);
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  hip_check(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  Arena arena;
  ArenaSwap swap{ctx};  // declared before the pool guard below: restores the context after the stream drained
  if (noalloc) {
    hipError_t e = hipSuccess;
    void* p = scratch_address(ctx->device, &e);
    if (!p) fail(LCC_ERR_DEVICE, std::string("address of the no-allocation scratch: ") + hipGetErrorString(e));
    arena.base = (char*)p;
    arena.cap = NOALLOC_BYTES;
    swap.engage(&arena);
  }
  Run R(ctx, st);
  if (opts) R.o = *opts; else default_opts(&R.o);
  check_opts(R.o);
  struct ProfGuard {
    lcc_ctx* c;
    explicit ProfGuard(lcc_ctx* x) : c(x) { g_prof_ctx = (x->prof_mask && !x->arena) ? x : nullptr; }
    ~ProfGuard() {
      g_prof_ctx = nullptr;
      for (auto& r : c->prof_recs) { c->ev_pool.push_back(r.a); c->ev_pool.push_back(r.b); }
      c->prof_recs.clear();
      for (auto& e : c->prof_open) if (e) { c->ev_pool.push_back(e); e = nullptr; }
    }
  } prof_guard(ctx);
  ctx->ensure_ws(g->n, g->nnz, st);
  if (noalloc) {  // the array keeps the previous call's contents: clear what must start at zero
    WS& w = ctx->w;
    zero_bytes(w.tg.held, (size_t)w.tg.held_cap * sizeof(uint32_t), st);
    zero_bytes(w.tg.status, (size_t)w.tg.status_cap * sizeof(unsigned long long), st);
    zero_bytes(w.tg.ticket, sizeof(uint32_t), st);
    zero_bytes(w.stripes, (size_t)NSTRIPE * STRIPE_W * sizeof(int64_t), st);
    w.tg.last = 0;
  }
  ctx->pool_reset();
  // on every exit, also a failure half-way: the stream is drained before the level pool is handed out again
  struct PoolGuard {
    lcc_ctx* c;
    hipStream_t s;
    ~PoolGuard() {
      (void)hipStreamSynchronize(s);
      c->pool_reset();
    }
  } guard{ctx, st};
  const int64_t n = g->n;
  if (n == 0) {  // lambda is still checked (modularity is undefined without weight); one level, no cluster
    Score s0{};
    const char* why = "";
    lcc_status ls = graph_score(lam, 0, 0, R.o, &s0, &why);
    if (ls != LCC_OK) fail(ls, why);
    fill_result(res, 0, 0, s0.p, s0.q, 0, 0, false, 1, 0);
    if (R.o.trace) R.o.trace->count = 0;
    return LCC_OK;
  }
  R.lv.reserve((size_t)R.o.max_levels + 2);
  if (g->mem == LCC_MEM_HOST) {  // the optional per-vertex inputs follow the graph to the device
    auto up = [&](const int32_t* src) -> const int32_t* {
      if (!src) return nullptr;
      int32_t* d = take<int32_t>(ctx, n);
      hip_check(hipMemcpyAsync(d, src, (size_t)n * 4, hipMemcpyHostToDevice, st), "input copy");
      return d;
    };
    init_labels = up(init_labels);
    constraint = up(constraint);
  }
  setup(R, g, lam, init_labels);
  R.lv[0].B = const_cast<int32_t*>(constraint);
  if (variant == LCC_LOUVAIN || variant == LCC_PLEIDEN) R.use_pingpong(n, g->nnz);
  int top = 0;
  if (variant == LCC_LOUVAIN || variant == LCC_PLOUVAIN) top = R.louvain(variant == LCC_PLOUVAIN, init_labels);
  else top = R.leiden(variant == LCC_PLEIDEN_PLUS, init_labels);
  // final compaction on level 0 and the exact objective (Eq. 1) of the result
  Level& L0 = R.lv[0];
  int64_t nc = R.count_labels(L0.C, n);
  int32_t* lab = (g->mem == LCC_MEM_DEVICE) ? labels_out : R.w.in_labels;
  launch_map_labels(L0.C, R.w.rank, n, lab, st);
  launch_cluster_weights(lab, L0.g.vw, n, R.w.W, st);
  launch_objective(L0.g, L0.b, lab, R.w.W, R.w.ctrl, st);
  R.read_ctrl("objective");
  if (ctx->prof_mask) prof_resolve(ctx, ctx->h_ctrl);
  __int128 N = (__int128)R.q * ctx->h_ctrl->obj_I - (__int128)R.p * (ctx->h_ctrl->obj_SW2 - L0.sum_w2);
  if (g->mem == LCC_MEM_HOST) {
    hip_check(hipMemcpyAsync(labels_out, lab, (size_t)n * 4, hipMemcpyDeviceToHost, st), "labels");
    R.sync("labels");
  }
  const bool mod = g->vw_mode == LCC_VW_WEIGHTED_DEGREE && lam.over_total_weight;
  fill_result(res, nc, N, R.p, R.q, L0.sum_w2, R.W, mod, top + 1, R.flags);
  if (R.o.trace) {
    R.emit_pass_records();
    std::vector<int64_t> out;
    for (size_t r = 0; r + 8 <= R.trace.size(); r += 8) {
      if (R.trace[r] != -1) {
        out.insert(out.end(), R.trace.begin() + r, R.trace.begin() + r + 8);
        continue;
      }
      const int lvl = (int)R.trace[r + 1], ph = (int)R.trace[r + 2], s = (int)R.trace[r + 4];
      const LMSlot& S = ctx->h_slots[s];
      for (int i = 1; i <= R.o.pass_limit; ++i) {
        int64_t Ni = R.q * S.I[i] - R.p * (S.SW2[i] - R.lv[lvl].sum_w2);
        int64_t rr[8] = {1, lvl, ph, i, S.nL[i], S.nM[i], Ni, 0};
        out.insert(out.end(), rr, rr + 8);
      }
    }
    lcc_trace* tr = R.o.trace;
    int64_t cnt = (int64_t)out.size() / 8;
    tr->count = cnt;
    if (tr->records) memcpy(tr->records, out.data(), (size_t)std::min(cnt, tr->capacity) * 64);
  }
  return LCC_OK;
}

// ---------------------------------------------------------------------------------------------------------
// Batched form: several device-resident graphs clustered in one pass over their union (Louvain / Louvain+).
// Graph k's vertices occupy ids [vb[k], vb[k+1]) and its entries [eb[k], eb[k+1]) of the union CSR.
// ---------------------------------------------------------------------------------------------------------
struct GDesc {
  const void* off;
  const int32_t* idx;
  const int32_t* w;
  const int64_t* vw;
  int64_t n, nnz, vb, eb;
  int32_t bits, mode;
};

// largest k < G with key(k) <= x (graphs with no vertices / entries are skipped naturally)
__device__ __forceinline__ int64_t find_graph(const GDesc* d, int64_t G, int64_t x, bool edges) {
  int64_t lo = 0, hi = G;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if ((edges ? d[mid].eb : d[mid].vb) <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t off_at(const GDesc& g, int64_t i) {
  return g.bits == 64 ? ((const int64_t*)g.off)[i] : (int64_t)((const int32_t*)g.off)[i];
}

__global__ void k_union_vertices(const GDesc* d, int64_t G, int64_t N, int64_t E, int64_t* off, int32_t* gid,
                                 int64_t* vwg, Ctrl* ctrl) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) off[N] = E;
  for (int64_t v = t0; v < N; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = find_graph(d, G, v, false);
    const GDesc& g = d[k];
    const int64_t vl = v - g.vb;
    const int64_t a = off_at(g, vl), b = off_at(g, vl + 1);
    if (b < a || (vl == 0 && a != 0) || (vl == g.n - 1 && b != g.nnz)) atomicOr(&ctrl->err_bits, ERRB_INVALID);
    off[v] = g.eb + a;
    gid[v] = (int32_t)k;
    if (g.mode == LCC_VW_GIVEN) vwg[v] = g.vw[vl];
  }
}

__global__ void k_union_edges(const GDesc* d, int64_t G, int64_t E, int32_t* idx, int32_t* w) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = find_graph(d, G, j, true);
    const GDesc& g = d[k];
    const int64_t jl = j - g.eb;
    const int32_t u = g.idx[jl];
    idx[j] = (u >= 0 && u < g.n) ? (int32_t)(g.vb + u) : -1;  // -1 fails the row validation
    w[j] = g.w ? g.w[jl] : 1;
  }
}

// labels_out[k][v - vb[k]] = compact label of v within graph k
__global__ void k_write_labels_seg(const int32_t* C, const int32_t* rank, const int32_t* gid, const int32_t* vbase,
                                   int32_t* const* outs, int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = gid[v];
    const int32_t b = vbase[k];
    outs[k][v - b] = rank[C[v]] - rank[b];
  }
}

bool leiden_family(lcc_variant v) { return v == LCC_PLEIDEN || v == LCC_PLEIDEN_PLUS; }

// graphs of one family (Louvain / Louvain+ or pLeiden / pLeiden+), untraced, whose union fits 32-bit vertex
// ids and 32-bit entry positions
bool fusable(const lcc_graph* gs, const lcc_variant* variants, int64_t count, const lcc_options* opts) {
  if (count < 2 || (opts && opts->trace)) return false;
  int64_t n = 0, e = 0;
  for (int64_t i = 0; i < count; ++i) {
    if (variants[i] < LCC_LOUVAIN || variants[i] > LCC_PLEIDEN_PLUS) return false;
    if (leiden_family(variants[i]) != leiden_family(variants[0])) return false;
    n += gs[i].n;
    e += gs[i].nnz;
  }
  return n < 2147483647LL && e < 2147483647LL;
}

lcc_status cluster_batch_fused(lcc_ctx* ctx, const lcc_graph* gs, const lcc_lambda* lams, const lcc_variant* variants,
                               int64_t G, const lcc_options* opts, void* stream, int32_t* const* labels_out,
                               lcc_result* res) {
  for (int64_t i = 0; i < G; ++i) {
    check_graph_args(&gs[i]);
    if (gs[i].n == 0 && gs[i].nnz != 0) fail(LCC_ERR_INVALID, "a graph without vertices has entries");
    if (gs[i].n > 0 && !labels_out[i]) fail(LCC_ERR_INVALID, "labels_out is NULL");
    if (variants[i] < LCC_LOUVAIN || variants[i] > LCC_PLEIDEN_PLUS) fail(LCC_ERR_INVALID, "unknown variant");
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  hip_check(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  Run R(ctx, st);
  if (opts) R.o = *opts; else default_opts(&R.o);
  check_opts(R.o);
  R.o.trace = nullptr;
  std::vector<int64_t> vb((size_t)G + 1, 0), eb((size_t)G + 1, 0);
  for (int64_t i = 0; i < G; ++i) { vb[i + 1] = vb[i] + gs[i].n; eb[i + 1] = eb[i] + gs[i].nnz; }
  const int64_t n = vb[G], nnz = eb[G];
  if (n == 0) {
    std::vector<Score> s0((size_t)G);
    for (int64_t i = 0; i < G; ++i) {
      const char* why = "";
      lcc_status ls = graph_score(lams[i], 0, 0, R.o, &s0[i], &why);
      if (ls != LCC_OK) fail(ls, std::string("graph ") + std::to_string(i) + ": " + why);
    }
    for (int64_t i = 0; i < G; ++i) fill_result(&res[i], 0, 0, s0[i].p, s0[i].q, 0, 0, false, 1, 0);
    return LCC_OK;
  }
  ctx->ensure_ws(n, nnz, st);
  ctx->pool_reset();
  // on every exit, also a failure half-way: the stream is drained before the level pool is handed out again
  struct PoolGuard {
    lcc_ctx* c;
    hipStream_t s;
    ~PoolGuard() {
      (void)hipStreamSynchronize(s);
      c->pool_reset();
    }
  } guard{ctx, st};
  WS& w = R.w;
  R.G = G;
  const bool leiden = leiden_family(variants[0]);
  // a Leiden graph may repeat each of its levels twice (no-progress retries): up to 3 union levels per level
  R.lv.reserve((size_t)(leiden ? 3 : 1) * R.o.max_levels + 2);
  // per-graph device arrays
  R.d_score = take<Score>(ctx, G);
  R.gI = take<int64_t>(ctx, (MAX_PASSES + 1) * G);
  R.gSW2 = take<int64_t>(ctx, (MAX_PASSES + 1) * G);
  R.gNbest = take<int64_t>(ctx, G);
  R.gN0 = take<int64_t>(ctx, G);
  R.gcopy = take<int32_t>(ctx, G);
  R.gact = take<uint8_t>(ctx, G);
  R.gtmp = take<int32_t>(ctx, G + 1);
  int8_t* gmode = take<int8_t>(ctx, G);
  GDesc* d_desc = take<GDesc>(ctx, G);
  int64_t* gW = take<int64_t>(ctx, 3 * G);  // W, W_E, sum w^2 per graph
  std::vector<GDesc> desc((size_t)G);
  std::vector<int8_t> hmode((size_t)G);
  bool any_given = false;
  std::vector<int32_t*> dev_out(labels_out, labels_out + G);  // host graphs: labels staged on the device
  for (int64_t i = 0; i < G; ++i) {
    const lcc_graph& g = gs[i];
    desc[i] = GDesc{g.offsets, g.indices, g.edge_w, g.vertex_w, g.n, g.nnz, vb[i], eb[i], g.offsets_bits,
                    (int32_t)g.vw_mode};
    if (g.mem == LCC_MEM_HOST && g.n > 0) {  // stage the graph's arrays in device memory
      auto up = [&](const void* src, size_t bytes) -> void* {
        void* d = ctx->pool_take(bytes);
        hip_check(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, st), "input copy");
        return d;
      };
      desc[i].off = up(g.offsets, (size_t)(g.n + 1) * (g.offsets_bits / 8));
      if (g.nnz) desc[i].idx = (const int32_t*)up(g.indices, (size_t)g.nnz * 4);
      if (g.nnz && g.edge_w) desc[i].w = (const int32_t*)up(g.edge_w, (size_t)g.nnz * 4);
      if (g.vw_mode == LCC_VW_GIVEN) desc[i].vw = (const int64_t*)up(g.vertex_w, (size_t)g.n * 8);
      dev_out[i] = take<int32_t>(ctx, g.n);
    }
    hmode[i] = (int8_t)g.vw_mode;
    any_given = any_given || g.vw_mode == LCC_VW_GIVEN;
  }
  hip_check(hipMemcpyAsync(d_desc, desc.data(), sizeof(GDesc) * G, hipMemcpyHostToDevice, st), "descriptors");
  hip_check(hipMemcpyAsync(gmode, hmode.data(), (size_t)G, hipMemcpyHostToDevice, st), "modes");
  // level 0: the union CSR in the workspace
  Level L0;
  L0.g.n = n;
  L0.g.nnz = nnz;
  L0.g.off = w.in_off;
  L0.g.idx = w.in_idx;
  L0.g.w = w.in_w;
  L0.g.vw = w.vw0;
  L0.gid = w.gid0;
  L0.vbase = take<int32_t>(ctx, G + 1);
  L0.hvb.resize((size_t)G + 1);
  for (int64_t i = 0; i <= G; ++i) L0.hvb[i] = (int32_t)vb[i];
  hip_check(hipMemcpyAsync(L0.vbase, L0.hvb.data(), (size_t)(G + 1) * 4, hipMemcpyHostToDevice, st), "vbase");
  L0.C = take<int32_t>(ctx, n);
  zero_bytes(w.ctrl, sizeof(Ctrl), st);
  k_union_vertices<<<grid1(n), BLOCK, 0, st>>>(d_desc, G, n, nnz, w.in_off, w.gid0, w.in_vwg, w.ctrl);
  if (nnz) k_union_edges<<<grid1(nnz), BLOCK, 0, st>>>(d_desc, G, nnz, w.in_idx, w.in_w);
  R.read_ctrl("union");
  if (ctx->h_ctrl->err_bits & ERRB_INVALID) fail(LCC_ERR_INVALID, "CSR offsets of a graph are not a valid row partition");
  R.lv.push_back(L0);
  Level& L = R.lv[0];
  {
    k_reset_level_counters<<<1, 1, 0, st>>>(w.ctrl);
    launch_buckets(L.g.off, n, w.list0, w.ctrl, ctx->bounds(), st);
    R.read_ctrl("buckets");
    Buckets& b = L.b;
    b.list = w.list0;
    for (int k = 0; k < NBUCKET; ++k) {
      b.count[k] = ctx->h_ctrl->bucket_count[k];
      b.off[k] = ctx->h_ctrl->bucket_off[k];
      b.edges[k] = ctx->h_ctrl->bucket_edges[k];
    }
    b.off[NBUCKET] = ctx->h_ctrl->bucket_off[NBUCKET];
    b.hub_chunks = ctx->h_ctrl->count3;
    b.hub_chunk_off = w.hub_off0;
    b.hub_ps = w.hub_ps; b.hub_pc = w.hub_pc; b.hub_pown = w.hub_pown; b.hub_acc = w.hub_acc; b.stripes = w.stripes;
    b.grid_cap = ctx->tune.grid_cap;
    b.hub_deg = ctx->tune.bucket_max[NBUCKET - 2];
    b.hash_shift = ctx->tune.hash_shift;
    b.count6_hi = ctx->h_ctrl->bucket6_hi;
    if (b.count[NBUCKET - 1])
      launch_hub_chunks(w.list0 + b.off[NBUCKET - 1], b.count[NBUCKET - 1], L.g.off, w.hub_cnt, w.hub_off0, w.scan_temp, st);
  }
  const auto sym_mark = ctx->pool_mark();  // the symmetry check's sort scratch is released below
  SymBuffers sb;
  int64_t max_nnz = 0;
  for (int64_t i = 0; i < G; ++i) max_nnz = std::max(max_nnz, gs[i].nnz);
  if (R.o.validate && (max_nnz <= SYM_SEARCH_MAX_NNZ || nnz <= SYM_SEARCH_MAX_AVG_DEG * n)) {
    sb.search = true;  // every graph's rows are local: the searches stay in cache
  } else if (R.o.validate) {
    sb.k0 = w.k0; sb.v0 = w.v0; sb.k1 = w.k1; sb.v1 = w.v1;
    sb.lo = w.cnt; sb.lbase = w.seg0; sb.scan_temp = w.scan_temp;
    sb.temp = ctx->pool_take(radix_temp_bytes(nnz));
  }
  launch_validate_rows(L.g, L.b, LCC_VW_UNIT, any_given ? w.in_vwg : nullptr, w.vw0, w.ctrl, st, sb, w.gid0, gmode,
                       w.t64b);
  launch_seg_sum(w.vw0, 0, L.vbase, G, gW, st);
  launch_seg_sum(w.t64b, 0, L.vbase, G, gW + G, st);
  L.sumw2g = gW + 2 * G;
  launch_seg_sum(w.vw0, 1, L.vbase, G, L.sumw2g, st);
  std::vector<int64_t> hW((size_t)(3 * G));
  hip_check(hipMemcpyAsync(hW.data(), gW, sizeof(int64_t) * 3 * G, hipMemcpyDeviceToHost, st), "graph sums");
  R.read_ctrl("validate rows");
  ctx->pool_release(sym_mark);
  const Ctrl& c = *ctx->h_ctrl;
  uint32_t e = c.err_bits;
  if (!R.o.validate) e &= ERRB_INVALID | ERRB_VW_TOO_BIG;
  if (e & ERRB_INVALID) fail(LCC_ERR_INVALID, "neighbour index out of range in a graph of the batch");
  if (e & ERRB_SELF_LOOP) fail(LCC_ERR_SELF_LOOP, "a row contains its own vertex");
  if (e & ERRB_UNSORTED) fail(LCC_ERR_UNSORTED, "a row is not strictly ascending");
  if (e & ERRB_WEIGHT) fail(LCC_ERR_WEIGHT, "an edge weight <= 0 or a vertex weight < 0");
  if ((e & ERRB_NOT_SYMMETRIC) || (sb.search && c.count0 != 0))
    fail(LCC_ERR_NOT_SYMMETRIC, "a graph of the batch is not symmetric");
  if (e & ERRB_VW_TOO_BIG) fail(LCC_ERR_OVERFLOW, "a vertex weight >= 2^31");
  std::vector<Score> sc((size_t)G);
  for (int64_t i = 0; i < G; ++i) {
    const char* why = "";
    lcc_status s = graph_score(lams[i], (uint64_t)hW[i], (uint64_t)hW[G + i], R.o, &sc[i], &why);
    if (s != LCC_OK) fail(s, std::string("graph ") + std::to_string(i) + ": " + why);
  }
  hip_check(hipMemcpyAsync(R.d_score, sc.data(), sizeof(Score) * G, hipMemcpyHostToDevice, st), "scores");
  // the method
  std::vector<uint8_t> plus((size_t)G);
  for (int64_t i = 0; i < G; ++i) plus[i] = variants[i] == LCC_PLOUVAIN || variants[i] == LCC_PLEIDEN_PLUS;
  std::vector<int> top((size_t)G, 0), levels((size_t)G, 1);
  std::vector<uint32_t> gflags((size_t)G, 0);
  if (leiden) {
    R.leiden_seg(plus, top, levels, gflags);
  } else {
    R.louvain_seg(plus, top, gflags);
    for (int64_t i = 0; i < G; ++i) levels[i] = top[i] + 1;
  }
  // per-graph compact labels and exact objective (Eq. 1) on level 0
  Level& F = R.lv[0];
  launch_label_rank(F.C, n, w.used, w.rank, w.scan_temp, st);
  int32_t** d_outs = take<int32_t*>(ctx, G);
  hip_check(hipMemcpyAsync(d_outs, dev_out.data(), sizeof(int32_t*) * G, hipMemcpyHostToDevice, st), "outputs");
  k_write_labels_seg<<<grid1(n), BLOCK, 0, st>>>(F.C, w.rank, F.gid, F.vbase, d_outs, n);
  launch_rebase(w.rank, F.vbase, G, R.gtmp, st);
  launch_cluster_weights(F.C, F.g.vw, n, w.W, st);
  launch_internal_per_vertex(F.g, F.b, F.C, w.t64a, st);
  int64_t* gobj = take<int64_t>(ctx, 2 * G);
  launch_seg_sum(w.t64a, 0, F.vbase, G, gobj, st);
  launch_seg_sum(w.W, 1, F.vbase, G, gobj + G, st);
  std::vector<int64_t> ho((size_t)(2 * G));
  std::vector<int32_t> hr((size_t)G + 1);
  hip_check(hipMemcpyAsync(ho.data(), gobj, sizeof(int64_t) * 2 * G, hipMemcpyDeviceToHost, st), "objective");
  hip_check(hipMemcpyAsync(hr.data(), R.gtmp, sizeof(int32_t) * (G + 1), hipMemcpyDeviceToHost, st), "counts");
  for (int64_t i = 0; i < G; ++i)
    if (gs[i].mem == LCC_MEM_HOST && gs[i].n > 0)
      hip_check(hipMemcpyAsync(labels_out[i], dev_out[i], (size_t)gs[i].n * 4, hipMemcpyDeviceToHost, st), "labels");
  R.sync("batch result");
  for (int64_t i = 0; i < G; ++i) {
    if (gs[i].n == 0) {
      fill_result(&res[i], 0, 0, sc[i].p, sc[i].q, 0, 0, false, 1, 0);
      continue;
    }
    const __int128 N = (__int128)sc[i].q * ho[i] - (__int128)sc[i].p * (ho[G + i] - hW[2 * G + i]);
    const bool mod = gs[i].vw_mode == LCC_VW_WEIGHTED_DEGREE && lams[i].over_total_weight;
    fill_result(&res[i], hr[i + 1] - hr[i], N, sc[i].p, sc[i].q, hW[2 * G + i], (uint64_t)hW[i], mod, levels[i],
                gflags[i]);
  }
  return LCC_OK;
}

template <typename F>
lcc_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LCC_ERR_OOM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return LCC_ERR_DEVICE;
  }
}

}  // namespace

// =========================================================================================================
// C-ABI
// =========================================================================================================
extern "C" {

lcc_status lcc_create(int device, lcc_alloc_fn alloc, lcc_free_fn free_fn, void* user, lcc_ctx** out) {
  return guarded([&]() -> lcc_status {
    if (!out) fail(LCC_ERR_INVALID, "out is NULL");
    if ((alloc == nullptr) != (free_fn == nullptr)) fail(LCC_ERR_INVALID, "alloc and free must both be set");
    int ndev = 0;
    hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) fail(LCC_ERR_INVALID, "no such device");
    hip_check(hipSetDevice(device), "hipSetDevice");
    if (device < MAX_DEVICES) {  // the no-allocation scratch's address on this device (its call reports errors)
      hipError_t e = hipSuccess;
      (void)scratch_address(device, &e);
    }
    lcc_ctx* c = new lcc_ctx();
    c->device = device;
    c->alloc = alloc;
    c->freef = free_fn;
    c->user = user;
    if (hipHostMalloc((void**)&c->h_ctrl, sizeof(Ctrl)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_slots, sizeof(LMSlot) * NSLOT) != hipSuccess) {
      if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
      if (c->h_slots) (void)hipHostFree(c->h_slots);
      delete c;
      fail(LCC_ERR_DEVICE, "pinned host allocation failed");
    }
    *out = c;
    return LCC_OK;
  });
}

lcc_status lcc_destroy(lcc_ctx* ctx) {
  return guarded([&]() -> lcc_status {
    if (!ctx) return LCC_OK;
    {
      std::lock_guard<std::mutex> lock(ctx->mu);
      (void)hipSetDevice(ctx->device);
      (void)hipDeviceSynchronize();
      ctx->dfree(ctx->ws_base);
      for (auto& c : ctx->pool.chunks) ctx->dfree(c.p);
      ctx->pool.chunks.clear();
      if (ctx->h_ctrl) (void)hipHostFree(ctx->h_ctrl);
      if (ctx->h_slots) (void)hipHostFree(ctx->h_slots);
      for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    }
    delete ctx;
    return LCC_OK;
  });
}

void lcc_default_options(lcc_options* opts) {
  if (opts) default_opts(opts);
}

lcc_status lcc_workspace_bytes(int64_t n, int64_t nnz, lcc_variant variant, size_t* bytes) {
  return guarded([&]() -> lcc_status {
    if (!bytes || n < 0 || nnz < 0) fail(LCC_ERR_INVALID, "bad arguments");
    if (variant < LCC_LOUVAIN || variant > LCC_PLEIDEN_PLUS) fail(LCC_ERR_INVALID, "unknown variant");
    *bytes = call_bytes(n, nnz, variant);
    return LCC_OK;
  });
}

lcc_status lcc_cluster(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                       const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res) {
  return guarded([&]() { return cluster_impl(ctx, g, lambda, variant, opts, stream, labels_out, res, nullptr); });
}

lcc_status lcc_cluster_noalloc(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                               const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res) {
  return guarded([&]() {
    return cluster_impl(ctx, g, lambda, variant, opts, stream, labels_out, res, nullptr, nullptr, true);
  });
}

lcc_status lcc_cluster_batch(lcc_ctx* ctx, const lcc_graph* gs, const lcc_lambda* lambdas,
                             const lcc_variant* variants, int64_t count, const lcc_options* opts, void* stream,
                             int32_t* const* labels_out, lcc_result* res) {
  return guarded([&]() -> lcc_status {
    if (count < 0 || (count > 0 && (!gs || !lambdas || !variants || !labels_out || !res)))
      fail(LCC_ERR_INVALID, "bad batch arguments");
    if (!ctx) fail(LCC_ERR_INVALID, "context is NULL");
    if (fusable(gs, variants, count, opts))
      return cluster_batch_fused(ctx, gs, lambdas, variants, count, opts, stream, labels_out, res);
    for (int64_t i = 0; i < count; ++i) {
      lcc_status s = cluster_impl(ctx, &gs[i], lambdas[i], variants[i], opts, stream, labels_out[i], &res[i], nullptr);
      if (s != LCC_OK) return s;
    }
    return LCC_OK;
  });
}

void lcc_default_tuning(lcc_tuning* t) {
  if (t) *t = initial_tuning();
}

lcc_status lcc_set_tuning(lcc_ctx* ctx, const lcc_tuning* t) {
  return guarded([&]() -> lcc_status {
    if (!ctx || !t) fail(LCC_ERR_INVALID, "bad arguments");
    for (int k = 0; k < NBUCKET - 1; ++k) {
      if (t->bucket_max[k] < 0 || t->bucket_max[k] > BUCKET_CAP[k])
        fail(LCC_ERR_INVALID, "bucket bound " + std::to_string(k) + " outside [0, " + std::to_string(BUCKET_CAP[k]) + "]");
      if (k > 0 && t->bucket_max[k] < t->bucket_max[k - 1]) fail(LCC_ERR_INVALID, "bucket bounds must not decrease");
    }
    if (t->grid_cap < 64 || t->grid_cap > 65536) fail(LCC_ERR_INVALID, "grid_cap outside [64, 65536]");
    if (t->hash_shift < 0 || t->hash_shift > 2) fail(LCC_ERR_INVALID, "hash_shift outside [0, 2]");
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->tune = *t;
    return LCC_OK;
  });
}

lcc_status lcc_get_tuning(lcc_ctx* ctx, lcc_tuning* t) {
  return guarded([&]() -> lcc_status {
    if (!ctx || !t) fail(LCC_ERR_INVALID, "bad arguments");
    std::lock_guard<std::mutex> lock(ctx->mu);
    *t = ctx->tune;
    return LCC_OK;
  });
}

lcc_status lcc_autotune(lcc_ctx* ctx, const lcc_graph* gs, const lcc_lambda* lambdas, const lcc_variant* variants,
                        int64_t count, const lcc_options* opts, void* stream, int32_t trials, lcc_tuning* best,
                        double* best_ms) {
  lcc_tuning start{};
  bool started = false;
  lcc_status st = guarded([&]() -> lcc_status {
    if (!ctx || !gs || !lambdas || !variants || !best || count < 1 || trials < 1)
      fail(LCC_ERR_INVALID, "bad autotune arguments");
    {
      std::lock_guard<std::mutex> lock(ctx->mu);
      start = ctx->tune;
      started = true;
    }
    // label scratch in each graph's memory space
    std::vector<int32_t*> outs((size_t)count);
    std::vector<std::vector<int32_t>> host_out((size_t)count);
    std::vector<lcc_result> res((size_t)count);
    int64_t dev_n = 0;
    for (int64_t i = 0; i < count; ++i)
      if (gs[i].mem == LCC_MEM_DEVICE) dev_n += std::max<int64_t>(gs[i].n, 1);
    int32_t* dev = dev_n ? (int32_t*)ctx->dalloc((size_t)dev_n * 4) : nullptr;
    struct Free { lcc_ctx* c; void* p; ~Free() { if (p) { (void)hipDeviceSynchronize(); c->dfree(p); } } } fr{ctx, dev};
    for (int64_t i = 0, o = 0; i < count; ++i) {
      if (gs[i].mem == LCC_MEM_DEVICE) {
        outs[(size_t)i] = dev + o;
        o += std::max<int64_t>(gs[i].n, 1);
      } else {
        host_out[(size_t)i].resize((size_t)std::max<int64_t>(gs[i].n, 1));
        outs[(size_t)i] = host_out[(size_t)i].data();
      }
    }
    auto run = [&](const lcc_tuning& t) -> double {
      {
        std::lock_guard<std::mutex> lock(ctx->mu);
        ctx->tune = t;
      }
      double ms = 0;
      for (int r = 0; r <= trials; ++r) {  // run 0 is the warm-up
        auto t0 = std::chrono::steady_clock::now();
        lcc_status s = count == 1 ? lcc_cluster(ctx, &gs[0], lambdas[0], variants[0], opts, stream, outs[0], &res[0])
                                  : lcc_cluster_batch(ctx, gs, lambdas, variants, count, opts, stream, outs.data(),
                                                      res.data());
        if (s != LCC_OK) fail(s, std::string("autotune run: ") + (lcc_last_error() ? lcc_last_error() : ""));
        double d = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (r == 1 || (r > 1 && d < ms)) ms = d;
      }
      return ms;
    };
    lcc_tuning cur = start, win = start;
    double win_ms = run(start);
    for (int32_t cap : {1024, 2048, 4096}) {  // workgroup caps with the current bounds
      if (cap == start.grid_cap) continue;
      lcc_tuning t = start;
      t.grid_cap = cap;
      double ms = run(t);
      if (ms < win_ms) { win_ms = ms; win = t; }
    }
    cur = win;
    // bucket layouts: each moves one class of rows to a bucket of larger capacity
    static const int64_t layouts[][NBUCKET - 1] = {
        {4, 8, 16, 32, 128, 1024, 8192},   // the default
        {0, 8, 16, 32, 128, 1024, 8192},   // no 4-lane groups
        {4, 8, 16, 16, 128, 1024, 8192},   // no 32-lane groups: degrees 17-32 to a wavefront
        {4, 8, 16, 32, 64, 1024, 8192},    // wavefront hash only up to degree 64
        {4, 8, 16, 32, 128, 512, 8192},    // the 8192-slot workgroups from degree 513
        {4, 8, 16, 32, 128, 1024, 4096},   // no 16384-slot workgroups: hub chunks from degree 4097
        {4, 8, 16, 32, 128, 1024, 2048},   // hub chunks from degree 2049
        {4, 8, 16, 32, 128, 1024, 1024},   // no 8192-slot workgroups: hub chunks from degree 1025
    };
    for (const auto& lay : layouts) {
      lcc_tuning t = cur;
      bool same = true;
      for (int k = 0; k < NBUCKET - 1; ++k) {
        same = same && t.bucket_max[k] == lay[k];
        t.bucket_max[k] = lay[k];
      }
      if (same) continue;
      double ms = run(t);
      if (ms < win_ms) { win_ms = ms; win = t; }
    }
    cur = win;
    for (int32_t hs = 0; hs <= 2; ++hs) {  // LDS hash sizes with the best layout
      if (hs == cur.hash_shift) continue;
      lcc_tuning t = cur;
      t.hash_shift = hs;
      double ms = run(t);
      if (ms < win_ms) { win_ms = ms; win = t; }
    }
    {
      std::lock_guard<std::mutex> lock(ctx->mu);
      ctx->tune = win;
    }
    *best = win;
    if (best_ms) *best_ms = win_ms;
    return LCC_OK;
  });
  if (st != LCC_OK && started) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->tune = start;
  }
  return st;
}

lcc_status lcc_objective_device(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lam, const int32_t* labels,
                                void* stream, lcc_result* res) {
  return guarded([&]() -> lcc_status {
    if (!ctx || !res) fail(LCC_ERR_INVALID, "bad arguments");
    check_graph_args(g);
    if (g->n > 0 && !labels) fail(LCC_ERR_INVALID, "labels is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    Run R(ctx, st);
    default_opts(&R.o);
    ctx->ensure_ws(g->n, g->nnz, st);
    ctx->pool_reset();
    // on every exit, also a failure half-way: the stream is drained before the level pool is handed out again
  struct PoolGuard {
    lcc_ctx* c;
    hipStream_t s;
    ~PoolGuard() {
      (void)hipStreamSynchronize(s);
      c->pool_reset();
    }
  } guard{ctx, st};
    if (g->n == 0) {
      fill_result(res, 0, 0, 0, 1, 0, 0, false, 0, 0);
      return LCC_OK;
    }
    const int32_t* lab = labels;
    if (g->mem == LCC_MEM_HOST) {
      hip_check(hipMemcpyAsync(R.w.in_labels, labels, (size_t)g->n * 4, hipMemcpyHostToDevice, st), "labels");
      lab = R.w.in_labels;
    }
    R.lv.reserve(2);
    setup(R, g, lam, lab);
    Level& L0 = R.lv[0];
    int64_t nc = R.count_labels(lab, g->n);
    launch_cluster_weights(lab, L0.g.vw, g->n, R.w.W, st);
    launch_objective(L0.g, L0.b, lab, R.w.W, R.w.ctrl, st);
    R.read_ctrl("objective");
    __int128 N = (__int128)R.q * ctx->h_ctrl->obj_I - (__int128)R.p * (ctx->h_ctrl->obj_SW2 - L0.sum_w2);
    const bool mod = g->vw_mode == LCC_VW_WEIGHTED_DEGREE && lam.over_total_weight;
    fill_result(res, nc, N, R.p, R.q, L0.sum_w2, R.W, mod, 1, 0);
    return LCC_OK;
  });
}

// Eq. 1 of a given clustering of a host graph, evaluated on the host in 128-bit integers.  It scores labels from
// any source and takes no part in the clustering calls.  The graph passes the same checks as for clustering,
// in the same order (offsets, rows, weights, symmetry); then the labels, lambda and the bound.
lcc_status lcc_objective(const lcc_graph* g, lcc_lambda lam, const int32_t* labels, lcc_result* res) {
  return guarded([&]() -> lcc_status {
    typedef unsigned __int128 u128;
    if (!res) fail(LCC_ERR_INVALID, "res is NULL");
    check_graph_args(g);
    if (g->mem != LCC_MEM_HOST) fail(LCC_ERR_INVALID, "lcc_objective takes a host graph (device graphs: lcc_objective_device)");
    const int64_t n = g->n, nnz = g->nnz;
    if (n > 0 && !labels) fail(LCC_ERR_INVALID, "labels is NULL");
    if (n == 0 && nnz == 0) {  // the empty clustering of the empty graph, as on the device
      fill_result(res, 0, 0, 0, 1, 0, 0, false, 0, 0);
      return LCC_OK;
    }
    const int64_t* o64 = g->offsets_bits == 64 ? (const int64_t*)g->offsets : nullptr;
    const int32_t* o32 = g->offsets_bits == 32 ? (const int32_t*)g->offsets : nullptr;
    auto off = [&](int64_t v) -> int64_t { return o64 ? o64[v] : (int64_t)o32[v]; };
    const int32_t* idx = g->indices;
    auto wt = [&](int64_t j) -> int64_t { return g->edge_w ? (int64_t)g->edge_w[j] : 1; };
    if (off(0) != 0 || off(n) != nnz) fail(LCC_ERR_INVALID, "offsets[0] != 0 or offsets[n] != nnz");
    for (int64_t v = 0; v < n; ++v)
      if (off(v + 1) < off(v)) fail(LCC_ERR_INVALID, "offsets decrease");
    for (int64_t v = 0; v < n; ++v)
      for (int64_t j = off(v); j < off(v + 1); ++j)
        if (idx[j] < 0 || idx[j] >= n) fail(LCC_ERR_INVALID, "neighbour index out of range");
    for (int64_t v = 0; v < n; ++v)
      for (int64_t j = off(v); j < off(v + 1); ++j) {
        if (idx[j] == v) fail(LCC_ERR_SELF_LOOP, "self-loop");
        if (j > off(v) && idx[j - 1] >= idx[j]) fail(LCC_ERR_UNSORTED, "row not strictly ascending");
      }
    for (int64_t j = 0; j < nnz; ++j)
      if (wt(j) <= 0) fail(LCC_ERR_WEIGHT, "edge weight <= 0");
    if (g->vw_mode == LCC_VW_GIVEN)
      for (int64_t v = 0; v < n; ++v)
        if (g->vertex_w[v] < 0) fail(LCC_ERR_WEIGHT, "vertex weight < 0");
    // every entry (v, u, w) has its reverse (u, v, w): binary search of v in the sorted row u
    for (int64_t v = 0; v < n; ++v)
      for (int64_t j = off(v); j < off(v + 1); ++j) {
        const int32_t u = idx[j];
        const int32_t* b = idx + off(u);
        const int32_t* e = idx + off(u + 1);
        const int32_t* f = std::lower_bound(b, e, (int32_t)v);
        if (f == e || *f != v || wt(f - idx) != wt(j)) fail(LCC_ERR_NOT_SYMMETRIC, "graph not symmetric");
      }
    for (int64_t v = 0; v < n; ++v)
      if (labels[v] < 0 || labels[v] >= n) fail(LCC_ERR_INVALID, "label outside [0, n)");
    // vertex weights; W < 2^63 keeps every square below 2^126
    std::vector<int64_t> vw((size_t)n);
    u128 W = 0, WE = 0;
    for (int64_t v = 0; v < n; ++v) {
      int64_t x = 1;
      if (g->vw_mode == LCC_VW_GIVEN) x = g->vertex_w[v];
      if (g->vw_mode == LCC_VW_WEIGHTED_DEGREE) {
        x = 0;
        for (int64_t j = off(v); j < off(v + 1); ++j) x += wt(j);
      }
      vw[(size_t)v] = x;
      W += (u128)x;
    }
    for (int64_t j = 0; j < nnz; ++j) WE += (u128)wt(j);
    const u128 LIM = (u128)1 << 126;
    if (W >> 63) fail(LCC_ERR_OVERFLOW, "total vertex weight >= 2^63");
    // lambda = p / q in lowest terms
    if (lam.den == 0) fail(LCC_ERR_LAMBDA, "lambda denominator is zero");
    u128 P = lam.num, Q = (u128)lam.den * (lam.over_total_weight ? W : 1);
    if (Q == 0 || P > Q) fail(LCC_ERR_LAMBDA, "lambda outside [0, 1] or undefined");
    if (P == 0) {
      Q = 1;
    } else {
      u128 a = P, b = Q;
      while (b) { u128 t = a % b; a = b; b = t; }
      P /= a;
      Q /= a;
    }
    if (Q >> 64) fail(LCC_ERR_OVERFLOW, "lambda denominator >= 2^64");
    // |N| <= q W_E + p W^2 < 2^126
    const u128 qWE = Q * WE, W2 = W * W;
    if (qWE >= LIM || (P && W2 > (LIM - 1 - qWE) / P)) fail(LCC_ERR_OVERFLOW, "q W_E + p W^2 >= 2^126");
    std::vector<uint64_t> Wc((size_t)n, 0);
    std::vector<uint8_t> seen((size_t)n, 0);
    int64_t nc = 0;
    u128 sum_w2 = 0;
    for (int64_t v = 0; v < n; ++v) {
      Wc[(size_t)labels[v]] += (uint64_t)vw[(size_t)v];
      sum_w2 += (u128)vw[(size_t)v] * (u128)vw[(size_t)v];
      if (!seen[(size_t)labels[v]]) { seen[(size_t)labels[v]] = 1; ++nc; }
    }
    u128 I = 0, SW2 = 0;
    for (int64_t v = 0; v < n; ++v)
      for (int64_t j = off(v); j < off(v + 1); ++j)
        if (labels[idx[j]] == labels[v]) I += (u128)wt(j);
    for (int64_t c = 0; c < n; ++c) SW2 += (u128)Wc[(size_t)c] * (u128)Wc[(size_t)c];
    const __int128 N = (__int128)(Q * I) - (__int128)(P * (SW2 - sum_w2));
    res->num_clusters = nc;
    res->obj_num_hi = (int64_t)(N >> 64);
    res->obj_num_lo = (uint64_t)N;
    res->obj_den = (uint64_t)Q;
    res->objective = (double)N / (double)Q;
    const bool mod = g->vw_mode == LCC_VW_WEIGHTED_DEGREE && lam.over_total_weight;
    res->modularity = mod && W > 0 ? (double)(N - (__int128)(P * sum_w2)) / ((double)Q * (double)W) : NAN;
    res->levels = 1;
    res->flags = 0;
    return LCC_OK;
  });
}

lcc_status lcc_profile_enable(lcc_ctx* ctx, uint64_t family_mask) {
  return guarded([&]() -> lcc_status {
    if (!ctx) fail(LCC_ERR_INVALID, "context is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->prof_mask = family_mask & ((1ull << PF_COUNT) - 1);
    return LCC_OK;
  });
}

lcc_status lcc_profile_read(lcc_ctx* ctx, lcc_kernel_stat* stats, int32_t capacity, int32_t* count, int32_t reset) {
  return guarded([&]() -> lcc_status {
    if (!ctx || !count || (capacity > 0 && !stats)) fail(LCC_ERR_INVALID, "bad arguments");
    std::lock_guard<std::mutex> lock(ctx->mu);
    int32_t k = 0;
    for (int f = 0; f < PF_COUNT; ++f) {
      if (k < capacity) {
        memset(&stats[k], 0, sizeof(stats[k]));
        snprintf(stats[k].name, sizeof(stats[k].name), "%s", PROF_NAMES[f]);
        stats[k].launches = ctx->prof_launches[f];
        stats[k].total_ms = ctx->prof_ms[f];
        stats[k].bytes = ctx->prof_bytes[f];
      }
      ++k;
      if (reset) { ctx->prof_launches[f] = 0; ctx->prof_ms[f] = 0; ctx->prof_bytes[f] = 0; }
    }
    *count = k;
    return LCC_OK;
  });
}

const char* lcc_status_string(lcc_status st) {
  switch (st) {
    case LCC_OK: return "ok";
    case LCC_ERR_INVALID: return "invalid argument or CSR structure";
    case LCC_ERR_NOT_SYMMETRIC: return "graph not symmetric";
    case LCC_ERR_SELF_LOOP: return "self-loop";
    case LCC_ERR_UNSORTED: return "row not strictly ascending";
    case LCC_ERR_WEIGHT: return "non-positive edge weight or negative vertex weight";
    case LCC_ERR_LAMBDA: return "lambda outside [0, 1] or undefined";
    case LCC_ERR_OVERFLOW: return "exactness bound exceeded";
    case LCC_ERR_OOM: return "out of device memory";
    case LCC_ERR_DEVICE: return "HIP runtime error";
    case LCC_ERR_BUSY: return "admission refused";
    case LCC_ERR_NOT_FOUND: return "unknown ticket";
  }
  return "unknown status";
}

const char* lcc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// Entry used by the server (server.hip): clustering with an initial clustering for pLeiden.
lcc_status lcc_cluster_ex(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                          const lcc_options* opts, void* stream, const int32_t* init_labels,
                          const int32_t* constraint, int32_t* labels_out, lcc_result* res) {
  return guarded([&]() {
    return cluster_impl(ctx, g, lambda, variant, opts, stream, labels_out, res, init_labels, constraint);
  });
}

lcc_status lcc_cluster_init_internal(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                                     const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res,
                                     const int32_t* init) {
  return guarded([&]() { return cluster_impl(ctx, g, lambda, variant, opts, stream, labels_out, res, init); });
}

int lcc_ctx_device_internal(const lcc_ctx* ctx) { return ctx->device; }

// Returns the context's workspace and level pool to its allocator (the next call allocates them again).  No
// call of the context may be running; its last call drained its stream before returning.
void lcc_ctx_release_internal(lcc_ctx* ctx) {
  std::lock_guard<std::mutex> lock(ctx->mu);
  (void)hipSetDevice(ctx->device);
  ctx->dfree(ctx->ws_base);
  ctx->ws_base = nullptr;
  ctx->ws_bytes = 0;
  ctx->ws_n = ctx->ws_nnz = -1;
  ctx->w = WS{};
  for (auto& c : ctx->pool.chunks) ctx->dfree(c.p);
  ctx->pool.chunks.clear();
  ctx->pool.cur = 0;
  ctx->pool.off = 0;
}
void lcc_ctx_allocator_internal(const lcc_ctx* ctx, lcc_alloc_fn* a, lcc_free_fn* f, void** user) {
  *a = ctx->alloc;
  *f = ctx->freef;
  *user = ctx->user;
}
