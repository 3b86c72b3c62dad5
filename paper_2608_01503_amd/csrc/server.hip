// Continuous-batching clustering server (lcc_server_* of include/lcc.h).
//
// The server owns S execution slots; each slot is a worker thread with its own context (workspace and level
// pool on the device) and its own HIP stream, so the sweeps of concurrently admitted jobs overlap on the GPU.
// A submitted job is copied to host memory and queued.  A free slot admits the oldest queued job whose
// device footprint (lcc_workspace_bytes) fits the unreserved part of the HBM budget; a job that does not fit
// yet is passed over by smaller ones at most a few times before it holds the next free slot, so a large
// request cannot starve.  When the admitted job is a small request, the slot also takes the other queued small
// requests of its family (Louvain / Louvain+, or pLeiden / pLeiden+) with the same options that fit the budget
// and runs them all as one fused batch (lcc_cluster_batch: one union graph per kernel launch), so a burst of small requests costs
// about one request's launches.  A finished slot releases its reservations at once and the next job joins
// without waiting for the others.  Results are bit-identical to a plain lcc_cluster call.
//
// Device memory is accounted per slot: every allocation of a slot's context goes through the slot's
// accounting allocator, which knows the bytes the slot holds.  A slot is charged the larger of what it holds
// and the footprint reserved for its running job, and the charges of all slots never exceed the budget: an
// allocation that would pass it (a job whose coarse levels outgrow the footprint estimate) is refused, the
// job is queued again at the head and rerun alone once the other slots are idle and have returned their
// memory.  An idle slot keeps its workspace for the next job (small jobs then allocate nothing) unless it
// holds more than its share of the budget or a queued job needs the memory, in which case it returns it.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/lcc.h"

lcc_status lcc_cluster_init_internal(lcc_ctx* ctx, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                                     const lcc_options* opts, void* stream, int32_t* labels_out, lcc_result* res,
                                     const int32_t* init);
int lcc_ctx_device_internal(const lcc_ctx* ctx);
void lcc_ctx_allocator_internal(const lcc_ctx* ctx, lcc_alloc_fn* a, lcc_free_fn* f, void** user);
void lcc_ctx_release_internal(lcc_ctx* ctx);

namespace {

// One slot per hardware queue a process gets by default (HIP's GPU_MAX_HW_QUEUES is 4): more streams than
// queues would share them.  LCC_SERVER_SLOTS (1-16) overrides it.
constexpr int DEFAULT_SLOTS = 4;
constexpr int MAX_SLOTS = 16;
constexpr int MAX_PASSED_OVER = 4;
constexpr int64_t FUSE_NNZ = (int64_t)1 << 22;        // requests up to this many entries may be fused
constexpr int64_t FUSE_TOTAL_NNZ = (int64_t)1 << 25;  // entries of one fused group
constexpr size_t FUSE_MAX = 256;                      // requests of one fused group

struct Job {
  uint64_t ticket = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> idx, w;
  std::vector<int64_t> vw;
  bool has_w = false;
  lcc_vw_mode vw_mode = LCC_VW_UNIT;
  lcc_lambda lam{};
  lcc_variant variant = LCC_PLOUVAIN;
  lcc_options opts{};
  bool has_opts = false;
  size_t footprint = 0;
  int passed_over = 0;
  bool alone = false;  // refused memory beyond the budget once: runs again with every other slot idle and empty
  bool done = false;
  lcc_status st = LCC_OK;
  std::vector<int32_t> labels;
  lcc_result res{};
};

// The accounting allocator of one slot: forwards to the parent context's allocator (or hipMalloc) and keeps
// the sizes of the slot's live allocations.
struct SlotAcct {
  lcc_server* srv = nullptr;
  int k = 0;
  lcc_alloc_fn a = nullptr;
  lcc_free_fn f = nullptr;
  void* user = nullptr;
  std::mutex amu;
  std::unordered_map<void*, size_t> sizes;
};

void* slot_alloc(size_t bytes, void* user);
void slot_free(void* p, void* user);

}  // namespace

struct lcc_server {
  lcc_ctx* parent = nullptr;
  size_t budget = 0;
  int nslots = DEFAULT_SLOTS;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Job>> queue;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  std::vector<lcc_ctx*> ctxs;
  std::vector<hipStream_t> streams;
  std::vector<std::unique_ptr<SlotAcct>> acct;
  // per slot, guarded by mu: bytes held, footprint reserved for the running job, running, asked to release
  std::vector<size_t> held, reserve;
  std::vector<char> busy, release_req, refused;
  bool alone_running = false;  // a job rerun alone is running: no other slot admits anything
  bool stop = false;
  uint64_t next_ticket = 1;

  size_t charge(int k) const { return std::max(held[k], reserve[k]); }
  size_t total_charge() const {
    size_t t = 0;
    for (int k = 0; k < nslots; ++k) t += charge(k);
    return t;
  }
  // Ask the idle slots (other than `self`) that hold memory to return it; true when some were asked.
  bool ask_idle_release(int self) {
    bool any = false;
    for (int x = 0; x < nslots; ++x)
      if (x != self && !busy[x] && held[x] > 0 && !release_req[x]) { release_req[x] = 1; any = true; }
    if (any) cv.notify_all();
    return any;
  }

  // Pick the job free slot k runs next (caller holds mu).  When a job fits only once memory retained by idle
  // slots (this one included) is returned, those slots are asked to return it and nothing is picked yet.
  std::shared_ptr<Job> pick(int k) {
    if (alone_running) return nullptr;
    for (size_t i = 0; i < queue.size(); ++i) {
      auto& j = queue[i];
      if (j->alone) {  // at the head: wait until every slot is idle and empty, nobody overtakes it
        bool others = held[k] > 0;
        for (int x = 0; x < nslots; ++x) others |= x != k && (busy[x] || held[x] > 0);
        if (others) {
          if (held[k] > 0) release_req[k] = 1;
          ask_idle_release(k);
          return nullptr;
        }
        alone_running = true;
      } else {
        const size_t rest = total_charge() - charge(k);
        if (rest + std::max(held[k], j->footprint) > budget) {
          // fits once idle slots return their memory: ask them, and let the job wait for it
          size_t idle = held[k];
          for (int x = 0; x < nslots; ++x)
            if (x != k && !busy[x]) idle += held[x];
          if (rest + held[k] - std::min(rest + held[k], idle) + j->footprint <= budget) {
            if (held[k] > 0) release_req[k] = 1;
            ask_idle_release(k);
            return nullptr;
          }
          if (j->passed_over >= MAX_PASSED_OVER) break;  // the head waits; nobody overtakes it any more
          continue;
        }
      }
      for (size_t x = 0; x < i; ++x) queue[x]->passed_over++;
      auto r = j;
      queue.erase(queue.begin() + (long)i);
      reserve[k] += r->footprint;
      return r;
    }
    return nullptr;
  }

  static bool fusable(const Job& j) { return j.nnz <= FUSE_NNZ; }
  // one fused group holds one family: Louvain / Louvain+ or pLeiden / pLeiden+
  static bool leiden(const Job& j) { return j.variant == LCC_PLEIDEN || j.variant == LCC_PLEIDEN_PLUS; }
  static bool same_opts(const Job& a, const Job& b) {
    return a.has_opts == b.has_opts && (!a.has_opts || memcmp(&a.opts, &b.opts, sizeof(lcc_options)) == 0);
  }

  // The admitted job plus the queued small jobs of its family that can join it (caller holds mu).
  std::vector<std::shared_ptr<Job>> pick_group(int k) {
    std::vector<std::shared_ptr<Job>> grp;
    auto head = pick(k);
    if (!head) return grp;
    grp.push_back(head);
    if (!fusable(*head) || head->alone) return grp;
    int64_t total = head->nnz;
    for (size_t i = 0; i < queue.size() && grp.size() < FUSE_MAX;) {
      auto& j = queue[i];
      const size_t rest = total_charge() - charge(k);
      if (fusable(*j) && !j->alone && leiden(*j) == leiden(*head) && same_opts(*head, *j) &&
          total + j->nnz <= FUSE_TOTAL_NNZ &&
          rest + std::max(held[k], reserve[k] + j->footprint) <= budget) {
        reserve[k] += j->footprint;
        total += j->nnz;
        grp.push_back(j);
        queue.erase(queue.begin() + (long)i);
      } else {
        ++i;
      }
    }
    return grp;
  }

  static lcc_graph host_graph(Job& j) {
    lcc_graph g{};
    g.n = j.n;
    g.nnz = j.nnz;
    g.offsets = j.off.data();
    g.offsets_bits = 64;
    g.indices = j.idx.data();
    g.edge_w = j.has_w ? j.w.data() : nullptr;
    g.vertex_w = j.vw_mode == LCC_VW_GIVEN ? j.vw.data() : nullptr;
    g.vw_mode = j.vw_mode;
    g.mem = LCC_MEM_HOST;
    j.labels.assign((size_t)std::max<int64_t>(j.n, 1), 0);
    return g;
  }

  void run_one(lcc_ctx* ctx, hipStream_t st, Job& j) {
    lcc_graph g = host_graph(j);
    j.st = lcc_cluster_init_internal(ctx, &g, j.lam, j.variant, j.has_opts ? &j.opts : nullptr, st,
                                     j.labels.data(), &j.res, nullptr);
  }

  void run_group(lcc_ctx* ctx, hipStream_t st, std::vector<std::shared_ptr<Job>>& grp) {
    if (grp.size() == 1) {
      run_one(ctx, st, *grp[0]);
      return;
    }
    const size_t m = grp.size();
    std::vector<lcc_graph> gs(m);
    std::vector<lcc_lambda> lams(m);
    std::vector<lcc_variant> vars(m);
    std::vector<int32_t*> outs(m);
    std::vector<lcc_result> res(m);
    for (size_t i = 0; i < m; ++i) {
      gs[i] = host_graph(*grp[i]);
      lams[i] = grp[i]->lam;
      vars[i] = grp[i]->variant;
      outs[i] = grp[i]->labels.data();
    }
    lcc_status s = lcc_cluster_batch(ctx, gs.data(), lams.data(), vars.data(), (int64_t)m,
                                     grp[0]->has_opts ? &grp[0]->opts : nullptr, st, outs.data(), res.data());
    if (s == LCC_OK) {
      for (size_t i = 0; i < m; ++i) { grp[i]->st = LCC_OK; grp[i]->res = res[i]; }
      return;
    }
    for (auto& j : grp) run_one(ctx, st, *j);  // some request is invalid: give each its own status
  }

  void release(int k) {
    lcc_ctx_release_internal(ctxs[k]);
    std::lock_guard<std::mutex> lock(mu);
    release_req[k] = 0;
  }

  void run_worker(int k) {
    lcc_ctx* ctx = ctxs[k];
    hipStream_t st = streams[k];
    for (;;) {
      std::vector<std::shared_ptr<Job>> grp;
      bool release_now = false;
      {
        std::unique_lock<std::mutex> lock(mu);
        cv.wait(lock, [&] {
          if (stop) return true;
          if (!release_req[k]) grp = pick_group(k);  // may ask this slot to return its memory first
          if (grp.empty() && release_req[k]) { release_now = true; return true; }
          return !grp.empty();
        });
        if (grp.empty() && !release_now) return;  // stopping
        if (!grp.empty()) { busy[k] = 1; refused[k] = 0; }
      }
      if (grp.empty()) {  // an idle slot asked to return its memory
        release(k);
        cv.notify_all();
        continue;
      }
      const bool was_alone = grp[0]->alone;
      run_group(ctx, st, grp);
      bool over;
      {
        std::lock_guard<std::mutex> lock(mu);
        over = held[k] > budget / (size_t)nslots;
      }
      if (over) lcc_ctx_release_internal(ctx);  // keep no more than this slot's share while idle
      {
        std::lock_guard<std::mutex> lock(mu);
        const bool again = refused[k] != 0;
        for (auto& j : grp) {
          if (again && j->st == LCC_ERR_OOM && !j->alone) {  // refused beyond the budget: rerun alone
            j->alone = true;
            j->st = LCC_OK;
            queue.push_front(j);
            continue;
          }
          j->done = true;
          // the host copy of the graph is no longer needed
          std::vector<int64_t>().swap(j->off);
          std::vector<int32_t>().swap(j->idx);
          std::vector<int32_t>().swap(j->w);
          std::vector<int64_t>().swap(j->vw);
        }
        reserve[k] = 0;
        busy[k] = 0;
        refused[k] = 0;
        release_req[k] = 0;
        if (was_alone) alone_running = false;
      }
      cv.notify_all();
    }
  }
};

namespace {

void* slot_alloc(size_t bytes, void* user) {
  auto* a = (SlotAcct*)user;
  lcc_server* s = a->srv;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    const int k = a->k;
    const size_t before = s->charge(k);
    const size_t after = std::max(s->held[k] + bytes, s->reserve[k]);
    if (s->total_charge() - before + after > s->budget) {
      s->refused[k] = 1;
      return nullptr;
    }
    s->held[k] += bytes;  // counted before the allocation, so concurrent checks see it
  }
  void* p = nullptr;
  if (a->a) p = a->a(bytes, a->user);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  if (!p) {
    std::lock_guard<std::mutex> lock(s->mu);
    s->held[a->k] -= bytes;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(a->amu);
  a->sizes[p] = bytes;
  return p;
}

void slot_free(void* p, void* user) {
  auto* a = (SlotAcct*)user;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lock(a->amu);
    auto it = a->sizes.find(p);
    if (it != a->sizes.end()) { bytes = it->second; a->sizes.erase(it); }
  }
  if (a->f) a->f(p, a->user);
  else (void)hipFree(p);
  std::lock_guard<std::mutex> lock(a->srv->mu);
  a->srv->held[a->k] -= std::min(bytes, a->srv->held[a->k]);
}

}  // namespace

extern "C" {

lcc_status lcc_server_create(lcc_ctx* ctx, size_t hbm_budget, lcc_server** out) {
  if (!ctx || !out || hbm_budget == 0) return LCC_ERR_INVALID;
  auto* s = new lcc_server();
  s->parent = ctx;
  s->budget = hbm_budget;
  if (const char* e = getenv("LCC_SERVER_SLOTS")) s->nslots = std::max(1, std::min(MAX_SLOTS, atoi(e)));
  s->held.assign((size_t)s->nslots, 0);
  s->reserve.assign((size_t)s->nslots, 0);
  s->busy.assign((size_t)s->nslots, 0);
  s->release_req.assign((size_t)s->nslots, 0);
  s->refused.assign((size_t)s->nslots, 0);
  int dev = lcc_ctx_device_internal(ctx);
  lcc_alloc_fn a;
  lcc_free_fn f;
  void* user;
  lcc_ctx_allocator_internal(ctx, &a, &f, &user);
  if (hipSetDevice(dev) != hipSuccess) { delete s; return LCC_ERR_DEVICE; }
  lcc_tuning tune;
  if (lcc_get_tuning(ctx, &tune) != LCC_OK) lcc_default_tuning(&tune);
  for (int k = 0; k < s->nslots; ++k) {
    auto ac = std::make_unique<SlotAcct>();
    ac->srv = s;
    ac->k = k;
    ac->a = a;
    ac->f = f;
    ac->user = user;
    s->acct.push_back(std::move(ac));
  }
  for (int k = 0; k < s->nslots; ++k) {
    lcc_ctx* c = nullptr;
    hipStream_t st = nullptr;
    if (lcc_create(dev, slot_alloc, slot_free, s->acct[k].get(), &c) != LCC_OK || hipStreamCreate(&st) != hipSuccess) {
      for (auto* x : s->ctxs) lcc_destroy(x);
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      if (c) lcc_destroy(c);
      delete s;
      return LCC_ERR_DEVICE;
    }
    (void)lcc_set_tuning(c, &tune);  // the slots run with the parent context's launch tuning
    s->ctxs.push_back(c);
    s->streams.push_back(st);
  }
  for (int k = 0; k < s->nslots; ++k) s->workers.emplace_back([s, k] { (void)hipSetDevice(lcc_ctx_device_internal(s->ctxs[k])); s->run_worker(k); });
  *out = s;
  return LCC_OK;
}

lcc_status lcc_submit(lcc_server* s, const lcc_graph* g, lcc_lambda lambda, lcc_variant variant,
                      const lcc_options* opts, uint64_t* ticket) {
  if (!s || !g || !ticket) return LCC_ERR_INVALID;
  if (g->n < 0 || g->nnz < 0 || !g->offsets || (g->nnz > 0 && !g->indices)) return LCC_ERR_INVALID;
  if (g->n > 2147483647LL || g->nnz > 2147483647LL) return LCC_ERR_INVALID;  // the clustering call's limits
  if (g->offsets_bits != 32 && g->offsets_bits != 64) return LCC_ERR_INVALID;
  if (g->vw_mode == LCC_VW_GIVEN && g->n > 0 && !g->vertex_w) return LCC_ERR_INVALID;
  size_t fp = 0;
  lcc_status st = lcc_workspace_bytes(g->n, g->nnz, variant, &fp);
  if (st != LCC_OK) return st;
  if (fp > s->budget) return LCC_ERR_BUSY;
  auto j = std::make_shared<Job>();
  j->n = g->n;
  j->nnz = g->nnz;
  j->vw_mode = g->vw_mode;
  j->lam = lambda;
  j->variant = variant;
  if (opts) { j->opts = *opts; j->opts.trace = nullptr; j->has_opts = true; }
  j->footprint = fp;
  const hipMemcpyKind kind = g->mem == LCC_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  j->off.resize((size_t)g->n + 1);
  if (g->offsets_bits == 64) {
    if (hipMemcpy(j->off.data(), g->offsets, (size_t)(g->n + 1) * 8, kind) != hipSuccess) return LCC_ERR_DEVICE;
  } else {
    std::vector<int32_t> o32((size_t)g->n + 1);
    if (hipMemcpy(o32.data(), g->offsets, (size_t)(g->n + 1) * 4, kind) != hipSuccess) return LCC_ERR_DEVICE;
    for (size_t i = 0; i < o32.size(); ++i) j->off[i] = o32[i];
  }
  j->idx.resize((size_t)std::max<int64_t>(g->nnz, 1));
  if (g->nnz && hipMemcpy(j->idx.data(), g->indices, (size_t)g->nnz * 4, kind) != hipSuccess) return LCC_ERR_DEVICE;
  if (g->edge_w) {
    j->has_w = true;
    j->w.resize((size_t)std::max<int64_t>(g->nnz, 1));
    if (g->nnz && hipMemcpy(j->w.data(), g->edge_w, (size_t)g->nnz * 4, kind) != hipSuccess) return LCC_ERR_DEVICE;
  }
  if (g->vw_mode == LCC_VW_GIVEN) {
    j->vw.resize((size_t)std::max<int64_t>(g->n, 1));
    if (g->n && hipMemcpy(j->vw.data(), g->vertex_w, (size_t)g->n * 8, kind) != hipSuccess) return LCC_ERR_DEVICE;
  }
  {
    std::lock_guard<std::mutex> lock(s->mu);
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv.notify_all();
  return LCC_OK;
}

lcc_status lcc_poll(lcc_server* s, uint64_t ticket, int* done, int32_t* labels_out, lcc_result* res) {
  if (!s || !done) return LCC_ERR_INVALID;
  std::shared_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return LCC_ERR_NOT_FOUND;
    j = it->second;
    if (!j->done) { *done = 0; return LCC_OK; }
    s->jobs.erase(it);
  }
  *done = 1;
  if (j->st != LCC_OK) return j->st;
  if (labels_out && j->n > 0) memcpy(labels_out, j->labels.data(), (size_t)j->n * 4);
  if (res) *res = j->res;
  return LCC_OK;
}

lcc_status lcc_server_destroy(lcc_server* s) {
  if (!s) return LCC_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto* c : s->ctxs) lcc_destroy(c);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return LCC_OK;
}

}  // extern "C"
