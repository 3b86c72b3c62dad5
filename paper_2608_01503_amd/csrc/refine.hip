// pLeidenR (Alg. 6, Lemmas 1-2): refinement of the clustering B by spanning trees.
//
//   U    = {u : w'(u, B[u]) >= 0}                               (q-scaled: q a(u,B[u]) - p w(u) (W_B - w(u)) >= 0)
//   A_v  = {v} plus neighbours u in U with B[u] = B[v] and w'(u,v) >= 0, in vertex-id order; H[v] = A_v[r] with
//          r = fmix64(s_t ^ 2v) mod |A_v|, s_t = t-th splitmix64 output of the seed (t counts refinement calls)
//   f(v) = fmix32(v ^ (s_t >> 32)), a bijection, K = 2^32; the edge to H[v] is kept iff f(H[v]) < f(v)
//   roots without children take f <- 2K - 1 - f and their own edge is tested again with the new values
//   trees: roots by following parents; members of non-trivial trees grouped by root and each tree sorted by f
//   commit: along each sorted tree, v_i is valid iff w'(v_i, X_{i-1}) >= 0 and w'(X_{i-1}, B) >= 0 where X_{i-1}
//          is the earlier part of the tree; w(X) and w(X, B \ X) come from prefix sums over the sorted order
//          (w(X_i, B \ X_i) = sum_{j <= i} a(v_j, B \ v_j) - 2 a(v_j, X_{j-1})); the longest all-valid prefix
//          takes the root's id, every other vertex keeps its own id.
#include "common.h"

namespace lcc {

namespace {

constexpr int HUB_BLOCK = 256;
constexpr int64_t K32 = (int64_t)1 << 32;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}
// persistent launches (at most 2048 workgroups looping over their share): one short workgroup per few
// vertices is bound by the workgroup dispatch rate
inline unsigned grp_blocks(const Buckets& bk, int64_t cnt, int G) {
  int64_t b = cdiv(cnt, BLOCK / G);
  return (unsigned)(b < 1 ? 1 : (b > bk.grid_cap ? bk.grid_cap : b));
}

__device__ __forceinline__ int find_chunk_owner(const int32_t* chunk_off, int64_t n7, int64_t blk) {
  int64_t lo = 0, hi = n7;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= blk) lo = mid; else hi = mid;
  }
  return (int)lo;
}

template <int G>
__device__ __forceinline__ int64_t gsum(int64_t x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

__device__ __forceinline__ uint64_t fkey(int32_t v, const RefSrc& rs, const uint8_t* flip) {
  uint64_t f = fmix32(rs.loc(v) ^ rs.fseed(v));
  return flip && flip[v] ? (uint64_t)(2 * K32 - 1) - f : f;
}

// a(v, B[v] \ v) and membership of U
template <int G>
__global__ __launch_bounds__(BLOCK) void k_aB_grp(const int32_t* list, int64_t cnt, DevGraph g, const int32_t* B,
                                                  const int64_t* WB, RefSrc rs, int64_t* aB, uint8_t* inU,
                                                  int64_t* nU) {
  __shared__ unsigned long long cu;  // |U| of this workgroup, one global atomic at the end
  if (threadIdx.x == 0) cu = 0;
  __syncthreads();
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int32_t bv = B[v];
    int64_t s = 0;
    for (int64_t j = g.off[v] + gl; j < g.off[v + 1]; j += G)
      if (B[g.idx[j]] == bv) s += g.w[j];
    s = gsum<G>(s);
    if (gl == 0) {
      aB[v] = s;
      int64_t wv = g.vw[v];
      const Score sc = rs.sc(v);
      bool u = rs.on(v) && sc.q * s - sc.p * wv * (WB[bv] - wv) >= 0;
      inU[v] = u;
      if (u) atomicAdd(&cu, 1ull);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && cu) atomicAdd((unsigned long long*)nU, cu);
}

__global__ __launch_bounds__(HUB_BLOCK) void k_aB_hub(const int32_t* hubs, const int32_t* chunk_off, int64_t n7,
                                                      DevGraph g, const int32_t* B, int64_t* aB) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int32_t bv = B[v];
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK_EDGES;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK_EDGES);
  int64_t s = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK)
    if (B[g.idx[j]] == bv) s += g.w[j];
  s = gsum<WAVE>(s);
  if ((threadIdx.x & (WAVE - 1)) == 0 && s) atomicAdd((unsigned long long*)&aB[v], (unsigned long long)s);
}

__global__ void k_hub_zero64(const int32_t* hubs, int64_t n7, int64_t* a) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n7; k += (int64_t)gridDim.x * blockDim.x)
    a[hubs[k]] = 0;
}

__global__ void k_hub_inU(const int32_t* hubs, int64_t n7, DevGraph g, const int32_t* B, const int64_t* WB,
                          RefSrc rs, const int64_t* aB, uint8_t* inU, int64_t* nU) {
  __shared__ unsigned long long cu;
  if (threadIdx.x == 0) cu = 0;
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n7; k += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = hubs[k];
    int64_t wv = g.vw[v];
    const Score sc = rs.sc(v);
    bool u = rs.on(v) && sc.q * aB[v] - sc.p * wv * (WB[B[v]] - wv) >= 0;
    inU[v] = u;
    if (u) atomicAdd(&cu, 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0 && cu) atomicAdd((unsigned long long*)nU, cu);
}

__device__ __forceinline__ bool qualifies(const DevGraph& g, const int32_t* B, const uint8_t* inU, const Score& sc,
                                          int64_t j, int32_t bv, int64_t wv) {
  int32_t u = g.idx[j];
  return inU[u] && B[u] == bv && sc.q * (int64_t)g.w[j] - sc.p * g.vw[u] * wv >= 0;
}

// Random candidate edge for rows of up to whole-wavefront groups: count, pick, locate (two sweeps).
template <int G>
__global__ __launch_bounds__(BLOCK) void k_choose_grp(const int32_t* list, int64_t cnt, DevGraph g, const int32_t* B,
                                                      const uint8_t* inU, RefSrc rs, int32_t* H) {
  const int gl = threadIdx.x % G;
  // the loop bound is the same for every lane of the workgroup: the ballots below see whole wavefronts
  for (int64_t gbase0 = (int64_t)blockIdx.x * (BLOCK / G); gbase0 < cnt; gbase0 += (int64_t)gridDim.x * (BLOCK / G)) {
  const int64_t gid = gbase0 + threadIdx.x / G;
  const bool active = gid < cnt;
  const int32_t v = active ? list[gid] : 0;
  const bool vin = active && inU[v];
  const int64_t j0 = active ? g.off[v] : 0, j1 = active ? g.off[v + 1] : 0;
  const int32_t bv = active ? B[v] : 0;
  const int64_t wv = active ? g.vw[v] : 0;
  const Score sc = rs.sc(v);
  // uniform trip count over the wavefront
  int64_t d = vin ? j1 - j0 : 0, dmax = d;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, WAVE));
  const int lane = threadIdx.x & (WAVE - 1);
  const int gbase = lane - gl;
  const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  int64_t total = 0, below = 0;
  for (int64_t o = 0; o < dmax; o += G) {
    int64_t j = j0 + o + gl;
    bool in = vin && j < j1;
    bool q = in && qualifies(g, B, inU, sc, j, bv, wv);
    uint64_t m = __ballot(q) & gmask;
    uint64_t mb = __ballot(q && g.idx[j] < v) & gmask;
    total += __popcll(m);
    below += __popcll(mb);
  }
  int64_t target = -1;  // index among qualifying neighbours, or -1 for v itself
  if (vin) {
    uint64_t r = fmix64(rs.seed(v) ^ ((uint64_t)rs.loc(v) << 1)) % (uint64_t)(total + 1);
    if ((int64_t)r != below) target = (int64_t)r < below ? (int64_t)r : (int64_t)r - 1;
  }
  int64_t seen = 0;
  int32_t found = -1;
  for (int64_t o = 0; o < dmax; o += G) {
    int64_t j = j0 + o + gl;
    bool in = vin && target >= 0 && j < j1;
    bool q = in && qualifies(g, B, inU, sc, j, bv, wv);
    uint64_t m = __ballot(q) & gmask;
    if (q && seen + __popcll(m & lt & gmask) == target) found = g.idx[j];
    seen += __popcll(m);
  }
  // the lane that found the target writes; otherwise lane 0 of the group writes v
  uint64_t fm = __ballot(found >= 0) & gmask;
  if (active) {
    if (fm) {
      if (found >= 0) H[v] = found;
    } else if (gl == 0) {
      H[v] = v;
    }
  }
  }
}

// hubs: per-chunk (qualifying count << 32 | qualifying count below v)
__global__ __launch_bounds__(HUB_BLOCK) void k_choose_hub_count(const int32_t* hubs, const int32_t* chunk_off,
                                                                int64_t n7, DevGraph g, const int32_t* B,
                                                                const uint8_t* inU, RefSrc rs, int64_t* pc) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  int64_t c = 0, cb = 0;
  if (inU[v]) {
    const int32_t bv = B[v];
    const int64_t wv = g.vw[v];
    const Score sc = rs.sc(v);
    const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK_EDGES;
    const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK_EDGES);
    for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK)
      if (qualifies(g, B, inU, sc, j, bv, wv)) {
        ++c;
        if (g.idx[j] < v) ++cb;
      }
  }
  __shared__ int64_t s1[HUB_BLOCK / WAVE], s2[HUB_BLOCK / WAVE];
  c = gsum<WAVE>(c);
  cb = gsum<WAVE>(cb);
  if ((threadIdx.x & (WAVE - 1)) == 0) { s1[threadIdx.x / WAVE] = c; s2[threadIdx.x / WAVE] = cb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t a = 0, b = 0;
    for (int w = 0; w < HUB_BLOCK / WAVE; ++w) { a += s1[w]; b += s2[w]; }
    pc[blockIdx.x] = (a << 32) | b;
  }
}

// per hub: pick r, find the chunk holding the target; tgt[k] = chunk << 32 | rank in chunk, or -1
__global__ void k_choose_hub_pick(const int32_t* hubs, const int32_t* chunk_off, int64_t n7, const uint8_t* inU,
                                  RefSrc rs, const int64_t* pc, int64_t* tgt, int32_t* H) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n7) return;
  int32_t v = hubs[k];
  tgt[k] = -1;
  if (!inU[v]) { H[v] = v; return; }
  int64_t total = 0, below = 0;
  for (int32_t c = chunk_off[k]; c < chunk_off[k + 1]; ++c) {
    total += pc[c] >> 32;
    below += pc[c] & 0xFFFFFFFF;
  }
  uint64_t r = fmix64(rs.seed(v) ^ ((uint64_t)rs.loc(v) << 1)) % (uint64_t)(total + 1);
  if ((int64_t)r == below) { H[v] = v; return; }
  int64_t t = (int64_t)r < below ? (int64_t)r : (int64_t)r - 1;
  for (int32_t c = chunk_off[k]; c < chunk_off[k + 1]; ++c) {
    int64_t cc = pc[c] >> 32;
    if (t < cc) { tgt[k] = ((int64_t)(c - chunk_off[k]) << 32) | t; return; }
    t -= cc;
  }
}

// per hub with a target: one workgroup scans the chunk in order
__global__ __launch_bounds__(HUB_BLOCK) void k_choose_hub_find(const int32_t* hubs, int64_t n7, DevGraph g,
                                                               const int32_t* B, const uint8_t* inU, RefSrc rs,
                                                               const int64_t* tgt, int32_t* H) {
  const int64_t k = blockIdx.x;
  const int64_t tg = tgt[k];
  if (tg < 0) return;
  const int32_t v = hubs[k];
  const int32_t bv = B[v];
  const int64_t wv = g.vw[v];
  const Score sc = rs.sc(v);
  const int64_t j0 = g.off[v] + (tg >> 32) * HUB_CHUNK_EDGES;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK_EDGES);
  const int64_t want = tg & 0xFFFFFFFF;
  __shared__ int64_t wc[HUB_BLOCK / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), wv_ = threadIdx.x / WAVE;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  int64_t seen = 0;
  for (int64_t jb = j0; jb < j1; jb += HUB_BLOCK) {
    int64_t j = jb + threadIdx.x;
    bool q = j < j1 && qualifies(g, B, inU, sc, j, bv, wv);
    uint64_t m = __ballot(q);
    if (lane == 0) wc[wv_] = __popcll(m);
    __syncthreads();
    int64_t pre = seen;
    for (int w = 0; w < wv_; ++w) pre += wc[w];
    if (q && pre + __popcll(m & lt) == want) H[v] = g.idx[j];
    for (int w = 0; w < HUB_BLOCK / WAVE; ++w) seen += wc[w];
    __syncthreads();
  }
}

__global__ void k_parents(int64_t n, const int32_t* H, RefSrc rs, int32_t* par, uint8_t* has_child) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t h = H[v];
    bool keep = h != (int32_t)v && fkey(h, rs, nullptr) < fkey((int32_t)v, rs, nullptr);
    par[v] = keep ? h : (int32_t)v;
    if (keep) has_child[h] = 1;
  }
}

__global__ void k_flip(int64_t n, const int32_t* par, const uint8_t* has_child, uint8_t* flip) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    flip[v] = par[v] == (int32_t)v && !has_child[v];
}

__global__ void k_reparent(int64_t n, const int32_t* H, RefSrc rs, const uint8_t* flip, int32_t* par) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t h = H[v];
    if (flip[v] && h != (int32_t)v && fkey(h, rs, flip) < fkey((int32_t)v, rs, flip)) par[v] = h;
  }
}

// Parent pointers strictly decrease the ordering value, so every chase ends at a root within n steps; the
// step bound only turns an impossible cycle into an error flag instead of a hang.
__global__ void k_roots(int64_t n, const int32_t* par, int32_t* root, int32_t* tsz, Ctrl* ctrl) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = (int32_t)v;
    int64_t steps = 0;
    while (par[x] != x && steps <= n) { x = par[x]; ++steps; }
    if (par[x] != x) atomicOr(&ctrl->err_bits, ERRB_INTERNAL);
    root[v] = x;
    atomicAdd(&tsz[x], 1);
  }
}

__global__ void k_members(int64_t n, const int32_t* root, const int32_t* tsz, uint8_t* member) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    member[v] = tsz[root[v]] > 1;
}

// positions of the trees of two or more members: the tree of root r gets tsz[r] of them
__global__ void k_tree_sizes(int64_t n, const int32_t* root, const int32_t* tsz, int32_t* gs) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    gs[v] = (root[v] == (int32_t)v && tsz[v] >= 2) ? tsz[v] : 0;
}

__global__ void k_tree_keys(int64_t n, const uint8_t* member, const int64_t* tpos, const int32_t* root,
                            RefSrc rs, const uint8_t* flip, uint64_t* keys, uint32_t* vals) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (!member[v]) continue;
    const int64_t p = tpos[v];
    keys[p] = ((uint64_t)(uint32_t)root[v] << 33) | fkey((int32_t)v, rs, flip);
    vals[p] = (uint32_t)v;
  }
}

// a(v, X_{<v}): edges to earlier vertices of the same tree
template <int G>
__global__ __launch_bounds__(BLOCK) void k_aX_grp(const int32_t* list, int64_t cnt, DevGraph g, const uint8_t* member,
                                                  const int32_t* root, RefSrc rs, const uint8_t* flip,
                                                  int64_t* aX) {
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    if (!member[v]) continue;  // uniform within the group
    const int32_t rv = root[v];
    const uint64_t fv = fkey(v, rs, flip);
    int64_t s = 0;
    for (int64_t j = g.off[v] + gl; j < g.off[v + 1]; j += G) {
      int32_t u = g.idx[j];
      if (root[u] == rv && fkey(u, rs, flip) < fv) s += g.w[j];
    }
    s = gsum<G>(s);
    if (gl == 0) aX[v] = s;
  }
}

__global__ __launch_bounds__(HUB_BLOCK) void k_aX_hub(const int32_t* hubs, const int32_t* chunk_off, int64_t n7,
                                                      DevGraph g, const uint8_t* member, const int32_t* root,
                                                      RefSrc rs, const uint8_t* flip, int64_t* aX) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  if (!member[v]) return;
  const int32_t rv = root[v];
  const uint64_t fv = fkey(v, rs, flip);
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK_EDGES;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK_EDGES);
  int64_t s = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK) {
    int32_t u = g.idx[j];
    if (root[u] == rv && fkey(u, rs, flip) < fv) s += g.w[j];
  }
  s = gsum<WAVE>(s);
  if ((threadIdx.x & (WAVE - 1)) == 0 && s) atomicAdd((unsigned long long*)&aX[v], (unsigned long long)s);
}

__global__ void k_sorted_terms(int64_t m, const uint32_t* sv, const int64_t* vw, const int64_t* aB,
                               const int64_t* aX, int64_t* tw, int64_t* tc, int32_t* pos_of) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = (int32_t)sv[i];
    tw[i] = vw[v];
    tc[i] = aB[v] - 2 * aX[v];
    pos_of[v] = (int32_t)i;
  }
}

__global__ void k_validity(int64_t m, const uint32_t* sv, const int32_t* root, const int32_t* pos_of,
                           const int64_t* pw, const int64_t* pc, const int64_t* aX, const int64_t* vw,
                           const int32_t* B, const int64_t* WB, RefSrc rs, int32_t* fail) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = (int32_t)sv[i];
    int32_t r = root[v];
    int64_t s = pos_of[r];
    int64_t wX = pw[i] - pw[s];
    int64_t cut = pc[i] - pc[s];
    const Score sc = rs.sc(r);
    int64_t c1 = sc.q * aX[v] - sc.p * vw[v] * wX;
    int64_t c2 = sc.q * cut - sc.p * wX * (WB[B[r]] - wX);
    if (c1 < 0 || c2 < 0) atomicMin(&fail[r], (int32_t)i);
  }
}

__global__ void k_commit(int64_t n, const uint8_t* member, const int32_t* root, const int32_t* pos_of,
                         const int32_t* fail, int32_t* R) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t r = root[v];
    R[v] = (member[v] && pos_of[v] < fail[r]) ? r : (int32_t)v;
  }
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

void refine(const DevGraph& g, const Buckets& b, const RefSrc& rs, const int32_t* B, int32_t* R, RefineBuffers& rb,
            Ctrl* ctrl, const std::function<void*(size_t)>& take, hipStream_t st) {
  const int64_t n = g.n;
  const int32_t* L = b.list;
  // constraint-cluster weights and U
  launch_cluster_weights(B, g.vw, n, rb.WB, st);
  k_set_i64<<<1, 1, 0, st>>>(&ctrl->refine_U, 0);
  if (b.count[0]) k_aB_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  if (b.count[1]) k_aB_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  if (b.count[2]) k_aB_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  if (b.count[3]) k_aB_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  int64_t nw = b.count[4] + b.count[5] + b.count[6];
  if (nw) k_aB_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  const int32_t* hubs = L + b.off[7];
  const int64_t n7 = b.count[7];
  if (n7) {
    k_hub_zero64<<<grid_for(n7), BLOCK, 0, st>>>(hubs, n7, rb.aB);
    k_aB_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, B, rb.aB);
    k_hub_inU<<<grid_for(n7), BLOCK, 0, st>>>(hubs, n7, g, B, rb.WB, rs, rb.aB, rb.inU, &ctrl->refine_U);
  }
  // random candidate edge
  if (b.count[0]) k_choose_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, B, rb.inU, rs, rb.H);
  if (b.count[1]) k_choose_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, B, rb.inU, rs, rb.H);
  if (b.count[2]) k_choose_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, B, rb.inU, rs, rb.H);
  if (b.count[3]) k_choose_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, B, rb.inU, rs, rb.H);
  if (nw) k_choose_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, B, rb.inU, rs, rb.H);
  if (n7) {
    k_choose_hub_count<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, B, rb.inU, rs, b.hub_ps);
    k_choose_hub_pick<<<grid_for(n7), BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, rb.inU, rs, b.hub_ps, b.hub_acc, rb.H);
    k_choose_hub_find<<<(unsigned)n7, HUB_BLOCK, 0, st>>>(hubs, n7, g, B, rb.inU, rs, b.hub_acc, rb.H);
    fill_i64(b.hub_acc, 0, n7, st);  // the per-hub accumulator is expected zero by the afterburner
  }
  // parents, singleton-tree fix, roots
  fill_u8(rb.has_child, 0, n, st);
  k_parents<<<grid_for(n), BLOCK, 0, st>>>(n, rb.H, rs, rb.par, rb.has_child);
  k_flip<<<grid_for(n), BLOCK, 0, st>>>(n, rb.par, rb.has_child, rb.flip);
  k_reparent<<<grid_for(n), BLOCK, 0, st>>>(n, rb.H, rs, rb.flip, rb.par);
  fill_i32(rb.tsz, 0, n, st);
  k_roots<<<grid_for(n), BLOCK, 0, st>>>(n, rb.par, rb.root, rb.tsz, ctrl);
  k_members<<<grid_for(n), BLOCK, 0, st>>>(n, rb.root, rb.tsz, rb.member);
  // members grouped by tree (each tree's range from a scan of the tree sizes), then every tree sorted by f;
  // pw, tmp64a and tmp64b serve as scratch here and get their own contents below
  int64_t* toff = rb.pw;
  auto* cursor = (unsigned long long*)rb.tmp64a;
  int64_t* tpos = rb.tmp64b;
  k_tree_sizes<<<grid_for(n), BLOCK, 0, st>>>(n, rb.root, rb.tsz, rb.tree_sz);
  scan_i32_i64(rb.tree_sz, toff, n, rb.scan_temp, st);
  // the member count is needed on the host to size the sort
  int64_t m = 0;
  device_check(hipMemcpyAsync(&m, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st), "tree members");
  device_check(hipStreamSynchronize(st), "tree members");
  k_set_i64<<<1, 1, 0, st>>>(&ctrl->refine_m, m);
  fill_i32(rb.fail, INT32_MAX, n, st);
  if (m > 0) {
    launch_group_place(rb.root, nullptr, rb.member, n, toff, n, cursor, tpos, st);
    k_tree_keys<<<grid_for(n), BLOCK, 0, st>>>(n, rb.member, tpos, rb.root, rs, rb.flip, rb.k0, rb.v0);
    segsort_pairs(rb.k0, rb.v0, rb.k1, rb.v1, m, toff, n, 33, rb.scan_temp, take, st);
    const uint32_t* sv = rb.v1;
    // a(v, X_{<v}) for tree members
    fill_i64(rb.aX, 0, n, st);
    if (b.count[0]) k_aX_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, rb.member, rb.root, rs, rb.flip, rb.aX);
    if (b.count[1]) k_aX_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, rb.member, rb.root, rs, rb.flip, rb.aX);
    if (b.count[2]) k_aX_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, rb.member, rb.root, rs, rb.flip, rb.aX);
    if (b.count[3]) k_aX_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, rb.member, rb.root, rs, rb.flip, rb.aX);
    if (nw) k_aX_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, rb.member, rb.root, rs, rb.flip, rb.aX);
    if (n7) k_aX_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, rb.member, rb.root, rs, rb.flip, rb.aX);
    k_sorted_terms<<<grid_for(m), BLOCK, 0, st>>>(m, sv, g.vw, rb.aB, rb.aX, rb.tmp64a, rb.tmp64b, rb.pos_of);
    scan_i64_i64(rb.tmp64a, rb.pw, m, rb.scan_temp, st);
    scan_i64_i64(rb.tmp64b, rb.pc, m, rb.scan_temp, st);
    k_validity<<<grid_for(m), BLOCK, 0, st>>>(m, sv, rb.root, rb.pos_of, rb.pw, rb.pc, rb.aX, g.vw, B, rb.WB, rs,
                                              rb.fail);
  }
  k_commit<<<grid_for(n), BLOCK, 0, st>>>(n, rb.member, rb.root, rb.pos_of, rb.fail, R);
}

}  // namespace lcc
