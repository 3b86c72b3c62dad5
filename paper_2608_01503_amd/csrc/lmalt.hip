// LocalMoveAlt (Sec. V-A): used when the synchronous local move leaves the objective unchanged.
//
// Every vertex that is not node optimal (its best destination strictly improves the objective) is a mover,
// taken in ascending vertex id with its destination fixed up front.  Applied one after another, mover i
// (v: A -> B) changes the objective by 2 g_i with
//   g_i = delta_i + q * sum over earlier movers u adjacent to v of w(u,v) * s(u, v)
//                 - p * w(v) * (F_B(i) - F_A(i)),
//   F_c(i) = sum over earlier movers u of w(u) ([D_u = c] - [C_u = c])    (the weight that flowed into c),
// s(u, v) = [D_u = B] - [C_u = B] - [D_u = A] + [C_u = A] (the afterburner pattern of Alg. 3; a move to a new
// singleton never meets another mover's cluster).  The adjacent sum is one pass over the movers' rows; the
// flows are prefix sums per cluster in mover order: one record per (mover, touched cluster) event and query,
// radix-sorted by (cluster, mover index, query before event) and scanned.  The shortest prefix with the
// largest total change is committed (it is non-empty: the first mover alone improves).
#include <algorithm>
#include <functional>

#include "common.h"

namespace lcc {

namespace {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

// movers: vertices that are not node optimal (in a union, only those of the graphs with act set)
__global__ void k_mover_flags(int64_t n, const VState* vs, uint8_t* mv, const int32_t* gid, const uint8_t* act) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    mv[v] = vs[v].d != D_NONE && (!act || act[gid[v]]);
}

__global__ void k_mover_list(int64_t n, const uint8_t* mv, const int32_t* pos, int32_t* list) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (mv[v]) list[pos[v]] = (int32_t)v;
}

// sign pattern of how an earlier mover (cu -> du) changes the gain of a later mover (cv -> dv)
__device__ __forceinline__ int pattern(int32_t cv, int32_t dv, int32_t cu, int32_t du) {
  int a = 0;
  if (cv == cu) a += 1;
  else if (dv == cu) a -= 1;
  if (du != D_EMPTY) {
    if (cv == du) a -= 1;
    else if (dv == du) a += 1;
  }
  return a;
}

// q-free adjacent part: adj[i] = sum over earlier adjacent movers u of w(u, v_i) s(u, v_i); one wavefront
// per mover (grid-stride), lanes over the row.  Rows of the hub bucket are left to k_gain_adj_hub.
__global__ __launch_bounds__(BLOCK) void k_gain_adj(const int32_t* list, int64_t k, DevGraph g, const VState* vs,
                                                    const uint8_t* mv, const int32_t* pos, int64_t hub_deg,
                                                    int64_t* adj) {
  const int lane = threadIdx.x & (WAVE - 1);
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE; i < k;
       i += (int64_t)gridDim.x * (BLOCK / WAVE)) {
    const int32_t v = list[i];
    if (g.off[v + 1] - g.off[v] > hub_deg) continue;  // uniform over the wavefront
    const VState me = vs[v];
    int64_t acc = 0;
    for (int64_t j = g.off[v] + lane; j < g.off[v + 1]; j += WAVE) {
      const int32_t u = g.idx[j];
      if (!mv[u] || pos[u] >= i) continue;
      const VState o = vs[u];
      acc += (int64_t)pattern(me.c, me.d, o.c, o.d) * g.w[j];
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
    if (lane == 0) adj[i] = acc;
  }
}

__device__ __forceinline__ int find_chunk_owner(const int32_t* chunk_off, int64_t n7, int64_t blk) {
  int64_t lo = 0, hi = n7;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= blk) lo = mid; else hi = mid;
  }
  return (int)lo;
}

// hub rows: one workgroup per edge chunk of a hub that is a mover, added into adj (zeroed beforehand)
__global__ __launch_bounds__(BLOCK) void k_gain_adj_hub(const int32_t* hubs, const int32_t* chunk_off, int64_t n7,
                                                        DevGraph g, const VState* vs, const uint8_t* mv,
                                                        const int32_t* pos, int64_t* adj) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  if (!mv[v]) return;
  const int64_t i = pos[v];
  const VState me = vs[v];
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK_EDGES;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK_EDGES);
  int64_t acc = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += BLOCK) {
    const int32_t u = g.idx[j];
    if (!mv[u] || pos[u] >= i) continue;
    const VState o = vs[u];
    acc += (int64_t)pattern(me.c, me.d, o.c, o.d) * g.w[j];
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0 && acc) atomicAdd((unsigned long long*)&adj[i], (unsigned long long)acc);
}

// Records of mover j (4 j .. 4 j + 3): event "leaves C" (-w), event "enters D" (+w), query at D, query at C.
// key = cluster << cs | j << 1 | (event ? 1 : 0) with cs = bits(k) + 1, so real keys use bits(n) + cs bits and
// the sort runs over one bit more; unused records (D = new singleton) get the largest key.
constexpr uint64_t NO_KEY = ~0ull;

__global__ void k_alt_records(const int32_t* list, int64_t k, int cs, const VState* vs, const int64_t* vw,
                              uint64_t* key, uint32_t* val, int64_t* evw) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = list[j];
    const VState s = vs[v];
    const int64_t w = vw[v];
    const uint64_t jj = (uint64_t)j << 1;
    const bool fresh = s.d == D_EMPTY;
    key[4 * j + 0] = ((uint64_t)(uint32_t)s.c << cs) | jj | 1;
    key[4 * j + 1] = fresh ? NO_KEY : (((uint64_t)(uint32_t)s.d << cs) | jj | 1);
    key[4 * j + 2] = fresh ? NO_KEY : (((uint64_t)(uint32_t)s.d << cs) | jj);
    key[4 * j + 3] = ((uint64_t)(uint32_t)s.c << cs) | jj;
    for (int t = 0; t < 4; ++t) val[4 * j + t] = (uint32_t)(4 * j + t);
    evw[4 * j + 0] = -w;
    evw[4 * j + 1] = fresh ? 0 : w;
    evw[4 * j + 2] = 0;
    evw[4 * j + 3] = 0;
  }
}

// sorted position p: x = the event weight (0 for queries), head = first record of a cluster
__global__ void k_alt_gather(const uint64_t* key, const uint32_t* val, const int64_t* evw, int64_t m, int cs,
                             int64_t* x, uint8_t* head) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    x[p] = (key[p] & 1) ? evw[val[p]] : 0;
    head[p] = p == 0 || (key[p] >> cs) != (key[p - 1] >> cs);
  }
}

// S = exclusive prefix of x, H = exclusive prefix of heads: segment of p = H[p] + head[p] - 1
__global__ void k_alt_base(const uint8_t* head, const int32_t* H, const int64_t* S, int64_t m, int64_t* base) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x)
    if (head[p]) base[H[p]] = S[p];
}

__global__ void k_alt_query(const uint64_t* key, const uint32_t* val, const uint8_t* head, const int32_t* H,
                            const int64_t* S, const int64_t* base, int64_t m, int64_t* F) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x)
    if (key[p] != NO_KEY && !(key[p] & 1)) F[val[p]] = S[p] - base[H[p] + head[p] - 1];
}

__global__ void k_gain(const int32_t* list, int64_t k, const VState* vs, const int64_t* vw, ScoreSrc ss,
                       const int64_t* adj, const int64_t* F, int64_t* gain) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = list[i];
    const VState me = vs[v];
    const Score sc = ss.at(v);
    const int64_t fB = me.d == D_EMPTY ? 0 : F[4 * i + 2];
    // half the exact objective change of the move (below 2^62): its terms are summed modulo 2^64
    gain[i] = (int64_t)((uint64_t)me.delta + (uint64_t)(sc.q * adj[i]) - (uint64_t)(sc.p * vw[v] * (fB - F[4 * i + 3])));
  }
}

// Shortest prefix with the largest strictly positive running sum.  S is the exclusive scan of the gains
// (S[i + 1] = running sum through mover i); one workgroup reduces (largest sum, then smallest index).
constexpr int BP_BLOCK = 1024;
__global__ __launch_bounds__(BP_BLOCK) void k_best_prefix(const int64_t* S, int64_t k, Ctrl* ctrl) {
  __shared__ int64_t sv[BP_BLOCK / WAVE], si[BP_BLOCK / WAVE];
  int64_t bv = 0, bi = INT64_MAX;  // no prefix yet; a prefix must beat 0
  for (int64_t i = threadIdx.x; i < k; i += BP_BLOCK) {
    const int64_t r = S[i + 1];
    if (r > bv || (r == bv && r > 0 && i < bi)) { bv = r; bi = i; }
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t ov = __shfl_xor(bv, o, WAVE), oi = __shfl_xor(bi, o, WAVE);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  if (lane == 0) { sv[wv] = bv; si[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BP_BLOCK / WAVE; ++w)
      if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) { bv = sv[w]; bi = si[w]; }
    ctrl->lmalt_best_k = bv > 0 ? bi + 1 : 0;
    ctrl->lmalt_best = bv > 0 ? bv : 0;
  }
}

// Union: the same per graph.  Graph k's movers are list positions [pos[vbase[k]], pos[vbase[k + 1]]) (pos is
// the exclusive scan of the mover flags), so its running sums are differences of S; they are formed modulo 2^64
// (exact: every graph's own running sums are below 2^63).  One workgroup per graph (grid-stride over graphs);
// best_k[k] = the length of graph k's committed prefix.
__global__ __launch_bounds__(BP_BLOCK) void k_best_prefix_seg(const int64_t* S, const int32_t* pos,
                                                              const int32_t* vbase, int64_t G, const uint8_t* act,
                                                              int64_t* best_k) {
  __shared__ int64_t sv[BP_BLOCK / WAVE], si[BP_BLOCK / WAVE];
  for (int64_t gk = blockIdx.x; gk < G; gk += gridDim.x) {
    if (!act[gk]) {
      if (threadIdx.x == 0) best_k[gk] = 0;
      continue;  // uniform over the workgroup
    }
    const int64_t i0 = pos[vbase[gk]], i1 = pos[vbase[gk + 1]];
    const uint64_t base = (uint64_t)S[i0];
    int64_t bv = 0, bi = INT64_MAX;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BP_BLOCK) {
      const int64_t r = (int64_t)((uint64_t)S[i + 1] - base);
      if (r > bv || (r == bv && r > 0 && i < bi)) { bv = r; bi = i; }
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const int64_t ov = __shfl_xor(bv, o, WAVE), oi = __shfl_xor(bi, o, WAVE);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) { sv[wv] = bv; si[wv] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < BP_BLOCK / WAVE; ++w)
        if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) { bv = sv[w]; bi = si[w]; }
      best_k[gk] = bv > 0 ? bi + 1 - i0 : 0;
    }
    __syncthreads();
  }
}

__global__ void k_commit_prefix_seg(int64_t n, uint8_t* keep, const int32_t* pos, const int32_t* gid,
                                    const int32_t* vbase, const int64_t* best_k) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = gid[v];
    keep[v] = keep[v] && pos[v] - pos[vbase[k]] < best_k[k];
  }
}

__global__ void k_commit_prefix(int64_t n, uint8_t* keep, const int32_t* pos, const Ctrl* ctrl) {
  const int64_t kb = ctrl->lmalt_best_k;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keep[v] = keep[v] && pos[v] < kb;
}

__global__ void k_set_counts(Ctrl* ctrl, int64_t k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctrl->lmalt_k = k;
    ctrl->lmalt_best_k = 0;
    ctrl->lmalt_best = 0;
  }
}

}  // namespace

// Precondition: bufs.C is the clustering, bufs.W its cluster weights.  On return bufs.C holds the result;
// ctrl->lmalt_k and ctrl->lmalt_best_k the mover count and the committed prefix.  take() hands out device
// scratch that stays valid until the call's stream has finished (sized by the mover count).  Returns false
// (nothing changed) when there are 2^30 movers or more.
bool lmalt(const DevGraph& g, const Buckets& b, const Score& sc, LMBuffers& bufs, LMSlot* slot, Ctrl* ctrl,
           int32_t* list, int64_t* gain, const std::function<void*(size_t)>& take, hipStream_t st,
           const AltSeg* seg) {
  const int64_t n = g.n;
  ScoreSrc ss;
  ss.s = sc;
  if (seg) ss = seg->ss;
  zero_bytes(slot, sizeof(LMSlot), st);
  launch_destinations_strict(g, b, ss, bufs, slot, st);
  k_mover_flags<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.vs, bufs.keep, seg ? ss.gid : nullptr, seg ? seg->act : nullptr);
  scan_u8_i32(bufs.keep, bufs.scan_a, n, bufs.scan_temp, nullptr, st);
  int32_t k32 = 0;
  hipMemcpyAsync(&k32, bufs.scan_a + n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  const int64_t k = k32;
  k_set_counts<<<1, 1, 0, st>>>(ctrl, k);
  if (k == 0) return true;
  if (4 * k > (int64_t)UINT32_MAX) return false;  // record ids are 32-bit
  k_mover_list<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.keep, bufs.scan_a, list);
  const int64_t m = 4 * k;
  auto* key0 = (uint64_t*)take((size_t)m * 8);
  auto* key1 = (uint64_t*)take((size_t)m * 8);
  auto* val0 = (uint32_t*)take((size_t)m * 4);
  auto* val1 = (uint32_t*)take((size_t)m * 4);
  auto* evw = (int64_t*)take((size_t)m * 8);
  auto* x = (int64_t*)take((size_t)m * 8);
  auto* S = (int64_t*)take((size_t)(m + 1) * 8);
  auto* head = (uint8_t*)take((size_t)m);
  auto* H = (int32_t*)take((size_t)(m + 1) * 4);
  auto* base = (int64_t*)take((size_t)m * 8);
  auto* F = (int64_t*)take((size_t)m * 8);
  auto* adj = (int64_t*)take((size_t)k * 8);
  void* stemp = take(scan_temp_bytes(m + 1));
  void* rtemp = take(radix_temp_bytes(m));
  auto* S2 = (int64_t*)take((size_t)(k + 1) * 8);
  const unsigned gw = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(k, BLOCK / WAVE), 2048));
  const int32_t* hubs = b.list + b.off[NBUCKET - 1];
  const int64_t n7 = b.count[NBUCKET - 1];
  if (n7) fill_i64(adj, 0, k, st);
  k_gain_adj<<<gw, BLOCK, 0, st>>>(list, k, g, bufs.vs, bufs.keep, bufs.scan_a, b.hub_deg, adj);
  if (n7) k_gain_adj_hub<<<(unsigned)b.hub_chunks, BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, bufs.vs, bufs.keep,
                                                                bufs.scan_a, adj);
  int kb = 1, nb = 1;
  while (((int64_t)1 << kb) < k) ++kb;
  while (((int64_t)1 << nb) < n) ++nb;
  const int cs = kb + 1;
  // real keys are below 2^(cs + nb); one more bit keeps NO_KEY (all ones in the sorted bits) strictly last
  int shifts[8], np = 0;
  for (int t = 0; t < cs + nb + 1 && np < 8; t += 8) shifts[np++] = t;
  k_alt_records<<<grid_for(k), BLOCK, 0, st>>>(list, k, cs, bufs.vs, g.vw, key0, val0, evw);
  const int which = radix_sort_pairs(key0, val0, key1, val1, m, shifts, np, rtemp, st);
  const uint64_t* ks = which ? key1 : key0;
  const uint32_t* vs_ = which ? val1 : val0;
  k_alt_gather<<<grid_for(m), BLOCK, 0, st>>>(ks, vs_, evw, m, cs, x, head);
  scan_i64_i64(x, S, m, stemp, st);
  scan_u8_i32(head, H, m, stemp, nullptr, st);
  k_alt_base<<<grid_for(m), BLOCK, 0, st>>>(head, H, S, m, base);
  k_alt_query<<<grid_for(m), BLOCK, 0, st>>>(ks, vs_, head, H, S, base, m, F);
  k_gain<<<grid_for(k), BLOCK, 0, st>>>(list, k, bufs.vs, g.vw, ss, adj, F, gain);
  scan_i64_i64(gain, S2, k, stemp, st);
  if (seg) {
    const int64_t G = seg->sg.G;
    k_best_prefix_seg<<<(unsigned)std::min<int64_t>(G, 4096), BP_BLOCK, 0, st>>>(S2, bufs.scan_a, ss.vbase, G, seg->act,
                                                                                 seg->best_k);
    k_commit_prefix_seg<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.keep, bufs.scan_a, ss.gid, ss.vbase, seg->best_k);
  } else {
    k_best_prefix<<<1, BP_BLOCK, 0, st>>>(S2, k, ctrl);
    k_commit_prefix<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.keep, bufs.scan_a, ctrl);
  }
  launch_apply_and_empty(g, b, bufs, seg ? seg->sg : SegLM{}, slot, st);
  return true;
}

}  // namespace lcc
