// Graph contraction (Alg. 4) as relabel + sort + segmented reduce, and the projections between levels.
//
// Coarse vertex x = rank of cluster id among the ids in use (ascending compaction by prefix scan).  Every
// fine entry (v, u, w) with map[v] != map[u] is emitted as key (map[v] << 32 | map[u]), value w, into coarse
// row x's range (per-row entry counts and grouped placement, segsort.hip); each row is then sorted by y, which
// brings equal keys together in (x, y) order; run heads become the coarse entries (neighbours ascending,
// weights summed from a prefix scan of the values, self-loops dropped).  The result is the canonical coarse
// CSR independent of scheduling.
#include "common.h"

namespace lcc {

namespace {

constexpr int HUB_BLOCK = 256;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}
// persistent launches (at most 2048 workgroups looping over their share of the vertices)
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

// In a union of graphs, gact (per graph, indexed through gid) restricts the labels to the graphs that go on
// to the next level; the other graphs' vertices map to -1 and produce no coarse vertex or entry.
__global__ void k_mark_used(const int32_t* labels, int64_t n, uint8_t* used, const int32_t* gid,
                            const uint8_t* gact) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (!gact || gact[gid[v]]) used[labels[v]] = 1;
}

__global__ void k_map(const int32_t* labels, const int32_t* rank, int64_t n, int32_t* map, const int32_t* gid,
                      const uint8_t* gact) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    map[v] = (!gact || gact[gid[v]]) ? rank[labels[v]] : -1;
}

// graph of each coarse vertex, and each graph's first coarse id (vbase_c[k] = rank[vbase[k]], k <= G)
__global__ void k_coarse_gid(const int32_t* map, const int32_t* gid, int64_t n, int32_t* cgid) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (map[v] >= 0) cgid[map[v]] = gid[v];
}

__global__ void k_rebase(const int32_t* rank, const int32_t* vbase, int64_t G, int32_t* vbase_c) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= G; k += (int64_t)gridDim.x * blockDim.x)
    vbase_c[k] = rank[vbase[k]];
}

__global__ __launch_bounds__(BLOCK) void k_coarse_vw(const int32_t* map, const int64_t* vw, int64_t n,
                                                     int64_t* cvw) {
  constexpr int SLOTS = 4096, T = 2048;
  __shared__ int32_t ak[SLOTS];
  __shared__ unsigned long long av[SLOTS];
  LdsAgg<SLOTS> agg{ak, av};
  for (int64_t t0 = (int64_t)blockIdx.x * T; t0 < n; t0 += (int64_t)gridDim.x * T) {
    agg.clear();
    __syncthreads();
    for (int k = threadIdx.x; k < T; k += BLOCK) {
      int64_t v = t0 + k;
      if (v >= n) break;
      if (map[v] >= 0) agg.add(map[v], vw[v]);
    }
    __syncthreads();
    agg.flush(cvw);
    __syncthreads();
  }
}

// cross-cluster entries per fine vertex; G lanes per vertex (G = 64 also covers whole-block rows by
// striding), hubs by chunks with atomics
template <int G>
__global__ __launch_bounds__(BLOCK) void k_cross_count_grp(const int32_t* list, int64_t cnt, DevGraph g,
                                                           const int32_t* map, int32_t* out) {
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int32_t x = map[v];
    int c = 0;
    for (int64_t j = g.off[v] + gl; j < g.off[v + 1]; j += G) c += map[g.idx[j]] != x;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, G);
    if (gl == 0) out[v] = c;
  }
}

__global__ __launch_bounds__(HUB_BLOCK) void k_cross_count_chunk(const int32_t* hubs, const int32_t* chunk_off,
                                                                 int64_t n7, int64_t chunk, DevGraph g,
                                                                 const int32_t* map, int32_t* out) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int32_t x = map[v];
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * chunk;
  const int64_t j1 = min(g.off[v + 1], j0 + chunk);
  int c = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK) c += map[g.idx[j]] != x;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0 && c) atomicAdd(&out[v], c);
}

// Emit (x << 32 | y, w); positions claimed per group with one atomic on the vertex cursor (the cursor
// starts at the vertex's exclusive prefix of cross entries).
template <int G>
__global__ __launch_bounds__(BLOCK) void k_cross_emit_grp(const int32_t* list, int64_t cnt, DevGraph g,
                                                          const int32_t* map, int64_t* cursor, uint64_t* keys,
                                                          uint32_t* vals) {
  const int gl = threadIdx.x % G;
  // the loop bound is the same for every lane of the workgroup: the ballots below see whole wavefronts
  for (int64_t gb0 = (int64_t)blockIdx.x * (BLOCK / G); gb0 < cnt; gb0 += (int64_t)gridDim.x * (BLOCK / G)) {
  const int64_t gid = gb0 + threadIdx.x / G;
  // groups past the end still execute the ballots (uniform control flow inside the wavefront)
  const bool active = gid < cnt;
  const int32_t v = active ? list[gid] : 0;
  const int64_t j0 = active ? g.off[v] : 0, j1 = active ? g.off[v + 1] : 0;
  // trip count must be uniform across the wavefront for the ballots: iterate to the wave's max degree
  int64_t d = j1 - j0;
  int64_t dmax = d;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, WAVE));
  const int32_t x = active ? map[v] : -1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int gbase = lane - gl;
  const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  for (int64_t off = 0; off < dmax; off += G) {
    int64_t j = j0 + off + gl;
    bool in = active && j < j1;
    int32_t y = in ? map[g.idx[j]] : -1;
    bool cross = in && y != x;
    uint64_t m = __ballot(cross) & gmask;
    int64_t base = 0;
    int leader = m ? __ffsll((unsigned long long)m) - 1 : gbase;
    if (m && lane == leader)
      base = (int64_t)atomicAdd((unsigned long long*)&cursor[v], (unsigned long long)__popcll(m));
    base = __shfl(base, leader, WAVE);
    if (cross) {
      int64_t p = base + __popcll(m & lt);
      keys[p] = ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
      vals[p] = (uint32_t)g.w[j];
    }
  }
  }
}

// rows handled by whole workgroups (bucket 6) or hub chunks: each wavefront claims its own positions
__global__ __launch_bounds__(HUB_BLOCK) void k_cross_emit_chunk(const int32_t* list, const int32_t* chunk_off,
                                                                int64_t nv, int64_t chunk, DevGraph g,
                                                                const int32_t* map, int64_t* cursor,
                                                                uint64_t* keys, uint32_t* vals) {
  int k;
  int64_t j0, j1;
  int32_t v;
  if (chunk_off) {
    k = find_chunk_owner(chunk_off, nv, blockIdx.x);
    v = list[k];
    j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * chunk;
    j1 = min(g.off[v + 1], j0 + chunk);
  } else {
    v = list[blockIdx.x];
    j0 = g.off[v];
    j1 = g.off[v + 1];
  }
  const int32_t x = map[v];
  const int lane = threadIdx.x & (WAVE - 1);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  const int wv = threadIdx.x / WAVE;
  for (int64_t jb = j0 + (int64_t)wv * WAVE; jb < j1; jb += HUB_BLOCK) {
    int64_t j = jb + lane;
    bool in = j < j1;
    int32_t y = in ? map[g.idx[j]] : -1;
    bool cross = in && y != x;
    uint64_t m = __ballot(cross);
    if (!m) continue;
    int leader = __ffsll((unsigned long long)m) - 1;
    int64_t base = 0;
    if (lane == leader) base = (int64_t)atomicAdd((unsigned long long*)&cursor[v], (unsigned long long)__popcll(m));
    base = __shfl(base, leader, WAVE);
    if (cross) {
      int64_t p = base + __popcll(m & lt);
      keys[p] = ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
      vals[p] = (uint32_t)g.w[j];
    }
  }
}

__global__ void k_zero_hub_counts(const int32_t* hubs, int64_t n7, int32_t* cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n7; k += (int64_t)gridDim.x * blockDim.x)
    cnt[hubs[k]] = 0;
}

__global__ void k_heads(const uint64_t* keys, int64_t m, uint8_t* head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || keys[i] != keys[i - 1]);
}

// run heads of the sorted keys become coarse entries: neighbour id, run start, row id
__global__ void k_heads_write(const uint64_t* keys, int64_t m, const uint8_t* head, const int32_t* uid,
                              int64_t nnzc, int32_t* cidx, int32_t* hstart, int32_t* ux) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    if (!head[i]) continue;
    uint64_t k = keys[i];
    int32_t u = uid[i];
    cidx[u] = (int32_t)(uint32_t)k;
    hstart[u] = (int32_t)i;
    ux[u] = (int32_t)(k >> 32);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) hstart[nnzc] = (int32_t)m;
}

// run weight = difference of the value prefix sums at consecutive run starts
__global__ void k_run_weights(const int64_t* pref, const int32_t* hstart, int64_t nnzc, int32_t* cw) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nnzc; u += (int64_t)gridDim.x * blockDim.x)
    cw[u] = (int32_t)(pref[hstart[u + 1]] - pref[hstart[u]]);
}

// row offsets: first entry whose row id is >= x (rows are sorted)
__global__ void k_row_offsets(const int32_t* ux, int64_t nnzc, int64_t nc, int64_t* coff) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= nc; x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnzc;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (ux[mid] < x) lo = mid + 1; else hi = mid;
    }
    coff[x] = lo;
  }
}

// vertices with map -1 (graphs of a union that stopped at this level) keep their clustering.  In a union a
// coarse label of graph k lies in k's coarse id range: it is moved to the same offset in k's fine id range.
__global__ void k_project(const int32_t* coarse_C, const int32_t* map, int64_t n, int32_t* fine_C,
                          const int32_t* gid, const int32_t* vbase_f, const int32_t* vbase_c) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = map[v];
    if (x < 0) continue;
    int32_t c = coarse_C[x];
    if (gid) c += vbase_f[gid[v]] - vbase_c[gid[v]];
    fine_C[v] = c;
  }
}

__global__ void k_downsample(const int32_t* B, const int32_t* rankB, const int32_t* map, int64_t n, int32_t* Cc,
                             const int32_t* gid, const int32_t* vbase_f, const int32_t* vbase_c,
                             const uint8_t* keep) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = map[v];
    if (x < 0) continue;
    if (!gid) {
      Cc[x] = rankB[B[v]];
    } else {
      const int32_t k = gid[v], bf = vbase_f[k];
      Cc[x] = (keep && keep[k] ? B[v] - bf : rankB[B[v]] - rankB[bf]) + vbase_c[k];
    }
  }
}

}  // namespace

void launch_label_rank(const int32_t* labels, int64_t n, uint8_t* used, int32_t* rank, void* temp,
                       hipStream_t st, const int32_t* gid, const uint8_t* gact) {
  fill_u8(used, 0, n, st);
  k_mark_used<<<grid_for(n), BLOCK, 0, st>>>(labels, n, used, gid, gact);
  scan_u8_i32(used, rank, n, temp, nullptr, st);
}

void launch_map_labels(const int32_t* labels, const int32_t* rank, int64_t n, int32_t* map, hipStream_t st,
                       const int32_t* gid, const uint8_t* gact) {
  k_map<<<grid_for(n), BLOCK, 0, st>>>(labels, rank, n, map, gid, gact);
}

void launch_coarse_gid(const int32_t* map, const int32_t* gid, int64_t n, int32_t* cgid, hipStream_t st) {
  k_coarse_gid<<<grid_for(n), BLOCK, 0, st>>>(map, gid, n, cgid);
}

void launch_rebase(const int32_t* rank, const int32_t* vbase, int64_t G, int32_t* vbase_c, hipStream_t st) {
  k_rebase<<<grid_for(G + 1), BLOCK, 0, st>>>(rank, vbase, G, vbase_c);
}

void launch_coarse_vw(const int32_t* map, const int64_t* vw, int64_t n, int64_t* cvw, hipStream_t st) {
  unsigned g = (unsigned)(cdiv(n, 2048) < 1 ? 1 : (cdiv(n, 2048) > 4096 ? 4096 : cdiv(n, 2048)));
  k_coarse_vw<<<g, BLOCK, 0, st>>>(map, vw, n, cvw);
}

void launch_cross_count(const DevGraph& g, const Buckets& b, const int32_t* map, int32_t* cnt, hipStream_t st) {
  const int32_t* L = b.list;
  if (b.count[0]) k_cross_count_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, map, cnt);
  if (b.count[1]) k_cross_count_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, map, cnt);
  if (b.count[2]) k_cross_count_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, map, cnt);
  if (b.count[3]) k_cross_count_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, map, cnt);
  int64_t nw = b.count[4] + b.count[5] + b.count[6];
  if (nw) k_cross_count_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, map, cnt);
  if (b.count[7]) {
    const int32_t* hubs = L + b.off[7];
    k_zero_hub_counts<<<grid_for(b.count[7]), BLOCK, 0, st>>>(hubs, b.count[7], cnt);
    k_cross_count_chunk<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, b.count[7],
                                                                     HUB_CHUNK_EDGES, g, map, cnt);
  }
}

void launch_cross_emit(const DevGraph& g, const Buckets& b, const int32_t* map, int64_t* cursor, uint64_t* keys,
                       uint32_t* vals, hipStream_t st) {
  const int32_t* L = b.list;
  if (b.count[0]) k_cross_emit_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, map, cursor, keys, vals);
  if (b.count[1]) k_cross_emit_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, map, cursor, keys, vals);
  if (b.count[2]) k_cross_emit_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, map, cursor, keys, vals);
  if (b.count[3]) k_cross_emit_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, map, cursor, keys, vals);
  int64_t nw = b.count[4] + b.count[5];
  if (nw) k_cross_emit_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, map, cursor, keys, vals);
  if (b.count[6]) k_cross_emit_chunk<<<(unsigned)b.count[6], HUB_BLOCK, 0, st>>>(L + b.off[6], nullptr, b.count[6], 0, g, map, cursor, keys, vals);
  if (b.count[7]) k_cross_emit_chunk<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(L + b.off[7], b.hub_chunk_off, b.count[7], HUB_CHUNK_EDGES, g, map, cursor, keys, vals);
}

void launch_heads(const uint64_t* keys, int64_t m, uint8_t* head, hipStream_t st) {
  k_heads<<<grid_for(m), BLOCK, 0, st>>>(keys, m, head);
}

void launch_coarse_write(const uint64_t* keys, const uint32_t* vals, const uint8_t* head, const int32_t* uid,
                         int64_t m, int64_t nnzc, int64_t nc, int64_t* pref, int32_t* hstart, int32_t* ux,
                         int32_t* cidx, int32_t* cw, int64_t* coff, void* temp, hipStream_t st) {
  scan_u32_i64(vals, pref, m, temp, st);
  k_heads_write<<<grid_for(m), BLOCK, 0, st>>>(keys, m, head, uid, nnzc, cidx, hstart, ux);
  k_run_weights<<<grid_for(nnzc), BLOCK, 0, st>>>(pref, hstart, nnzc, cw);
  k_row_offsets<<<grid_for(nc + 1), BLOCK, 0, st>>>(ux, nnzc, nc, coff);
}

void launch_project(const int32_t* coarse_C, const int32_t* map, int64_t n, int32_t* fine_C, hipStream_t st,
                    const int32_t* gid, const int32_t* vbase_f, const int32_t* vbase_c) {
  k_project<<<grid_for(n), BLOCK, 0, st>>>(coarse_C, map, n, fine_C, gid, vbase_f, vbase_c);
}

void launch_downsample(const int32_t* B, const int32_t* rankB, const int32_t* map, int64_t n, int32_t* Cc,
                       hipStream_t st, const int32_t* gid, const int32_t* vbase_f, const int32_t* vbase_c,
                       const uint8_t* keep) {
  k_downsample<<<grid_for(n), BLOCK, 0, st>>>(B, rankB, map, n, Cc, gid, vbase_f, vbase_c, keep);
}

}  // namespace lcc
