// LocalMoveAlt (Sec. V-A): used when the synchronous local move leaves the objective unchanged.
//
// Every vertex that is not node optimal (its best destination strictly improves the objective) is a mover,
// taken in ascending vertex id with its destination fixed up front.  The exact objective change of applying
// the movers one after another is delta_i adjusted by EVERY earlier mover j -- the afterburner rule of Alg. 3
// with w'(u,v) = w(u,v) - lambda w(u) w(v) over all pairs, adjacent or not.  The shortest prefix with the
// largest total change is committed (it is non-empty: the first mover alone improves).  One workgroup per
// mover sums over the earlier movers; the edge weight w(v_j, v_i) is found by binary search in v_i's sorted
// row only when the cluster pattern of the pair makes it matter.
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

__global__ void k_mover_flags(int64_t n, const VState* vs, uint8_t* mv) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    mv[v] = vs[v].d != D_NONE;
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

__global__ __launch_bounds__(BLOCK) void k_gain(const int32_t* list, int64_t k, DevGraph g, const VState* vs,
                                                Score sc, int64_t* gain) {
  const int64_t i = blockIdx.x;
  const int32_t vi = list[i];
  const VState me = vs[vi];
  const int64_t wi = g.vw[vi];
  const int64_t rb = g.off[vi], re = g.off[vi + 1];
  int64_t acc = 0;
  for (int64_t j = threadIdx.x; j < i; j += BLOCK) {
    const int32_t vj = list[j];
    const VState o = vs[vj];
    int a = pattern(me.c, me.d, o.c, o.d);
    if (a == 0) continue;
    int64_t lo = rb, hi = re;
    while (lo < hi) {
      int64_t mid = lo + ((hi - lo) >> 1);
      if (g.idx[mid] < vj) lo = mid + 1; else hi = mid;
    }
    int64_t w = (lo < re && g.idx[lo] == vj) ? (int64_t)g.w[lo] : 0;
    acc += (int64_t)a * (sc.q * w - sc.p * g.vw[vj] * wi);
  }
  __shared__ int64_t ws[BLOCK / WAVE];
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0) ws[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < BLOCK / WAVE; ++w) t += ws[w];
    gain[i] = me.delta + t;
  }
}

// shortest prefix with the largest positive running sum (one workgroup)
__global__ __launch_bounds__(BLOCK) void k_best_prefix(const int64_t* gain, int64_t k, Ctrl* ctrl) {
  __shared__ int64_t wsum[BLOCK / WAVE];
  __shared__ int64_t s_carry, s_best, s_bestk;
  if (threadIdx.x == 0) { s_carry = 0; s_best = 0; s_bestk = 0; }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  for (int64_t b0 = 0; b0 < k; b0 += BLOCK) {
    int64_t i = b0 + threadIdx.x;
    int64_t x = i < k ? gain[i] : 0;
    int64_t inc = x;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      int64_t y = __shfl_up(inc, o, WAVE);
      if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    int64_t before = s_carry;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    int64_t run = before + inc;  // running sum through item i
    __syncthreads();
    // serial max over this chunk in item order (ties keep the earliest)
    __shared__ int64_t runs[BLOCK];
    runs[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int t = 0; t < BLOCK && b0 + t < k; ++t)
        if (runs[t] > s_best) { s_best = runs[t]; s_bestk = b0 + t + 1; }
      s_carry = runs[min((int64_t)BLOCK, k - b0) - 1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl->lmalt_best_k = s_bestk;
    ctrl->lmalt_best = s_best;
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

// Precondition: bufs.C is the clustering, bufs.W / bufs.sz its cluster weights and sizes.  On return bufs.C
// holds the result; ctrl->lmalt_k and ctrl->lmalt_best_k the mover count and the committed prefix.
void lmalt(const DevGraph& g, const Buckets& b, const Score& sc, LMBuffers& bufs, LMSlot* slot, Ctrl* ctrl,
           int32_t* list, int64_t* gain, hipStream_t st) {
  const int64_t n = g.n;
  zero_bytes(slot, sizeof(LMSlot), st);
  launch_destinations_strict(g, b, sc, bufs, slot, st);
  k_mover_flags<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.vs, bufs.keep);
  scan_u8_i32(bufs.keep, bufs.scan_a, n, bufs.scan_temp, nullptr, st);
  int32_t k32 = 0;
  hipMemcpyAsync(&k32, bufs.scan_a + n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  const int64_t k = k32;
  k_set_counts<<<1, 1, 0, st>>>(ctrl, k);
  if (k == 0) return;
  k_mover_list<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.keep, bufs.scan_a, list);
  k_gain<<<(unsigned)k, BLOCK, 0, st>>>(list, k, g, bufs.vs, sc, gain);
  k_best_prefix<<<1, BLOCK, 0, st>>>(gain, k, ctrl);
  k_commit_prefix<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.keep, bufs.scan_a, ctrl);
  launch_apply_and_empty(g, bufs, slot, st);
}

}  // namespace lcc
