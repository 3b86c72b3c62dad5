// Grouped placement and segmented sorting, for the two sorts of the hot path whose keys are (segment, key
// inside the segment): the contraction's (coarse row x, neighbour y) entries (Alg. 4) and pLeidenR's tree
// members by (root, ordering f) (Alg. 6).
//
// Instead of an LSD radix sort over every key bit, the items are first placed into their segment's range
// (sizes are known up front, so the range of segment s starts at an exclusive scan of the sizes; items of one
// tile claim space with one global atomic per distinct segment), and then each segment is sorted on its own,
// by size class: up to 16 or 64 items by ranking in a group of 16 or 64 lanes (shuffles, no LDS), up to 128 by
// a bitonic network in the registers of one wavefront, up to 512 by a bitonic network in LDS (one workgroup),
// and the longer segments in place by an LSD radix sort over the key bits inside the segment (tile histograms
// laid out by segment).
// Equal keys may end in any order; the callers either have unique keys or sum equal keys' values.
#include <algorithm>
#include <functional>

#include "common.h"

namespace lcc {

namespace {

constexpr int PL_TILE = 2048;            // items per placement tile
constexpr int PL_SLOTS = 2 * PL_TILE;    // LDS hash of the tile's segments

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}
inline unsigned tile_blocks(int64_t tiles, int64_t cap) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, cap));
}

// The tile's LDS hash also lists its occupied slots (each wavefront appends its new slots with one LDS
// atomic): the per-tile flush and the reset for the next tile visit only those, not the whole table.
// Probes key g into the table; returns the slot, and whether g took a new one, for a converged wavefront
// (lanes with act false probe nothing).
__device__ __forceinline__ int pl_claim(int32_t* hk, uint16_t* hl, int* hn, bool act, int32_t g) {
  int h = -1, claimed = 0;
  if (act) {
    uint32_t x = fmix32((uint32_t)g) & (PL_SLOTS - 1);
    for (int probe = 0; probe < PL_SLOTS; ++probe) {
      const int32_t prev = atomicCAS(&hk[x], -1, g);
      if (prev == -1 || prev == g) { claimed = prev == -1; break; }
      x = (x + 1) & (PL_SLOTS - 1);
    }
    h = (int)x;
  }
  const uint64_t m = __ballot(claimed);
  if (m) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(hn, __popcll(m));
    base = __shfl(base, leader, WAVE);
    if (claimed) hl[base + __popcll(m & ((1ull << lane) - 1))] = (uint16_t)h;
  }
  return h;
}

// out[grp[i]] += cnt[i] for grp[i] >= 0
__global__ __launch_bounds__(BLOCK) void k_group_sum(const int32_t* grp, const int32_t* cnt, int64_t n,
                                                     int64_t* out) {
  __shared__ int32_t hk[PL_SLOTS];
  __shared__ unsigned long long hv[PL_SLOTS];
  __shared__ uint16_t hl[PL_TILE];  // a tile has at most PL_TILE distinct keys
  __shared__ int hn;
  constexpr int IPT = PL_TILE / BLOCK;
  for (int s = threadIdx.x; s < PL_SLOTS; s += BLOCK) { hk[s] = -1; hv[s] = 0; }
  if (threadIdx.x == 0) hn = 0;
  __syncthreads();
  for (int64_t t0 = (int64_t)blockIdx.x * PL_TILE; t0 < n; t0 += (int64_t)gridDim.x * PL_TILE) {  // uniform
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int64_t i = t0 + (int64_t)k * BLOCK + threadIdx.x;
      const int32_t g = i < n ? grp[i] : -1;
      const int32_t c = i < n ? cnt[i] : 0;
      const bool act = g >= 0 && c > 0;
      const int h = pl_claim(hk, hl, &hn, act, g);
      if (act) atomicAdd(&hv[h], (unsigned long long)c);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < hn; j += BLOCK) {
      const int sl = hl[j];
      atomicAdd((unsigned long long*)&out[hk[sl]], hv[sl]);
      hk[sl] = -1;
      hv[sl] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) hn = 0;
    __syncthreads();
  }
}

// Item i (grp[i] >= 0, mask[i] set when mask is given) receives pos[i], the start of cnt[i] positions (1 when
// cnt is null) inside its segment; cursor[s] starts at segment s's first position and is advanced.
__global__ __launch_bounds__(BLOCK) void k_group_place(const int32_t* grp, const int32_t* cnt, const uint8_t* mask,
                                                       int64_t n, unsigned long long* cursor, int64_t* pos) {
  __shared__ int32_t hk[PL_SLOTS];
  __shared__ unsigned long long hs[PL_SLOTS];  // the tile's total per segment, then the base it claimed
  __shared__ uint16_t hl[PL_TILE];
  __shared__ int hn;
  constexpr int IPT = PL_TILE / BLOCK;
  for (int s = threadIdx.x; s < PL_SLOTS; s += BLOCK) { hk[s] = -1; hs[s] = 0; }
  if (threadIdx.x == 0) hn = 0;
  __syncthreads();
  for (int64_t t0 = (int64_t)blockIdx.x * PL_TILE; t0 < n; t0 += (int64_t)gridDim.x * PL_TILE) {  // uniform
    int slot[IPT];
    unsigned long long in_tile[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int64_t i = t0 + (int64_t)k * BLOCK + threadIdx.x;
      bool act = i < n && (!mask || mask[i]);
      const int32_t g = act ? grp[i] : -1;
      const unsigned long long c = !act ? 0ull : cnt ? (unsigned long long)(cnt[i] > 0 ? cnt[i] : 0) : 1ull;
      act = act && g >= 0 && c != 0;
      const int h = pl_claim(hk, hl, &hn, act, g);
      slot[k] = act ? h : -1;
      in_tile[k] = act ? atomicAdd(&hs[h], c) : 0ull;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < hn; j += BLOCK) {
      const int sl = hl[j];
      hs[sl] = atomicAdd(&cursor[hk[sl]], hs[sl]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (slot[k] >= 0) pos[t0 + (int64_t)k * BLOCK + threadIdx.x] = (int64_t)(hs[slot[k]] + in_tile[k]);
    __syncthreads();
    for (int j = threadIdx.x; j < hn; j += BLOCK) {
      const int sl = hl[j];
      hk[sl] = -1;
      hs[sl] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) hn = 0;
    __syncthreads();
  }
}

__global__ void k_copy_u64(const int64_t* src, int64_t n, unsigned long long* dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (unsigned long long)src[i];
}

// Segments by size class: 1 (1..16 items), 2 (17..64), 3 (65..128), 4 (129..SEG_MED), 5 (longer); empty ones
// need nothing.
constexpr int SEG_MED = 512;
constexpr int NCLASS = 6;
constexpr int C_LONG = NCLASS - 1;

__device__ __forceinline__ int seg_class(int64_t sz) {
  return sz <= 0 ? 0 : sz <= 16 ? 1 : sz <= 64 ? 2 : sz <= 128 ? 3 : sz <= SEG_MED ? 4 : C_LONG;
}

// lists[c][..] = the segments of class c (in any order); counts[c] = their number.  Each workgroup counts the
// classes of all its segments first and claims one range per class with one global atomic (same-address
// atomics serialise, so not one per tile), then writes its segments into those ranges.  Within a wavefront,
// the lanes of a class are counted by ballot and added with one LDS atomic.
__global__ __launch_bounds__(BLOCK) void k_seg_classify(const int64_t* off, int64_t nseg, int32_t* lists,
                                                        unsigned long long* counts) {
  __shared__ unsigned int lc[NCLASS];
  __shared__ unsigned long long base[NCLASS];
  const int lane = threadIdx.x & (WAVE - 1);
  const uint64_t lt = (1ull << lane) - 1;
  if (threadIdx.x < NCLASS) lc[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t s0 = (int64_t)blockIdx.x * BLOCK; s0 < nseg; s0 += (int64_t)gridDim.x * BLOCK) {  // uniform
    const int64_t s = s0 + threadIdx.x;
    const int c = s < nseg ? seg_class(off[s + 1] - off[s]) : 0;
#pragma unroll
    for (int k = 1; k < NCLASS; ++k) {
      const uint64_t m = __ballot(c == k);
      if (lane == 0 && m) atomicAdd(&lc[k], (unsigned int)__popcll(m));
    }
  }
  __syncthreads();
  if (threadIdx.x > 0 && threadIdx.x < NCLASS) {
    base[threadIdx.x] = lc[threadIdx.x] ? atomicAdd(&counts[threadIdx.x], (unsigned long long)lc[threadIdx.x]) : 0;
    lc[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t s0 = (int64_t)blockIdx.x * BLOCK; s0 < nseg; s0 += (int64_t)gridDim.x * BLOCK) {
    const int64_t s = s0 + threadIdx.x;
    const int c = s < nseg ? seg_class(off[s + 1] - off[s]) : 0;
#pragma unroll
    for (int k = 1; k < NCLASS; ++k) {
      const uint64_t m = __ballot(c == k);
      if (!m) continue;  // uniform over the wavefront
      const int leader = __ffsll((unsigned long long)m) - 1;
      unsigned int b = 0;
      if (lane == leader) b = atomicAdd(&lc[k], (unsigned int)__popcll(m));
      b = __shfl(b, leader, WAVE);
      if (c == k) lists[(int64_t)k * nseg + (int64_t)(base[k] + b + (unsigned int)__popcll(m & lt))] = (int32_t)s;
    }
  }
}

// Segments of at most G items, one group of G lanes each: every item's rank in its segment is the number of
// smaller keys (ties by position), found with G shuffles.
template <int G>
__global__ __launch_bounds__(BLOCK) void k_seg_rank(const int32_t* list, const unsigned long long* count,
                                                    const int64_t* off, const uint64_t* kin, const uint32_t* vin,
                                                    uint64_t* kout, uint32_t* vout) {
  const int64_t cnt = (int64_t)*count;
  const int gl = threadIdx.x % G;
  for (int64_t q = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / G; q < cnt; q += (int64_t)gridDim.x * (BLOCK / G)) {
    const int64_t s = list[q];
    const int64_t b = off[s], sz = off[s + 1] - b;
    const bool in = gl < sz;
    const uint64_t key = in ? kin[b + gl] : ~0ull;
    const uint32_t val = in ? vin[b + gl] : 0u;
    int rank = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const uint64_t kk = __shfl(key, k, G);
      rank += (kk < key) || (kk == key && k < gl);
    }
    if (in) {
      kout[b + rank] = key;
      vout[b + rank] = val;
    }
  }
}

// Segments of 65..128 items, one wavefront each, bitonic in registers: lane l holds items l and l + 64, pairs
// 64 apart meet inside a lane, closer pairs across lanes by shuffles.  Padding keys are all ones.
__global__ __launch_bounds__(BLOCK) void k_seg_wave_bitonic(const int32_t* list, const unsigned long long* count,
                                                            const int64_t* off, const uint64_t* kin,
                                                            const uint32_t* vin, uint64_t* kout, uint32_t* vout) {
  const int64_t cnt = (int64_t)*count;
  const int lane = threadIdx.x & (WAVE - 1);
  for (int64_t q = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE; q < cnt; q += (int64_t)gridDim.x * (BLOCK / WAVE)) {
    const int64_t s = list[q];
    const int64_t b = off[s], sz = off[s + 1] - b;
    uint64_t k0 = lane < sz ? kin[b + lane] : ~0ull, k1 = lane + WAVE < sz ? kin[b + lane + WAVE] : ~0ull;
    uint32_t v0 = lane < sz ? vin[b + lane] : 0u, v1 = lane + WAVE < sz ? vin[b + lane + WAVE] : 0u;
    for (int size = 2; size <= 2 * WAVE; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        if (stride == WAVE) {  // items l and l + 64: ascending, since (l & 128) == 0
          if (k0 > k1) {
            const uint64_t tk = k0; k0 = k1; k1 = tk;
            const uint32_t tv = v0; v0 = v1; v1 = tv;
          }
        } else {
          const bool lower = (lane & stride) == 0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            uint64_t& k = h ? k1 : k0;
            uint32_t& v = h ? v1 : v0;
            const int i = lane + h * WAVE;
            const uint64_t pk = __shfl_xor(k, stride, WAVE);
            const uint32_t pv = __shfl_xor(v, stride, WAVE);
            const bool asc = (i & size) == 0;
            const bool take = lower == asc ? pk < k : pk > k;  // the lower slot keeps the min when ascending
            if (take) { k = pk; v = pv; }
          }
        }
      }
    }
    if (lane < sz) { kout[b + lane] = k0; vout[b + lane] = v0; }
    if (lane + WAVE < sz) { kout[b + lane + WAVE] = k1; vout[b + lane + WAVE] = v1; }
  }
}

// ascending bitonic sort of N (a power of two, <= SEG_MED) keys with their values, in LDS
__device__ __forceinline__ void bitonic_lds(uint64_t* k, uint32_t* v, int N) {
  for (int size = 2; size <= N; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < N / 2; i += BLOCK) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == asc) {
          k[lo] = b;
          k[hi] = a;
          const uint32_t t = v[lo];
          v[lo] = v[hi];
          v[hi] = t;
        }
      }
    }
  __syncthreads();
}

// Segments of 129..SEG_MED items, one workgroup each, bitonic in LDS (the radix passes of the long segments
// beat the network beyond a few hundred items).
__global__ __launch_bounds__(BLOCK) void k_seg_bitonic(const int32_t* list, const unsigned long long* count,
                                                       const int64_t* off, const uint64_t* kin, const uint32_t* vin,
                                                       uint64_t* kout, uint32_t* vout) {
  __shared__ uint64_t sk[SEG_MED];
  __shared__ uint32_t sv[SEG_MED];
  const int64_t cnt = (int64_t)*count;
  for (int64_t q = blockIdx.x; q < cnt; q += gridDim.x) {
    const int64_t s = list[q];
    const int64_t b = off[s], sz = off[s + 1] - b;
    int N = 1;
    while (N < sz) N <<= 1;
    for (int i = threadIdx.x; i < N; i += BLOCK) {
      sk[i] = i < sz ? kin[b + i] : ~0ull;
      sv[i] = i < sz ? vin[b + i] : 0u;
    }
    bitonic_lds(sk, sv, N);
    for (int i = threadIdx.x; i < sz; i += BLOCK) {
      kout[b + i] = sk[i];
      vout[b + i] = sv[i];
    }
    __syncthreads();
  }
}

// Long segments are sorted in place by an LSD radix sort over the key bits inside the segment only: the
// tiles of every long segment keep per-tile digit counts laid out as (segment rank, digit, tile), so one
// exclusive scan over them gives each item's position in the concatenation of the long segments, which maps
// back into its own segment's range.
constexpr int SR_TILE = 4096;

__global__ void k_seg_long_sizes(const int32_t* list, int64_t nlong, const int64_t* off, int64_t* size,
                                 int64_t* ntile) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nlong; r += (int64_t)gridDim.x * blockDim.x) {
    size[r] = off[list[r] + 1] - off[list[r]];
    ntile[r] = cdiv(size[r], SR_TILE);
  }
}

struct LongTile {
  int64_t r, t, nt, b, e;  // segment rank, tile of the segment, tiles of the segment, item range
};

__device__ __forceinline__ LongTile long_tile(int64_t g, const int64_t* toff, int64_t nlong, const int32_t* list,
                                              const int64_t* off) {
  int64_t lo = 0, hi = nlong - 1;  // last r with toff[r] <= g
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  LongTile lt;
  lt.r = lo;
  lt.t = g - toff[lo];
  lt.nt = toff[lo + 1] - toff[lo];
  const int64_t s = list[lo];
  lt.b = off[s] + lt.t * SR_TILE;
  lt.e = min(off[s + 1], lt.b + SR_TILE);
  return lt;
}

__global__ __launch_bounds__(BLOCK) void k_segradix_hist(const uint64_t* keys, const int64_t* off, const int32_t* list,
                                                         const int64_t* toff, int64_t nlong, int shift,
                                                         uint32_t* hist) {
  __shared__ uint32_t cnt[256];
  const LongTile lt = long_tile(blockIdx.x, toff, nlong, list, off);
  cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = lt.b + threadIdx.x; i < lt.e; i += BLOCK) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[256 * toff[lt.r] + (int64_t)threadIdx.x * lt.nt + lt.t] = cnt[threadIdx.x];
}

// Stable scatter of one tile: items in rounds of 256 in index order; a lane's rank among same-digit items of
// its round is the count of lower lanes of its wavefront with the same digit (ballot match) plus the counts of
// the earlier wavefronts.
__global__ __launch_bounds__(BLOCK) void k_segradix_scatter(const uint64_t* kin, const uint32_t* vin,
                                                            const int64_t* off, const int32_t* list,
                                                            const int64_t* toff, const int64_t* loff, int64_t nlong,
                                                            int shift, const uint32_t* offs, uint64_t* kout,
                                                            uint32_t* vout) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[BLOCK / WAVE][256];
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid & (WAVE - 1);
  const LongTile lt = long_tile(blockIdx.x, toff, nlong, list, off);
  base[tid] = offs[256 * toff[lt.r] + (int64_t)tid * lt.nt + lt.t];
  const int64_t to_array = off[list[lt.r]] - loff[lt.r];  // position in the concatenation -> in the array
  const uint64_t lm = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  for (int64_t r0 = lt.b; r0 < lt.e; r0 += BLOCK) {  // block-uniform
#pragma unroll
    for (int k = 0; k < BLOCK / WAVE; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const int64_t i = r0 + tid;
    const bool valid = i < lt.e;
    const uint64_t key = valid ? kin[i] : 0;
    const uint32_t val = valid ? vin[i] : 0;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      mask &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t prank = (uint32_t)__popcll(mask & lm);
    if (valid && prank == 0) wcnt[wv][d] = (uint32_t)__popcll(mask);
    __syncthreads();
    {
      uint32_t run = base[tid];
#pragma unroll
      for (int k = 0; k < BLOCK / WAVE; ++k) {
        const uint32_t c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const int64_t dst = to_array + (int64_t)(wcnt[wv][d] + prank);
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(BLOCK) void k_seg_long_copy(const uint64_t* kin, const uint32_t* vin, const int64_t* off,
                                                         const int32_t* list, const int64_t* toff, int64_t nlong,
                                                         uint64_t* kout, uint32_t* vout) {
  const LongTile lt = long_tile(blockIdx.x, toff, nlong, list, off);
  for (int64_t i = lt.b + threadIdx.x; i < lt.e; i += BLOCK) {
    kout[i] = kin[i];
    vout[i] = vin[i];
  }
}

}  // namespace

void launch_group_sum(const int32_t* grp, const int32_t* cnt, int64_t n, int64_t* out, hipStream_t st) {
  k_group_sum<<<tile_blocks(cdiv(n, PL_TILE), 4096), BLOCK, 0, st>>>(grp, cnt, n, out);
}

void launch_group_place(const int32_t* grp, const int32_t* cnt, const uint8_t* mask, int64_t n, const int64_t* start,
                        int64_t nseg, unsigned long long* cursor, int64_t* pos, hipStream_t st) {
  k_copy_u64<<<grid_for(nseg), BLOCK, 0, st>>>(start, nseg, cursor);
  k_group_place<<<tile_blocks(cdiv(n, PL_TILE), 4096), BLOCK, 0, st>>>(grp, cnt, mask, n, cursor, pos);
}

void segsort_pairs(uint64_t* kin, uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t m,
                   const int64_t* off, int64_t nseg, int low_bits, void* scan_temp,
                   const std::function<void*(size_t)>& take, hipStream_t st) {
  if (m <= 0 || nseg <= 0) return;
  auto* counts = (unsigned long long*)take(NCLASS * sizeof(unsigned long long));
  auto* lists = (int32_t*)take((size_t)NCLASS * nseg * sizeof(int32_t));
  zero_bytes(counts, NCLASS * sizeof(unsigned long long), st);
  k_seg_classify<<<tile_blocks(cdiv(nseg, BLOCK), 512), BLOCK, 0, st>>>(off, nseg, lists, counts);
  unsigned long long hc[NCLASS] = {};
  device_check(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st), "segment classes");
  device_check(hipStreamSynchronize(st), "segment classes");
  if (hc[1]) k_seg_rank<16><<<tile_blocks(cdiv((int64_t)hc[1], BLOCK / 16), 4096), BLOCK, 0, st>>>(
      lists + 1 * nseg, counts + 1, off, kin, vin, kout, vout);
  if (hc[2]) k_seg_rank<64><<<tile_blocks(cdiv((int64_t)hc[2], BLOCK / 64), 4096), BLOCK, 0, st>>>(
      lists + 2 * nseg, counts + 2, off, kin, vin, kout, vout);
  if (hc[3]) k_seg_wave_bitonic<<<tile_blocks(cdiv((int64_t)hc[3], BLOCK / WAVE), 4096), BLOCK, 0, st>>>(
      lists + 3 * nseg, counts + 3, off, kin, vin, kout, vout);
  if (hc[4]) k_seg_bitonic<<<tile_blocks((int64_t)hc[4], 2048), BLOCK, 0, st>>>(lists + 4 * nseg, counts + 4, off,
                                                                                 kin, vin, kout, vout);
  const int64_t nlong = (int64_t)hc[C_LONG];
  if (nlong == 0) return;
  // long segments, in place: passes alternate between (kin, vin) and (kout, vout) on their ranges
  const int32_t* list = lists + C_LONG * nseg;
  auto* size = (int64_t*)take((size_t)nlong * 8);
  auto* ntile = (int64_t*)take((size_t)nlong * 8);
  auto* loff = (int64_t*)take((size_t)(nlong + 1) * 8);
  auto* toff = (int64_t*)take((size_t)(nlong + 1) * 8);
  k_seg_long_sizes<<<grid_for(nlong), BLOCK, 0, st>>>(list, nlong, off, size, ntile);
  scan_i64_i64(size, loff, nlong, scan_temp, st);
  scan_i64_i64(ntile, toff, nlong, scan_temp, st);
  int64_t T = 0;
  device_check(hipMemcpyAsync(&T, toff + nlong, sizeof(int64_t), hipMemcpyDeviceToHost, st), "long tiles");
  device_check(hipStreamSynchronize(st), "long tiles");
  auto* hist = (uint32_t*)take((size_t)(256 * T + 1) * 4);
  auto* offs = (uint32_t*)take((size_t)(256 * T + 1) * 4);
  uint64_t* ka = kin;
  uint32_t* va = vin;
  uint64_t* kb = kout;
  uint32_t* vb = vout;
  int np = 0;
  for (int sh = 0; sh < low_bits; sh += 8, ++np) {
    k_segradix_hist<<<(unsigned)T, BLOCK, 0, st>>>(ka, off, list, toff, nlong, sh, hist);
    scan_u32_u32(hist, offs, 256 * T, scan_temp, st);
    k_segradix_scatter<<<(unsigned)T, BLOCK, 0, st>>>(ka, va, off, list, toff, loff, nlong, sh, offs, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != kout) k_seg_long_copy<<<(unsigned)T, BLOCK, 0, st>>>(ka, va, off, list, toff, nlong, kout, vout);
}

}  // namespace lcc
