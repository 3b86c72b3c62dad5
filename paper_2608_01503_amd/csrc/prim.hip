// Device-wide primitives for gfx950: exclusive scans (reduce-then-scan over 2048-element tiles) and a stable
// LSD radix sort of (uint64 key, uint32 value) pairs with 8-bit digits (per-tile histograms, a scan of the
// digit-major histogram, and a stable scatter whose in-tile ranks come from wavefront ballots).
#include "common.h"

namespace lcc {

namespace {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;  // 2048
constexpr int RADIX_TILE = 4096;               // 16 rounds of 256 items

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over the block; returns the block total in *total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* total) {
  __shared__ T wsum[BLOCK / WAVE];
  int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  T inc = wave_incl_scan(x);
  if (lane == WAVE - 1) wsum[wv] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < BLOCK / WAVE; ++k) {
    T s = wsum[k];
    if (k < wv) before += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

template <typename In, typename Out>
__global__ __launch_bounds__(BLOCK) void k_tile_reduce(const In* in, int64_t n, Out* sums, const int64_t* cond) {
  if (cond && *cond == 0) return;
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  Out s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += (Out)in[base + k];
  Out tot;
  block_excl_scan<Out>(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place by one block; sums[nt] = grand total.
template <typename Out>
__global__ __launch_bounds__(BLOCK) void k_scan_sums(Out* sums, int64_t nt, const int64_t* cond) {
  if (cond && *cond == 0) return;
  Out carry = 0;
  for (int64_t b0 = 0; b0 < nt; b0 += BLOCK) {
    int64_t i = b0 + threadIdx.x;
    Out x = i < nt ? sums[i] : 0;
    Out tot;
    Out ex = block_excl_scan<Out>(x, &tot);
    if (i < nt) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

template <typename In, typename Out>
__global__ __launch_bounds__(BLOCK) void k_tile_scan(const In* in, Out* out, int64_t n, const Out* sums,
                                                     int64_t nt, const int64_t* cond) {
  if (cond && *cond == 0) return;
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  Out v[SCAN_ITEMS];
  Out s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? (Out)in[base + k] : (Out)0;
    s += v[k];
  }
  Out tot;
  Out run = block_excl_scan<Out>(s, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nt];
}

// Whole scan by one workgroup (tiles in sequence with a carry): small inputs take one launch instead of
// three.
template <typename In, typename Out>
__global__ __launch_bounds__(BLOCK) void k_scan_small(const In* in, Out* out, int64_t n, const int64_t* cond) {
  if (cond && *cond == 0) return;
  Out carry = 0;
  for (int64_t t0 = 0; t0 < n; t0 += SCAN_TILE) {
    const int64_t base = t0 + (int64_t)threadIdx.x * SCAN_ITEMS;
    Out v[SCAN_ITEMS];
    Out s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      v[k] = (base + k < n) ? (Out)in[base + k] : (Out)0;
      s += v[k];
    }
    Out tot;
    Out run = block_excl_scan<Out>(s, &tot) + carry;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
template <typename In, typename Out>
void scan_impl(const In* in, Out* out, int64_t n, void* temp, const int64_t* cond, hipStream_t st) {
  int64_t nt = cdiv(n, SCAN_TILE);
  Out* sums = (Out*)temp;
  if (nt == 0) {
    k_fill<Out><<<1, 1, 0, st>>>(out, (Out)0, 1);
    return;
  }
  if (nt <= 8) {
    k_scan_small<In, Out><<<1, BLOCK, 0, st>>>(in, out, n, cond);
    return;
  }
  k_tile_reduce<In, Out><<<(unsigned)nt, BLOCK, 0, st>>>(in, n, sums, cond);
  k_scan_sums<Out><<<1, BLOCK, 0, st>>>(sums, nt, cond);
  k_tile_scan<In, Out><<<(unsigned)nt, BLOCK, 0, st>>>(in, out, n, sums, nt, cond);
}

// ---------------------------------------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(BLOCK) void k_radix_hist(const uint64_t* keys, int64_t m, int shift, uint32_t* hist,
                                                      int64_t ntiles) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t t0 = (int64_t)blockIdx.x * RADIX_TILE;
  for (int r = 0; r < RADIX_TILE / BLOCK; ++r) {
    int64_t i = t0 + r * BLOCK + threadIdx.x;
    if (i < m) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter.  Items of a tile are taken in rounds of 256 (one per thread, in index order); within a
// round, a lane's rank among same-digit items is the number of lower lanes of its wavefront with the same
// digit (ballot match over the 8 digit bits) plus the counts of the earlier wavefronts of the round.  Each
// item first goes to its place in the tile sorted by digit, in LDS; the sorted tile is then written out with
// consecutive threads on consecutive positions of each digit's run, so the stores coalesce instead of
// scattering every round's items over 256 digit runs.
__global__ __launch_bounds__(BLOCK) void k_radix_scatter(const uint64_t* kin, const uint32_t* vin, int64_t m,
                                                         int shift, const uint32_t* hist, const uint32_t* offs,
                                                         int64_t ntiles, uint64_t* kout, uint32_t* vout) {
  __shared__ uint64_t tk[RADIX_TILE];
  __shared__ uint32_t tv[RADIX_TILE];
  __shared__ uint32_t lbase[256];  // first position of each digit in the sorted tile
  __shared__ uint32_t lrun[256];   // next free position of each digit in the sorted tile
  __shared__ uint32_t gbase[256];  // first global position of this tile's items of each digit
  __shared__ uint32_t wcnt[BLOCK / WAVE][256];
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid & (WAVE - 1);
  const int64_t t0 = (int64_t)blockIdx.x * RADIX_TILE;
  gbase[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
  {  // the tile's digit counts (from the histogram pass), exclusive-scanned over the digits
    uint32_t tot = 0;
    const uint32_t c = hist[(int64_t)tid * ntiles + blockIdx.x];
    const uint32_t ex = block_excl_scan<uint32_t>(c, &tot);
    lbase[tid] = ex;
    lrun[tid] = ex;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  const int items = (int)min<int64_t>(RADIX_TILE, m - t0);
  for (int r = 0; r * BLOCK < items; ++r) {  // block-uniform
#pragma unroll
    for (int k = 0; k < BLOCK / WAVE; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const int li = r * BLOCK + tid;
    const bool valid = li < items;
    const uint64_t key = valid ? kin[t0 + li] : 0;
    const uint32_t val = valid ? vin[t0 + li] : 0;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((d >> b) & 1u);
      mask &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t prank = (uint32_t)__popcll(mask & lt);
    if (valid && prank == 0) wcnt[wv][d] = (uint32_t)__popcll(mask);
    __syncthreads();
    {
      uint32_t run = lrun[tid];
#pragma unroll
      for (int k = 0; k < BLOCK / WAVE; ++k) {
        uint32_t c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      lrun[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wcnt[wv][d] + prank;
      tk[pos] = key;
      tv[pos] = val;
    }
    __syncthreads();  // every wavefront has read its offsets before the next round clears them
  }
  for (int p = tid; p < items; p += BLOCK) {
    const uint64_t key = tk[p];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    const uint32_t dst = gbase[d] + ((uint32_t)p - lbase[d]);
    kout[dst] = key;
    vout[dst] = tv[p];
  }
}

// Whole sort of at most RADIX_TILE pairs by one workgroup in LDS: every pass is a histogram, a scan of the 256
// digit counts and the stable ballot-ranked scatter above, between two LDS buffers.  The result is written to
// (k0, v0).
struct RadixShifts {
  int s[8];
};

__global__ __launch_bounds__(BLOCK) void k_radix_small(uint64_t* k0, uint32_t* v0, int64_t m, RadixShifts sh,
                                                       int npass) {
  __shared__ uint64_t kb[2][RADIX_TILE];
  __shared__ uint32_t vb[2][RADIX_TILE];
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[BLOCK / WAVE][256];
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid & (WAVE - 1);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  for (int64_t i = tid; i < m; i += BLOCK) { kb[0][i] = k0[i]; vb[0][i] = v0[i]; }
  int cur = 0;
  for (int p = 0; p < npass; ++p) {
    const int shift = sh.s[p];
    cnt[tid] = 0;
    __syncthreads();
    for (int64_t i = tid; i < m; i += BLOCK) atomicAdd(&cnt[(uint32_t)(kb[cur][i] >> shift) & 255u], 1u);
    __syncthreads();
    {
      uint32_t tot;
      run[tid] = block_excl_scan<uint32_t>(cnt[tid], &tot);
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < m; r0 += BLOCK) {  // block-uniform
#pragma unroll
      for (int k = 0; k < BLOCK / WAVE; ++k) wcnt[k][tid] = 0;
      __syncthreads();
      const int64_t i = r0 + tid;
      const bool valid = i < m;
      const uint64_t key = valid ? kb[cur][i] : 0;
      const uint32_t val = valid ? vb[cur][i] : 0;
      const uint32_t d = (uint32_t)(key >> shift) & 255u;
      uint64_t mask = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        uint64_t bal = __ballot((d >> b) & 1u);
        mask &= ((d >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t prank = (uint32_t)__popcll(mask & lt);
      if (valid && prank == 0) wcnt[wv][d] = (uint32_t)__popcll(mask);
      __syncthreads();
      {
        uint32_t rr = run[tid];
#pragma unroll
        for (int k = 0; k < BLOCK / WAVE; ++k) {
          uint32_t c = wcnt[k][tid];
          wcnt[k][tid] = rr;
          rr += c;
        }
        run[tid] = rr;
      }
      __syncthreads();
      if (valid) {
        const uint32_t dst = wcnt[wv][d] + prank;
        kb[cur ^ 1][dst] = key;
        vb[cur ^ 1][dst] = val;
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  for (int64_t i = tid; i < m; i += BLOCK) { k0[i] = kb[cur][i]; v0[i] = vb[cur][i]; }
}

__global__ void k_iota(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}
__global__ void k_copy32(int32_t* d, const int32_t* s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void k_off32to64(const int32_t* in, int64_t* out, int64_t n1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int64_t)in[i];
}

inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return (size_t)(cdiv(n, SCAN_TILE) + 2) * sizeof(int64_t); }

void scan_u8_i32(const uint8_t* in, int32_t* out, int64_t n, void* temp, const int64_t* cond, hipStream_t st) {
  scan_impl<uint8_t, int32_t>(in, out, n, temp, cond, st);
}
void scan_i32_i32(const int32_t* in, int32_t* out, int64_t n, void* temp, hipStream_t st) {
  scan_impl<int32_t, int32_t>(in, out, n, temp, nullptr, st);
}
void scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st) {
  scan_impl<int32_t, int64_t>(in, out, n, temp, nullptr, st);
}
void scan_i64_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st) {
  scan_impl<int64_t, int64_t>(in, out, n, temp, nullptr, st);
}
void scan_u32_i64(const uint32_t* in, int64_t* out, int64_t n, void* temp, hipStream_t st) {
  scan_impl<uint32_t, int64_t>(in, out, n, temp, nullptr, st);
}
void scan_u32_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t st) {
  scan_impl<uint32_t, uint32_t>(in, out, n, temp, nullptr, st);
}

// temp: histogram (256 * ntiles + 1 uint32), its scan, and the scan's own temp.
size_t radix_temp_bytes(int64_t m) {
  int64_t nt = cdiv(m, RADIX_TILE);
  size_t h = (size_t)(256 * nt + 1) * sizeof(uint32_t);
  h = (h + 255) & ~(size_t)255;
  return 2 * h + scan_temp_bytes(256 * nt + 1);
}

int radix_sort_pairs(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t m, const int* shifts,
                     int npass, void* temp, hipStream_t st) {
  if (m <= 0 || npass <= 0) return 0;
  if (m <= RADIX_TILE && npass <= 8) {
    RadixShifts sh{};
    for (int p = 0; p < npass; ++p) sh.s[p] = shifts[p];
    k_radix_small<<<1, BLOCK, 0, st>>>(k0, v0, m, sh, npass);
    return 0;
  }
  int64_t nt = cdiv(m, RADIX_TILE);
  size_t h = (size_t)(256 * nt + 1) * sizeof(uint32_t);
  h = (h + 255) & ~(size_t)255;
  uint32_t* hist = (uint32_t*)temp;
  uint32_t* offs = (uint32_t*)((char*)temp + h);
  void* stemp = (char*)temp + 2 * h;
  uint64_t* ki = k0; uint32_t* vi = v0; uint64_t* ko = k1; uint32_t* vo = v1;
  for (int p = 0; p < npass; ++p) {
    k_radix_hist<<<(unsigned)nt, BLOCK, 0, st>>>(ki, m, shifts[p], hist, nt);
    scan_impl<uint32_t, uint32_t>(hist, offs, 256 * nt, stemp, nullptr, st);
    k_radix_scatter<<<(unsigned)nt, BLOCK, 0, st>>>(ki, vi, m, shifts[p], hist, offs, nt, ko, vo);
    uint64_t* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
  }
  return (npass & 1) ? 1 : 0;
}

__global__ void k_store_count(const int32_t* src, int64_t* dst) { *dst = *src; }

void store_count(const int32_t* src, int64_t* dst, hipStream_t st) { k_store_count<<<1, 1, 0, st>>>(src, dst); }

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill<int32_t><<<grid_for(n), BLOCK, 0, st>>>(p, v, n);
}
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill<int64_t><<<grid_for(n), BLOCK, 0, st>>>(p, v, n);
}
void zero_bytes(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  if ((bytes & 7) == 0 && ((uintptr_t)p & 7) == 0) fill_i64((int64_t*)p, 0, (int64_t)(bytes / 8), st);
  else fill_u8((uint8_t*)p, 0, (int64_t)bytes, st);
}

void fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_fill<uint8_t><<<grid_for(n), BLOCK, 0, st>>>(p, v, n);
}
void iota_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n > 0) k_iota<<<grid_for(n), BLOCK, 0, st>>>(p, n);
}
void copy_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t st) {
  if (n > 0) k_copy32<<<grid_for(n), BLOCK, 0, st>>>(dst, src, n);
}
void offsets32_to_64(const int32_t* in, int64_t* out, int64_t n1, hipStream_t st) {
  if (n1 > 0) k_off32to64<<<grid_for(n1), BLOCK, 0, st>>>(in, out, n1);
}

}  // namespace lcc
