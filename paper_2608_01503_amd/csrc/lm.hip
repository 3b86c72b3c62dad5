// Local move (Alg. 2), afterburner filter (Alg. 3), update, objective, degree buckets and CSR validation.
//
// Integer form (lambda = p / q in lowest terms, every w' scaled by q):
//   a(v,c) = sum of w(u,v) over neighbours u with C[u] = c        W_c = sum of w(u) over cluster c
//   S(v,c) = q a(v,c) - p w(v) W_c            (c != C[v])         S_cur = q a(v,C[v]) - p w(v) (W_C[v] - w(v))
//   N(C)   = q I(C) - p (sum_c W_c^2 - sum_v w(v)^2)              (lambdaCC = N / q, Eq. 1)
// The host guarantees q W_E + p W^2 < 2^62, so every score, every objective numerator and every sum of
// afterburner adjustments is below 2^62 (2^63 for the adjustment sums) in magnitude and fits in int64, a delta
// (a difference of two scores) below 2^63.  What can reach 2^64 -- the difference of two deltas in the tie test,
// a delta plus its adjustments -- is formed in 128 bits, as is the temperature test (a rational phi times a
// score).  Sums whose final value fits but whose partial sums need not (the change of the sum of squared
// cluster weights) are accumulated modulo 2^64, which leaves the final value exact.
//
// Work decomposition per degree bucket (see common.h): groups of G lanes (G = 4..32, one neighbour per lane,
// neighbour clusters aggregated by register shuffles), one wavefront per vertex with an LDS open-addressing
// hash (degree <= 128), one workgroup per vertex with an LDS hash (degree <= 1024: 128 threads, <= 4096: 512
// threads), and hub vertices split into 2048-edge chunks processed by independent workgroups with a global-memory hash in the edge arena.
#include <algorithm>
#include <initializer_list>
#include <utility>

#include "common.h"

namespace lcc {

namespace {

constexpr int HUB_CHUNK = (int)HUB_CHUNK_EDGES;  // edges of a hub handled by one workgroup
constexpr int HUB_LDS_BITS = 12;     // its LDS pre-aggregation table: 2 * HUB_CHUNK slots
constexpr int HUB_BLOCK = 256;
constexpr int BIG_BLOCK = 256;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------------------------------------
// reductions over a group of G lanes (G <= 64: shuffles; G == BLOCK-sized: shuffles + LDS)
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ bool better(int64_t s2, int32_t c2, int64_t s, int32_t c) {
  return s2 > s || (s2 == s && c2 < c);
}

// Partner of butterfly step K (K = 0, 1, ...) inside aligned groups of G lanes.  Groups of at most 16 lanes
// use DPP lane moves (register to register, no LDS): two quad permutations (lane ^ 1, lane ^ 2), the row half
// mirror (lane i of an 8-lane half-row <-> lane 7 - i) and the row mirror (i <-> 15 - i).  The mirror partners
// are not xor partners, but each step pairs every lane with one in the other half of its 2^(K+1)-lane block,
// whose lanes all hold the same value after the earlier steps: an all-reduction of a commutative and
// associative operation gets the same result.  Wider groups use shuffles.
constexpr int DPP_GROUP_STEP[4] = {0xB1, 0x4E, 0x141, 0x140};

template <int G, int K>
__device__ __forceinline__ int32_t gx32(int32_t x) {
  if constexpr (G <= 16) return __builtin_amdgcn_update_dpp(0, x, DPP_GROUP_STEP[K], 0xf, 0xf, false);
  else return __shfl_xor(x, 1 << K, G);
}
template <int G, int K>
__device__ __forceinline__ int64_t gx64(int64_t x) {
  if constexpr (G <= 16) {
    const int32_t lo = gx32<G, K>((int32_t)(uint32_t)(uint64_t)x);
    const int32_t hi = gx32<G, K>((int32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
  } else {
    return __shfl_xor(x, 1 << K, G);
  }
}

// Lane K of every aligned group of G lanes (G = 4: quad permutation; 8 and 16: row broadcasts; else shuffle).
template <int G, int K>
__device__ __forceinline__ int32_t gbcast32(int32_t x) {
  if constexpr (G == 4) {
    return __builtin_amdgcn_update_dpp(0, x, K | (K << 2) | (K << 4) | (K << 6), 0xf, 0xf, false);
  } else if constexpr (G == 8) {
    const int32_t lo = __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xf, 0xf, false);      // row_newbcast:K
    const int32_t hi = __builtin_amdgcn_update_dpp(0, x, 0x150 + K + 8, 0xf, 0xf, false);  // row_newbcast:K+8
    return (threadIdx.x & 8) ? hi : lo;
  } else if constexpr (G == 16) {
    return __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xf, 0xf, false);
  } else {
    return __shfl(x, K, G);
  }
}

template <int G, int K = 0>
__device__ __forceinline__ void argmax_steps(int64_t& s, int32_t& c) {
  if constexpr ((1 << K) < G) {
    const int64_t s2 = gx64<G, K>(s);
    const int32_t c2 = gx32<G, K>(c);
    if (better(s2, c2, s, c)) { s = s2; c = c2; }
    argmax_steps<G, K + 1>(s, c);
  }
}
template <int G, int K = 0>
__device__ __forceinline__ int64_t sum_steps(int64_t x) {
  if constexpr ((1 << K) < G) return sum_steps<G, K + 1>(x + gx64<G, K>(x));
  else return x;
}

template <int G>
__device__ __forceinline__ void argmax_reduce(int64_t& s, int32_t& c) {
  if constexpr (G <= WAVE) {
    argmax_steps<G>(s, c);
  } else {
    __shared__ int64_t ss[G / WAVE];
    __shared__ int32_t cc[G / WAVE];
    argmax_reduce<WAVE>(s, c);
    int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) { ss[wv] = s; cc[wv] = c; }
    __syncthreads();
    s = ss[0]; c = cc[0];
#pragma unroll
    for (int k = 1; k < G / WAVE; ++k)
      if (better(ss[k], cc[k], s, c)) { s = ss[k]; c = cc[k]; }
    __syncthreads();
  }
}

template <int G>
__device__ __forceinline__ int64_t sum_reduce(int64_t x) {
  if constexpr (G <= WAVE) {
    return sum_steps<G>(x);
  } else {
    __shared__ int64_t ss[G / WAVE];
    x = sum_reduce<WAVE>(x);
    int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) ss[wv] = x;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int k = 0; k < G / WAVE; ++k) t += ss[k];
    __syncthreads();
    return t;
  }
}

// Destination and candidacy of one vertex from its own score and its best neighbouring cluster
// (Alg. 2: argmax, the empty-cluster rule, the temperature rule w'(v,D) >= (1 - phi) w'(v,C[v])).
// strict != 0 replaces the temperature rule by "the move strictly improves" (node optimality, Sec. V-A).
struct Verdict {
  int32_t d;
  int64_t delta;
  bool cand;
};
__device__ __forceinline__ Verdict decide(int64_t scur, int64_t sbest, int32_t cbest, uint32_t pa, uint32_t pb,
                                          int strict) {
  int32_t d;
  int64_t sd;
  if (scur < 0 && (cbest == INT32_MAX || sbest < 0)) {
    d = D_EMPTY;
    sd = 0;
  } else if (cbest == INT32_MAX) {
    return {D_NONE, 0, false};
  } else {
    d = cbest;
    sd = sbest;
  }
  int64_t delta = sd - scur;
  bool cand = strict ? (delta > 0) : ((__int128)pb * sd >= (__int128)(pb - pa) * scur);
  return {cand ? d : D_NONE, cand ? delta : 0, cand};
}

// this workgroup's stripe of the counter partials (see NSTRIPE)
__device__ __forceinline__ unsigned long long* stripe(int64_t* S, int ct) {
  return (unsigned long long*)&S[(int64_t)(blockIdx.x & (NSTRIPE - 1)) * STRIPE_W + ct];
}

// Per-thread counter partials: each thread adds into registers, and the workgroup reduces them once at its end
// (one stripe atomic per counter), instead of an LDS atomic per vertex on one shared address.
struct VtxAcc {
  int64_t ncand = 0;
  int64_t own = 0;
  int64_t bytes = 0;
};
// every thread of the workgroup (BS threads) calls this once, at the end of the kernel; counter ids < 0 are
// not counted
template <int BS>
__device__ __forceinline__ void acc_flush(const VtxAcc& a, int64_t* S, int ct_ncand, int ct_own = -1,
                                          int ct_bytes = -1) {
  const int64_t c = ct_ncand >= 0 ? sum_reduce<BS>(a.ncand) : 0;
  const int64_t o = ct_own >= 0 ? sum_reduce<BS>(a.own) : 0;
  const int64_t b = ct_bytes >= 0 ? sum_reduce<BS>(a.bytes) : 0;
  if (threadIdx.x == 0) {
    if (c) atomicAdd(stripe(S, ct_ncand), (unsigned long long)c);
    if (o) atomicAdd(stripe(S, ct_own), (unsigned long long)o);
    if (b) atomicAdd(stripe(S, ct_bytes), (unsigned long long)b);
  }
}

// Destinations of the counters a fold adds up (null: not folded; its stripes stay as they are).
struct FoldDst {
  int64_t* d[CT_COUNT];
};

// Adds the stripes of every counter that has a destination into it and clears those stripes; run by one
// workgroup of 1024 threads.  The stripes are read as 8192 pieces of 16 bytes, thread t taking pieces t,
// t + 1024, ..., t + 7168: every load instruction of a wavefront covers 1 KB of consecutive bytes, and piece p
// holds counters 2 (p mod 8) and 2 (p mod 8) + 1 of stripe p / 8, so a thread always sees the same two
// counters.  Ends with a barrier: the destinations are final for every thread afterwards.
__device__ __forceinline__ void fold_block(int64_t* S, const FoldDst& f) {
  static_assert(NSTRIPE == 1024 && STRIPE_W == 16 && CT_COUNT <= STRIPE_W, "8 pieces per stripe, 8 per thread");
  __shared__ int64_t part[1024 / WAVE][STRIPE_W];
  const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
  const int c0 = 2 * (t & 7), c1 = c0 + 1;
  const bool f0 = c0 < CT_COUNT && f.d[c0], f1 = c1 < CT_COUNT && f.d[c1];
  int64_t a0 = 0, a1 = 0;
  if (f0 || f1) {
    longlong2* P = (longlong2*)S;
    longlong2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = P[t + 1024 * k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (f0) a0 += v[k].x;
      if (f1) a1 += v[k].y;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((f0 && v[k].x) || (f1 && v[k].y)) {
        longlong2 z = v[k];
        if (f0) z.x = 0;
        if (f1) z.y = 0;
        P[t + 1024 * k] = z;
      }
    }
  }
  if (__ballot(a0 != 0 || a1 != 0)) {  // stripes past the launches' workgroup counts are zero: most skip
#pragma unroll
    for (int o = 8; o < WAVE; o <<= 1) {  // lanes with equal t mod 8 hold the same two counters
      a0 += __shfl_xor(a0, o, WAVE);
      a1 += __shfl_xor(a1, o, WAVE);
    }
  }
  if (lane < 8) { part[wv][c0] = a0; part[wv][c1] = a1; }
  __syncthreads();
  if (t < CT_COUNT && f.d[t]) {
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 1024 / WAVE; ++k) s += part[k][t];
    if (s) *f.d[t] += s;
  }
  __syncthreads();
}

__device__ __forceinline__ void finish_vertex(int32_t v, int32_t cv, int64_t wv, int64_t own, int64_t sbest,
                                              int32_t cbest, const Score& sc, const int64_t* W, uint32_t pa,
                                              uint32_t pb, int strict, VState* vs, VtxAcc& va,
                                              int64_t* ownv) {
  int64_t scur = sc.q * own - sc.p * wv * (W[cv] - wv);
  Verdict vd = decide(scur, sbest, cbest, pa, pb, strict);
  VState o;
  o.c = cv;
  o.d = vd.d;
  o.delta = vd.delta;
  vs[v] = o;
  va.ncand += vd.cand ? 1 : 0;
  va.own += own;
  if (ownv) ownv[v] = own;
}

// Algorithmic bytes of the enumeration (diagnostics): a vertex's row (index, weight and the neighbour's
// cluster: 12 bytes per entry), its own state (56 bytes) and one cluster weight per other cluster (8 bytes each).
__device__ __forceinline__ int64_t enum_bytes(int64_t deg, int64_t np) { return 12 * deg + 56 + 8 * np; }

__device__ __forceinline__ uint32_t hslot(int32_t c, int bits) {
  return ((uint32_t)c * 2654435761u) >> (32 - bits);
}

__device__ __forceinline__ int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

// log2 of the LDS hash capacity for a row of degree d: pow2ceil(2 d) << shift slots (at least 2), at most the
// kernel's table of `slots`; the bucket bounds keep 2 d <= slots, so the load factor never exceeds 1/2
__device__ __forceinline__ int table_bits(int64_t d, int shift, int slots) {
  int bits = ceil_log2(2 * d);
  if (bits < 1) bits = 1;
  bits += shift;
  const int cap = ceil_log2(slots);
  return bits < cap ? bits : cap;
}

__device__ __forceinline__ int find_chunk_owner(const int32_t* chunk_off, int64_t n7, int64_t blk) {
  int64_t lo = 0, hi = n7;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= blk) lo = mid; else hi = mid;
  }
  return (int)lo;
}


// ---------------------------------------------------------------------------------------------------------
// Row helpers.  Every lane keeps U edges (or table slots) in flight: the index loads, then the dependent
// gathers, are issued back to back before any of them is consumed, so one lane's gathers overlap instead of
// forming a serial chain.
// ---------------------------------------------------------------------------------------------------------
constexpr int U = 4;

// Sum of x over the 64 lanes of a fully active wavefront, returned to every lane.  A row-local Hillis-Steele
// scan by DPP row shifts (1, 2, 4, 8), then the two row broadcasts carry rows 0-2 into rows 1-3, so lane 63
// holds the total: register-to-register moves only, no LDS round trips.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  int v = (int)x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ void lds_insert(int32_t* hk, uint32_t* hv, int bits, int32_t c, uint32_t wt) {
  const uint32_t mask = (1u << bits) - 1;
  uint32_t h = hslot(c, bits);
  for (uint32_t probe = 0; probe <= mask; ++probe) {  // the table has room for every distinct key
    int32_t prev = atomicCAS(&hk[h], -1, c);
    if (prev == -1 || prev == c) { atomicAdd(&hv[h], wt); return; }
    h = (h + 1) & mask;
  }
}

// a(v, c) for the edges b + t, b + t + S, ... < e into the LDS table; edges into v's own cluster cv are
// summed in registers (returned) instead.  Many lanes of a wavefront often carry the same cluster id (clusters
// grow over the passes), and same-address LDS atomics serialise: before inserting, each batch combines the
// lanes holding the two most frequent-looking keys (the first remaining lane's key, twice) with a ballot and
// a wavefront sum, and one lane inserts the total.  The loop is uniform over the wavefront (lanes past the
// end carry no key) so the ballots and shuffles see every lane.
__device__ __forceinline__ int64_t insert_row(const DevGraph& g, const int32_t* C, int64_t b, int64_t e, int t,
                                              int S, int32_t cv, int32_t* hk, uint32_t* hv, int bits,
                                              const int32_t* cons, int32_t bv) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t tw = t - lane;  // first lane of this wavefront
  int64_t own = 0;
  for (int64_t j0 = b + t, jw = b + tw; jw < e; j0 += (int64_t)S * U, jw += (int64_t)S * U) {
    // Lanes past the end read the row's last entry (jw < e, so it exists) and drop it afterwards: every load
    // and gather is issued unconditionally, back to back, with no per-load branch.
    int32_t us[U], cs[U];
    uint32_t ws[U];
    bool ok[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t j = j0 + (int64_t)k * S;
      ok[k] = j < e;
      const int64_t jc = ok[k] ? j : e - 1;
      us[k] = g.idx[jc];
      ws[k] = (uint32_t)g.w[jc];
    }
    if (cons) {
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (cons[us[k]] != bv) ok[k] = false;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) cs[k] = C[us[k]];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      int32_t key = ok[k] ? cs[k] : -1;
      uint32_t val = ok[k] ? ws[k] : 0u;
      if (key == cv) { own += val; key = -1; }
#pragma unroll
      for (int round = 0; round < 2; ++round) {
        uint64_t act = __ballot(key >= 0);
        if (!act) break;
        int lead = __ffsll((unsigned long long)act) - 1;
        int32_t lk = __builtin_amdgcn_readlane(key, lead);
        uint64_t m = __ballot(key == lk);
        if (__popcll(m) < 2) break;  // no sharing left worth combining
        uint32_t part = wave_sum_u32(key == lk ? val : 0u);
        if (lane == lead) lds_insert(hk, hv, bits, lk, part);
        if (key == lk) key = -1;
      }
      if (key >= 0) lds_insert(hk, hv, bits, key, val);
    }
  }
  return own;
}

struct Best {
  int64_t s;
  int32_t c;
  int64_t own;
  int64_t np;
};

__device__ __forceinline__ Best best_init() { return Best{INT64_MIN, INT32_MAX, 0, 0}; }

// slots t, t + S, ... < cap: best other cluster, weight to the own cluster, number of other clusters
__device__ __forceinline__ void scan_table(const int32_t* hk, const uint32_t* hv, int cap, int t, int S, int32_t cv,
                                           int64_t wv, const int64_t* W, const Score& sc, Best& r) {
  for (int s0 = t; s0 < cap; s0 += S * U) {
    int32_t ks[U];
    int64_t as[U], Ws[U];
    // every read stays inside the table (clamped slot) and is issued unconditionally, so the 2 U LDS reads
    // go out back to back and are waited for once; slots past the end are then masked off
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int sl = s0 + k * S;
      const int slc = sl < cap ? sl : cap - 1;
      const int32_t kk = hk[slc];
      const uint32_t vv = hv[slc];
      ks[k] = sl < cap ? kk : -1;
      as[k] = ks[k] >= 0 ? (int64_t)vv : 0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) Ws[k] = W[ks[k] >= 0 ? ks[k] : cv];  // empty slots read W[cv] and are skipped
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (ks[k] < 0) continue;
      if (ks[k] == cv) { r.own += as[k]; continue; }
      ++r.np;
      int64_t val = sc.q * as[k] - sc.p * wv * Ws[k];
      if (better(val, ks[k], r.s, r.c)) { r.s = val; r.c = ks[k]; }
    }
  }
}

// reduction of Best over G lanes (G <= 64) or a block of G threads; the result is valid in lane / thread 0
template <int G, int K = 0>
__device__ __forceinline__ void best_steps(Best& r) {
  if constexpr ((1 << K) < G) {
    const int64_t s2 = gx64<G, K>(r.s);
    const int32_t c2 = gx32<G, K>(r.c);
    r.own += gx64<G, K>(r.own);
    r.np += gx64<G, K>(r.np);
    if (better(s2, c2, r.s, r.c)) { r.s = s2; r.c = c2; }
    best_steps<G, K + 1>(r);
  }
}

template <int G>
__device__ __forceinline__ void best_reduce(Best& r) {
  constexpr int WD = G < WAVE ? G : WAVE;
  best_steps<WD>(r);
  if constexpr (G > WAVE) {
    __shared__ Best sb[G / WAVE];
    if ((threadIdx.x & (WAVE - 1)) == 0) sb[threadIdx.x / WAVE] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 1; k < G / WAVE; ++k) {
        r.own += sb[k].own;
        r.np += sb[k].np;
        if (better(sb[k].s, sb[k].c, r.s, r.c)) { r.s = sb[k].s; r.c = sb[k].c; }
      }
    }
  }
}

// singleton pass: best neighbour u by S = q w(u,v) - p w(v) w(u)
template <int UU = U>
__device__ __forceinline__ void single_row(const DevGraph& g, const Score& sc, int64_t b, int64_t e, int t, int S,
                                           int64_t wv, Best& r, const int32_t* cons, int32_t bv) {
  for (int64_t j0 = b + t; j0 < e; j0 += (int64_t)S * UU) {
    // lanes past the end read the row's last entry (j0 < e) and drop it: loads issued without branches
    int32_t us[UU];
    int64_t ws[UU], vu[UU];
    bool ok[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      const int64_t j = j0 + (int64_t)k * S;
      ok[k] = j < e;
      const int64_t jc = ok[k] ? j : e - 1;
      us[k] = g.idx[jc];
      ws[k] = g.w[jc];
    }
    if (cons) {
#pragma unroll
      for (int k = 0; k < UU; ++k)
        if (cons[us[k]] != bv) ok[k] = false;
    }
#pragma unroll
    for (int k = 0; k < UU; ++k) vu[k] = g.vw[us[k]];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      if (!ok[k]) continue;
      int64_t val = sc.q * ws[k] - sc.p * wv * vu[k];
      if (better(val, us[k], r.s, r.c)) { r.s = val; r.c = us[k]; }
    }
  }
}

// internal weight of v: sum of w(u,v) over neighbours in v's cluster
template <int UU = U>
__device__ __forceinline__ int64_t internal_row(const DevGraph& g, const int32_t* C, int64_t b, int64_t e, int t,
                                                int S, int32_t cv) {
  int64_t acc = 0;
  for (int64_t j0 = b + t; j0 < e; j0 += (int64_t)S * UU) {
    // lanes past the end read the row's last entry (j0 < e) and drop it: loads issued without branches
    int32_t cs[UU];
    int64_t ws[UU];
    bool ok[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      const int64_t j = j0 + (int64_t)k * S;
      ok[k] = j < e;
      const int64_t jc = ok[k] ? j : e - 1;
      cs[k] = g.idx[jc];
      ws[k] = g.w[jc];
    }
#pragma unroll
    for (int k = 0; k < UU; ++k) cs[k] = C[cs[k]];
#pragma unroll
    for (int k = 0; k < UU; ++k)
      if (ok[k] && cs[k] == cv) acc += ws[k];
  }
  return acc;
}

// ---------------------------------------------------------------------------------------------------------
// Pass bookkeeping (single thread)
// ---------------------------------------------------------------------------------------------------------

// Start of pass i: decide whether it repeats pass i-1 exactly (pass i-1 moved nothing and the temperature
// is unchanged), and reset the pass counters.
// Launched with one workgroup of 1024 threads: first folds the counters the previous pass left in the stripes.
__global__ __launch_bounds__(1024) void k_pass_begin(LMSlot* s, int i, int same_phi, int64_t* S, FoldDst f) {
  fold_block(S, f);
  if (threadIdx.x != 0) return;
  s->copy = 0;
  s->n_empty = 0;
  if (i >= 2 && same_phi && s->nM[i - 1] == 0) {
    s->skip[i] = 1;
    s->nL[i] = s->nL[i - 1];
    s->nM[i] = 0;
    s->I[i - 1] = s->I[i - 2];
    s->SW2[i] = s->SW2[i - 1];
  } else {
    s->skip[i] = 0;
    s->nL[i] = 0;
    s->nM[i] = 0;
    s->I[i - 1] = 0;
    s->SW2[i] = s->SW2[i - 1];  // a single graph's moves add their change (a union recomputes it)
  }
}

// Best-so-far check of state k (Alg. 2: C_out <- C when lambdaCC(C) > lambdaCC(C_out)).  Skipped when state
// k equals state k-1, which was checked already.
// One workgroup of 1024 threads: first folds the counters the state's sums are waiting for.
__global__ __launch_bounds__(1024) void k_best(LMSlot* s, int k, int skipk, int64_t p, int64_t q, int64_t sum_w2,
                                               int64_t* S, FoldDst f) {
  fold_block(S, f);
  if (threadIdx.x != 0) return;
  s->copy = 0;
  if (skipk >= 0 && s->skip[skipk]) return;
  int64_t N = q * s->I[k] - p * (s->SW2[k] - sum_w2);
  if (k == 0) {
    s->N0 = N;
    s->Nbest = N;
  } else if (N > s->Nbest) {
    s->Nbest = N;
    s->copy = 1;
  }
}

__global__ void k_copy_if(const LMSlot* s, const int32_t* C, int32_t* Cout, int64_t n) {
  if (!s->copy) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Cout[i] = C[i];
}

// One workgroup of 1024 threads: first folds the counters of the last pass.
__global__ __launch_bounds__(1024) void k_final_state(LMSlot* s, int last, int64_t* S, FoldDst f) {
  fold_block(S, f);
  if (threadIdx.x != 0) return;
  if (s->skip[last]) s->I[last] = s->I[last - 1];
  else s->I[last] = 0;
}

// ---------------------------------------------------------------------------------------------------------
// Singleton pass (first coarsening pass, Sec. IV-A: clusters are the vertices, no enumeration)
// ---------------------------------------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(BLOCK) void k_single_grp(const int32_t* list, int64_t cnt, DevGraph g, ScoreSrc ss,
                                                      uint32_t pa, uint32_t pb, VState* vs, LMSlot* slot,
                                                      int pass, int64_t* S) {
  VtxAcc va;
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int64_t wv = g.vw[v];
    const Score sc = ss.at(v);
    Best r = best_init();
    single_row<G <= 16 ? 1 : U>(g, sc, g.off[v], g.off[v + 1], gl, G, wv, r, ss.cons, ss.con(v));
    best_reduce<G>(r);
    if (gl == 0) finish_vertex(v, v, wv, 0, r.s, r.c, sc, g.vw, pa, pb, 0, vs, va, ss.ownv);
  }
  acc_flush<BLOCK>(va, S, CT_NCAND, -1);
}

template <int G>
__global__ __launch_bounds__(G) void k_single_blk(const int32_t* list, int64_t cnt, DevGraph g, ScoreSrc ss,
                                                  uint32_t pa, uint32_t pb, VState* vs, LMSlot* slot, int pass,
                                                  int64_t* S) {
  VtxAcc va;
  for (int64_t vi = blockIdx.x; vi < cnt; vi += gridDim.x) {
    const int32_t v = list[vi];
    const int64_t wv = g.vw[v];
    const Score sc = ss.at(v);
    Best r = best_init();
    single_row(g, sc, g.off[v], g.off[v + 1], threadIdx.x, G, wv, r, ss.cons, ss.con(v));
    best_reduce<G>(r);
    if (threadIdx.x == 0) finish_vertex(v, v, wv, 0, r.s, r.c, sc, g.vw, pa, pb, 0, vs, va, ss.ownv);
    __syncthreads();
  }
  acc_flush<G>(va, S, CT_NCAND, -1);
}

// Hub chunk of the singleton pass: partial argmax per chunk.
__global__ __launch_bounds__(HUB_BLOCK) void k_single_hub(const int32_t* hubs, const int32_t* chunk_off,
                                                          int64_t n7, DevGraph g, ScoreSrc ss, int64_t* ps,
                                                          int32_t* pc) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const Score sc = ss.at(v);
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK);
  const int64_t wv = g.vw[v];
  const int32_t bv = ss.con(v);
  int64_t bs = INT64_MIN;
  int32_t bcl = INT32_MAX;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK) {
    int32_t u = g.idx[j];
    if (ss.cons && ss.cons[u] != bv) continue;
    int64_t s = sc.q * (int64_t)g.w[j] - sc.p * wv * g.vw[u];
    if (better(s, u, bs, bcl)) { bs = s; bcl = u; }
  }
  argmax_reduce<HUB_BLOCK>(bs, bcl);
  if (threadIdx.x == 0) { ps[blockIdx.x] = bs; pc[blockIdx.x] = bcl; }
}

// ---------------------------------------------------------------------------------------------------------
// General pass: enumerate neighbour clusters and take the argmax (Alg. 2 with DS = Enumerate(G, C))
// ---------------------------------------------------------------------------------------------------------

// Every lane of the group sees every lane's (cluster, weight) in turn and sums the weights of its own cluster;
// a lane stays leader when no earlier lane holds its cluster.
template <int G, int K = 0>
__device__ __forceinline__ void pair_sweep(int32_t c, int32_t wt, bool has, int gl, int64_t& acc, bool& leader) {
  if constexpr (K < G) {
    const int32_t ck = gbcast32<G, K>(c);
    const int32_t wk = gbcast32<G, K>(wt);
    if (has && ck == c) {
      acc += wk;
      if (K < gl) leader = false;
    }
    pair_sweep<G, K + 1>(c, wt, has, gl, acc, leader);
  }
}

// degree <= G: lane l holds neighbour l; clusters aggregated by an all-pairs sweep of the group.  Workgroup
// bid of nblk walks the list.
template <int G>
__device__ __forceinline__ void enum_grp_blocks(const int32_t* list, int64_t cnt, unsigned bid, unsigned nblk,
                                                const DevGraph& g, const int32_t* C, const int64_t* W,
                                                const ScoreSrc& ss, uint32_t pa, uint32_t pb, int strict,
                                                VState* vs, VtxAcc& va) {
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)bid * (BLOCK / G) + threadIdx.x / G; gid < cnt; gid += (int64_t)nblk * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int64_t b = g.off[v];
    const int d = (int)(g.off[v + 1] - b);
    const int32_t cv = C[v];
    const int64_t wv = g.vw[v];
    const Score sc = ss.at(v);
    const int32_t u = gl < d ? g.idx[b + gl] : -1;
    const bool has = u >= 0 && (!ss.cons || ss.cons[u] == ss.cons[v]);
    const int32_t c = has ? C[u] : -1;
    const int32_t wt = has ? g.w[b + gl] : 0;
    int64_t acc = 0;
    bool leader = has;
    pair_sweep<G>(c, wt, has, gl, acc, leader);
    int64_t own = (leader && c == cv) ? acc : 0;
    int64_t bs = INT64_MIN;
    int32_t bcl = INT32_MAX;
    if (leader && c != cv) {
      bs = sc.q * acc - sc.p * wv * W[c];
      bcl = c;
      va.bytes += 8;
    }
    argmax_reduce<G>(bs, bcl);
    own = sum_reduce<G>(own);
    if (gl == 0) {
      finish_vertex(v, cv, wv, own, bs, bcl, sc, W, pa, pb, strict, vs, va, ss.ownv);
      va.bytes += enum_bytes(d, 0);
    }
  }
}

template <int G>
__global__ __launch_bounds__(BLOCK) void k_enum_grp(const int32_t* list, int64_t cnt, DevGraph g,
                                                    const int32_t* C, const int64_t* W, ScoreSrc ss, uint32_t pa,
                                                    uint32_t pb, int strict, VState* vs, LMSlot* slot, int pass,
                                                    int64_t* S, int ct_own, int ct_pairs) {
  VtxAcc va;
  if (slot && slot->skip[pass]) return;
  enum_grp_blocks<G>(list, cnt, blockIdx.x, gridDim.x, g, C, W, ss, pa, pb, strict, vs, va);
  acc_flush<BLOCK>(va, S, slot ? CT_NCAND : -1, ct_own, ct_pairs);
}

// The sub-wave group buckets in one launch: the workgroups are split in ranges, one per bucket, so the buckets
// run side by side instead of one launch after another (each with its own tail).
constexpr int NGRP = 3;
struct GrpSet {
  const int32_t* list[NGRP];
  int64_t cnt[NGRP];
  unsigned nb[NGRP];  // workgroups of each bucket (0: none)
};
__device__ __forceinline__ int grp_set_bucket(const GrpSet& q, unsigned& bid) {
  bid = blockIdx.x;
  int k = 0;
  while (k < NGRP - 1 && bid >= q.nb[k]) bid -= q.nb[k++];
  return k;
}

// buckets 0-2: rows of at most 4, 8 and 16 entries (the 32-lane bucket keeps a launch of its own: merged
// with it, the lattice and kNN graphs ran slower)
__global__ __launch_bounds__(BLOCK) void k_enum_grps(GrpSet q, DevGraph g, const int32_t* C, const int64_t* W,
                                                     ScoreSrc ss, uint32_t pa, uint32_t pb, int strict, VState* vs,
                                                     LMSlot* slot, int pass, int64_t* S, int ct_own, int ct_pairs0) {
  VtxAcc va;
  if (slot && slot->skip[pass]) return;
  unsigned bid;
  const int k = grp_set_bucket(q, bid);  // uniform over the workgroup
  if (k == 0) enum_grp_blocks<4>(q.list[0], q.cnt[0], bid, q.nb[0], g, C, W, ss, pa, pb, strict, vs, va);
  else if (k == 1) enum_grp_blocks<8>(q.list[1], q.cnt[1], bid, q.nb[1], g, C, W, ss, pa, pb, strict, vs, va);
  else enum_grp_blocks<16>(q.list[2], q.cnt[2], bid, q.nb[2], g, C, W, ss, pa, pb, strict, vs, va);
  acc_flush<BLOCK>(va, S, slot ? CT_NCAND : -1, ct_own, ct_pairs0 >= 0 ? ct_pairs0 + k : -1);
}

// Orders a wavefront's own LDS accesses around a phase change of its private table: every LDS operation of
// the wavefront has completed (lgkmcnt 0) and the compiler moves no memory access across.  No other wavefront
// is involved, so no workgroup barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt left at their maximum
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront per vertex, LDS open-addressing hash of capacity pow2ceil(2 d) <= SLOTS.  Every wavefront owns
// its table and walks its own vertices: the wavefronts of a workgroup never wait for each other.
template <int SLOTS>
__global__ __launch_bounds__(BLOCK) void k_enum_wave(const int32_t* list, int64_t cnt, DevGraph g,
                                                     const int32_t* C, const int64_t* W, ScoreSrc ss, uint32_t pa,
                                                     uint32_t pb, int strict, VState* vs, LMSlot* slot,
                                                     int pass, int64_t* S, int ct_own, int ct_pairs,
                                                     int hshift) {
  __shared__ int32_t hk[BLOCK / WAVE][SLOTS];
  __shared__ uint32_t hv[BLOCK / WAVE][SLOTS];
  VtxAcc va;
  if (slot && slot->skip[pass]) return;
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  int32_t* tk = hk[wv];
  uint32_t* tv = hv[wv];
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / WAVE)) {
    const int32_t v = list[gid];
    const int64_t b = g.off[v], e = g.off[v + 1];
    const int32_t cv = C[v];
    const int64_t wvt = g.vw[v];
    const int bits = table_bits(e - b, hshift, SLOTS);
    for (int sl = lane; sl < (1 << bits); sl += WAVE) { tk[sl] = -1; tv[sl] = 0; }
    wave_lds_sync();
    const int64_t own_reg = insert_row(g, C, b, e, lane, WAVE, cv, tk, tv, bits, ss.cons, ss.con(v));
    wave_lds_sync();
    const Score sc = ss.at(v);
    Best r = best_init();
    scan_table(tk, tv, 1 << bits, lane, WAVE, cv, wvt, W, sc, r);
    r.own += own_reg;
    best_reduce<WAVE>(r);
    if (lane == 0) {
      finish_vertex(v, cv, wvt, r.own, r.s, r.c, sc, W, pa, pb, strict, vs, va, ss.ownv);
      va.bytes += enum_bytes(e - b, r.np);
    }
    wave_lds_sync();  // the scan's reads are done before the next vertex clears the table
  }
  acc_flush<BLOCK>(va, S, slot ? CT_NCAND : -1, ct_own, ct_pairs);
}

// One workgroup of BS threads per vertex sharing an LDS hash of capacity pow2ceil(2 d) <= SLOTS.
template <int BS, int SLOTS>
__global__ __launch_bounds__(BS) void k_enum_blk(const int32_t* list, int64_t cnt, DevGraph g, const int32_t* C,
                                                 const int64_t* W, ScoreSrc ss, uint32_t pa, uint32_t pb,
                                                 int strict, VState* vs, LMSlot* slot, int pass,
                                                 int64_t* S, int ct_own, int ct_pairs, int hshift) {
  __shared__ int32_t hk[SLOTS];
  __shared__ uint32_t hv[SLOTS];
  VtxAcc va;
  if (slot && slot->skip[pass]) return;
  for (int64_t vi = blockIdx.x; vi < cnt; vi += gridDim.x) {
    const int32_t v = list[vi];
    const int64_t b = g.off[v], e = g.off[v + 1];
    const int32_t cv = C[v];
    const int64_t wvt = g.vw[v];
    const int bits = table_bits(e - b, hshift, SLOTS);
    for (int sl = threadIdx.x; sl < (1 << bits); sl += BS) { hk[sl] = -1; hv[sl] = 0; }
    __syncthreads();
    const int64_t own_reg = insert_row(g, C, b, e, threadIdx.x, BS, cv, hk, hv, bits, ss.cons, ss.con(v));
    __syncthreads();
    const Score sc = ss.at(v);
    Best r = best_init();
    scan_table(hk, hv, 1 << bits, threadIdx.x, BS, cv, wvt, W, sc, r);
    r.own += own_reg;
    best_reduce<BS>(r);
    if (threadIdx.x == 0) {
      finish_vertex(v, cv, wvt, r.own, r.s, r.c, sc, W, pa, pb, strict, vs, va, ss.ownv);
      va.bytes += enum_bytes(e - b, r.np);
    }
    __syncthreads();
  }
  acc_flush<BS>(va, S, slot ? CT_NCAND : -1, ct_own, ct_pairs);
}

// Hubs: global-memory hash of 2 d 64-bit slots (cluster << 32 | weight sum) at slot offset 2 off[v] of the
// edge arena.  A hub's weight sums stay below 2^32 (the total edge weight does), so adding a weight to a slot
// never carries into its key.  Chunk k of a hub owns the 2 * HUB_CHUNK slots that start at
// 2 (off[v] + k HUB_CHUNK) for clearing and scanning; insertions probe the whole table.
constexpr unsigned long long HUB_EMPTY = 0xFFFFFFFF00000000ull;

__device__ __forceinline__ uint32_t hub_slot(int32_t c, int64_t cap) {
  return (uint32_t)(((uint64_t)fmix32((uint32_t)c) * (uint64_t)cap) >> 32);
}

__global__ __launch_bounds__(HUB_BLOCK) void k_hub_clear(const int32_t* hubs, const int32_t* chunk_off,
                                                         int64_t n7, const int64_t* off, uint32_t* arena,
                                                         const LMSlot* slot, int pass) {
  if (slot && pass >= 0 && slot->skip[pass]) return;
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int64_t s0 = 2 * (off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK);
  const int64_t s1 = min(2 * off[v + 1], s0 + 2 * HUB_CHUNK);
  unsigned long long* tab = (unsigned long long*)arena;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += HUB_BLOCK) tab[s] = HUB_EMPTY;
}

// Each chunk first aggregates its edges by cluster in LDS (a hub's neighbours often share few clusters), then
// inserts one entry per distinct cluster into the hub's global table.
__global__ __launch_bounds__(HUB_BLOCK) void k_hub_insert(const int32_t* hubs, const int32_t* chunk_off,
                                                          int64_t n7, DevGraph g, const int32_t* C,
                                                          uint32_t* arena, const LMSlot* slot, int pass,
                                                          const int32_t* cons) {
  if (slot && slot->skip[pass]) return;
  constexpr int S = 2 * HUB_CHUNK;
  static_assert(S == (1 << HUB_LDS_BITS), "the LDS table holds 2 slots per chunk edge");
  __shared__ int32_t lk[S];
  __shared__ uint32_t lv[S];
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int64_t base = g.off[v];
  const int64_t cap = 2 * (g.off[v + 1] - base);
  const int64_t j0 = base + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK);
  for (int s = threadIdx.x; s < S; s += HUB_BLOCK) { lk[s] = -1; lv[s] = 0; }
  __syncthreads();
  // own-cluster edges also go through the table here (the scan reads the hub's own weight from it)
  const int64_t own = insert_row(g, C, j0, j1, threadIdx.x, HUB_BLOCK, -3, lk, lv, HUB_LDS_BITS, cons, cons ? cons[v] : 0);
  (void)own;
  __syncthreads();
  // one atomic per entry: an add when the slot already holds the key, else a compare-and-swap of the whole
  // slot from empty (a slot read as empty may be stale; the swap then reports its real content)
  unsigned long long* tab = (unsigned long long*)arena + 2 * base;
  for (int s = threadIdx.x; s < S; s += HUB_BLOCK) {
    int32_t c = lk[s];
    if (c < 0) continue;
    const unsigned long long wt = lv[s];
    const unsigned long long mine = ((unsigned long long)(uint32_t)c << 32) | wt;
    int64_t h = hub_slot(c, cap);
    for (int64_t probe = 0; probe < cap; ++probe) {
      unsigned long long cur = tab[h];
      if (cur == HUB_EMPTY) {
        cur = atomicCAS(&tab[h], HUB_EMPTY, mine);
        if (cur == HUB_EMPTY) break;
      }
      if ((uint32_t)(cur >> 32) == (uint32_t)c) { atomicAdd(&tab[h], wt); break; }
      if (++h == cap) h = 0;
    }
  }
}

// Scan this chunk's share of the table: partial best and own weight; clears the slots for the next pass.
__global__ __launch_bounds__(HUB_BLOCK) void k_hub_scan(const int32_t* hubs, const int32_t* chunk_off,
                                                        int64_t n7, DevGraph g, const int32_t* C,
                                                        const int64_t* W, ScoreSrc ss, uint32_t* arena,
                                                        int64_t* ps, int32_t* pc, int64_t* pown,
                                                        const LMSlot* slot, int pass, int64_t* S,
                                                        int ct_pairs) {
  if (slot && slot->skip[pass]) return;
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const Score sc = ss.at(v);
  const int32_t cv = C[v];
  const int64_t wvt = g.vw[v];
  const int64_t s0 = 2 * (g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK);
  const int64_t s1 = min(2 * g.off[v + 1], s0 + 2 * HUB_CHUNK);
  int64_t own = 0, bs = INT64_MIN, np_ = 0;
  int32_t bcl = INT32_MAX;
  unsigned long long* tab = (unsigned long long*)arena;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += HUB_BLOCK) {
    const unsigned long long e = tab[s];
    if (e == HUB_EMPTY) continue;
    tab[s] = HUB_EMPTY;
    const int32_t c = (int32_t)(uint32_t)(e >> 32);
    const int64_t a = (int64_t)(uint32_t)e;
    if (c == cv) { own = a; continue; }
    ++np_;
    int64_t sc_ = sc.q * a - sc.p * wvt * W[c];
    if (better(sc_, c, bs, bcl)) { bs = sc_; bcl = c; }
  }
  argmax_reduce<HUB_BLOCK>(bs, bcl);
  own = sum_reduce<HUB_BLOCK>(own);
  np_ = sum_reduce<HUB_BLOCK>(np_);
  if (threadIdx.x == 0) {
    ps[blockIdx.x] = bs; pc[blockIdx.x] = bcl; pown[blockIdx.x] = own;
    if (ct_pairs >= 0 && np_) atomicAdd(stripe(S, ct_pairs), (unsigned long long)(8 * np_));
  }
}

// Combine the chunks of each hub (pown may be null: singleton pass).  off (the level's offsets) and ct_bytes
// (a counter id, or -1) count the hub rows' algorithmic bytes.
__global__ void k_hub_final(const int32_t* hubs, const int32_t* chunk_off, int64_t n7, const int64_t* vw,
                            const int32_t* C, const int64_t* W, ScoreSrc ss, uint32_t pa, uint32_t pb, int strict,
                            const int64_t* ps, const int32_t* pc, const int64_t* pown, VState* vs,
                            LMSlot* slot, int pass, int64_t* S, int ct_own, const int64_t* off = nullptr,
                            int ct_bytes = -1) {
  VtxAcc va;
  if (slot && slot->skip[pass]) return;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n7) {
    int32_t v = hubs[k];
    int64_t bs = INT64_MIN, own = 0;
    int32_t bcl = INT32_MAX;
    for (int32_t ch = chunk_off[k]; ch < chunk_off[k + 1]; ++ch) {
      if (better(ps[ch], pc[ch], bs, bcl)) { bs = ps[ch]; bcl = pc[ch]; }
      if (pown) own += pown[ch];
    }
    int32_t cv = C ? C[v] : v;
    finish_vertex(v, cv, vw[v], own, bs, bcl, ss.at(v), C ? W : vw, pa, pb, strict, vs, va, ss.ownv);
    if (off) va.bytes += enum_bytes(off[v + 1] - off[v], 0);
  }
  acc_flush<BLOCK>(va, S, slot ? CT_NCAND : -1, ct_own, ct_bytes);
}

// ---------------------------------------------------------------------------------------------------------
// Afterburner filter (Alg. 3).  For candidate v, every adjacent candidate u ordered before v adjusts delta_v
// by +-q w'(u,v); v is kept when the adjusted delta is >= 0.  Order: larger delta first; deltas within the
// tie window are ordered by the splitmix64 hash of the vertex id.
// ---------------------------------------------------------------------------------------------------------
// u and v are graph-local ids (the level id minus the graph's first id in a union of graphs).
__device__ __forceinline__ bool before(int32_t u, int64_t du, int32_t v, int64_t dv, int64_t tie) {
  const __int128 diff = (__int128)du - dv;  // two deltas below 2^63 each: their difference needs 65 bits
  const __int128 ad = diff < 0 ? -diff : diff;
  if (ad <= tie) return fmix64((uint64_t)(uint32_t)u) < fmix64((uint64_t)(uint32_t)v);
  return diff > 0;
}

__device__ __forceinline__ int64_t ab_adjust(int32_t cv, int32_t dv, int32_t cu, int32_t du, int64_t wq) {
  int64_t a = 0;
  if (cv == cu) a += wq;
  else if (dv == cu) a -= wq;
  if (du != D_EMPTY) {
    if (cv == du) a -= wq;
    else if (dv == du) a += wq;
  }
  return a;
}

__device__ __forceinline__ int ab_pattern(int32_t cv, int32_t dv, int32_t cu, int32_t du) {
  int a = 0;
  if (cv == cu) a += 1;
  else if (dv == cu) a -= 1;
  if (du != D_EMPTY) {
    if (cv == du) a -= 1;
    else if (dv == du) a += 1;
  }
  return a;
}

// sum of the adjustments of candidate v over the edges b + t, b + t + S, ... < e
template <int UU = U>
__device__ __forceinline__ int64_t ab_row(const DevGraph& g, const VState* vs, const Score& sc, int32_t base,
                                          int64_t b, int64_t e, int t, int S, int32_t v, const VState& me,
                                          int64_t wv) {
  int64_t acc = 0;
  for (int64_t j0 = b + t; j0 < e; j0 += (int64_t)S * UU) {
    // lanes past the end read the row's last entry (j0 < e) and drop it: loads issued without branches
    int32_t us[UU];
    int64_t ws[UU];
    bool ok[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      const int64_t j = j0 + (int64_t)k * S;
      ok[k] = j < e;
      const int64_t jc = ok[k] ? j : e - 1;
      us[k] = g.idx[jc];
      ws[k] = g.w[jc];
    }
    VState os[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) os[k] = vs[us[k]];
    int pat[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) {
      pat[k] = 0;
      if (ok[k] && os[k].d != D_NONE && before(us[k] - base, os[k].delta, v - base, me.delta, sc.tie))
        pat[k] = ab_pattern(me.c, me.d, os[k].c, os[k].d);
    }
    int64_t vu[UU];
#pragma unroll
    for (int k = 0; k < UU; ++k) vu[k] = pat[k] ? g.vw[us[k]] : 0;
#pragma unroll
    for (int k = 0; k < UU; ++k)
      if (pat[k]) acc += (int64_t)pat[k] * (sc.q * ws[k] - sc.p * vu[k] * wv);
  }
  return acc;
}

template <int G>
__device__ __forceinline__ void ab_grp_blocks(const int32_t* list, int64_t cnt, unsigned bid, unsigned nblk,
                                              const DevGraph& g, const VState* vs, const ScoreSrc& ss, uint8_t* keep,
                                              VtxAcc& va) {
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)bid * (BLOCK / G) + threadIdx.x / G; gid < cnt; gid += (int64_t)nblk * (BLOCK / G)) {
    const int32_t v = list[gid];
    const VState me = vs[v];
    if (me.d == D_NONE) {
      if (gl == 0) keep[v] = 0;
    } else {
      int64_t acc = ab_row<G <= 16 ? 1 : U>(g, vs, ss.at(v), ss.base(v), g.off[v], g.off[v + 1], gl, G, v, me, g.vw[v]);
      acc = sum_reduce<G>(acc);
      if (gl == 0) {
        bool k = (__int128)me.delta + acc >= 0;
        keep[v] = k;
        if (k) va.ncand += 1;
      }
    }
  }
}

template <int G>
__global__ __launch_bounds__(BLOCK) void k_ab_grp(const int32_t* list, int64_t cnt, DevGraph g, const VState* vs,
                                                  ScoreSrc ss, uint8_t* keep, LMSlot* slot, int pass,
                                                  int64_t* S) {
  VtxAcc va;
  if (slot->skip[pass]) return;
  ab_grp_blocks<G>(list, cnt, blockIdx.x, gridDim.x, g, vs, ss, keep, va);
  acc_flush<BLOCK>(va, S, CT_NM, -1);
}

// buckets 0-2 in one launch, as for the enumeration
__global__ __launch_bounds__(BLOCK) void k_ab_grps(GrpSet q, DevGraph g, const VState* vs, ScoreSrc ss, uint8_t* keep,
                                                   LMSlot* slot, int pass, int64_t* S) {
  VtxAcc va;
  if (slot->skip[pass]) return;
  unsigned bid;
  const int k = grp_set_bucket(q, bid);  // uniform over the workgroup
  if (k == 0) ab_grp_blocks<4>(q.list[0], q.cnt[0], bid, q.nb[0], g, vs, ss, keep, va);
  else if (k == 1) ab_grp_blocks<8>(q.list[1], q.cnt[1], bid, q.nb[1], g, vs, ss, keep, va);
  else ab_grp_blocks<16>(q.list[2], q.cnt[2], bid, q.nb[2], g, vs, ss, keep, va);
  acc_flush<BLOCK>(va, S, CT_NM, -1);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ab_blk(const int32_t* list, int64_t cnt, DevGraph g, const VState* vs,
                                               ScoreSrc ss, uint8_t* keep, LMSlot* slot, int pass,
                                               int64_t* S) {
  VtxAcc va;
  if (slot->skip[pass]) return;
  for (int64_t vi = blockIdx.x; vi < cnt; vi += gridDim.x) {
    const int32_t v = list[vi];
    const VState me = vs[v];
    if (me.d == D_NONE) {  // uniform over the block
      if (threadIdx.x == 0) keep[v] = 0;
      continue;
    }
    int64_t acc = ab_row(g, vs, ss.at(v), ss.base(v), g.off[v], g.off[v + 1], threadIdx.x, BS, v, me, g.vw[v]);
    acc = sum_reduce<BS>(acc);
    if (threadIdx.x == 0) {
      bool k = (__int128)me.delta + acc >= 0;
      keep[v] = k;
      if (k) va.ncand += 1;
    }
  }
  acc_flush<BS>(va, S, CT_NM, -1);
}

__global__ __launch_bounds__(HUB_BLOCK) void k_ab_hub(const int32_t* hubs, const int32_t* chunk_off, int64_t n7,
                                                      DevGraph g, const VState* vs, ScoreSrc ss, int64_t* hacc,
                                                      const LMSlot* slot, int pass) {
  if (slot->skip[pass]) return;
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const VState me = vs[v];
  if (me.d == D_NONE) return;
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK);
  const int64_t wv = g.vw[v];
  int64_t acc = ab_row(g, vs, ss.at(v), ss.base(v), j0, j1, threadIdx.x, HUB_BLOCK, v, me, wv);
  acc = sum_reduce<HUB_BLOCK>(acc);
  if (threadIdx.x == 0 && acc) atomicAdd((unsigned long long*)&hacc[k], (unsigned long long)acc);
}

__global__ void k_ab_hub_final(const int32_t* hubs, int64_t n7, const VState* vs, int64_t* hacc, uint8_t* keep,
                               LMSlot* slot, int pass, int64_t* S) {
  VtxAcc va;
  if (slot->skip[pass]) return;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n7) {
    int32_t v = hubs[k];
    VState me = vs[v];
    bool kp = me.d != D_NONE && (__int128)me.delta + hacc[k] >= 0;
    keep[v] = kp;
    hacc[k] = 0;
    if (kp) va.ncand += 1;
  }
  acc_flush<BLOCK>(va, S, CT_NM, -1);
}

// Ablations of the symmetry breaking (Table 2): every candidate kept (mode 1), or the minimum label heuristic
// in odd passes (mode 2: kept only when moving to a lower cluster id or to a new singleton).
__global__ void k_keep_rule(const int32_t* list, int64_t cnt, const VState* vs, int mode, int pass, uint8_t* keep,
                            LMSlot* slot, int64_t* S) {
  VtxAcc va;
  if (slot->skip[pass]) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = list[i];
    const VState s = vs[v];
    bool k = s.d != D_NONE;
    if (k && mode == 2 && (pass & 1)) k = s.d == D_EMPTY || s.d < s.c;
    keep[v] = k;
    if (k) va.ncand += 1;
  }
  acc_flush<BLOCK>(va, S, CT_NM, -1);
}

// ---------------------------------------------------------------------------------------------------------
// Update (the update step of Alg. 2): simultaneous moves with integer atomics on the cluster
// weights and sizes.  Movers to a new singleton take the ids left unused by all other moves, smallest first,
// in ascending vertex order.
// ---------------------------------------------------------------------------------------------------------
constexpr int APPLY_PER = 2;                   // vertices per thread and tile (their loads overlap)
constexpr int APPLY_TILE = APPLY_PER * BLOCK;  // vertices per workgroup tile
constexpr int AGG_SLOTS = 4096;                // LDS aggregation table of the cluster-weight changes
constexpr int AGG_BLOCKS = 768;                // workgroups of the aggregating kernels (3 per CU fit the LDS)
// The table keeps accumulating over a workgroup's tiles and is flushed only before it could pass half full (a
// tile adds at most 2 APPLY_TILE keys): a heavy cluster then receives one global atomic per workgroup, not per
// tile (same-address atomics serialise).
constexpr int AGG_FLUSH_AT = AGG_SLOTS / 2 - 2 * APPLY_TILE;
static_assert(AGG_FLUSH_AT >= 0, "the table must hold the keys of a tile");

// LDS aggregation table that also lists its occupied slots: a flush visits only those and leaves the table
// empty behind it, so neither the flush nor the next tile pays for the whole table.
struct AggList {
  int32_t* keys;
  unsigned long long* vals;
  uint16_t* used;  // occupied slots, in claim order (the table stays at most half full)
  int* nused;
  __device__ __forceinline__ void clear_all() {
    for (int s = threadIdx.x; s < AGG_SLOTS; s += blockDim.x) { keys[s] = -1; vals[s] = 0; }
    if (threadIdx.x == 0) *nused = 0;
  }
  // Adds v to key k when act; called by every lane of a converged wavefront.  Returns 1 when k took a new
  // slot; the new slots of the wavefront are appended to the list with one LDS atomic.
  __device__ __forceinline__ int add(bool act, int32_t k, int64_t v) {
    int claimed = 0;
    uint32_t h = 0;
    if (act) {
      h = ((uint32_t)k * 2654435761u) & (AGG_SLOTS - 1);
      for (int probe = 0; probe < AGG_SLOTS; ++probe) {
        const int32_t prev = atomicCAS(&keys[h], -1, k);
        if (prev == -1 || prev == k) {
          atomicAdd(&vals[h], (unsigned long long)v);
          claimed = prev == -1;
          break;
        }
        h = (h + 1) & (AGG_SLOTS - 1);
      }
    }
    const uint64_t m = __ballot(claimed);
    if (m) {
      const int lane = threadIdx.x & (WAVE - 1);
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(nused, __popcll(m));
      base = __shfl(base, leader, WAVE);
      if (claimed) used[base + __popcll(m & ((1ull << lane) - 1))] = (uint16_t)h;
    }
    return claimed;
  }
  // Adds every listed entry into out (sq: also returns this thread's share of the change of the sum of
  // squares, as LdsAgg::flush_sq) and empties those slots.  Call between workgroup barriers; the caller then
  // resets the list count.
  __device__ __forceinline__ int64_t flush(int64_t* out, bool sq) {
    const int n = *nused;
    uint64_t d = 0;  // modulo 2^64: the changes of all workgroups add up to a value that fits
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int s = used[i];
      const int32_t k = keys[s];
      const unsigned long long v = vals[s];
      if (v) {
        const int64_t old = (int64_t)atomicAdd((unsigned long long*)&out[k], v);
        if (sq) d += (uint64_t)(2 * old * (int64_t)v + (int64_t)v * (int64_t)v);  // modulo 2^64
      }
      keys[s] = -1;
      vals[s] = 0;
    }
    return (int64_t)d;
  }
};

// sq (optional) receives the change of sum_c W_c^2 made by the moves (a single graph's state bookkeeping);
// slot->n_empty becomes nonzero when some kept move goes to a new singleton.
__global__ __launch_bounds__(BLOCK) void k_apply(int64_t n, const uint8_t* keep, const VState* vs,
                                                 const int64_t* vw, int32_t* C, int64_t* W, uint8_t* empty,
                                                 LMSlot* slot, int pass, int64_t* S, int track_sq) {
  if (slot && slot->skip[pass]) return;
  uint64_t dsq = 0;  // modulo 2^64 (see AggList::flush)
  __shared__ int32_t ak[AGG_SLOTS];
  __shared__ unsigned long long av[AGG_SLOTS];
  __shared__ uint16_t au[AGG_SLOTS / 2];
  __shared__ int an;
  __shared__ unsigned long long ne;
  AggList agg{ak, av, au, &an};
  if (threadIdx.x == 0) ne = 0;
  agg.clear_all();
  __syncthreads();
  int used = 0;  // distinct keys in the table (uniform over the workgroup)
  for (int64_t t0 = (int64_t)blockIdx.x * APPLY_TILE; t0 < n; t0 += (int64_t)gridDim.x * APPLY_TILE) {
    uint8_t kp[APPLY_PER];
#pragma unroll
    for (int k = 0; k < APPLY_PER; ++k) {
      const int64_t v = t0 + k * BLOCK + threadIdx.x;
      kp[k] = v < n ? keep[v] : 0;
    }
    VState sv[APPLY_PER];
    int64_t wv[APPLY_PER];
#pragma unroll
    for (int k = 0; k < APPLY_PER; ++k) {
      const int64_t v = t0 + k * BLOCK + threadIdx.x;
      sv[k] = VState{0, D_NONE, 0};
      wv[k] = 0;
      if (kp[k]) { sv[k] = vs[v]; wv[k] = vw[v]; }
    }
    int64_t claims = 0;
#pragma unroll
    for (int k = 0; k < APPLY_PER; ++k) {
      const int64_t v = t0 + k * BLOCK + threadIdx.x;
      const bool mv = kp[k] && sv[k].d != D_EMPTY;  // a move into an existing cluster
      claims += agg.add(kp[k], sv[k].c, -wv[k]);
      claims += agg.add(mv, sv[k].d, wv[k]);
      if (v < n) {
        if (mv) C[v] = sv[k].d;
        if (kp[k] && !mv) atomicAdd(&ne, 1ull);
        empty[v] = (uint8_t)(kp[k] && !mv);
      }
    }
    used += (int)sum_reduce<BLOCK>(claims);  // its barriers also complete this tile's table updates
    if (used > AGG_FLUSH_AT) {
      dsq += (uint64_t)agg.flush(W, track_sq);
      __syncthreads();
      if (threadIdx.x == 0) an = 0;
      __syncthreads();
      used = 0;
    }
  }
  if (used) dsq += (uint64_t)agg.flush(W, track_sq);
  __syncthreads();
  if (threadIdx.x == 0 && ne && slot) slot->n_empty = 1;  // consumers only test it against zero
  if (track_sq) {
    const int64_t tot = sum_reduce<BLOCK>((int64_t)dsq);
    if (threadIdx.x == 0 && tot) atomicAdd(stripe(S, CT_SQ), (unsigned long long)tot);
  }
}

// Free cluster ids are the ids that no vertex holds once every move except those to a new singleton is
// applied.  A held id is marked with this pass's tag (marks of earlier passes carry older tags).
__global__ void k_free_mark(int64_t n, const int32_t* C, const uint8_t* empty, uint32_t* held, uint32_t tag,
                            const LMSlot* slot) {
  if (slot->n_empty == 0) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (!empty[v]) held[C[v]] = tag;
}

// The free ids in ascending order (freelist) and, for a union, every id's rank among them (rank[n] = count).
__global__ __launch_bounds__(BLOCK) void k_free_list(int64_t n, const uint32_t* held, uint32_t tag,
                                                     int32_t* freelist, int32_t* rank, unsigned long long* status,
                                                     uint32_t* ticket, uint32_t lbtag, uint32_t nt,
                                                     const LMSlot* slot) {
  if (slot->n_empty == 0) return;
  __shared__ uint32_t sh_t, sh_p, wsum[BLOCK / WAVE];
  const uint32_t draws = nt + gridDim.x;
  for (uint32_t t = lb_next(ticket, draws, &sh_t); t < nt; t = lb_next(ticket, draws, &sh_t)) {
    const int64_t base = (int64_t)t * LB_TILE + (int64_t)threadIdx.x * LB_ITEMS;
    uint32_t f[LB_ITEMS], s = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
      f[k] = (base + k < n && held[base + k] != tag) ? 1u : 0u;
      s += f[k];
    }
    uint32_t tot;
    const uint32_t ex = lb_block_excl(s, &tot, wsum);
    uint32_t run = lb_prefix(status, t, lbtag, tot, &sh_p) + ex;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
      if (base + k < n) {
        if (rank) rank[base + k] = (int32_t)run;
        if (f[k]) freelist[run] = (int32_t)(base + k);
      }
      run += f[k];
    }
    if (rank && base < n && base + LB_ITEMS >= n) rank[n] = (int32_t)run;
  }
}

// Movers to a new singleton take the free ids in ascending vertex order: the i-th mover takes freelist[i].
// For a union only the movers' ranks are written (rank, rank[n] = count); k_assign_empty_seg assigns.
__global__ __launch_bounds__(BLOCK) void k_assign_empty(int64_t n, const uint8_t* empty, const int32_t* freelist,
                                                        const int64_t* vw, int32_t* C, int64_t* W, int32_t* rank,
                                                        unsigned long long* status, uint32_t* ticket,
                                                        uint32_t lbtag, uint32_t nt, const LMSlot* slot,
                                                        int64_t* sq) {
  if (slot->n_empty == 0) return;
  int64_t dsq = 0;  // each new singleton adds w(v)^2 to sum_c W_c^2
  __shared__ uint32_t sh_t, sh_p, wsum[BLOCK / WAVE];
  const uint32_t draws = nt + gridDim.x;
  for (uint32_t t = lb_next(ticket, draws, &sh_t); t < nt; t = lb_next(ticket, draws, &sh_t)) {
    const int64_t base = (int64_t)t * LB_TILE + (int64_t)threadIdx.x * LB_ITEMS;
    uint32_t f[LB_ITEMS], s = 0;
    if (base + LB_ITEMS <= n) {
      const uint64_t e8 = *(const uint64_t*)(empty + base);  // base is a multiple of 8
#pragma unroll
      for (int k = 0; k < LB_ITEMS; ++k) f[k] = (uint32_t)(e8 >> (8 * k)) & 0xFFu ? 1u : 0u;
    } else {
#pragma unroll
      for (int k = 0; k < LB_ITEMS; ++k) f[k] = (base + k < n && empty[base + k]) ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) s += f[k];
    uint32_t tot;
    const uint32_t ex = lb_block_excl(s, &tot, wsum);
    uint32_t run = lb_prefix(status, t, lbtag, tot, &sh_p) + ex;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
      const int64_t v = base + k;
      if (v < n) {
        if (rank) {
          rank[v] = (int32_t)run;
        } else if (f[k]) {
          const int32_t c = freelist[run];
          C[v] = c;
          W[c] = vw[v];  // a free id has weight 0
          dsq += vw[v] * vw[v];
        }
      }
      run += f[k];
    }
    if (rank && base < n && base + LB_ITEMS >= n) rank[n] = (int32_t)run;
  }
  if (sq) {
    dsq = sum_reduce<BLOCK>(dsq);
    if (threadIdx.x == 0 && dsq) atomicAdd((unsigned long long*)sq, (unsigned long long)dsq);
  }
}

// sum over cluster ids of W_c^2
__global__ void k_sw2(const int64_t* W, int64_t n, int64_t* out, const LMSlot* slot, int pass) {
  if (slot && pass >= 0 && slot->skip[pass]) return;
  int64_t s = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = W[c];
    s += x * x;
  }
  s = sum_reduce<BLOCK>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)out, (unsigned long long)s);
}

// ---------------------------------------------------------------------------------------------------------
// Objective: ordered internal edge weight I(C) = sum over edges (u,v) with C[u] = C[v] of w(u,v)
// ---------------------------------------------------------------------------------------------------------
// one total over all rows (counter CT_INT of the stripes S), or per_v[v] per row when per_v is not null
template <int G>
__global__ __launch_bounds__(BLOCK) void k_internal_grp(const int32_t* list, int64_t cnt, DevGraph g,
                                                        const int32_t* C, int64_t* S, const int32_t* skip,
                                                        int64_t* per_v) {
  if (skip && *skip) return;
  const int gl = threadIdx.x % G;
  int64_t s = 0;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    int64_t x = internal_row<G <= 16 ? 1 : U>(g, C, g.off[v], g.off[v + 1], gl, G, C[v]);
    if (per_v) {
      x = sum_reduce<G>(x);
      if (gl == 0) per_v[v] = x;
    } else {
      s += x;
    }
  }
  if (per_v) return;
  s = sum_reduce<BLOCK>(s);
  if (threadIdx.x == 0 && s) atomicAdd(stripe(S, CT_INT), (unsigned long long)s);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_internal_blk(const int32_t* list, int64_t cnt, DevGraph g, const int32_t* C,
                                                     int64_t* S, const int32_t* skip, int64_t* per_v) {
  if (skip && *skip) return;
  int64_t s = 0;
  for (int64_t vi = blockIdx.x; vi < cnt; vi += gridDim.x) {
    const int32_t v = list[vi];
    int64_t x = internal_row(g, C, g.off[v], g.off[v + 1], threadIdx.x, BS, C[v]);
    if (per_v) {
      x = sum_reduce<BS>(x);
      if (threadIdx.x == 0) per_v[v] = x;
    } else {
      s += x;
    }
  }
  if (per_v) return;
  s = sum_reduce<BS>(s);
  if (threadIdx.x == 0 && s) atomicAdd(stripe(S, CT_INT), (unsigned long long)s);
}

__global__ __launch_bounds__(HUB_BLOCK) void k_internal_hub(const int32_t* hubs, const int32_t* chunk_off,
                                                            int64_t n7, DevGraph g, const int32_t* C, int64_t* S,
                                                            const int32_t* skip, int64_t* per_v) {
  if (skip && *skip) return;
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int32_t cv = C[v];
  const int64_t j0 = g.off[v] + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK);
  int64_t s = internal_row(g, C, j0, j1, threadIdx.x, HUB_BLOCK, cv);
  s = sum_reduce<HUB_BLOCK>(s);
  if (threadIdx.x == 0 && s) atomicAdd(per_v ? (unsigned long long*)&per_v[v] : stripe(S, CT_INT), (unsigned long long)s);
}

// per_v[hubs[k]] = 0 before the hub chunks add into it
__global__ void k_zero_listed(const int32_t* list, int64_t cnt, int64_t* per_v, const int32_t* skip) {
  if (skip && *skip) return;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += (int64_t)gridDim.x * blockDim.x)
    per_v[list[k]] = 0;
}

// ---------------------------------------------------------------------------------------------------------
// Union of graphs: per-graph sums and the per-graph best-so-far decision
// ---------------------------------------------------------------------------------------------------------

// out[k] = sum of x[i] (square: x[i]^2) over i in [vbase[k], vbase[k+1]); one workgroup per graph.  When pass
// `pass` repeats the previous one (slot->skip), the previous state's sums are copied from prev instead.
__global__ __launch_bounds__(BLOCK) void k_seg_sum(const int64_t* x, int square, const int32_t* vbase, int64_t G,
                                                   int64_t* out, const int64_t* prev, const LMSlot* slot,
                                                   int pass) {
  const bool skip = slot && pass >= 0 && slot->skip[pass];
  for (int64_t k = blockIdx.x; k < G; k += gridDim.x) {
    if (skip) {
      if (threadIdx.x == 0) out[k] = prev[k];
      continue;
    }
    int64_t s = 0;
    for (int64_t i = (int64_t)vbase[k] + threadIdx.x; i < vbase[k + 1]; i += BLOCK) {
      int64_t v = x[i];
      s += square ? v * v : v;
    }
    s = sum_reduce<BLOCK>(s);
    if (threadIdx.x == 0) out[k] = s;
  }
}

// Best-so-far check of state k for every graph (Alg. 2: C_out <- C when the graph's objective improves).
__global__ void k_best_seg(SegLM sg, const LMSlot* slot, int k, int skipk) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < sg.G; g += (int64_t)gridDim.x * blockDim.x) {
    sg.copy[g] = 0;
    if (skipk >= 0 && slot->skip[skipk]) continue;
    const Score sc = sg.score[g];
    const int64_t N = sc.q * sg.I[(int64_t)k * sg.G + g] - sc.p * (sg.SW2[(int64_t)k * sg.G + g] - sg.sumw2[g]);
    if (k == 0) {
      sg.N0[g] = N;
      sg.Nbest[g] = N;
    } else if (N > sg.Nbest[g]) {
      sg.Nbest[g] = N;
      sg.copy[g] = 1;
    }
  }
}

__global__ void k_copy_if_seg(const int32_t* copy, const int32_t* gid, const int32_t* C, int32_t* Cout, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (copy[gid[i]]) Cout[i] = C[i];
}

// Movers to a new singleton in a union: the i-th mover of graph k (ascending id) takes the i-th free id of
// graph k; both lists are ascending over the whole union and each graph's share is a contiguous run.
__global__ void k_assign_empty_seg(int64_t n, const uint8_t* empty, const int32_t* rank_free,
                                   const int32_t* rank_mv, const int32_t* freelist, const int32_t* gid,
                                   const int32_t* vbase, const int64_t* vw, int32_t* C, int64_t* W,
                                   const LMSlot* slot) {
  if (slot->n_empty == 0) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (!empty[v]) continue;
    const int32_t b = vbase[gid[v]];
    const int32_t c = freelist[rank_free[b] + (rank_mv[v] - rank_mv[b])];
    C[v] = c;
    W[c] = vw[v];
  }
}

__global__ __launch_bounds__(BLOCK) void k_cluster_weights(const int32_t* C, const int64_t* vw, int64_t n,
                                                           int64_t* W) {
  constexpr int PER = 4, T = PER * BLOCK;  // one key per vertex: a tile adds at most T keys
  static_assert(AGG_SLOTS / 2 - T >= 0, "the table must hold the keys of a tile");
  __shared__ int32_t ak[AGG_SLOTS];
  __shared__ unsigned long long av[AGG_SLOTS];
  __shared__ uint16_t au[AGG_SLOTS / 2];
  __shared__ int an;
  AggList agg{ak, av, au, &an};
  agg.clear_all();
  __syncthreads();
  int used = 0;  // as in k_apply: flushed before the table could pass half full
  for (int64_t t0 = (int64_t)blockIdx.x * T; t0 < n; t0 += (int64_t)gridDim.x * T) {
    int32_t c[PER];
    int64_t w[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t v = t0 + k * BLOCK + threadIdx.x;
      c[k] = v < n ? C[v] : -1;
      w[k] = v < n ? vw[v] : 0;
    }
    int64_t claims = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) claims += agg.add(c[k] >= 0, c[k], w[k]);
    used += (int)sum_reduce<BLOCK>(claims);
    if (used > AGG_SLOTS / 2 - T) {
      agg.flush(W, false);
      __syncthreads();
      if (threadIdx.x == 0) an = 0;
      __syncthreads();
      used = 0;
    }
  }
  if (used) agg.flush(W, false);
}

__global__ void k_copy_vw(const int64_t* vw, int64_t* W, int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    W[v] = vw[v];
}

__global__ void k_zero_i64(int64_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------------------------------------------------------
// Degree buckets
// ---------------------------------------------------------------------------------------------------------
__global__ void k_bucket_count(const int64_t* off, int64_t n, Ctrl* ctrl, const int32_t* gid, const uint8_t* gact,
                               BucketBounds bb) {
  __shared__ unsigned long long cnt[NBUCKET], edg[NBUCKET];
  __shared__ unsigned long long chunks, hi6;
  if (threadIdx.x < NBUCKET) { cnt[threadIdx.x] = 0; edg[threadIdx.x] = 0; }
  if (threadIdx.x == 0) { chunks = 0; hi6 = 0; }
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (gact && !gact[gid[v]]) continue;
    int64_t d = off[v + 1] - off[v];
    int b = bucket_of(d, bb);
    atomicAdd(&cnt[b], 1ull);
    if (d) atomicAdd(&edg[b], (unsigned long long)d);
    if (b == NBUCKET - 1) atomicAdd(&chunks, (unsigned long long)cdiv(d, HUB_CHUNK));
    if (b == NBUCKET - 2 && d > B6_SPLIT) atomicAdd(&hi6, 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0 && hi6) atomicAdd((unsigned long long*)&ctrl->bucket6_hi, hi6);
  if (threadIdx.x < NBUCKET && cnt[threadIdx.x])
    atomicAdd((unsigned long long*)&ctrl->bucket_count[threadIdx.x], cnt[threadIdx.x]);
  if (threadIdx.x < NBUCKET && edg[threadIdx.x])
    atomicAdd((unsigned long long*)&ctrl->bucket_edges[threadIdx.x], edg[threadIdx.x]);
  if (threadIdx.x == 0 && chunks) atomicAdd((unsigned long long*)&ctrl->count3, chunks);
}

__global__ void k_bucket_offsets(Ctrl* ctrl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t s = 0;
  for (int b = 0; b < NBUCKET; ++b) {
    ctrl->bucket_off[b] = s;
    ctrl->bucket_cursor[b] = s;
    s += ctrl->bucket_count[b];
  }
  ctrl->bucket_off[NBUCKET] = s;
  ctrl->bucket6_cursor_hi = ctrl->bucket_off[NBUCKET - 1] - ctrl->bucket6_hi;
}

// Bucket lists: per workgroup tile, LDS counts per bucket, one global atomic per bucket, positions inside
// the tile from LDS atomics (the order inside a bucket does not affect any result).  Rows of bucket 6 longer
// than B6_SPLIT go to the end of its list (a list of their own, index NBUCKET here), so the two table sizes of
// that bucket each walk only their own rows.
__global__ __launch_bounds__(BLOCK) void k_bucket_scatter(const int64_t* off, int64_t n, int32_t* list,
                                                          Ctrl* ctrl, const int32_t* gid, const uint8_t* gact,
                                                          BucketBounds bb) {
  __shared__ uint32_t cnt[NBUCKET + 1];
  __shared__ int64_t base[NBUCKET + 1];
  constexpr int T = 4 * BLOCK;
  for (int64_t t0 = (int64_t)blockIdx.x * T; t0 < n; t0 += (int64_t)gridDim.x * T) {
    if (threadIdx.x <= NBUCKET) cnt[threadIdx.x] = 0;
    __syncthreads();
    int b[4];
    uint32_t r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int64_t v = t0 + k * BLOCK + threadIdx.x;
      b[k] = -1;
      if (v < n && (!gact || gact[gid[v]])) {
        const int64_t d = off[v + 1] - off[v];
        b[k] = bucket_of(d, bb);
        if (b[k] == NBUCKET - 2 && d > B6_SPLIT) b[k] = NBUCKET;
      }
      if (b[k] >= 0) r[k] = atomicAdd(&cnt[b[k]], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET && cnt[threadIdx.x])
      base[threadIdx.x] = (int64_t)atomicAdd((unsigned long long*)&ctrl->bucket_cursor[threadIdx.x],
                                             (unsigned long long)cnt[threadIdx.x]);
    if (threadIdx.x == NBUCKET && cnt[NBUCKET])
      base[NBUCKET] = (int64_t)atomicAdd((unsigned long long*)&ctrl->bucket6_cursor_hi,
                                         (unsigned long long)cnt[NBUCKET]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (b[k] >= 0) list[base[b[k]] + r[k]] = (int32_t)(t0 + k * BLOCK + threadIdx.x);
    __syncthreads();
  }
}

__global__ void k_hub_chunk_counts(const int32_t* hubs, int64_t n7, const int64_t* off, int32_t* cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n7; k += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = hubs[k];
    cnt[k] = (int32_t)cdiv(off[v + 1] - off[v], HUB_CHUNK);
  }
}

// ---------------------------------------------------------------------------------------------------------
// Validation of the CSR (setup, Sec. II): offsets first, then one pass over the rows checking index range,
// self-loops, strict ascending order and positive weights.  Symmetry is checked by a multiset fingerprint:
// with rows strictly ascending, the graph is symmetric iff the multiset of stored (u, v, w) equals that of
// (v, u, w); the sums (mod 2^64) of a 64-bit hash of (u, v, w) and of (v, u, w) over the stored entries are
// compared (an asymmetric input passes only on a hash collision).
// ---------------------------------------------------------------------------------------------------------
__global__ void k_validate_offsets(const int64_t* off, int64_t n, int64_t nnz, Ctrl* ctrl) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    if (off[0] != 0 || off[n] != nnz) atomicOr(&ctrl->err_bits, ERRB_INVALID);
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (off[v + 1] < off[v]) atomicOr(&ctrl->err_bits, ERRB_INVALID);
}

// Exact symmetry, two ways (the driver picks one per call; both give the same verdict):
//  - by transposition: every entry j = (v, u, w) of row v is also written as the key (u << 32 | v) with value
//    w.  A stable sort of these pairs by u alone keeps, for each u, the entries in the order of their rows v,
//    so the sorted sequence is the transposed CSR in canonical order; the graph is symmetric iff it equals the
//    CSR itself entry by entry (k_sym_compare).  Cost: a few streaming passes, whatever the layout.
//  - by search (keys == null, search set): vertices are ranked by (row length, id); every entry (v, u) whose
//    target u ranks below v must find (u, v) of the same weight in row u (binary search, rows ascending), and
//    these entries must be exactly as many as those whose target ranks above.  The first condition maps them
//    one-to-one onto entries (u, v) whose target v ranks above u (rows hold no duplicate); with equal counts
//    that map is onto, so every entry has its reverse.  Each search runs in the shorter row of its pair: cheap
//    when the rows a search visits are in cache (graphs of a few million entries, or a union of such graphs),
//    line-miss bound otherwise.
// A row that is not ascending is reported as unsorted first.
struct EdgeCheck {
  uint32_t err = 0;
  int64_t balance = 0;  // entries towards a lower-ranked vertex minus entries towards a higher-ranked one
  int64_t ws = 0;
  int64_t lower = 0;    // entries towards a lower vertex id
};

__device__ __forceinline__ bool found_in_row(const DevGraph& g, int64_t lo, int64_t end, int32_t v, int32_t wt) {
  int64_t hi = end;
  while (lo < hi) {  // first position holding an id >= v
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (g.idx[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < end && g.idx[lo] == v && g.w[lo] == wt;
}

// entry j = (v, u) of row v, which starts at rb and holds dv entries
__device__ __forceinline__ void check_edge(const DevGraph& g, int32_t v, int64_t j, int64_t rb, int64_t dv,
                                           EdgeCheck& ec, bool search) {
  int32_t u = g.idx[j];
  int32_t wt = g.w[j];
  ec.ws += wt;
  ec.lower += u < v;
  if (u < 0 || u >= g.n) { ec.err |= ERRB_INVALID; return; }
  if (u == v) { ec.err |= ERRB_SELF_LOOP; return; }
  if (j > rb && g.idx[j - 1] >= u) ec.err |= ERRB_UNSORTED;
  if (wt <= 0) ec.err |= ERRB_WEIGHT;
  if (!search) return;
  const int64_t bu = g.off[u], eu = g.off[u + 1], du = eu - bu;
  if (du < dv || (du == dv && u < v)) {
    ++ec.balance;
    if (!found_in_row(g, bu, eu, v, wt)) ec.err |= ERRB_NOT_SYMMETRIC;
  } else {
    --ec.balance;
  }
}

// Symmetry by transposition of the upper half.  Row v's entries towards higher ids (the upper entries; a
// suffix of the ascending row, after its lo[v] lower entries) are written as pairs (u << 32 | v, w), packed
// in entry order: entry j goes to j - lbase[v] - lo[v], lbase = exclusive scan of lo.  Sorted stably by u,
// the pairs of target u list their sources ascending, so a symmetric graph gives exactly row u's lower part:
// position p must hold u with lbase[u] <= p < lbase[u] + lo[u], the source at idx[off[u] + p - lbase[u]] and the
// same weight, and there must be as many lower entries as upper ones (nnz / 2 each).  Positions map to distinct
// lower entries, so equal counts make the pairing a bijection.
template <int G>
__global__ __launch_bounds__(BLOCK) void k_sym_emit_grp(const int32_t* list, int64_t cnt, DevGraph g,
                                                        const int32_t* lo, const int64_t* lbase, uint64_t* keys,
                                                        uint32_t* vals) {
  const int gl = threadIdx.x % G;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int64_t rb = g.off[v], re = g.off[v + 1];
    const int64_t shift = lbase[v] + lo[v];
    for (int64_t j = rb + lo[v] + gl; j < re; j += G) {
      keys[j - shift] = ((uint64_t)(uint32_t)g.idx[j] << 32) | (uint32_t)v;
      vals[j - shift] = (uint32_t)g.w[j];
    }
  }
}

// hub rows: each chunk writes the upper entries of its own edge range
__global__ __launch_bounds__(HUB_BLOCK) void k_sym_emit_hub(const int32_t* hubs, const int32_t* chunk_off, int64_t n7,
                                                            DevGraph g, const int32_t* lo, const int64_t* lbase,
                                                            uint64_t* keys, uint32_t* vals) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int64_t rb = g.off[v];
  const int64_t j0 = max(rb + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK, rb + lo[v]);
  const int64_t j1 = min(g.off[v + 1], rb + (int64_t)(blockIdx.x - chunk_off[k] + 1) * HUB_CHUNK);
  const int64_t shift = lbase[v] + lo[v];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK) {
    keys[j - shift] = ((uint64_t)(uint32_t)g.idx[j] << 32) | (uint32_t)v;
    vals[j - shift] = (uint32_t)g.w[j];
  }
}

__global__ __launch_bounds__(BLOCK) void k_sym_compare(DevGraph g, const uint64_t* ks, const uint32_t* vs, int64_t m,
                                                       const int32_t* lo, const int64_t* lbase, Ctrl* ctrl) {
  bool bad = false;
  if (blockIdx.x == 0 && threadIdx.x == 0) bad = g.nnz != 2 * m || lbase[g.n] != m;
  for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < m; p += (int64_t)gridDim.x * BLOCK) {
    const uint64_t key = ks[p];
    const int64_t u = (int64_t)(key >> 32);
    const int32_t v = (int32_t)(uint32_t)key;
    if (u >= g.n) { bad = true; continue; }
    const int64_t r = p - lbase[u];
    if (r < 0 || r >= lo[u]) { bad = true; continue; }
    const int64_t j = g.off[u] + r;
    bad |= v != g.idx[j] || vs[p] != (uint32_t)g.w[j];
  }
  if (bad) atomicOr(&ctrl->err_bits, ERRB_NOT_SYMMETRIC);
}

// vertex-weight mode of a vertex (per graph in a union), and the optional per-vertex weighted-degree output
struct VwSrc {
  int mode;
  const int32_t* gid;
  const int8_t* gmode;
  int64_t* rowsum;
  __device__ __forceinline__ int at(int32_t v) const { return gmode ? (int)gmode[gid[v]] : mode; }
};

__device__ __forceinline__ int64_t vertex_weight(int vw_mode, int64_t ws, const int64_t* vw_given, int32_t v,
                                                 uint32_t& err) {
  if (vw_mode == 1) return ws;
  if (vw_mode == 2) return 1;
  int64_t x = vw_given[v];
  if (x < 0) err |= ERRB_WEIGHT;
  if (x >= ((int64_t)1 << 31)) err |= ERRB_VW_TOO_BIG;
  return x;
}

__device__ __forceinline__ void flush_check(EdgeCheck ec, int64_t wsum, Ctrl* ctrl) {
  // block-wide: every thread calls this
  const int64_t bal = sum_reduce<BLOCK>(ec.balance);
  wsum = sum_reduce<BLOCK>(wsum);
  if (ec.err) atomicOr(&ctrl->err_bits, ec.err);
  if (threadIdx.x == 0) {
    if (bal) atomicAdd((unsigned long long*)&ctrl->count0, (unsigned long long)bal);
    if (wsum) atomicAdd((unsigned long long*)&ctrl->sum_we, (unsigned long long)wsum);
  }
}

template <int G>
__global__ __launch_bounds__(BLOCK) void k_validate_grp(const int32_t* list, int64_t cnt, DevGraph g, VwSrc vm,
                                                        const int64_t* vw_given, int64_t* vw_out, Ctrl* ctrl,
                                                        int32_t* lo, bool search) {
  const int gl = threadIdx.x % G;
  EdgeCheck ec;
  int64_t wsum = 0;
  for (int64_t gid = (int64_t)blockIdx.x * (BLOCK / G) + threadIdx.x / G; gid < cnt;
       gid += (int64_t)gridDim.x * (BLOCK / G)) {
    const int32_t v = list[gid];
    const int64_t rb = g.off[v], re = g.off[v + 1];
    const int64_t ws0 = ec.ws, lo0 = ec.lower;
    for (int64_t j = rb + gl; j < re; j += G) check_edge(g, v, j, rb, re - rb, ec, search);
    int64_t ws = sum_reduce<G>(ec.ws - ws0);
    const int64_t nlo = lo ? sum_reduce<G>(ec.lower - lo0) : 0;
    if (gl == 0) {
      if (lo) lo[v] = (int32_t)nlo;
      vw_out[v] = vertex_weight(vm.at(v), ws, vw_given, v, ec.err);
      if (vm.rowsum) vm.rowsum[v] = ws;
      wsum += ws;
    }
  }
  flush_check(ec, wsum, ctrl);
}

__global__ __launch_bounds__(BIG_BLOCK) void k_validate_blk(const int32_t* list, int64_t cnt, DevGraph g, VwSrc vm,
                                                            const int64_t* vw_given, int64_t* vw_out, Ctrl* ctrl,
                                                            int32_t* lo, bool search) {
  EdgeCheck ec;
  int64_t wsum = 0;
  for (int64_t vi = blockIdx.x; vi < cnt; vi += gridDim.x) {
    const int32_t v = list[vi];
    const int64_t rb = g.off[v], re = g.off[v + 1];
    const int64_t ws0 = ec.ws, lo0 = ec.lower;
    for (int64_t j = rb + threadIdx.x; j < re; j += BIG_BLOCK) check_edge(g, v, j, rb, re - rb, ec, search);
    int64_t ws = sum_reduce<BIG_BLOCK>(ec.ws - ws0);
    const int64_t nlo = lo ? sum_reduce<BIG_BLOCK>(ec.lower - lo0) : 0;
    if (threadIdx.x == 0) {
      if (lo) lo[v] = (int32_t)nlo;
      vw_out[v] = vertex_weight(vm.at(v), ws, vw_given, v, ec.err);
      if (vm.rowsum) vm.rowsum[v] = ws;
      wsum += ws;
    }
  }
  flush_check(ec, wsum, ctrl);
}

// hubs: chunk sums of the weighted degree land in hsum[k] (zeroed beforehand)
__global__ __launch_bounds__(HUB_BLOCK) void k_validate_hub(const int32_t* hubs, const int32_t* chunk_off,
                                                            int64_t n7, DevGraph g, int64_t* hsum, Ctrl* ctrl,
                                                            int32_t* lo, bool search) {
  const int k = find_chunk_owner(chunk_off, n7, blockIdx.x);
  const int32_t v = hubs[k];
  const int64_t rb = g.off[v];
  const int64_t j0 = rb + (int64_t)(blockIdx.x - chunk_off[k]) * HUB_CHUNK;
  const int64_t j1 = min(g.off[v + 1], j0 + HUB_CHUNK);
  EdgeCheck ec;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += HUB_BLOCK) check_edge(g, v, j, rb, g.off[v + 1] - rb, ec, search);
  int64_t ws = sum_reduce<HUB_BLOCK>(ec.ws);
  if (threadIdx.x == 0 && ws) atomicAdd((unsigned long long*)&hsum[k], (unsigned long long)ws);
  if (lo) {  // lo of a hub is zeroed beforehand; its chunks add their counts
    const int64_t nlo = sum_reduce<HUB_BLOCK>(ec.lower);
    if (threadIdx.x == 0 && nlo) atomicAdd(&lo[v], (int32_t)nlo);
  }
  flush_check(ec, threadIdx.x == 0 ? ws : 0, ctrl);
}

__global__ void k_validate_hub_final(const int32_t* hubs, int64_t n7, VwSrc vm, const int64_t* vw_given,
                                     int64_t* hsum, int64_t* vw_out, Ctrl* ctrl) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n7) return;
  int32_t v = hubs[k];
  uint32_t err = 0;
  vw_out[v] = vertex_weight(vm.at(v), hsum[k], vw_given, v, err);
  if (vm.rowsum) vm.rowsum[v] = hsum[k];
  hsum[k] = 0;
  if (err) atomicOr(&ctrl->err_bits, err);
}

__global__ void k_vertex_sums(const int64_t* vw, int64_t n, Ctrl* ctrl) {
  int64_t s = 0, s2 = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = vw[v];
    s += x;
    s2 += x * x;
  }
  s = sum_reduce<BLOCK>(s);
  s2 = sum_reduce<BLOCK>(s2);
  if (threadIdx.x == 0) {
    if (s) atomicAdd((unsigned long long*)&ctrl->sum_w, (unsigned long long)s);
    if (s2) atomicAdd((unsigned long long*)&ctrl->sum_w2, (unsigned long long)s2);
  }
}

__global__ __launch_bounds__(1024) void k_fold(int64_t* S, FoldDst f) { fold_block(S, f); }

inline unsigned grid_for(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}
// kernels that end in one global atomic per workgroup on a shared counter: few workgroups, so the atomics
// on that one address do not serialise behind each other
inline unsigned red_blocks(int64_t n) {
  int64_t g = cdiv(n, BLOCK);
  return (unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

// Persistent launches: workgroups loop over their share of the vertices.  Launching one short workgroup per
// vertex (or per few vertices) is bound by the workgroup dispatch rate, not by memory.
// The local move takes twice the level's grid cap (4096 workgroups by default); the workgroup-per-vertex
// kernels of bucket 6 take a quarter of that.
inline unsigned grp_blocks(const Buckets& b, int64_t cnt, int G) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(cnt, BLOCK / G), 2 * (int64_t)b.grid_cap));
}
inline unsigned vtx_blocks(const Buckets& b, int64_t cnt, int64_t cap_div = 1) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cnt, 2 * (int64_t)b.grid_cap / cap_div));
}
// persistent workgroups of a single-pass scan over nt tiles
inline unsigned lb_blocks(uint32_t nt) { return (unsigned)std::max<uint32_t>(1, std::min<uint32_t>(nt, 1024)); }

// Fold the listed counters (id, destination; a null destination folds nothing) of the stripes S: now, with a
// fold kernel, or, when `pending` is given, by the next bookkeeping kernel (k_pass_begin, k_best or
// k_final_state), which folds its FoldDst before anything reads the destinations.
void fold(int64_t* S, std::initializer_list<std::pair<int, int64_t*>> m, hipStream_t st, FoldDst* pending = nullptr) {
  FoldDst f{};
  bool any = false;
  for (const auto& e : m)
    if (e.second) { f.d[e.first] = e.second; any = true; }
  if (pending) {
    for (int ct = 0; ct < CT_COUNT; ++ct)
      if (f.d[ct]) pending->d[ct] = f.d[ct];
  } else if (any) {
    k_fold<<<1, 1024, 0, st>>>(S, f);
  }
}

// Hub chunk scratch lives at the end of the per-chunk partial arrays.
struct HubScratch {
  int64_t* ps;
  int32_t* pc;
  int64_t* pown;
  int64_t* hacc;
};

}  // namespace

// =========================================================================================================
// Host launchers
// =========================================================================================================

void launch_validate_offsets(const int64_t* off, int64_t n, int64_t nnz, Ctrl* ctrl, hipStream_t st) {
  k_validate_offsets<<<grid_for(n), BLOCK, 0, st>>>(off, n, nnz, ctrl);
}

void launch_validate_rows(const DevGraph& g, const Buckets& b, int vw_mode, const int64_t* vw_given,
                          int64_t* vw_out, Ctrl* ctrl, hipStream_t st, const SymBuffers& sb, const int32_t* gid,
                          const int8_t* gmode, int64_t* rowsum) {
  const int32_t* L = b.list;
  const VwSrc vm{vw_mode, gid, gmode, rowsum};
  const bool tr = sb.k0 && g.nnz > 0;  // symmetry by transposition: the rows' lower counts first
  int32_t* lo = tr ? sb.lo : nullptr;
  const int64_t nw = b.count[4] + b.count[5];
  const int32_t* hubs = L + b.off[7];
  if (tr && b.count[7]) fill_i32(lo, 0, g.n, st);  // hub rows add their chunks' counts
  if (b.count[0]) k_validate_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (b.count[1]) k_validate_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (b.count[2]) k_validate_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (b.count[3]) k_validate_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (nw) k_validate_grp<64><<<grp_blocks(b, nw, 64), BLOCK, 0, st>>>(L + b.off[4], nw, g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (b.count[6]) k_validate_blk<<<vtx_blocks(b, b.count[6]), BIG_BLOCK, 0, st>>>(L + b.off[6], b.count[6], g, vm, vw_given, vw_out, ctrl, lo, sb.search);
  if (b.count[7]) {
    fill_i64(b.hub_acc, 0, b.count[7], st);
    k_validate_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, b.count[7], g, b.hub_acc, ctrl, lo, sb.search);
    k_validate_hub_final<<<grid_for(b.count[7]), BLOCK, 0, st>>>(hubs, b.count[7], vm, vw_given, b.hub_acc, vw_out, ctrl);
  }
  if (tr) {  // the upper entries packed, sorted by their target and compared with the rows' lower parts
    scan_i32_i64(lo, sb.lbase, g.n, sb.scan_temp, st);
    const int64_t m = g.nnz / 2;
    const int32_t* lc = lo;
    if (b.count[0]) k_sym_emit_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, lc, sb.lbase, sb.k0, sb.v0);
    if (b.count[1]) k_sym_emit_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, lc, sb.lbase, sb.k0, sb.v0);
    if (b.count[2]) k_sym_emit_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, lc, sb.lbase, sb.k0, sb.v0);
    if (b.count[3]) k_sym_emit_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, lc, sb.lbase, sb.k0, sb.v0);
    if (nw + b.count[6]) k_sym_emit_grp<64><<<grp_blocks(b, nw + b.count[6], 64), BLOCK, 0, st>>>(L + b.off[4], nw + b.count[6], g, lc, sb.lbase, sb.k0, sb.v0);
    if (b.count[7]) k_sym_emit_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, b.count[7], g, lc, sb.lbase, sb.k0, sb.v0);
    int bits = 1;
    while (((int64_t)1 << bits) < g.n) ++bits;
    int shifts[4];
    const int npass = (bits + 7) / 8;
    for (int k = 0; k < npass; ++k) shifts[k] = 32 + 8 * k;
    const int which = m > 0 ? radix_sort_pairs(sb.k0, sb.v0, sb.k1, sb.v1, m, shifts, npass, sb.temp, st) : 0;
    k_sym_compare<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(m, BLOCK), 16384)), BLOCK, 0, st>>>(
        g, which ? sb.k1 : sb.k0, which ? sb.v1 : sb.v0, m, lc, sb.lbase, ctrl);
  }
}

void launch_buckets(const int64_t* off, int64_t n, int32_t* list, Ctrl* ctrl, const BucketBounds& bb, hipStream_t st,
                    const int32_t* gid, const uint8_t* gact) {
  k_bucket_count<<<red_blocks(n), BLOCK, 0, st>>>(off, n, ctrl, gid, gact, bb);
  k_bucket_offsets<<<1, 1, 0, st>>>(ctrl);
  k_bucket_scatter<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 4 * BLOCK), 8192)), BLOCK, 0, st>>>(off, n, list, ctrl, gid, gact, bb);
}

void launch_hub_chunks(const int32_t* hubs, int64_t n7, const int64_t* off, int32_t* cnt, int32_t* chunk_off,
                       void* temp, hipStream_t st) {
  if (n7 == 0) return;
  k_hub_chunk_counts<<<grid_for(n7), BLOCK, 0, st>>>(hubs, n7, off, cnt);
  scan_i32_i32(cnt, chunk_off, n7, temp, st);
}

void launch_vertex_sums(const int64_t* vw, int64_t n, Ctrl* ctrl, hipStream_t st) {
  k_vertex_sums<<<red_blocks(n), BLOCK, 0, st>>>(vw, n, ctrl);
}

void launch_cluster_weights(const int32_t* C, const int64_t* vw, int64_t n, int64_t* W, hipStream_t st) {
  fill_i64(W, 0, n, st);
  k_cluster_weights<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 4 * BLOCK), AGG_BLOCKS)), BLOCK, 0, st>>>(C, vw, n, W);
}

static void launch_internal(const DevGraph& g, const Buckets& b, const int32_t* C, int64_t* out,
                            const int32_t* skip, hipStream_t st, int64_t* per_v = nullptr,
                            FoldDst* pending = nullptr) {
  const int32_t* L = b.list;
  int64_t* S = b.stripes;
  if (b.count[0]) k_internal_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, C, S, skip, per_v);
  if (b.count[1]) k_internal_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, C, S, skip, per_v);
  if (b.count[2]) k_internal_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, C, S, skip, per_v);
  if (b.count[3]) k_internal_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, C, S, skip, per_v);
  if (b.count[4]) k_internal_grp<32><<<grp_blocks(b, b.count[4], 32), BLOCK, 0, st>>>(L + b.off[4], b.count[4], g, C, S, skip, per_v);
  if (b.count[5]) k_internal_grp<64><<<grp_blocks(b, b.count[5], 64), BLOCK, 0, st>>>(L + b.off[5], b.count[5], g, C, S, skip, per_v);
  if (b.count[6]) k_internal_blk<BIG_BLOCK><<<vtx_blocks(b, b.count[6]), BIG_BLOCK, 0, st>>>(L + b.off[6], b.count[6], g, C, S, skip, per_v);
  if (b.count[7]) {
    if (per_v) k_zero_listed<<<grid_for(b.count[7]), BLOCK, 0, st>>>(L + b.off[7], b.count[7], per_v, skip);
    k_internal_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(L + b.off[7], b.hub_chunk_off, b.count[7], g, C, S, skip, per_v);
  }
  if (!per_v) fold(S, {{CT_INT, out}}, st, pending);
}

void launch_internal_per_vertex(const DevGraph& g, const Buckets& b, const int32_t* C, int64_t* out,
                                hipStream_t st) {
  launch_internal(g, b, C, nullptr, nullptr, st, out);
}

static unsigned seg_blocks(int64_t G) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(G, 4096)); }

void launch_seg_sum(const int64_t* x, int square, const int32_t* vbase, int64_t G, int64_t* out, hipStream_t st) {
  if (G > 0) k_seg_sum<<<seg_blocks(G), BLOCK, 0, st>>>(x, square, vbase, G, out, nullptr, nullptr, -1);
}

void launch_objective(const DevGraph& g, const Buckets& b, const int32_t* C, const int64_t* W, Ctrl* ctrl,
                      hipStream_t st) {
  k_zero_i64<<<1, 1, 0, st>>>(&ctrl->obj_I);
  k_zero_i64<<<1, 1, 0, st>>>(&ctrl->obj_SW2);
  launch_internal(g, b, C, &ctrl->obj_I, nullptr, st);
  k_sw2<<<red_blocks(g.n), BLOCK, 0, st>>>(W, g.n, &ctrl->obj_SW2, nullptr, -1);
}

static const int32_t* L_hubs(const Buckets& b);
static HubScratch hub_scratch(const Buckets& b);

// One pass of destinations + candidacy.  singleton: first coarsening pass (C = identity).
static void launch_destinations(const DevGraph& g, const Buckets& b, const ScoreSrc& sc, uint32_t pa, uint32_t pb,
                                int strict, bool singleton, LMBuffers& bufs, LMSlot* slot, int pass,
                                int64_t* own_sum, const HubScratch& hs, hipStream_t st,
                                FoldDst* pending = nullptr) {
  const int32_t* L = b.list;
  const int32_t* C = bufs.C;
  const int64_t* W = bufs.W;
  VState* vs = bufs.vs;
  const int32_t* hubs = L + b.off[7];
  const int64_t n7 = b.count[7];
  int64_t* S = b.stripes;
  if (singleton) {
    double sb = 0;
    for (int k = 0; k < NBUCKET; ++k) sb += 16.0 * (double)b.edges[k] + 48.0 * (double)b.count[k];
    prof_begin(PF_SINGLE, st);
    if (b.count[0]) k_single_grp<4><<<grp_blocks(b, b.count[0], 4), BLOCK, 0, st>>>(L + b.off[0], b.count[0], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[1]) k_single_grp<8><<<grp_blocks(b, b.count[1], 8), BLOCK, 0, st>>>(L + b.off[1], b.count[1], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[2]) k_single_grp<16><<<grp_blocks(b, b.count[2], 16), BLOCK, 0, st>>>(L + b.off[2], b.count[2], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[3]) k_single_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[4]) k_single_grp<32><<<grp_blocks(b, b.count[4], 32), BLOCK, 0, st>>>(L + b.off[4], b.count[4], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[5]) k_single_grp<64><<<grp_blocks(b, b.count[5], 64), BLOCK, 0, st>>>(L + b.off[5], b.count[5], g, sc, pa, pb, vs, slot, pass, S);
    if (b.count[6]) k_single_blk<BIG_BLOCK><<<vtx_blocks(b, b.count[6]), BIG_BLOCK, 0, st>>>(L + b.off[6], b.count[6], g, sc, pa, pb, vs, slot, pass, S);
    if (n7) {
      k_single_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, sc, hs.ps, hs.pc);
      k_hub_final<<<grid_for(n7), BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g.vw, nullptr, nullptr, sc, pa, pb, 0,
                                                 hs.ps, hs.pc, nullptr, vs, slot, pass, S, -1);
    }
    prof_end(PF_SINGLE, sb, st);
    fold(S, {{CT_NCAND, &slot->nL[pass]}}, st, pending);
    return;
  }
  int64_t* P = strict ? nullptr : bufs.enum_bytes;  // algorithmic-byte counters (diagnostics), per bucket
  const int co = own_sum ? CT_OWN : -1;
  auto cp = [&](int k) { return P ? CT_PAIRS + k : -1; };
  // the launches count their algorithmic bytes on the device; they join the timing tallies when the call ends
#define LCC_ENUM(k, launch)                      \
  if (b.count[k]) {                              \
    prof_begin(PF_ENUM_B0 + k, st);              \
    launch;                                      \
    prof_end(PF_ENUM_B0 + k, 0.0, st);           \
  }
  {  // buckets 0-2 in one launch (its time is family 0's, its bytes those of the three buckets)
    GrpSet q{};
    unsigned nb = 0;
    for (int k = 0; k < 3; ++k) {
      q.list[k] = L + b.off[k];
      q.cnt[k] = b.count[k];
      q.nb[k] = b.count[k] ? grp_blocks(b, b.count[k], 4 << k) : 0;
      nb += q.nb[k];
    }
    if (nb) {
      prof_begin(PF_ENUM_B0, st);
      k_enum_grps<<<nb, BLOCK, 0, st>>>(q, g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(0));
      prof_end(PF_ENUM_B0, 0.0, st);
    }
  }
  LCC_ENUM(3, (k_enum_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(3))))
  LCC_ENUM(4, (k_enum_wave<LDS_SLOTS_B4><<<grp_blocks(b, b.count[4], WAVE), BLOCK, 0, st>>>(L + b.off[4], b.count[4], g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(4), b.hash_shift)))
  LCC_ENUM(5, (k_enum_blk<128, LDS_SLOTS_B5><<<vtx_blocks(b, b.count[5]), 128, 0, st>>>(L + b.off[5], b.count[5], g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(5), b.hash_shift)))
  // bucket 6: rows up to B6_SPLIT on 512 threads and an 8192-slot table; when a tuning raises the bucket's
  // bound, the longer rows (the tail of the bucket's list) on 1024 threads and a 16384-slot table
  const int64_t n6 = b.count[6] - b.count6_hi;
  if (n6) {
    prof_begin(PF_ENUM_B0 + 6, st);
    k_enum_blk<512, LDS_SLOTS_B6><<<vtx_blocks(b, n6, 4), 512, 0, st>>>(L + b.off[6], n6, g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(6), b.hash_shift);
    prof_end(PF_ENUM_B0 + 6, 0.0, st);
  }
  if (b.count6_hi) {
    prof_begin(PF_ENUM_B0 + 6, st);
    k_enum_blk<1024, LDS_SLOTS_B6X><<<vtx_blocks(b, b.count6_hi, 4), 1024, 0, st>>>(L + b.off[6] + n6, b.count6_hi, g, C, W, sc, pa, pb, strict, vs, slot, pass, S, co, cp(6), b.hash_shift);
    prof_end(PF_ENUM_B0 + 6, 0.0, st);
  }
#undef LCC_ENUM
  if (n7) {
    unsigned nc = (unsigned)b.hub_chunks;
    prof_begin(PF_ENUM_B0 + 7, st);
    k_hub_insert<<<nc, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, C, bufs.arena, slot, pass, sc.cons);
    k_hub_scan<<<nc, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g, C, W, sc, bufs.arena, hs.ps, hs.pc, hs.pown, slot, pass,
                                         S, cp(7));
    k_hub_final<<<grid_for(n7), BLOCK, 0, st>>>(hubs, b.hub_chunk_off, n7, g.vw, C, W, sc, pa, pb, strict, hs.ps,
                                               hs.pc, hs.pown, vs, slot, pass, S, co, g.off, cp(7));
    prof_end(PF_ENUM_B0 + 7, 0.0, st);
  }
  fold(S, {{CT_NCAND, slot ? &slot->nL[pass] : nullptr}, {CT_OWN, own_sum}, {CT_PAIRS + 0, P ? P + 0 : nullptr},
           {CT_PAIRS + 1, P ? P + 1 : nullptr}, {CT_PAIRS + 2, P ? P + 2 : nullptr}, {CT_PAIRS + 3, P ? P + 3 : nullptr},
           {CT_PAIRS + 4, P ? P + 4 : nullptr}, {CT_PAIRS + 5, P ? P + 5 : nullptr}, {CT_PAIRS + 6, P ? P + 6 : nullptr},
           {CT_PAIRS + 7, P ? P + 7 : nullptr}}, st, pending);
}

static const int32_t* L_hubs(const Buckets& b) { return b.list + b.off[7]; }

static HubScratch hub_scratch(const Buckets& b) {
  HubScratch hs;
  hs.ps = b.hub_ps;
  hs.pc = b.hub_pc;
  hs.pown = b.hub_pown;
  hs.hacc = b.hub_acc;
  return hs;
}

static void launch_afterburner(const DevGraph& g, const Buckets& b, const ScoreSrc& sc, LMBuffers& bufs,
                               LMSlot* slot, int pass, const HubScratch& hs, hipStream_t st) {
  const int32_t* L = b.list;
  const VState* vs = bufs.vs;
  uint8_t* keep = bufs.keep;
  {  // buckets 0-2 in one launch
    GrpSet q{};
    unsigned nb = 0;
    for (int k = 0; k < 3; ++k) {
      q.list[k] = L + b.off[k];
      q.cnt[k] = b.count[k];
      q.nb[k] = b.count[k] ? grp_blocks(b, b.count[k], 4 << k) : 0;
      nb += q.nb[k];
    }
    if (nb) k_ab_grps<<<nb, BLOCK, 0, st>>>(q, g, vs, sc, keep, slot, pass, b.stripes);
  }
  if (b.count[3]) k_ab_grp<32><<<grp_blocks(b, b.count[3], 32), BLOCK, 0, st>>>(L + b.off[3], b.count[3], g, vs, sc, keep, slot, pass, b.stripes);
  // degree 33-128 rows in half-wavefront groups (one pass of U = 4 loads covers them), longer ones per wavefront
  if (b.count[4]) k_ab_grp<32><<<grp_blocks(b, b.count[4], 32), BLOCK, 0, st>>>(L + b.off[4], b.count[4], g, vs, sc, keep, slot, pass, b.stripes);
  if (b.count[5]) k_ab_grp<64><<<grp_blocks(b, b.count[5], 64), BLOCK, 0, st>>>(L + b.off[5], b.count[5], g, vs, sc, keep, slot, pass, b.stripes);
  if (b.count[6]) k_ab_blk<BIG_BLOCK><<<vtx_blocks(b, b.count[6]), BIG_BLOCK, 0, st>>>(L + b.off[6], b.count[6], g, vs, sc, keep, slot, pass, b.stripes);
  if (b.count[7]) {
    const int32_t* hubs = L + b.off[7];
    k_ab_hub<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(hubs, b.hub_chunk_off, b.count[7], g, vs, sc, hs.hacc, slot, pass);
    k_ab_hub_final<<<grid_for(b.count[7]), BLOCK, 0, st>>>(hubs, b.count[7], vs, hs.hacc, keep, slot, pass, b.stripes);
  }
}

// track_sq: keep slot->SW2[pass] (set to the previous state's value by k_pass_begin) up to date from the
// moves instead of recomputing it from all cluster weights
static void apply_and_empty(const DevGraph& g, const Buckets& b, LMBuffers& bufs, const SegLM& sg, LMSlot* slot,
                            int pass, bool track_sq, hipStream_t st, FoldDst* pending = nullptr) {
  const int64_t n = g.n;
  int64_t* sq = track_sq ? &slot->SW2[pass] : nullptr;
  unsigned ga = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, APPLY_TILE), AGG_BLOCKS));
  k_apply<<<ga, BLOCK, 0, st>>>(n, bufs.keep, bufs.vs, g.vw, bufs.C, bufs.W, bufs.empty, slot, pass, b.stripes,
                                track_sq ? 1 : 0);
  // the kept moves (afterburner or keep rule) and the sum-of-squares change
  fold(b.stripes, {{CT_NM, slot ? &slot->nM[pass] : nullptr}, {CT_SQ, sq}}, st, pending);
  // free ids and ranks of the movers to a new singleton; all no-ops unless some vertex moved to a new
  // singleton in this pass
  // all three tags are taken before the first launch: a wrap-around (which clears the tagged words) can then
  // only come before the marks are written, never between the marks and their readers
  Tagged& tg = *bufs.tg;
  uint32_t tags[3];
  next_tags(tg, 3, tags, st);
  const uint32_t mark = tags[0];
  k_free_mark<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.C, bufs.empty, tg.held, mark, slot);
  const uint32_t nt = (uint32_t)cdiv(n, LB_TILE);
  const unsigned gl = lb_blocks(nt);
  k_free_list<<<gl, BLOCK, 0, st>>>(n, tg.held, mark, bufs.freelist, sg.G ? bufs.scan_a : nullptr, tg.status,
                                    tg.ticket, tags[1], nt, slot);
  k_assign_empty<<<gl, BLOCK, 0, st>>>(n, bufs.empty, bufs.freelist, g.vw, bufs.C, bufs.W,
                                       sg.G ? bufs.scan_b : nullptr, tg.status, tg.ticket, tags[2], nt,
                                       slot, sq);
  if (sg.G)
    k_assign_empty_seg<<<grid_for(n), BLOCK, 0, st>>>(n, bufs.empty, bufs.scan_a, bufs.scan_b, bufs.freelist, sg.gid,
                                                     sg.vbase, g.vw, bufs.C, bufs.W, slot);
}

// Objective bookkeeping of state k after pass `pass` (union: per graph).
static void state_sums_sw2(const SegLM& sg, const int64_t* W, int64_t n, LMSlot* slot, int k, int pass,
                           hipStream_t st) {
  if (sg.G) {
    const int64_t G = sg.G;
    k_seg_sum<<<seg_blocks(G), BLOCK, 0, st>>>(W, 1, sg.vbase, G, sg.SW2 + (int64_t)k * G,
                                              k ? sg.SW2 + (int64_t)(k - 1) * G : nullptr, pass >= 0 ? slot : nullptr, pass);
  } else if (pass < 0) {  // the starting state; later states follow from the moves (apply_and_empty)
    k_sw2<<<red_blocks(n), BLOCK, 0, st>>>(W, n, &slot->SW2[k], nullptr, pass);
  }
}

// pend: counters still in the stripes that this check's sums need (folded here, then cleared)
static void best_so_far(const SegLM& sg, LMSlot* slot, const LMParams& prm, LMBuffers& bufs, int64_t n, int k,
                        int skipk, hipStream_t st, int64_t* S, FoldDst& pend) {
  if (sg.G) {
    bool any = false;
    for (int ct = 0; ct < CT_COUNT; ++ct) any = any || pend.d[ct];
    if (any) k_fold<<<1, 1024, 0, st>>>(S, pend);
    pend = FoldDst{};
    k_best_seg<<<grid_for(sg.G), BLOCK, 0, st>>>(sg, slot, k, skipk);
    if (k > 0) k_copy_if_seg<<<grid_for(n), BLOCK, 0, st>>>(sg.copy, sg.gid, bufs.C, bufs.Cout, n);
  } else {
    k_best<<<1, 1024, 0, st>>>(slot, k, skipk, prm.sc.p, prm.sc.q, prm.sum_w2, S, pend);
    pend = FoldDst{};
    if (k > 0) k_copy_if<<<grid_for(n), BLOCK, 0, st>>>(slot, bufs.C, bufs.Cout, n);
  }
}

void local_move(const DevGraph& g, const Buckets& b, const LMParams& prm, bool singleton, LMBuffers& bufs,
                LMSlot* slot, Ctrl* ctrl, hipStream_t st) {
  (void)ctrl;
  const int64_t n = g.n;
  const HubScratch hs = hub_scratch(b);
  const SegLM& sg = prm.seg;
  const int64_t G = sg.G;
  ScoreSrc sc;
  sc.s = prm.sc;
  sc.cons = prm.cons;
  if (G) { sc.tab = sg.score; sc.gid = sg.gid; sc.vbase = sg.vbase; sc.ownv = sg.ownv; }
  zero_bytes(slot, sizeof(LMSlot), st);
  // starting state: cluster weights, sizes, C_out = C, sum of squared cluster weights (state 0)
  if (singleton) {
    iota_i32(bufs.C, n, st);
    k_copy_vw<<<grid_for(n), BLOCK, 0, st>>>(g.vw, bufs.W, n);
  } else {
    launch_cluster_weights(bufs.C, g.vw, n, bufs.W, st);
  }
  copy_i32(bufs.Cout, bufs.C, n, st);
  if (G) {  // vertices outside the bucket lists never move and add nothing to their graph's sums
    fill_u8(bufs.keep, 0, n, st);
    fill_i64(sg.ownv, 0, n, st);
  }
  state_sums_sw2(sg, bufs.W, n, slot, 0, -1, st);
  if (b.count[7])
    k_hub_clear<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(L_hubs(b), b.hub_chunk_off, b.count[7], g.off,
                                                             bufs.arena, nullptr, -1);
  // Counters the kernels leave in the stripes are folded by the next bookkeeping kernel of a single graph
  // (no launch of their own); a union folds them at once.
  int64_t* S = b.stripes;
  FoldDst pend{};
  FoldDst* pp = G ? nullptr : &pend;
  for (int i = 1; i <= prm.pass_limit; ++i) {
    // a pass that kept no move repeats exactly when the next one has the same temperature (and, under the
    // minimum label heuristic, never: its rule alternates between passes)
    int same_phi = i >= 2 && prm.phi_num[i] == prm.phi_num[i - 1] && prm.phi_den[i] == prm.phi_den[i - 1] &&
                   prm.symmetry != 2;
    k_pass_begin<<<1, 1024, 0, st>>>(slot, i, same_phi, S, pend);
    pend = FoldDst{};
    bool single_now = singleton && i == 1;
    launch_destinations(g, b, sc, prm.phi_num[i], prm.phi_den[i], 0, single_now, bufs, slot, i,
                        &slot->I[i - 1], hs, st, pp);
    if (G)  // internal weight of state i-1 per graph, from the own-cluster weights the pass just summed
      k_seg_sum<<<seg_blocks(G), BLOCK, 0, st>>>(sg.ownv, 0, sg.vbase, G, sg.I + (int64_t)(i - 1) * G,
                                                i >= 2 ? sg.I + (int64_t)(i - 2) * G : nullptr, slot, i);
    // best-so-far check of the state this pass started from (state i-1)
    best_so_far(sg, slot, prm, bufs, n, i - 1, i, st, S, pend);
    if (prm.symmetry == 0) {
      launch_afterburner(g, b, sc, bufs, slot, i, hs, st);
    } else {
      const int64_t nl = b.off[NBUCKET];
      k_keep_rule<<<red_blocks(nl), BLOCK, 0, st>>>(b.list, nl, bufs.vs, prm.symmetry, i, bufs.keep, slot,
                                                    b.stripes);
    }
    apply_and_empty(g, b, bufs, sg, slot, i, G == 0, st, pp);
    state_sums_sw2(sg, bufs.W, n, slot, i, i, st);
  }
  const int last = prm.pass_limit;
  if (last >= 1) {
    k_final_state<<<1, 1024, 0, st>>>(slot, last, S, pend);
    pend = FoldDst{};
    if (G) {
      launch_internal(g, b, bufs.C, nullptr, &slot->skip[last], st, sg.ownv);
      k_seg_sum<<<seg_blocks(G), BLOCK, 0, st>>>(sg.ownv, 0, sg.vbase, G, sg.I + (int64_t)last * G,
                                                sg.I + (int64_t)(last - 1) * G, slot, last);
    } else {
      launch_internal(g, b, bufs.C, &slot->I[last], &slot->skip[last], st, nullptr, &pend);
    }
    best_so_far(sg, slot, prm, bufs, n, last, last, st, S, pend);
  } else {
    best_so_far(sg, slot, prm, bufs, n, 0, -1, st, S, pend);
  }
}

void next_tags(Tagged& t, int k, uint32_t* out, hipStream_t st) {
  if (t.last > UINT32_MAX - (uint32_t)k) {  // fewer than k tags left: clear the tagged words, number from 1
    zero_bytes(t.held, (size_t)t.held_cap * sizeof(uint32_t), st);
    zero_bytes(t.status, (size_t)t.status_cap * sizeof(unsigned long long), st);
    t.last = 0;
  }
  for (int i = 0; i < k; ++i) out[i] = ++t.last;
}

uint32_t next_tag(Tagged& t, hipStream_t st) {
  uint32_t x;
  next_tags(t, 1, &x, st);
  return x;
}

void launch_apply_and_empty(const DevGraph& g, const Buckets& b, LMBuffers& bufs, const SegLM& sg, LMSlot* slot,
                            hipStream_t st) {
  apply_and_empty(g, b, bufs, sg, slot, 0, false, st);
}

void launch_destinations_strict(const DevGraph& g, const Buckets& b, const ScoreSrc& ss, LMBuffers& bufs,
                                LMSlot* slot, hipStream_t st) {
  const HubScratch hs = hub_scratch(b);
  if (b.count[7])
    k_hub_clear<<<(unsigned)b.hub_chunks, HUB_BLOCK, 0, st>>>(L_hubs(b), b.hub_chunk_off, b.count[7], g.off,
                                                             bufs.arena, nullptr, -1);
  launch_destinations(g, b, ss, 0, 1, 1, false, bufs, slot, 0, nullptr, hs, st);
}

}  // namespace lcc
