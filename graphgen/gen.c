/*
 * Seeded synthetic graph generators: planted-partition SBM, R-MAT, 2-D lattice.
 *
 * These produce the inputs that both the CPU oracle and the GPU library are
 * run on.  They contain none of the clustering method's arithmetic: they only
 * draw random edges and build a symmetric CSR (rows ascending, neighbours
 * ascending and unique, no self-loops, duplicate edges merged by summing
 * their integer weights).
 *
 * Randomness is counter based, so the output does not depend on the number
 * of OpenMP threads:
 *   fmix64  = the splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014)
 *   key(seed, stream) = fmix64(seed ^ fmix64(stream + GOLDEN))
 *   draw(key, ctr)    = fmix64(key + (ctr + 1) * GOLDEN)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t fmix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27; z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t rkey(uint64_t seed, uint64_t stream) { return fmix64(seed ^ fmix64(stream + GOLDEN)); }
static inline uint64_t rdraw(uint64_t key, uint64_t ctr) { return fmix64(key + (ctr + 1) * GOLDEN); }
/* uniform in (0, 1] with 53 random bits */
static inline double runif(uint64_t x) { return ((double)(x >> 11) + 1.0) * (1.0 / 9007199254740992.0); }
static inline uint64_t prob_threshold(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return UINT64_MAX;
  return (uint64_t)ldexp(p, 64);
}

typedef struct { int32_t v; int32_t w; } nbr_t;

static int cmp_nbr(const void* a, const void* b) {
  int32_t x = ((const nbr_t*)a)->v, y = ((const nbr_t*)b)->v;
  return (x > y) - (x < y);
}

/* Build a symmetric CSR from an undirected pair list.  Self-loops are dropped,
 * parallel edges merged (weights summed).  Outputs are malloc'd; the caller
 * frees them with gen_free.  Returns the number of directed entries, or -1 on
 * allocation failure or weight overflow. */
static int64_t build_csr(int64_t n, int64_t m, const int32_t* pu, const int32_t* pv, const int32_t* pw,
                         int64_t** out_off, int32_t** out_idx, int32_t** out_w) {
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    if (pu[e] == pv[e]) continue;
    __atomic_fetch_add(&deg[pu[e]], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[pv[e]], 1, __ATOMIC_RELAXED);
  }
  int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!off) { free(deg); return -1; }
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
  int64_t tot = off[n];
  nbr_t* nb = (nbr_t*)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(nbr_t));
  if (!nb) { free(deg); free(off); return -1; }
  memcpy(deg, off, (size_t)n * sizeof(int64_t)); /* deg becomes the cursor */
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = pu[e], v = pv[e];
    if (u == v) continue;
    int64_t a = __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
    int64_t b = __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
    nb[a].v = v; nb[a].w = pw ? pw[e] : 1;
    nb[b].v = u; nb[b].w = pw ? pw[e] : 1;
  }
  /* sort each row, merge duplicates; cnt[i] = unique count */
  int64_t* cnt = deg;
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : overflow)
  for (int64_t i = 0; i < n; ++i) {
    nbr_t* r = nb + off[i];
    int64_t d = off[i + 1] - off[i];
    if (d > 1) qsort(r, (size_t)d, sizeof(nbr_t), cmp_nbr);
    int64_t k = 0;
    for (int64_t j = 0; j < d; ++j) {
      if (k > 0 && r[k - 1].v == r[j].v) {
        int64_t s = (int64_t)r[k - 1].w + r[j].w;
        if (s > INT32_MAX) overflow = 1;
        r[k - 1].w = (int32_t)s;
      } else {
        r[k++] = r[j];
      }
    }
    cnt[i] = k;
  }
  if (overflow) { free(deg); free(off); free(nb); return -1; }
  int64_t* noff = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!noff) { free(deg); free(off); free(nb); return -1; }
  noff[0] = 0;
  for (int64_t i = 0; i < n; ++i) noff[i + 1] = noff[i] + cnt[i];
  int64_t nnz = noff[n];
  int32_t* idx = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  int32_t* w = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!idx || !w) { free(deg); free(off); free(nb); free(noff); free(idx); free(w); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    const nbr_t* r = nb + off[i];
    for (int64_t j = 0; j < noff[i + 1] - noff[i]; ++j) {
      idx[noff[i] + j] = r[j].v;
      w[noff[i] + j] = r[j].w;
    }
  }
  free(deg); free(off); free(nb);
  *out_off = noff; *out_idx = idx; *out_w = w;
  return nnz;
}

void gen_free(void* p) { free(p); }

/* Planted partition: vertex i in block i / block_size.  Each unordered pair
 * (i, j), i < j, is an edge independently with probability p_in inside a
 * block and p_out across.  Pairs are visited by geometric skipping along each
 * row (row i draws from its own counter stream), unit weights. */
int64_t gen_sbm(int64_t n_blocks, int64_t block_size, double p_in, double p_out, uint64_t seed,
                int64_t* n_out, int64_t** off, int32_t** idx, int32_t** w) {
  int64_t n = n_blocks * block_size;
  *n_out = n;
  /* first pass counts edges per row, second writes them */
  int64_t* rc = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!rc) return -1;
  for (int pass = 0; pass < 2; ++pass) {
    int32_t *pu = NULL, *pv = NULL;
    int64_t m = 0;
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) { int64_t c = rc[i]; rc[i] = m; m += c; }
      rc[n] = m;
      pu = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
      pv = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
      if (!pu || !pv) { free(pu); free(pv); free(rc); return -1; }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      uint64_t key = rkey(seed, (uint64_t)i);
      uint64_t ctr = 0;
      int64_t blk_end = (i / block_size + 1) * block_size;
      int64_t cnt = 0, pos = pass ? rc[i] : 0;
      for (int seg = 0; seg < 2; ++seg) {
        double p = seg == 0 ? p_in : p_out;
        int64_t lo = seg == 0 ? i + 1 : blk_end, hi = seg == 0 ? blk_end : n;
        if (p <= 0.0 || lo >= hi) continue;
        double lq = log1p(-p);
        int64_t j = lo - 1;
        for (;;) {
          int64_t gap = 1;
          if (p < 1.0) {
            double g = floor(log(runif(rdraw(key, ctr++))) / lq);
            if (g > (double)(hi - j)) break;
            gap = (int64_t)g + 1;
          }
          j += gap;
          if (j >= hi) break;
          if (pass) { pu[pos + cnt] = (int32_t)i; pv[pos + cnt] = (int32_t)j; }
          ++cnt;
        }
      }
      if (!pass) rc[i] = cnt;
    }
    if (pass == 1) {
      int64_t r = build_csr(n, m, pu, pv, NULL, off, idx, w);
      free(pu); free(pv); free(rc);
      return r;
    }
  }
  return -1;
}

/* R-MAT: edge e in [0, edge_factor * 2^scale) descends `scale` levels of the
 * adjacency quadtree; at level k it takes quadrant (0,0),(0,1),(1,0),(1,1) with
 * probabilities (a, b, c, d) using draw(key(seed, e), k).  Then symmetrised,
 * self-loops dropped, duplicates merged by summing weight 1 per occurrence. */
int64_t gen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                 int64_t* n_out, int64_t** off, int32_t** idx, int32_t** w) {
  int64_t n = (int64_t)1 << scale;
  int64_t m = edge_factor * n;
  *n_out = n;
  uint64_t ta = prob_threshold(a), tb = prob_threshold(a + b), tc = prob_threshold(a + b + c);
  int32_t* pu = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  int32_t* pv = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  if (!pu || !pv) { free(pu); free(pv); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t key = rkey(seed, (uint64_t)e);
    uint32_t u = 0, v = 0;
    for (int k = 0; k < scale; ++k) {
      uint64_t r = rdraw(key, (uint64_t)k);
      uint32_t bu = 0, bv = 0;
      if (r < ta) { bu = 0; bv = 0; }
      else if (r < tb) { bu = 0; bv = 1; }
      else if (r < tc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    pu[e] = (int32_t)u; pv[e] = (int32_t)v;
  }
  int64_t r = build_csr(n, m, pu, pv, NULL, off, idx, w);
  free(pu); free(pv);
  return r;
}

/* rows x cols 4-neighbour lattice, vertex id = r * cols + c.  Undirected edge
 * ids: right edges r*(cols-1)+c first, then down edges.  Exactly
 * floor(M * del_frac) edges are deleted, chosen as the prefix of a seeded
 * Fisher-Yates shuffle; the rest get weight 1 + draw % (w_max) (uniform in
 * [1, w_max]). */
int64_t gen_lattice(int64_t rows, int64_t cols, double del_frac, int32_t w_max, uint64_t seed,
                    int64_t* n_out, int64_t** off, int32_t** idx, int32_t** w) {
  int64_t n = rows * cols;
  *n_out = n;
  int64_t mr = rows * (cols - 1), md = (rows - 1) * cols, M = mr + md;
  int64_t k = (int64_t)floor((double)M * del_frac);
  int64_t* perm = (int64_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(int64_t));
  uint8_t* del = (uint8_t*)calloc((size_t)(M > 0 ? M : 1), 1);
  if (!perm || !del) { free(perm); free(del); return -1; }
  for (int64_t e = 0; e < M; ++e) perm[e] = e;
  uint64_t kd = rkey(seed, 1);
  for (int64_t i = 0; i < k; ++i) {
    int64_t j = i + (int64_t)(rdraw(kd, (uint64_t)i) % (uint64_t)(M - i));
    int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    del[perm[i]] = 1;
  }
  free(perm);
  int64_t m = M - k;
  int32_t* pu = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t* pv = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t* pw = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!pu || !pv || !pw) { free(del); free(pu); free(pv); free(pw); return -1; }
  uint64_t kw = rkey(seed, 2);
  int64_t t = 0;
  for (int64_t e = 0; e < M; ++e) {
    if (del[e]) continue;
    int64_t a, b;
    if (e < mr) { int64_t r = e / (cols - 1), c = e % (cols - 1); a = r * cols + c; b = a + 1; }
    else { int64_t x = e - mr; int64_t r = x / cols, c = x % cols; a = r * cols + c; b = a + cols; }
    pu[t] = (int32_t)a; pv[t] = (int32_t)b;
    pw[t] = 1 + (int32_t)(rdraw(kw, (uint64_t)e) % (uint64_t)w_max);
    ++t;
  }
  free(del);
  int64_t r = build_csr(n, m, pu, pv, pw, off, idx, w);
  free(pu); free(pv); free(pw);
  return r;
}

/* Build a CSR from a caller-supplied undirected pair list (used for small
 * hand-made graphs and kNN graphs assembled in Python). */
int64_t gen_from_pairs(int64_t n, int64_t m, const int32_t* pu, const int32_t* pv, const int32_t* pw,
                       int64_t** off, int32_t** idx, int32_t** w) {
  return build_csr(n, m, pu, pv, pw, off, idx, w);
}

/* ---------------------------------------------------------------------------------------------------
 * k-nearest-neighbour graphs of Gaussian-mixture points (the batched workload).
 *
 * Points live on an integer grid of 1/8 unit so that every distance is an exact integer:
 *   normal draw  = Irwin-Hall sum of twelve 16-bit uniforms minus 6 * 65536   (unit 1/65536, sd ~ 1)
 *   mean[c][d]   = 3 * normal(key_means, c * dim + d)                          (sd 3)
 *   component(i) = high 32 bits of draw(key_pts, i * (3 dim + 1)) scaled to [0, K)
 *   x[i][d]      = clamp(floor((mean + normal) / 8192 + 1/2), -127, 127)      (unit 1/8)
 * with key_means = key(seed, 2 graph) and key_pts = key(seed, 2 graph + 1).  Only integer operations, so
 * any implementation of this recipe gives the same points.
 * ------------------------------------------------------------------------------------------------- */
static inline int64_t irwin_hall12(uint64_t key, uint64_t ctr0) {
  int64_t s = 0;
  for (int t = 0; t < 3; ++t) {
    uint64_t x = rdraw(key, ctr0 + (uint64_t)t);
    s += (int64_t)(x & 0xFFFF) + (int64_t)((x >> 16) & 0xFFFF) + (int64_t)((x >> 32) & 0xFFFF) + (int64_t)(x >> 48);
  }
  return s - 6 * 65536;
}

void gen_knn_points(int64_t n, int32_t dim, int32_t K, uint64_t seed, uint64_t graph, int8_t* out) {
  const uint64_t km = rkey(seed, 2 * graph), kp = rkey(seed, 2 * graph + 1);
  int64_t* mean = (int64_t*)malloc((size_t)K * dim * sizeof(int64_t));
  for (int64_t c = 0; c < K; ++c)
    for (int64_t d = 0; d < dim; ++d) mean[c * dim + d] = 3 * irwin_hall12(km, 3 * (uint64_t)(c * dim + d));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t base = (uint64_t)i * (uint64_t)(3 * dim + 1);
    const uint64_t cx = rdraw(kp, base);
    const int64_t c = (int64_t)(((cx >> 32) * (uint64_t)K) >> 32);
    for (int64_t d = 0; d < dim; ++d) {
      int64_t a = mean[c * dim + d] + irwin_hall12(kp, base + 1 + 3 * (uint64_t)d);
      int64_t x = (a + 4096) >> 13;
      if (x > 127) x = 127;
      if (x < -127) x = -127;
      out[i * dim + d] = (int8_t)x;
    }
  }
  free(mean);
}

/* Exact k nearest neighbours of every point by brute force: squared distances are integers, ties go to the
 * lower index.  nbr[i*k + t], d2[i*k + t] in ascending (distance, index) order.  Requires n > k. */
void gen_knn(const int8_t* pts, int64_t n, int32_t dim, int32_t k, int32_t* nbr, int64_t* d2) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    int64_t* bd = d2 + i * k;
    int32_t* bj = nbr + i * k;
    int cnt = 0;
    const int8_t* pi = pts + i * dim;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const int8_t* pj = pts + j * dim;
      int64_t s = 0;
      for (int d = 0; d < dim; ++d) {
        int64_t t = (int64_t)pi[d] - pj[d];
        s += t * t;
      }
      if (cnt == k && s >= bd[k - 1]) continue;  /* (s, j) is not below the current k-th: j > its index */
      int pos = cnt < k ? cnt++ : k - 1;
      while (pos > 0 && bd[pos - 1] > s) {
        bd[pos] = bd[pos - 1];
        bj[pos] = bj[pos - 1];
        --pos;
      }
      bd[pos] = s;
      bj[pos] = (int32_t)j;
    }
  }
}
