/*
 * CPU oracle for synchronous multilevel LambdaCC clustering -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded and exact (every product and comparison in 128-bit integers).  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it.  It shares no code with the
 * GPU library.  Each function names the part of the paper it follows:
 *
 *   Eq. 1 and the signed graph w'          -> objective(), score arithmetic
 *   Alg. 2 (synchronous local move)        -> lm_pass(), local_move()
 *   Alg. 3 (afterburner filter)            -> inside lm_pass()
 *   Alg. 4 (graph contraction)             -> contract()
 *   Alg. 6 (pLeidenR)                      -> refine()
 *   Sec. V-A (alternate local move)        -> lmalt()
 *   Alg. 1 (Louvain / Louvain+)            -> run_louvain()
 *   Alg. 5 (pLeiden)                       -> run_leiden()
 *
 * Integer form used throughout (lambda = p / q in lowest terms, w' scaled by q):
 *   a(v,c)  = sum of w(u,v) over neighbours u of v with C[u] = c
 *   W_c     = sum of w(u) over members u of cluster c
 *   S(v,c)  = q a(v,c) - p w(v) W_c                      (= q w'(v, C_c) for c != C[v])
 *   S_cur   = q a(v,C[v]) - p w(v) (W_C[v] - w(v))        (= q w'(v, C[v]))
 *   N(C)    = q * sum_{ordered internal pairs} w'(u,v)    (lambdaCC = N / q, Eq. 1)
 *           = q I(C) - p (sum_c W_c^2 - sum_v w(v)^2)
 *   moving v from A to B changes N by 2 (S(v,B) - S(v,A)).
 *
 * Readings of points the paper leaves open are listed in the design notes; the ones that shape the code
 * are repeated at the function that takes them.
 */
#include "lcc_oracle.h"

#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

typedef struct {
  int64_t n;
  const int64_t* off;
  const int32_t* idx;
  const int32_t* ew; /* NULL => all 1 */
  const int64_t* vw;
  const int32_t* B;  /* constraint clustering of the coarsening local move (Sec. IV-D), NULL => none */
} ograph;

static inline int64_t EW(const ograph* g, int64_t j) { return g->ew ? g->ew[j] : 1; }

/* splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014) */
uint64_t orc_fmix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 27; z *= 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* MurmurHash3 32-bit finaliser (Appleby), a bijection on 32-bit words */
uint32_t orc_fmix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85EBCA6BU;
  h ^= h >> 13; h *= 0xC2B2AE35U;
  return h ^ (h >> 16);
}
/* t-th output (t = 0, 1, ...) of the splitmix64 generator seeded with `seed` */
static uint64_t seed_stream(uint64_t seed, uint64_t t) {
  return orc_fmix64(seed + (t + 1) * 0x9E3779B97F4A7C15ULL);
}

static void* xcalloc(size_t n, size_t s) {
  void* p = calloc(n ? n : 1, s);
  if (!p) abort(); /* the oracle is test infrastructure: out of memory is fatal */
  return p;
}
static void* xmalloc(size_t n) {
  void* p = malloc(n ? n : 1);
  if (!p) abort();
  return p;
}

static i128 i128_abs(i128 x) { return x < 0 ? -x : x; }
static void put128(i128 x, int64_t* hl) {
  hl[0] = (int64_t)(x >> 64);
  hl[1] = (int64_t)(uint64_t)x;
}

/* ---------------------------------------------------------------------------------------------------
 * Setup (Sec. II): validate the symmetric CSR, derive vertex weights, fix lambda = p / q.
 * Check order: arguments, structure, self-loops, sortedness, weights, symmetry, weight totals (total edge
 * weight < 2^32, so every weighted degree and coarse edge weight is < 2^31; given vertex weights < 2^31),
 * lambda, exactness bound.
 * ------------------------------------------------------------------------------------------------- */
static int64_t find_in_row(const ograph* g, int64_t row, int32_t key) {
  int64_t lo = g->off[row], hi = g->off[row + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->idx[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < g->off[row + 1] && g->idx[lo] == key) ? lo : -1;
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) { uint64_t t = a % b; a = b; b = t; }
  return a;
}

int orc_setup(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
              int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int64_t* vw_out,
              uint64_t* pq) {
  if (n < 0 || n > 2147483647LL || !off) return ORC_ERR_INVALID;
  if (vw_mode != ORC_VW_GIVEN && vw_mode != ORC_VW_WEIGHTED_DEGREE && vw_mode != ORC_VW_UNIT) return ORC_ERR_INVALID;
  if (vw_mode == ORC_VW_GIVEN && n > 0 && !vw_in) return ORC_ERR_INVALID;
  if (off[0] != 0) return ORC_ERR_INVALID;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return ORC_ERR_INVALID;
  int64_t nnz = off[n];
  if (nnz > 0 && !idx) return ORC_ERR_INVALID;
  ograph g = {n, off, idx, ew, NULL};
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = off[v]; j < off[v + 1]; ++j)
      if (idx[j] < 0 || idx[j] >= n) return ORC_ERR_INVALID;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = off[v]; j < off[v + 1]; ++j)
      if (idx[j] == v) return ORC_ERR_SELF_LOOP;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = off[v] + 1; j < off[v + 1]; ++j)
      if (idx[j] <= idx[j - 1]) return ORC_ERR_UNSORTED;
  for (int64_t j = 0; j < nnz; ++j)
    if (EW(&g, j) <= 0) return ORC_ERR_WEIGHT;
  if (vw_mode == ORC_VW_GIVEN)
    for (int64_t v = 0; v < n; ++v)
      if (vw_in[v] < 0) return ORC_ERR_WEIGHT;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = off[v]; j < off[v + 1]; ++j) {
      int64_t r = find_in_row(&g, idx[j], (int32_t)v);
      if (r < 0 || EW(&g, r) != EW(&g, j)) return ORC_ERR_NOT_SYMMETRIC;
    }
  i128 WE = 0, W = 0;
  for (int64_t j = 0; j < nnz; ++j) WE += EW(&g, j);
  if (WE >= ((i128)1 << 32)) return ORC_ERR_OVERFLOW; /* every weighted degree < 2^31 */
  if (vw_mode == ORC_VW_GIVEN)
    for (int64_t v = 0; v < n; ++v)
      if (vw_in[v] >= ((int64_t)1 << 31)) return ORC_ERR_OVERFLOW;
  for (int64_t v = 0; v < n; ++v) {
    int64_t x;
    if (vw_mode == ORC_VW_GIVEN) x = vw_in[v];
    else if (vw_mode == ORC_VW_UNIT) x = 1;
    else { x = 0; for (int64_t j = off[v]; j < off[v + 1]; ++j) x += EW(&g, j); }
    vw_out[v] = x;
    W += x;
  }
  if (lam_den == 0) return ORC_ERR_LAMBDA;
  i128 P = lam_num, Q = (i128)lam_den * (lam_over_total ? W : 1);
  if (Q <= 0 || P > Q) return ORC_ERR_LAMBDA;
  if (Q >= ((i128)1 << 64)) return ORC_ERR_OVERFLOW;
  uint64_t p = (uint64_t)P, q = (uint64_t)Q;
  if (p == 0) q = 1;
  else { uint64_t d = gcd_u64(p, q); p /= d; q /= d; }
  /* admission bound of the library (every score and objective numerator of the method stays below 2^62 in
   * magnitude); the oracle itself computes in 128 bits throughout */
  if ((i128)q * WE + (i128)p * W * W >= ((i128)1 << 62)) return ORC_ERR_OVERFLOW;
  pq[0] = p; pq[1] = q;
  return ORC_OK;
}

/* ---------------------------------------------------------------------------------------------------
 * Objective, Eq. 1: sum over clusters of sum over ordered pairs u != v of w(u,v) - lambda w(u) w(v),
 * scaled by q.  I(C) counts each internal undirected edge twice (E holds both directions).
 * ------------------------------------------------------------------------------------------------- */
static i128 objective(const ograph* g, i128 p, i128 q, const int32_t* C) {
  int64_t n = g->n;
  int64_t* Wc = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  i128 I = 0, sumw2 = 0, sumW2 = 0;
  for (int64_t v = 0; v < n; ++v) {
    Wc[C[v]] += g->vw[v];
    sumw2 += (i128)g->vw[v] * g->vw[v];
    for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j)
      if (C[g->idx[j]] == C[v]) I += EW(g, j);
  }
  for (int64_t c = 0; c < n; ++c) sumW2 += (i128)Wc[c] * Wc[c];
  free(Wc);
  return q * I - p * (sumW2 - sumw2);
}

void orc_objective(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                   uint64_t p, uint64_t q, const int32_t* C, int64_t* N_hi_lo) {
  ograph g = {n, off, idx, ew, vw};
  put128(objective(&g, p, q, C), N_hi_lo);
}

/* ---------------------------------------------------------------------------------------------------
 * Afterburner ordering (Sec. IV-A): larger deltas first; two deltas whose objective changes 2 delta / q
 * differ by less than epsilon are ordered by a hash of the vertex id (splitmix64 finaliser), then by id.
 * A zero difference always counts as a tie, so the relation is total on distinct vertices.
 * ------------------------------------------------------------------------------------------------- */
static int before(int64_t u, i128 du, int64_t v, i128 dv, i128 q, uint32_t eps_num, uint32_t eps_den) {
  i128 diff = du - dv;
  int tie = (diff == 0) || ((i128)2 * eps_den * i128_abs(diff) < (i128)eps_num * q);
  if (!tie) return du > dv;
  uint64_t hu = orc_fmix64((uint64_t)u), hv = orc_fmix64((uint64_t)v);
  if (hu != hv) return hu < hv;
  return u < v;
}

/* Scratch for one pass. */
typedef struct {
  int64_t* acc;     /* dense a(v, c) accumulator over cluster ids */
  int32_t* touched; /* cluster ids with acc != 0 */
  int64_t* Wc;
  int64_t* size;
  i128* delta;
  i128* dadj;       /* delta after the afterburner adjustment */
  int32_t* D;
  uint8_t* cand;
  uint8_t* keep;
} scratch;

static void scratch_init(scratch* s, int64_t n) {
  s->acc = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  s->touched = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  s->Wc = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  s->size = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  s->delta = (i128*)xcalloc((size_t)n, sizeof(i128));
  s->dadj = (i128*)xcalloc((size_t)n, sizeof(i128));
  s->D = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  s->cand = (uint8_t*)xcalloc((size_t)n, 1);
  s->keep = (uint8_t*)xcalloc((size_t)n, 1);
}
static void scratch_free(scratch* s) {
  free(s->acc); free(s->touched); free(s->Wc); free(s->size);
  free(s->delta); free(s->dadj); free(s->D); free(s->cand); free(s->keep);
}

static void cluster_weights(const ograph* g, const int32_t* C, int64_t* Wc, int64_t* size) {
  memset(Wc, 0, (size_t)g->n * sizeof(int64_t));
  memset(size, 0, (size_t)g->n * sizeof(int64_t));
  for (int64_t v = 0; v < g->n; ++v) { Wc[C[v]] += g->vw[v]; size[C[v]] += 1; }
}

/* Destination of v (Alg. 2, the argmax and the empty-cluster rule).  Candidate destinations are the
 * clusters adjacent to v other than C[v] (under a constraint clustering B only through neighbours u with
 * B[u] = B[v]: the new Louvain+ iteration of Sec. IV-D); ties go to the lowest cluster id.  If v's own contribution is
 * negative and no adjacent cluster scores >= 0, D = EMPTY with score 0.  Returns 0 when v has no
 * destination at all.  Writes *S_cur and *S_D. */
static int destination(const ograph* g, i128 p, i128 q, const int32_t* C, scratch* s, int64_t v,
                       int32_t* D, i128* S_cur, i128* S_D) {
  int64_t nt = 0;
  for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j) {
    if (g->B && g->B[g->idx[j]] != g->B[v]) continue;
    int32_t c = C[g->idx[j]];
    if (s->acc[c] == 0) s->touched[nt++] = c;
    s->acc[c] += EW(g, j);
  }
  int64_t wv = g->vw[v];
  int32_t cv = C[v];
  i128 scur = q * s->acc[cv] - p * (i128)wv * (s->Wc[cv] - wv);
  int32_t best = ORC_NONE;
  i128 sbest = 0;
  for (int64_t k = 0; k < nt; ++k) {
    int32_t c = s->touched[k];
    if (c == cv) continue;
    i128 sc = q * s->acc[c] - p * (i128)wv * s->Wc[c];
    if (best == ORC_NONE || sc > sbest || (sc == sbest && c < best)) { best = c; sbest = sc; }
  }
  for (int64_t k = 0; k < nt; ++k) s->acc[s->touched[k]] = 0;
  *S_cur = scur;
  if (scur < 0 && (best == ORC_NONE || sbest < 0)) { *D = ORC_EMPTY; *S_D = 0; return 1; }
  if (best == ORC_NONE) { *D = ORC_NONE; *S_D = 0; return 0; }
  *D = best; *S_D = sbest;
  return 1;
}

/* Apply the kept moves simultaneously.  Movers to EMPTY take the ids left unused once every other move
 * is applied, in ascending order, handed out in ascending vertex order. */
static void apply_moves(const ograph* g, int32_t* C, const int32_t* D, const uint8_t* keep, int64_t* size) {
  int64_t n = g->n;
  memset(size, 0, (size_t)n * sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) {
    if (keep[v] && D[v] == ORC_EMPTY) continue;
    int32_t c = keep[v] ? D[v] : C[v];
    size[c] += 1;
  }
  int64_t next_free = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (!keep[v]) continue;
    if (D[v] == ORC_EMPTY) {
      while (size[next_free] != 0) ++next_free;
      C[v] = (int32_t)next_free++;
    } else {
      C[v] = D[v];
    }
  }
}

/* One pass of Alg. 2 from the snapshot C, with temperature phi = phi_num / phi_den, followed by the
 * symmetry breaking (the afterburner filter of Alg. 3, or an ablation of Table 2) and the update.  `pass` is
 * the 1-based pass number (the minimum label heuristic is active in odd passes).  Counts |L| and |M|. */
static void lm_pass(const ograph* g, i128 p, i128 q, uint32_t phi_num, uint32_t phi_den, uint32_t eps_num,
                    uint32_t eps_den, int symmetry, int pass, int32_t* C, scratch* s, int64_t* counts) {
  int64_t n = g->n;
  cluster_weights(g, C, s->Wc, s->size);
  int64_t nL = 0, nM = 0;
  for (int64_t v = 0; v < n; ++v) {
    i128 scur, sd;
    s->cand[v] = 0;
    s->keep[v] = 0;
    s->delta[v] = 0;
    s->dadj[v] = 0;
    if (!destination(g, p, q, C, s, v, &s->D[v], &scur, &sd)) continue;
    s->delta[v] = sd - scur;
    /* candidate test: w'(v, D) >= (1 - phi) w'(v, C[v]) */
    if ((i128)phi_den * sd >= (i128)(phi_den - phi_num) * scur) { s->cand[v] = 1; ++nL; }
  }
  if (symmetry != ORC_SYM_AFTERBURNER) {
    for (int64_t v = 0; v < n; ++v) {
      if (!s->cand[v]) continue;
      s->dadj[v] = s->delta[v];
      int ok = 1;
      if (symmetry == ORC_SYM_MLH && (pass & 1)) ok = s->D[v] == ORC_EMPTY || s->D[v] < C[v];
      if (ok) { s->keep[v] = 1; ++nM; }
    }
    apply_moves(g, C, s->D, s->keep, s->size);
    counts[0] = nL;
    counts[1] = nM;
    return;
  }
  /* Alg. 3: adjust delta_v by every adjacent candidate ordered before v */
  for (int64_t v = 0; v < n; ++v) {
    if (!s->cand[v]) continue;
    i128 d = s->delta[v];
    int32_t cv = C[v], dv = s->D[v];
    for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j) {
      int32_t u = g->idx[j];
      if (!s->cand[u] || !before(u, s->delta[u], v, s->delta[v], q, eps_num, eps_den)) continue;
      i128 wq = q * EW(g, j) - p * (i128)g->vw[u] * g->vw[v];
      int32_t cu = C[u], du = s->D[u];
      if (cv == cu) d += wq;
      else if (dv == cu) d -= wq;
      if (du != ORC_EMPTY && cv == du) d -= wq;
      else if (du != ORC_EMPTY && dv == du) d += wq;
    }
    s->dadj[v] = d;
    if (d >= 0) { s->keep[v] = 1; ++nM; }
  }
  apply_moves(g, C, s->D, s->keep, s->size);
  counts[0] = nL;
  counts[1] = nM;
}

void orc_lm_pass(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                 uint64_t p, uint64_t q, uint32_t phi_num, uint32_t phi_den, uint32_t eps_num,
                 uint32_t eps_den, int32_t symmetry, int32_t pass, int32_t* C, int32_t* D, int64_t* delta_hi,
                 uint64_t* delta_lo, int64_t* dadj_hi, uint64_t* dadj_lo, uint8_t* cand, uint8_t* keep,
                 int64_t* counts) {
  ograph g = {n, off, idx, ew, vw};
  scratch s;
  scratch_init(&s, n);
  lm_pass(&g, p, q, phi_num, phi_den, eps_num, eps_den, symmetry, pass, C, &s, counts);
  for (int64_t v = 0; v < n; ++v) {
    if (D) D[v] = s.D[v];
    if (delta_hi) delta_hi[v] = (int64_t)(s.delta[v] >> 64);
    if (delta_lo) delta_lo[v] = (uint64_t)s.delta[v];
    if (dadj_hi) dadj_hi[v] = (int64_t)(s.dadj[v] >> 64);
    if (dadj_lo) dadj_lo[v] = (uint64_t)s.dadj[v];
    if (cand) cand[v] = s.cand[v];
    if (keep) keep[v] = s.keep[v];
  }
  scratch_free(&s);
}

/* ---------------------------------------------------------------------------------------------------
 * Trace records: {kind, level, phase, pass, a, b, c, d}
 * ------------------------------------------------------------------------------------------------- */
enum { TR_LMPASS = 1, TR_LEVEL = 2, TR_LMALT = 3, TR_REFINE = 4 };
typedef struct { int64_t* buf; int64_t cap; int64_t count; } tracer;

static void trace_rec(tracer* t, int64_t kind, int64_t level, int64_t phase, int64_t pass, int64_t a,
                      int64_t b, int64_t c, int64_t d) {
  if (!t || !t->buf) return;
  if (t->count < t->cap) {
    int64_t* r = t->buf + 8 * t->count;
    r[0] = kind; r[1] = level; r[2] = phase; r[3] = pass; r[4] = a; r[5] = b; r[6] = c; r[7] = d;
  }
  t->count++;
}

static void phi_of_pass(const orc_opts* o, int pass, uint32_t* num, uint32_t* den) {
  for (int k = 0; k < o->n_phi; ++k)
    if ((uint32_t)pass <= o->phi_until[k]) { *num = o->phi_num[k]; *den = o->phi_den[k]; return; }
  *num = o->phi_num[o->n_phi - 1];
  *den = o->phi_den[o->n_phi - 1];
}

/* LocalMovePasses (Alg. 2): pass_limit passes from C; C_out keeps the best clustering seen (strict
 * improvement of the objective).  The next pass continues from C, not from C_out.  On return C holds
 * C_out; returns N(C_out). */
static i128 local_move(const ograph* g, i128 p, i128 q, const orc_opts* o, int32_t* C, tracer* tr,
                       int64_t level, int64_t phase) {
  int64_t n = g->n;
  scratch s;
  scratch_init(&s, n);
  int32_t* Cout = (int32_t*)xmalloc((size_t)n * sizeof(int32_t));
  memcpy(Cout, C, (size_t)n * sizeof(int32_t));
  i128 Nbest = objective(g, p, q, C);
  for (int i = 1; i <= o->pass_limit; ++i) {
    uint32_t pn, pd;
    phi_of_pass(o, i, &pn, &pd);
    int64_t counts[2];
    lm_pass(g, p, q, pn, pd, o->eps_num, o->eps_den, o->symmetry, i, C, &s, counts);
    i128 N = objective(g, p, q, C);
    trace_rec(tr, TR_LMPASS, level, phase, i, counts[0], counts[1], (int64_t)N, 0);
    if (N > Nbest) { Nbest = N; memcpy(Cout, C, (size_t)n * sizeof(int32_t)); }
  }
  memcpy(C, Cout, (size_t)n * sizeof(int32_t));
  free(Cout);
  scratch_free(&s);
  return Nbest;
}

void orc_local_move(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                    uint64_t p, uint64_t q, const orc_opts* opts, int32_t* C, int64_t* N_hi_lo) {
  ograph g = {n, off, idx, ew, vw};
  put128(local_move(&g, p, q, opts, C, NULL, 0, 0), N_hi_lo);
}

/* Ascending compaction of the labels in use: map[c] = rank of c among used ids.  Returns the count. */
static int64_t compact_labels(int64_t n, const int32_t* C, int32_t* map_of_id) {
  uint8_t* used = (uint8_t*)xcalloc((size_t)n, 1);
  for (int64_t v = 0; v < n; ++v) used[C[v]] = 1;
  int64_t k = 0;
  for (int64_t c = 0; c < n; ++c) map_of_id[c] = used[c] ? (int32_t)k++ : -1;
  free(used);
  return k;
}

/* ---------------------------------------------------------------------------------------------------
 * Graph contraction (Sec. III-A, Alg. 4): one coarse vertex per cluster with w(x) = w(C_x); an edge
 * (x, y) of weight w(C_x, C_y) whenever that is positive, in both directions; no self-loops.  The
 * internal ordered weight is kept in s(x) instead (objective offset), sq(x) = sum of w(v)^2 at level 0.
 * Canonical layout: rows by coarse id, neighbours ascending.
 * ------------------------------------------------------------------------------------------------- */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

int64_t orc_contract(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                     const int64_t* s_in, const int64_t* sq_in, const int32_t* map, int64_t nc,
                     int64_t* coff, int32_t* cidx, int32_t* cw, int64_t* cvw, int64_t* cs, int64_t* csq) {
  /* members of each coarse vertex, ascending fine id */
  int64_t* moff = (int64_t*)xcalloc((size_t)nc + 1, sizeof(int64_t));
  int64_t* mem = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) moff[map[v] + 1]++;
  for (int64_t x = 0; x < nc; ++x) moff[x + 1] += moff[x];
  int64_t* cur = (int64_t*)xcalloc((size_t)nc + 1, sizeof(int64_t));
  memcpy(cur, moff, (size_t)(nc + 1) * sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) mem[cur[map[v]]++] = v;
  free(cur);
  int64_t* acc = (int64_t*)xcalloc((size_t)nc, sizeof(int64_t));
  int32_t* touched = (int32_t*)xcalloc((size_t)nc, sizeof(int32_t));
  int64_t e = 0;
  coff[0] = 0;
  for (int64_t x = 0; x < nc; ++x) {
    int64_t nt = 0, wsum = 0, ssum = 0, sqsum = 0;
    for (int64_t k = moff[x]; k < moff[x + 1]; ++k) {
      int64_t v = mem[k];
      wsum += vw[v];
      ssum += s_in ? s_in[v] : 0;
      sqsum += sq_in ? sq_in[v] : vw[v] * vw[v];
      for (int64_t j = off[v]; j < off[v + 1]; ++j) {
        int32_t y = map[idx[j]];
        int64_t wt = ew ? ew[j] : 1;
        if (y == x) { ssum += wt; continue; }
        if (acc[y] == 0) touched[nt++] = y;
        acc[y] += wt;
      }
    }
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int64_t k = 0; k < nt; ++k) {
      cidx[e] = touched[k];
      cw[e] = (int32_t)acc[touched[k]];
      acc[touched[k]] = 0;
      ++e;
    }
    coff[x + 1] = e;
    cvw[x] = wsum;
    if (cs) cs[x] = ssum;
    if (csq) csq[x] = sqsum;
  }
  free(acc); free(touched); free(moff); free(mem);
  return e;
}

/* ---------------------------------------------------------------------------------------------------
 * pLeidenR (Alg. 6, Lemmas 1-2).
 *   U    = vertices with w'(u, B[u]) >= 0.
 *   A_v  = {v} plus neighbours u in U with B[u] = B[v] and w'(u, v) >= 0, taken in vertex-id order;
 *          H[v] = A_v[r], r = fmix64(s_t ^ 2v) mod |A_v|  (s_t = t-th splitmix64 output of the seed).
 *   f(v) = fmix32(v ^ (s_t >> 32)), injective, K = 2^32.
 *   Edges towards a higher-f vertex are dropped (v is then a root).  Roots without children (singleton
 *   trees) take f <- 2K - 1 - f (order-equivalent to the paper's 2K - f, kept within 33 bits) and their
 *   own edge is tested again with the new values.
 *   Each tree is sorted by f (root first); the longest prefix whose every vertex v_i passes
 *   w'(v_i, X_{i-1}) >= 0 and w'(X_{i-1}, B) >= 0 (X_{i-1} = earlier prefix) becomes one cluster
 *   labelled by the root id; every later vertex stays a singleton labelled by its own id.
 * ------------------------------------------------------------------------------------------------- */
typedef struct { uint64_t key; int32_t v; } tkey;
static int cmp_tkey(const void* a, const void* b) {
  uint64_t x = ((const tkey*)a)->key, y = ((const tkey*)b)->key;
  return (x > y) - (x < y);
}

static void refine(const ograph* g, i128 p, i128 q, const int32_t* B, uint64_t seed, uint64_t t,
                   int32_t* R, int32_t* parent_out, int32_t* root_out, int64_t* fkey_out, int64_t* counts) {
  int64_t n = g->n;
  uint64_t st = seed_stream(seed, t);
  uint32_t fseed = (uint32_t)(st >> 32);
  int64_t* WB = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) WB[B[v]] += g->vw[v];
  int64_t* aB = (int64_t*)xcalloc((size_t)n, sizeof(int64_t)); /* a(v, B[v] \ v) */
  uint8_t* inU = (uint8_t*)xcalloc((size_t)n, 1);
  int64_t nU = 0;
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j)
      if (B[g->idx[j]] == B[v]) aB[v] += EW(g, j);
    i128 sv = q * aB[v] - p * (i128)g->vw[v] * (WB[B[v]] - g->vw[v]);
    inU[v] = sv >= 0;
    nU += inU[v];
  }
  /* random candidate edge */
  int32_t* H = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  int32_t* list = (int32_t*)xcalloc((size_t)n + 1, sizeof(int32_t));
  for (int64_t v = 0; v < n; ++v) {
    H[v] = (int32_t)v;
    if (!inU[v]) continue;
    int64_t k = 0;
    int inserted = 0;
    for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j) {
      int32_t u = g->idx[j];
      if (!inserted && u > v) { list[k++] = (int32_t)v; inserted = 1; }
      if (!inU[u] || B[u] != B[v]) continue;
      if (q * EW(g, j) - p * (i128)g->vw[u] * g->vw[v] < 0) continue;
      list[k++] = u;
    }
    if (!inserted) list[k++] = (int32_t)v;
    uint64_t r = orc_fmix64(st ^ ((uint64_t)v << 1)) % (uint64_t)k;
    H[v] = list[r];
  }
  free(list);
  /* ordering and parents */
  int64_t* f = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) f[v] = orc_fmix32((uint32_t)v ^ fseed);
  int32_t* par = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  for (int64_t v = 0; v < n; ++v) par[v] = (H[v] != v && f[H[v]] < f[v]) ? H[v] : (int32_t)v;
  uint8_t* has_child = (uint8_t*)xcalloc((size_t)n, 1);
  for (int64_t v = 0; v < n; ++v) if (par[v] != v) has_child[par[v]] = 1;
  const int64_t K = (int64_t)1 << 32;
  uint8_t* flipped = (uint8_t*)xcalloc((size_t)n, 1);
  for (int64_t v = 0; v < n; ++v)
    if (par[v] == v && !has_child[v]) { flipped[v] = 1; f[v] = 2 * K - 1 - f[v]; }
  for (int64_t v = 0; v < n; ++v)
    if (flipped[v] && H[v] != v && f[H[v]] < f[v]) par[v] = H[v];
  free(has_child);
  /* roots by following parents */
  int32_t* root = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  for (int64_t v = 0; v < n; ++v) {
    int32_t x = (int32_t)v;
    while (par[x] != x) x = par[x];
    root[v] = x;
  }
  /* tree sizes; serialise non-trivial trees sorted by (root, f) */
  int64_t* tsz = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) tsz[root[v]]++;
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v) if (tsz[root[v]] > 1) ++m;
  tkey* ord = (tkey*)xcalloc((size_t)m, sizeof(tkey));
  m = 0;
  for (int64_t v = 0; v < n; ++v)
    if (tsz[root[v]] > 1) { ord[m].key = ((uint64_t)root[v] << 33) | (uint64_t)f[v]; ord[m].v = (int32_t)v; ++m; }
  qsort(ord, (size_t)m, sizeof(tkey), cmp_tkey);
  for (int64_t v = 0; v < n; ++v) R[v] = (int32_t)v;
  /* commit the longest well-connected prefix of each tree */
  int64_t i = 0;
  while (i < m) {
    int32_t r0 = root[ord[i].v];
    int64_t j = i;
    while (j < m && root[ord[j].v] == r0) ++j;
    int64_t wX = 0, cutX = 0; /* w(X_{k-1}) and w(X_{k-1}, B \ X_{k-1}) */
    int64_t WBr = WB[B[r0]];
    int64_t k;
    for (k = i; k < j; ++k) {
      int32_t v = ord[k].v;
      int64_t aX = 0; /* a(v, X_{k-1}): edges to earlier vertices of the same tree */
      for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
        int32_t u = g->idx[e];
        if (root[u] == r0 && f[u] < f[v]) aX += EW(g, e);
      }
      i128 c1 = q * aX - p * (i128)g->vw[v] * wX;
      i128 c2 = q * cutX - p * (i128)wX * (WBr - wX);
      if (c1 < 0 || c2 < 0) break;
      R[v] = r0;
      wX += g->vw[v];
      cutX += aB[v] - 2 * aX;
    }
    i = j;
  }
  if (parent_out) memcpy(parent_out, par, (size_t)n * sizeof(int32_t));
  if (root_out) memcpy(root_out, root, (size_t)n * sizeof(int32_t));
  if (fkey_out) memcpy(fkey_out, f, (size_t)n * sizeof(int64_t));
  if (counts) { counts[0] = nU; counts[1] = m; }
  free(ord); free(tsz); free(root); free(flipped); free(par); free(f); free(H); free(inU); free(aB); free(WB);
}

void orc_refine(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                uint64_t p, uint64_t q, const int32_t* B, uint64_t seed, uint64_t t, int32_t* R_out,
                int32_t* parent, int32_t* root, int64_t* fkey) {
  ograph g = {n, off, idx, ew, vw};
  refine(&g, p, q, B, seed, t, R_out, parent, root, fkey, NULL);
}

/* ---------------------------------------------------------------------------------------------------
 * LocalMoveAlt (Sec. V-A): every vertex that is not node optimal (its destination per Alg. 2 without the
 * temperature rule improves the objective), in ascending id, with its destination fixed up front.  The
 * moves are applied one after another to a copy; each one's exact objective change accounts for every
 * earlier move, adjacent or not.  The shortest prefix with the largest total change is committed; movers
 * to EMPTY take fresh ids as in the synchronous update.
 * ------------------------------------------------------------------------------------------------- */
static void lmalt(const ograph* g, i128 p, i128 q, int32_t* C, int64_t* counts) {
  int64_t n = g->n;
  scratch s;
  scratch_init(&s, n);
  cluster_weights(g, C, s.Wc, s.size);
  int64_t k = 0;
  int32_t* mv = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  int32_t* dst = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  for (int64_t v = 0; v < n; ++v) {
    int32_t D;
    i128 scur, sd;
    if (!destination(g, p, q, C, &s, v, &D, &scur, &sd)) continue;
    if (sd - scur > 0) { mv[k] = (int32_t)v; dst[k] = D; ++k; }
  }
  counts[0] = k;
  counts[1] = 0;
  if (k == 0) { free(mv); free(dst); scratch_free(&s); return; }
  /* sequential simulation on labels extended with fresh ids n, n+1, ... for EMPTY */
  int32_t* Cs = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  memcpy(Cs, C, (size_t)n * sizeof(int32_t));
  int64_t* Ws = (int64_t*)xcalloc((size_t)(n + k), sizeof(int64_t));
  memcpy(Ws, s.Wc, (size_t)n * sizeof(int64_t));
  i128 run = 0, best = 0;
  int64_t bestk = 0;
  for (int64_t i = 0; i < k; ++i) {
    int32_t v = mv[i];
    int64_t wv = g->vw[v];
    int32_t from = Cs[v];
    int32_t to = dst[i] == ORC_EMPTY ? (int32_t)(n + i) : dst[i];
    int64_t a_from = 0, a_to = 0;
    for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j) {
      int32_t c = Cs[g->idx[j]];
      if (c == from) a_from += EW(g, j);
      if (c == to) a_to += EW(g, j);
    }
    i128 s_from = q * a_from - p * (i128)wv * (Ws[from] - wv);
    i128 s_to = q * a_to - p * (i128)wv * Ws[to];
    run += 2 * (s_to - s_from);
    Ws[from] -= wv;
    Ws[to] += wv;
    Cs[v] = to;
    if (run > best) { best = run; bestk = i + 1; }
  }
  /* commit the prefix */
  memset(s.keep, 0, (size_t)n);
  for (int64_t i = 0; i < bestk; ++i) { s.keep[mv[i]] = 1; s.D[mv[i]] = dst[i]; }
  apply_moves(g, C, s.D, s.keep, s.size);
  counts[1] = bestk;
  free(Cs); free(Ws); free(mv); free(dst);
  scratch_free(&s);
}

void orc_lmalt(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
               uint64_t p, uint64_t q, int32_t* C, int64_t* counts) {
  ograph g = {n, off, idx, ew, vw};
  lmalt(&g, p, q, C, counts);
}

/* ---------------------------------------------------------------------------------------------------
 * Multilevel drivers
 * ------------------------------------------------------------------------------------------------- */
typedef struct {
  ograph g;
  int64_t *off, *vw; /* owned (NULL at level 0) */
  int32_t *idx, *ew;
  int32_t* map;      /* fine vertex -> coarse vertex of the next level */
  int32_t* C;        /* clustering of this level */
  int32_t* Bown;     /* constraint of the coarse vertices (owned, NULL at level 0 or unconstrained) */
} level_t;

static void level_free(level_t* L, int owned) {
  if (owned) { free(L->off); free(L->vw); free(L->idx); free(L->ew); free(L->Bown); }
  free(L->map);
  free(L->C);
}

static int64_t count_distinct(int64_t n, const int32_t* C) {
  uint8_t* used = (uint8_t*)xcalloc((size_t)n, 1);
  int64_t k = 0;
  for (int64_t v = 0; v < n; ++v) if (!used[C[v]]) { used[C[v]] = 1; ++k; }
  free(used);
  return k;
}

/* contract level l into level l+1 by the compact map of `labels` */
static void make_next_level(level_t* lv, int64_t l, const int32_t* labels, int64_t* nc_out) {
  level_t* L = &lv[l];
  int64_t n = L->g.n;
  int32_t* id_map = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  int64_t nc = compact_labels(n, labels, id_map);
  L->map = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
  for (int64_t v = 0; v < n; ++v) L->map[v] = id_map[labels[v]];
  free(id_map);
  level_t* N = &lv[l + 1];
  memset(N, 0, sizeof(*N));
  int64_t nnz = L->g.off[n];
  N->off = (int64_t*)xcalloc((size_t)nc + 1, sizeof(int64_t));
  N->idx = (int32_t*)xcalloc((size_t)nnz, sizeof(int32_t));
  N->ew = (int32_t*)xcalloc((size_t)nnz, sizeof(int32_t));
  N->vw = (int64_t*)xcalloc((size_t)nc, sizeof(int64_t));
  orc_contract(n, L->g.off, L->g.idx, L->g.ew, L->g.vw, NULL, NULL, L->map, nc, N->off, N->idx, N->ew,
               N->vw, NULL, NULL);
  N->g.n = nc; N->g.off = N->off; N->g.idx = N->idx; N->g.ew = N->ew; N->g.vw = N->vw;
  if (L->g.B) {  /* a coarse vertex lies inside one constraint cluster: it inherits that cluster */
    N->Bown = (int32_t*)xcalloc((size_t)nc, sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) N->Bown[L->map[v]] = L->g.B[v];
    N->g.B = N->Bown;
  }
  N->C = (int32_t*)xcalloc((size_t)nc, sizeof(int32_t));
  *nc_out = nc;
}

/* Alg. 1: Louvain (no uncoarsening) and Louvain+ (local move again after each projection).
 * init (optional): the level-0 local move starts from it instead of singletons (the iteration the Leiden
 * authors describe).  A constraint clustering lv[0].g.B (optional) confines the coarsening local moves to
 * clusters inside one constraint cluster; the uncoarsening local moves are free (the iteration of Sec. IV-D). */
static int run_louvain(level_t* lv, i128 p, i128 q, const orc_opts* o, int plus, const int32_t* init,
                       tracer* tr, int64_t* top, uint32_t* flags) {
  int64_t l = 0;
  for (;;) {
    level_t* L = &lv[l];
    int64_t n = L->g.n;
    for (int64_t v = 0; v < n; ++v) L->C[v] = (l == 0 && init) ? init[v] : (int32_t)v;
    i128 N = local_move(&L->g, p, q, o, L->C, tr, l, 0);
    int64_t nc = count_distinct(n, L->C);
    trace_rec(tr, TR_LEVEL, l, 0, 0, n, L->g.off[n], nc, (int64_t)N);
    if (nc == n) break;
    if (l + 1 >= o->max_levels) { *flags |= ORC_FLAG_LEVEL_CAP; break; }
    int64_t nc2;
    make_next_level(lv, l, L->C, &nc2);
    ++l;
  }
  *top = l;
  for (int64_t k = l - 1; k >= 0; --k) {
    level_t* L = &lv[k];
    for (int64_t v = 0; v < L->g.n; ++v) L->C[v] = lv[k + 1].C[L->map[v]];
    if (plus) {
      ograph free_g = L->g;
      free_g.B = NULL;
      i128 N = local_move(&free_g, p, q, o, L->C, tr, k, 1);
      trace_rec(tr, TR_LEVEL, k, 1, 0, L->g.n, L->g.off[L->g.n], count_distinct(L->g.n, L->C), (int64_t)N);
    }
  }
  return 0;
}

/* Alg. 5: pLeiden (and pLeiden+ with the uncoarsening local move).  When refinement leaves the level
 * unchanged three times in a row the loop stops with a flag (a guard the paper does not need to state). */
static int run_leiden(level_t* lv, i128 p, i128 q, const orc_opts* o, int plus, const int32_t* init,
                      tracer* tr, int64_t* top, uint32_t* flags) {
  int64_t l = 0;
  uint64_t t = 0;
  int noprog = 0;
  {
    level_t* L = &lv[0];
    for (int64_t v = 0; v < L->g.n; ++v) L->C[v] = init ? init[v] : (int32_t)v;
  }
  for (;;) {
    level_t* L = &lv[l];
    int64_t n = L->g.n;
    i128 N0 = objective(&L->g, p, q, L->C);
    i128 N = local_move(&L->g, p, q, o, L->C, tr, l, 0);
    if (N == N0) {
      int64_t cnt[2];
      lmalt(&L->g, p, q, L->C, cnt);
      N = objective(&L->g, p, q, L->C);
      trace_rec(tr, TR_LMALT, l, 0, 0, cnt[0], cnt[1], (int64_t)N, 0);
    }
    int64_t nc = count_distinct(n, L->C);
    trace_rec(tr, TR_LEVEL, l, 0, 0, n, L->g.off[n], nc, (int64_t)N);
    if (nc == n) break;
    if (l + 1 >= o->max_levels) { *flags |= ORC_FLAG_LEVEL_CAP; break; }
    int32_t* R = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
    int64_t rc[2];
    refine(&L->g, p, q, L->C, o->seed, t, R, NULL, NULL, NULL, rc);
    int64_t nR = count_distinct(n, R);
    trace_rec(tr, TR_REFINE, l, 0, 0, nR, (int64_t)t, rc[0], rc[1]);
    ++t;
    if (nR == n) {
      free(R);
      if (++noprog >= 3) { *flags |= ORC_FLAG_REFINE_NO_PROGRESS; break; }
      continue; /* same level again with the next refinement seed */
    }
    noprog = 0;
    int64_t nc2;
    make_next_level(lv, l, R, &nc2);
    free(R);
    /* Downsample: coarse vertex x inherits the (compacted) cluster of its members */
    int32_t* id_map = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
    compact_labels(n, L->C, id_map);
    for (int64_t v = 0; v < n; ++v) lv[l + 1].C[L->map[v]] = id_map[L->C[v]];
    free(id_map);
    ++l;
  }
  *top = l;
  for (int64_t k = l - 1; k >= 0; --k) {
    level_t* L = &lv[k];
    for (int64_t v = 0; v < L->g.n; ++v) L->C[v] = lv[k + 1].C[L->map[v]];
    if (plus) {
      i128 N = local_move(&L->g, p, q, o, L->C, tr, k, 1);
      trace_rec(tr, TR_LEVEL, k, 1, 0, L->g.n, L->g.off[L->g.n], count_distinct(L->g.n, L->C), (int64_t)N);
    }
  }
  return 0;
}

static void default_opts(orc_opts* o) {
  memset(o, 0, sizeof(*o));
  o->pass_limit = 6;
  o->n_phi = 2;
  o->phi_num[0] = 3; o->phi_den[0] = 4; o->phi_until[0] = 4;
  o->phi_num[1] = 1; o->phi_den[1] = 4; o->phi_until[1] = 6;
  o->eps_num = 1; o->eps_den = 10;
  o->seed = 1;
  o->max_levels = 64;
}

int orc_cluster(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
                int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int variant,
                const orc_opts* opts, int32_t* labels_out, int64_t* result, int64_t* trace,
                int64_t trace_cap, int64_t* trace_count) {
  return orc_cluster_ex(n, off, idx, ew, vw_in, vw_mode, lam_num, lam_den, lam_over_total, variant, opts, NULL,
                        NULL, labels_out, result, trace, trace_cap, trace_count);
}

int orc_cluster_ex(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
                   int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int variant,
                   const orc_opts* opts, const int32_t* init, const int32_t* constraint, int32_t* labels_out,
                   int64_t* result, int64_t* trace, int64_t trace_cap, int64_t* trace_count) {
  orc_opts o;
  if (opts) o = *opts; else default_opts(&o);
  if (o.max_levels <= 0 || o.max_levels > 1024 || o.pass_limit < 0 || o.n_phi < 1 || o.n_phi > 8 ||
      o.eps_den == 0 || o.symmetry < ORC_SYM_AFTERBURNER || o.symmetry > ORC_SYM_MLH)
    return ORC_ERR_INVALID;
  for (int k = 0; k < o.n_phi; ++k)
    if (o.phi_den[k] == 0 || o.phi_num[k] > o.phi_den[k]) return ORC_ERR_INVALID;
  if (variant < ORC_LOUVAIN || variant > ORC_PLEIDEN_PLUS) return ORC_ERR_INVALID;
  if (constraint && (init || variant == ORC_PLEIDEN || variant == ORC_PLEIDEN_PLUS)) return ORC_ERR_INVALID;
  int64_t* vw = (int64_t*)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  uint64_t pq[2];
  int st = orc_setup(n, off, idx, ew, vw_in, vw_mode, lam_num, lam_den, lam_over_total, vw, pq);
  if (st != ORC_OK) { free(vw); return st; }
  if (init)
    for (int64_t v = 0; v < n; ++v)
      if (init[v] < 0 || init[v] >= n) { free(vw); return ORC_ERR_INVALID; }
  i128 p = pq[0], q = pq[1];
  tracer tr = {trace, trace_cap, 0};
  level_t* lv = (level_t*)xcalloc((size_t)o.max_levels + 1, sizeof(level_t));
  lv[0].g.n = n; lv[0].g.off = off; lv[0].g.idx = idx; lv[0].g.ew = ew; lv[0].g.vw = vw; lv[0].g.B = constraint;
  lv[0].C = (int32_t*)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int64_t top = 0;
  uint32_t flags = 0;
  if (n > 0) {
    if (variant == ORC_LOUVAIN || variant == ORC_PLOUVAIN)
      run_louvain(lv, p, q, &o, variant == ORC_PLOUVAIN, init, &tr, &top, &flags);
    else
      run_leiden(lv, p, q, &o, variant == ORC_PLEIDEN_PLUS, init, &tr, &top, &flags);
  }
  int32_t* id_map = (int32_t*)xcalloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int64_t nc = n > 0 ? compact_labels(n, lv[0].C, id_map) : 0;
  for (int64_t v = 0; v < n; ++v) labels_out[v] = id_map[lv[0].C[v]];
  i128 N = n > 0 ? objective(&lv[0].g, p, q, labels_out) : 0;
  free(id_map);
  for (int64_t l = 0; l <= top; ++l) level_free(&lv[l], l > 0);
  free(lv);
  free(vw);
  result[0] = nc;
  result[1] = (int64_t)(N >> 64);
  result[2] = (int64_t)(uint64_t)N;
  result[3] = top + 1;
  result[4] = flags;
  result[5] = (int64_t)q;
  result[6] = (int64_t)p;
  if (trace_count) *trace_count = tr.count;
  return ORC_OK;
}
