/*
 * CPU oracle for synchronous multilevel LambdaCC clustering (pLouvain / Louvain+ and pLeiden).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded reference the GPU library is
 * checked against.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the GPU library.
 *
 * All arithmetic is exact: integer weights, 128-bit products and comparisons.
 */
#ifndef LCC_ORACLE_H
#define LCC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LOUVAIN = 0, ORC_PLOUVAIN = 1, ORC_PLEIDEN = 2, ORC_PLEIDEN_PLUS = 3 };
enum { ORC_VW_GIVEN = 0, ORC_VW_WEIGHTED_DEGREE = 1, ORC_VW_UNIT = 2 };
enum { ORC_OK = 0, ORC_ERR_INVALID = -1, ORC_ERR_NOT_SYMMETRIC = -2, ORC_ERR_SELF_LOOP = -3,
       ORC_ERR_UNSORTED = -4, ORC_ERR_WEIGHT = -5, ORC_ERR_LAMBDA = -6, ORC_ERR_OVERFLOW = -7,
       ORC_ERR_OOM = -8 };
enum { ORC_FLAG_LEVEL_CAP = 1, ORC_FLAG_REFINE_NO_PROGRESS = 2 };
#define ORC_EMPTY (-2) /* destination "new singleton cluster" */
#define ORC_NONE (-1)  /* no destination */

typedef struct {
  int32_t pass_limit;                                 /* 6 */
  int32_t n_phi;                                      /* phases of the temperature schedule */
  uint32_t phi_num[8], phi_den[8], phi_until[8];      /* phase k covers passes <= phi_until[k] */
  uint32_t eps_num, eps_den;                          /* afterburner tie window, 1/10 */
  uint64_t seed;                                      /* refinement randomness */
  int32_t max_levels;                                 /* 64 */
  int32_t symmetry;                                   /* ORC_SYM_*: afterburner (default) or an ablation */
} orc_opts;

/* Symmetry breaking of the local move (Sec. IV-A; the ablations of Table 2):
 *   ORC_SYM_AFTERBURNER  Alg. 3
 *   ORC_SYM_NONE         every candidate moves
 *   ORC_SYM_MLH          minimum label heuristic in odd passes (a candidate moves only to a cluster of lower
 *                        id than its own, or to a new singleton), every candidate moves in even passes */
enum { ORC_SYM_AFTERBURNER = 0, ORC_SYM_NONE = 1, ORC_SYM_MLH = 2 };

/* Full clustering: setup (validation, vertex weights, lambda = p/q), then the chosen variant.
 * labels_out[n]: compact labels 0..c-1.  result[0..5] = {num_clusters, N_hi, N_lo (objective numerator,
 * lambdaCC = N / q, as int128), levels, flags, q}.  result[6] = p.
 * trace: records of 8 int64 {kind, level, phase, pass, a, b, c, d}; may be NULL. */
int orc_cluster(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
                int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int variant,
                const orc_opts* opts, int32_t* labels_out, int64_t* result, int64_t* trace,
                int64_t trace_cap, int64_t* trace_count);

/* As orc_cluster, with the iteration inputs (Sec. II-B, Sec. IV-D), each optional:
 *   init        n labels in [0, n): pLeiden / pLeiden+ start from this clustering (Alg. 5's C_in); Louvain /
 *               Louvain+ start the level-0 local move from it instead of singletons
 *   constraint  n labels (any int32): Louvain / Louvain+ only, and not together with init; the coarsening
 *               local moves may only join clusters whose members share the vertex's constraint label, the
 *               uncoarsening local moves are free */
int orc_cluster_ex(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
                   int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int variant,
                   const orc_opts* opts, const int32_t* init, const int32_t* constraint, int32_t* labels_out,
                   int64_t* result, int64_t* trace, int64_t trace_cap, int64_t* trace_count);

/* Setup only: validate, derive vertex weights into vw_out[n], lambda into pq[2] (reduced). */
int orc_setup(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw_in,
              int vw_mode, uint64_t lam_num, uint64_t lam_den, int lam_over_total, int64_t* vw_out,
              uint64_t* pq);

/* Phase functions on a level graph with resolved vertex weights vw and lambda p/q.  Labels in [0, n). */
void orc_objective(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                   uint64_t p, uint64_t q, const int32_t* C, int64_t* N_hi_lo);

/* One synchronous local-move pass from C (updated in place).  Outputs per vertex: D (cluster id, ORC_EMPTY
 * or ORC_NONE), delta and afterburner-adjusted delta (hi/lo of int128), cand flag, keep flag.
 * counts[0] = |L|, counts[1] = |M|.  Any output pointer may be NULL. */
void orc_lm_pass(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                 uint64_t p, uint64_t q, uint32_t phi_num, uint32_t phi_den, uint32_t eps_num,
                 uint32_t eps_den, int32_t symmetry, int32_t pass, int32_t* C, int32_t* D, int64_t* delta_hi,
                 uint64_t* delta_lo, int64_t* dadj_hi, uint64_t* dadj_lo, uint8_t* cand, uint8_t* keep,
                 int64_t* counts);

/* LocalMovePasses from C (in place: C becomes C_out).  Returns the objective of C_out in N_hi_lo. */
void orc_local_move(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                    uint64_t p, uint64_t q, const orc_opts* opts, int32_t* C, int64_t* N_hi_lo);

/* Contraction by a compact map (values in [0, nc)).  Output arrays sized by the caller: coff[nc+1],
 * cidx/cw[nnz], cvw[nc], cs[nc] (internal ordered weight incl. the fine s), csq[nc].  s_in/sq_in may be
 * NULL (level 0: s = 0, sq = w^2).  Returns the coarse nnz. */
int64_t orc_contract(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                     const int64_t* s_in, const int64_t* sq_in, const int32_t* map, int64_t nc,
                     int64_t* coff, int32_t* cidx, int32_t* cw, int64_t* cvw, int64_t* cs, int64_t* csq);

/* pLeidenR with constraint B and refinement call index t.  R_out[n]: refined labels (root id or own id).
 * Debug outputs (may be NULL): parent[n], root[n], fkey[n] (the final 33-bit ordering value). */
void orc_refine(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
                uint64_t p, uint64_t q, const int32_t* B, uint64_t seed, uint64_t t, int32_t* R_out,
                int32_t* parent, int32_t* root, int64_t* fkey);

/* LocalMoveAlt from C (in place).  counts[0] = non-node-optimal vertices, counts[1] = committed prefix. */
void orc_lmalt(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* ew, const int64_t* vw,
               uint64_t p, uint64_t q, int32_t* C, int64_t* counts);

uint64_t orc_fmix64(uint64_t x);
uint32_t orc_fmix32(uint32_t x);

#ifdef __cplusplus
}
#endif
#endif
