/*
 * Link & Code reference oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of what the Link & Code search path
 * computes, and of the index build that produces its inputs.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header or table with the GPU library.
 *
 * Paper: Douze, Sablayrolles, Jegou, "Link and code: Fast indexing with
 * graphs and compact regression codes", CVPR 2018 (arXiv 1804.09996).
 *
 * Index layout written by the builder (all arrays owned by the caller):
 *   codes   [n][code_stride] u8      PQ code of every vector (Sec. 4.1)
 *   adj0    [n][deg0] i32            level-0 links, -1 padded, each list sorted
 *                                    by (||x_i - q(x_j)||^2, j) ascending
 *                                    (Sec. 4.2: ordered by increasing distance)
 *   level   [n] i8                   node level (Sec. 2, Sec. 4.1)
 *   up_base [n] i32                  first upper row of node i, -1 if level 0;
 *                                    the row of level l >= 1 is up_base[i]+l-1
 *   adj_up  [rows][deg_up] i32       upper-level links, -1 padded
 *   beta    [m_beta][n_beta][k+1] f32  regression codebook (Sec. 4.3), one per
 *                                    block of d_pad / m_beta coordinates (the
 *                                    product codebook of Eq. 9; m_beta = 1 is
 *                                    the single codebook of Eq. 5-8)
 *   beta_idx[n][m_beta] u8           selected entry per vector and block
 *   coarse  (optional)               2-level codec (Sec. 5.1): first-level
 *                                    centroids [2][k][d_pad/2] f32 and codes
 *                                    [n][2] u16; the PQ codes then encode the
 *                                    residual
 *
 * Parity: unpinned functions are marked "parity unpinned" below; every other
 * function is pinned by a CPU test against a closed form, brute force or a
 * library routine.
 */
#ifndef LC_ORACLE_H
#define LC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* First level of the 2-level residual codec (Sec. 3.3 / Sec. 5.1): a product
 * quantizer over the two halves of the (projected) vector, k centroids each;
 * the PQ codes then encode the residual, so that
 * q(x) = [C1[0][c0(x)], C1[1][c1(x)]] + PQ(residual).  k = 0: one-level codec. */
typedef struct {
  int32_t k;
  const float *cent;     /* [2][k][d_pad/2] */
  const uint16_t *codes; /* [n][2] */
} orc_coarse;

typedef struct {
  int32_t n, d, d_pad, m, ksub, code_stride;
  int32_t deg0, deg_up, k_reg, n_beta;
  int32_t entry, max_level;
  int32_t m_beta; /* regression-codebook blocks, divides m */
  const float *proj;       /* [d_pad][d] or NULL when d_pad == d */
  const float *centroids;  /* [m][ksub][dsub] */
  const uint8_t *codes;
  const int32_t *adj0;
  const int32_t *up_base;
  const int32_t *adj_up;
  const float *beta;
  const uint8_t *beta_idx;
  orc_coarse coarse; /* k = 0: one-level codec */
} orc_index;

/* k-means (Lloyd) in float64, used for PQ (Sec. 3.3) and for initialising the
 * regression codebook (Sec. 4.3).  init[c] picks the seed rows.  sse_hist
 * receives iters+1 values: the SSE after each assignment step. */
int orc_kmeans(const double *x, int64_t n, int dim, int k, const int64_t *init, int iters,
               int nthreads, double *cent, int32_t *assign, double *sse_hist);

/* y' = P y in float64 (or a copy when proj is NULL). */
void orc_project(const float *proj, int d_pad, int d, const float *y, double *out);

/* PQ training on (projected) training vectors; centroids rounded to f32. */
int orc_pq_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int m,
                 int ksub, const int64_t *init /*[m][ksub]*/, int iters, int nthreads,
                 float *cent /*[m][ksub][dsub]*/, double *sse_hist /*[m][iters+1] or NULL*/);

/* PQ encoding: per-subspace argmin in float64, lowest index on ties. */
int orc_pq_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                  int ksub, const float *cent, int nthreads, uint8_t *codes, int code_stride);

/* level_i = min(cap, floor(-ln(U_i) / ln(ratio))).  Returns the row count
 * sum_i level_i needed for adj_up. */
int64_t orc_levels(const double *u, int64_t n, int ratio, int cap, int8_t *level);

/* Batched nested-graph build over PQ-coded vectors (Sec. 2, Sec. 4.1, Sec. 5.1).
 * Fills adj0, up_base, adj_up, *entry, *max_level.  Pinned through the build
 * trace below: every candidate list equals an independent best-first search
 * of the graph as it stood at the start of its batch, every selection meets
 * the shrinking rule's defining properties checked pair by pair, every
 * reverse-link merge covers the old list plus its new links and is ordered by
 * the distance from the owner's own vector, and replaying the trace gives the
 * final lists. */
int orc_hnsw_build(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                   int ksub, const float *cent, const uint8_t *codes, int code_stride,
                   const int8_t *level, int deg0, int deg_up, int ef_construction, int nthreads,
                   int32_t *adj0, int32_t *up_base, int32_t *adj_up, int32_t *entry,
                   int32_t *max_level, const orc_coarse *cq /* NULL: one-level codec */);

/* Build trace (test infrastructure): while buf is set, orc_hnsw_build
 * appends one record per list update, in execution order (sequential with one
 * thread):
 *   [kind, level, owner, nc, nout, cand[nc], out[nout], by_test[nout]]
 * kind 0: selection of a new node's list at a level (cand = its search
 *         result W, sorted by (distance, id));
 * kind 1: a reverse-link merge that overflowed the list and re-ran the
 *         selection from the owner's vector (cand = old list, then new links);
 * kind 2: a reverse-link merge that fit (out = cand sorted by distance);
 * kind 3: start of a batch (owner = batch size, cand = the batch's nodes).
 * by_test[i] = 1 when out[i] was kept by the shrinking test, 0 when it
 * filled a free slot.  orc_build_trace(NULL, 0) stops recording;
 * orc_build_trace_used() is the words written, or -1 once cap overflowed. */
void orc_build_trace(int32_t *buf, int64_t cap);
int64_t orc_build_trace_used(void);

/* Least squares (Sec. 4.2, Eq. 4): beta minimising ||x - G beta||^2 given
 * A = G^T G and c = G^T x; Cholesky, else eigen pseudo-inverse. */
int orc_lsq_solve(const double *a, const double *c, int p, double *beta);

/* Regression-codebook training (Sec. 4.3, Eq. 6-8), one codebook per block of
 * d_pad / m_beta coordinates (Eq. 9; m_beta divides m).  beta receives
 * [m_beta][n_beta][k+1]; loss_hist [m_beta][em_iters+1] values of L'(B) after
 * each assignment step. */
int orc_beta_train(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj,
                   int d_pad, int m, int ksub, const float *cent, const uint8_t *codes,
                   int code_stride, const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta,
                   const int64_t *init, int km_iters, int em_iters, int nthreads, float *beta,
                   double *loss_hist, const orc_coarse *cq);

/* Shared 0-byte regression weights (Sec. 4.2, Eq. 3-5) over the given ids. */
int orc_beta_shared(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj,
                    int d_pad, int m, int ksub, const float *cent, const uint8_t *codes,
                    int code_stride, const int32_t *adj0, int deg0, int k_reg, double *beta,
                    const orc_coarse *cq);

/* Assignment (Sec. 4.3, Eq. 7) with the stored f32 codebook, lowest index on
 * ties, block by block; beta_idx receives [n][m_beta]. */
int orc_beta_assign(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                    int ksub, const float *cent, const uint8_t *codes, int code_stride,
                    const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta, const float *beta,
                    int nthreads, uint8_t *beta_idx, const orc_coarse *cq);

/* 2-level residual codec (Sec. 3.3 "residual" codecs; Sec. 5.1 "two-level
 * encodings"): the first level is trained with orc_pq_train(m = 2, ksub = k).
 * Encoding: per half, the nearest first-level centroid in float64 (lowest index
 * on ties) into codes [n][2], and, when resid is not NULL, the residual
 * P x - c rounded to f32 into resid [n][d_pad], which the second-level PQ
 * (orc_pq_train / orc_pq_encode with proj NULL, d = d_pad) trains on and encodes. */
int orc_coarse_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int k,
                      const float *cent, int nthreads, uint16_t *codes, float *resid);

/* Per-node term of the 2-level asymmetric distance: with c the first-level and
 * r the second-level reconstruction, ||y - c - r||^2 = ||y - c||^2
 * - 2 <y, r> + (||c + r||^2 - ||c||^2); norm[i] receives the last term, in
 * float64 rounded to f32. */
int orc_coarse_norms(const orc_index *ix, float *norm /*[n]*/);

/* Per-query ADC table LUT[s][c] = ||y'^s - C[s][c]||^2 in float64.  For a
 * 2-level codec the oracle takes the asymmetric distance by its definition,
 * ||y' - q(x)||^2, and the "table" is y' itself (its first d_pad entries). */
void orc_lut(const orc_index *ix, const float *y, double *lut /*[m][ksub]*/);

/* Full search (Sec. 2 and Sec. 4.1): greedy descent on the upper levels,
 * best-first walk on level 0 with W bounded by ef_eff = max(ef_q, S), the
 * S-entry short-list, regression refinement (Eq. 5 / Eq. 7) and top-K by
 * (distance, id).  Outputs may be NULL when not wanted. */
int orc_search(const orc_index *ix, const float *q, int64_t nq, const int32_t *ef, int32_t S,
               int32_t K, int nthreads, int32_t *out_ids, double *out_d, int32_t *cand_ids,
               double *cand_adc, int32_t *cand_n, int32_t *stats);

/* The same with the paper's budget T on distance computations (Sec. 3.1):
 * max_d > 0 stops a query's level-0 walk right after its max_d-th distance
 * evaluation (D = min(max_d, D of the unbounded walk)); 0 = no budget. */
int orc_search_capped(const orc_index *ix, const float *q, int64_t nq, const int32_t *ef, int32_t S,
                      int32_t K, int32_t max_d, int nthreads, int32_t *out_ids, double *out_d,
                      int32_t *cand_ids, double *cand_adc, int32_t *cand_n, int32_t *stats);

/* The search's first stage (Sec. 2: greedy descent on the upper levels, then
 * the best-first walk on level 0 with W bounded by ef_eff = max(ef_q, S),
 * and the S-entry short-list) with the caller's ADC tables in place of
 * orc_lut's: tables double [nq][m][ksub], a node's key being the sum of its
 * codes' entries.  One-level codec only (-1 for a 2-level index); outputs as
 * orc_search's first-stage outputs. */
int orc_walk_tables(const orc_index *ix, const double *tables, int64_t nq, const int32_t *ef, int32_t S,
                    int nthreads, int32_t *cand_ids, double *cand_adc, int32_t *cand_n, int32_t *stats);

/* Refined squared distance ||y' - x~_i||^2 for any id, x~_i = sum_j beta_j q(g_j(i))
 * block by block (Eq. 5, Eq. 9). */
double orc_refined_distance(const orc_index *ix, const float *y, int32_t i);

/* Sequence of expanded ids of one query's level-0 walk (for trace diffs).
 * Returns the number written (<= cap). */
int32_t orc_walk_trace(const orc_index *ix, const float *y, int32_t ef_eff, int32_t *trace,
                       int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
