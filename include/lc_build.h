/*
 * liblc_build — host-side construction of a Link & Code index in the layout
 * that include/lc.h binds (codes, adj0, up_base/adj_up, beta, beta_idx).
 *
 * Paper: Douze, Sablayrolles, Jegou, "Link and code: Fast indexing with graphs
 * and compact regression codes", CVPR 2018 (arXiv 1804.09996).
 *
 * All pointers are HOST pointers owned by the caller; outputs are written in
 * place.  Functions return 0 on success, a negative value on invalid
 * arguments (-1) or allocation failure (-2).  `nthreads` worker threads are
 * used; every result is independent of the thread count.  Random draws
 * (k-means seeds, level uniforms, training subsets) are inputs.
 */
#ifndef LC_BUILD_H
#define LC_BUILD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Product quantizer (Sec. 3.3; Sec. 4.1 "Vector approximation"): per
 * sub-space k-means with 256 centroids on the (projected) training vectors,
 * seeded with the rows init[s][0..255], `iters` Lloyd iterations; an empty
 * cluster is re-seeded with the point of largest error.
 * centroids: f32 [m][256][d_pad/m]. */
int lcb_pq_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int m,
                 const int64_t *init, int iters, int nthreads, float *centroids);

/* PQ codes (nearest centroid per sub-space, lowest index on ties):
 * codes u8 [n][code_stride]. */
int lcb_pq_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                  const float *centroids, int nthreads, uint8_t *codes, int code_stride);

/* 2-level residual codec (Sec. 3.3 residual codecs; Sec. 5.1 two-level
 * encodings): a first-level product quantizer over the two halves of the
 * (projected) vector, k centroids each (k <= 65536; PQ2 x log2 k), whose
 * residual the PQ of lcb_pq_train / lcb_pq_encode then encodes (called with
 * proj NULL and d = d_pad on the residuals).
 * lcb_coarse_train: per-half k-means seeded by init [2][k] -> cent f32 [2][k][d_pad/2].
 * lcb_coarse_encode: nearest centroid per half (lowest index on ties) ->
 * codes u16 [n][2], and the residuals P x - c -> resid f32 [n][d_pad].
 * lcb_coarse_decode: the reconstructions q(x) = c + r -> rec f32 [n][d_pad]
 * (either output may be NULL), and the per-node term of the decomposed
 * asymmetric distance, ||c + r||^2 - ||c||^2 -> norm f32 [n].
 * The graph build and the regression codebook take rec (their last argument)
 * in place of the PQ decoding; NULL there means the one-level codec. */
int lcb_coarse_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int k,
                     const int64_t *init, int iters, int nthreads, float *cent);
int lcb_coarse_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int k,
                      const float *cent, int nthreads, uint16_t *codes, float *resid);
int lcb_coarse_decode(int64_t n, int d_pad, int m, const float *centroids, const uint8_t *codes,
                      int code_stride, int k, const float *cent, const uint16_t *ccodes, int nthreads,
                      float *rec, float *norm);

/* Node levels (Sec. 2 geometric layers, Sec. 4.1 ratio between levels):
 * level_i = min(cap, floor(-ln(u_i) / ln(ratio))).  Returns sum_i level_i,
 * the number of upper-level rows. */
int64_t lcb_levels(const double *u, int64_t n, int ratio, int cap, int8_t *level);

/* Nested graph over the coded vectors (Sec. 2; Sec. 4.1 "Graph-based
 * structure"; Sec. 5.1): nodes are inserted by level (descending) then id, in
 * batches of clamp(inserted / 16, 1, 4096) searched against the graph as it
 * stood before the batch, with asymmetric distances from the raw vector; the
 * links of a node are chosen by the shrinking heuristic and filled up to the
 * degree with the nearest rejected candidates; reverse links re-shrink a full
 * list from its owner's raw vector.  Level-0 lists are sorted by increasing
 * distance to their owner (Sec. 4.2).  Outputs: adj0 i32 [n][deg0], up_base
 * i32 [n], adj_up i32 [rows][deg_up], *entry, *max_level. */
int lcb_graph_build(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                    const float *centroids, const uint8_t *codes, int code_stride,
                    const int8_t *level, int deg0, int deg_up, int ef_construction, int nthreads,
                    int32_t *adj0, int32_t *up_base, int32_t *adj_up, int32_t *entry,
                    int32_t *max_level, const float *rec);

/* lcb_graph_build with upper_only = 1: the same batches, stopped before the
 * first batch that starts with a level-0 node (every later node is then a
 * level-0 node, so the rest of the build only searches and links level 0:
 * lc_graph_insert on the GPU continues it from *next_pos, the position in the
 * insertion order where it stopped, with the same batch sizes).  upper_only = 0
 * is lcb_graph_build; *next_pos (if given) is then n. */
int lcb_graph_build_part(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                         const float *centroids, const uint8_t *codes, int code_stride,
                         const int8_t *level, int deg0, int deg_up, int ef_construction, int nthreads,
                         int32_t *adj0, int32_t *up_base, int32_t *adj_up, int32_t *entry,
                         int32_t *max_level, const float *rec, int upper_only, int64_t *next_pos);

/* Regression codebook (Sec. 4.3, Eq. 6-8) in float64 on the training ids:
 * per-vector least squares initialises a k-means (km_iters), then em_iters
 * rounds of assignment (Eq. 7) and per-cluster least squares (Eq. 8).  With
 * m_beta > 1 (m_beta divides m) one codebook per block of d_pad / m_beta
 * coordinates, each trained on its block alone from the same seeds (the
 * product codebook, Eq. 9).
 * beta: f32 [m_beta][n_beta][k_reg+1]; loss_hist (optional)
 * [m_beta][em_iters+1] values. */
int lcb_beta_train(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj,
                   int d_pad, int m, const float *centroids, const uint8_t *codes, int code_stride,
                   const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta, const int64_t *init,
                   int km_iters, int em_iters, int nthreads, float *beta, double *loss_hist,
                   const float *rec);

/* Codebook entry of every vector and block (Sec. 4.3, Eq. 7 per block) with
 * the f32 codebooks: beta_idx u8 [n][m_beta]. */
int lcb_beta_assign(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                    const float *centroids, const uint8_t *codes, int code_stride,
                    const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta, const float *beta,
                    int nthreads, uint8_t *beta_idx, const float *rec);

/* Learned rotation ahead of the product quantizer (OPQ: the codec of Sec. 4.1
 * and Sec. 5.1 rotates the vectors before PQ).  Starting from init_proj
 * [d_pad][d] (orthonormal columns; NULL = identity, d_pad == d only), repeat
 * opq_iters times: project the training vectors, train the PQ (km_iters Lloyd
 * iterations, seeded by init [m][256] the first time, warm after), and replace
 * the rotation by the P with orthonormal columns minimising
 * sum_i ||P x_i - q(P x_i)||^2 for those reconstructions (orthogonal
 * Procrustes: P = S^T (S S^T)^(-1/2), S = X^T Yhat).  proj_out [d_pad][d];
 * mse_hist (optional) opq_iters+1 values of the mean distortion, the last for
 * the returned rotation's PQ.  Independent of nthreads.  Returns 0, -1 on bad
 * arguments, 2 if a rotation step meets a rank-deficient S. */
int lcb_opq_train(const float *train, int64_t n, int d, int d_pad, int m, const float *init_proj,
                  const int64_t *init, int opq_iters, int km_iters, int nthreads, float *proj_out,
                  double *mse_hist);

/* The Procrustes step alone: P [D][d] from S [d][D] (0, or 1 if S is rank
 * deficient). */
int lcb_procrustes(const double *S, int d, int D, double *P);

#ifdef __cplusplus
}
#endif
#endif
