/*
 * liblc — Link & Code search on AMD Instinct MI355X (gfx950).
 *
 * Paper: M. Douze, A. Sablayrolles, H. Jegou, "Link and code: Fast indexing
 * with graphs and compact regression codes", CVPR 2018 (arXiv 1804.09996).
 *
 * The search path has three calls, each one or more HIP kernels on the
 * caller's stream:
 *   lc_build_lut  per-query product-quantizer distance tables (Sec. 4.1,
 *                 asymmetric distance computation).
 *   lc_search     greedy descent on the upper graph levels, then a
 *                 best-first walk on level 0 whose nodes hold only PQ codes
 *                 (Sec. 2; Sec. 4.1 "Graph-based structure"); returns the
 *                 short-list of the first stage (Sec. 4.1 "Refinement
 *                 strategy").
 *   lc_refine     re-ranks the short-list with the regression refinement
 *                 x~ = sum_j beta_j q(g_j(x)) (Sec. 4.2 Eq. 5 with a beta taken
 *                 from the learned codebook of Sec. 4.3, Eq. 7, or one beta per
 *                 block of coordinates from the product codebook, Eq. 9) and
 *                 keeps the top K by (squared L2 distance, id).
 *
 * Conventions (all calls):
 *  - Distances are squared Euclidean (Sec. 2 works with d = l2).
 *  - Ids are int32; -1 marks "no entry".  Keys are ordered by (distance, id).
 *  - Every data pointer is a DEVICE pointer owned by the caller; the library
 *    never allocates, frees or copies device memory and never synchronises
 *    the stream.  `stream` is a hipStream_t (NULL = the null stream).
 *  - Arguments are validated on the host before anything is launched; a
 *    failed check returns LC_EINVAL / LC_ENOTSUP / LC_ENOSPC and launches
 *    nothing.  A launch error returns LC_EHIP; faults inside a kernel surface
 *    at the caller's next synchronisation.
 *  - The bound index is immutable, so calls on different streams may run
 *    concurrently (each with its own workspace).
 *  - Results do not depend on nq, on the batch a query is in, or on the
 *    launch schedule.
 */
#ifndef LC_H
#define LC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LC_OK = 0,
  LC_EINVAL = 1,  /* a null pointer, a size out of range, inconsistent shapes */
  LC_ENOSPC = 2,  /* workspace too small                                     */
  LC_ENOTSUP = 3, /* shape the kernels do not support (e.g. m % 8 != 0)       */
  LC_EHIP = 4     /* HIP runtime or launch error                              */
};

enum { LC_LUT_F32 = 0, LC_LUT_F16 = 1 };
enum { LC_REFINE_F32 = 0, LC_REFINE_BF16_RESCORE = 1 };

/* Borrowed device views of an index (the caller keeps the memory alive).
 * Layout (row-major, all device memory):
 *   proj      f32 [d_pad][d]    projection with orthonormal columns applied
 *                               before PQ: required when d_pad > d (a
 *                               rotation ahead of the product quantizer, as
 *                               OPQ does, Sec. 5.1), optional when d_pad == d
 *                               (e.g. a learned rotation), NULL for none
 *   centroids f32 [m][256][dsub], dsub = d_pad / m (8-bit PQ, Sec. 3.3)
 *   codes     u8  [n][code_stride], code_stride = next power of two >= m
 *   adj0      i32 [n][deg0]      level-0 links, -1 padded at the end, each
 *                               list sorted by increasing distance to its
 *                               owner (Sec. 4.2 orders g_1..g_k that way)
 *   up_base   i32 [n]            first upper row of node i, -1 on level 0;
 *                               the row of level l >= 1 is up_base[i] + l - 1
 *   adj_up    i32 [n_up_rows][deg_up]  upper-level links, -1 padded
 *   beta      f32 [m_beta][n_beta][k_reg + 1]  regression codebooks (Sec. 4.3):
 *                               m_beta = 1 is the codebook of Eq. 6-8; with
 *                               m_beta > 1 the d_pad coordinates are cut into
 *                               m_beta equal blocks of m / m_beta whole
 *                               sub-spaces, each with its own codebook (the
 *                               product codebook of Eq. 9)
 *   beta_idx  u8  [n][m_beta]    codebook entry of every vector and block
 *                               (1 byte per block, Sec. 4.3)
 * entry is the single node of the top level, max_level its level (Sec. 2). */
typedef struct {
  int32_t n, d, d_pad, m, ksub, code_stride, deg0, deg_up, k_reg, n_beta;
  int32_t entry, max_level, m_beta;
  int64_t n_up_rows;
  const float *proj;
  const float *centroids;
  const uint8_t *codes;
  const int32_t *adj0;
  const int32_t *up_base;
  const int32_t *adj_up;
  const float *beta;
  const uint8_t *beta_idx;
  /* 2-level residual codec (Sec. 3.3 residual codecs; Sec. 5.1 two-level
   * encodings), or coarse_k = 0 for the one-level PQ codec.  A vector is
   * q(x) = [C1[0][c0], C1[1][c1]] + PQ(codes): a first-level product
   * quantizer over the two halves of the (projected) vector, coarse_k
   * centroids each (coarse_k <= 65536, d_pad even), and the PQ codes encode
   * the residual. */
  int32_t coarse_k;
  const float *coarse_cent;      /* [2][coarse_k][d_pad/2] */
  const uint16_t *coarse_codes;  /* [n][2] (c0, c1), 4-byte aligned */
  const float *coarse_norm;      /* [n] ||c + r||^2 - ||c||^2, the node's term of the distance */
} lc_index_view;

typedef struct lc_index lc_index;

/* Validate the view and keep a host-side copy of it (host memory only; the
 * device arrays are borrowed).  Requires ksub == 256, m % 8 == 0, m <= 64,
 * d_pad % m == 0, dsub <= 16, deg0 <= 32, deg_up <= 32, 1 <= k_reg <= deg0,
 * 1 <= n_beta <= 256, m_beta >= 1 dividing m, 0 <= entry < n.  Returns LC_OK
 * and *out, or an error
 * code and *out = NULL. */
int lc_index_bind(const lc_index_view *view, lc_index **out);
void lc_index_release(lc_index *ix);

/* Elements of lut_dtype per query row of a distance table: m * 256 for the
 * one-level codec; for the 2-level codec the row holds m * 256 entries of
 * lut_dtype, then 2 * coarse_k float32 entries, and is padded to a multiple
 * of 256 bytes (layout below).  0 for a NULL index or another type. */
int64_t lc_lut_stride(const lc_index *ix, int lut_dtype);

/* Distance tables, Sec. 4.1 (asymmetric distances):
 *   LUT[q][s][c] = || (P y_q)^s - C[s][c] ||^2,  s < m, c < 256.
 * q:   f32 [nq][d] queries.
 * lut: LC_LUT_F32 -> f32 [nq][m][256];
 *      LC_LUT_F16 -> f16 [nq][m][256] holding LUT[q][s][c] / lut_scale[q][s]
 *      rounded to nearest, with lut_scale f32 [nq][m] a power of two per
 *      (query, sub-space) that maps the largest entry of the row to at most
 *      2^15 (precision form; lut_scale is NULL for F32).
 * 2-level codec (coarse_k > 0): with z = P y_q, c the first-level and r the
 * second-level reconstruction,
 * ||z - c - r||^2 = ||z^0 - c^0||^2 + ||z^1 - c^1||^2 - 2 <z, r> + coarse_norm,
 * so row q of lut (lc_lut_stride(ix, lut_dtype) elements) holds [m][256]
 * entries -2 <z^s, C[s][c]> (LC_LUT_F16: divided by lut_scale[q][s], a power
 * of two mapping the row's largest magnitude to at most 2^15), then
 * [2][coarse_k] float32 entries ||z^h - C1[h][c]||^2, then zero padding;
 * lc_search adds a node's two first-level entries and its coarse_norm to the
 * sum over its codes, and clamps the result at 0.
 * lut must be 16-byte aligned (LC_EINVAL otherwise).  nq == 0 is a no-op. */
int lc_build_lut(const lc_index *ix, const float *q, int64_t nq, int lut_dtype, void *lut,
                 float *lut_scale, void *stream);

/* Bytes of workspace lc_search needs for nq queries with every ef <= ef_max
 * and short-list S.  The workspace must be zero-filled before its first use;
 * lc_search leaves it zero-filled again when it returns. */
size_t lc_search_workspace_bytes(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S);

/* First stage (Sec. 2 walk + Sec. 4.1 short-list).  For every query q:
 *   1. greedy descent from `entry` on levels max_level..1: move to the
 *      neighbour with the smallest key while it beats the current key;
 *   2. best-first walk on level 0 with a pool W of at most
 *      ef_eff = max(ef[q], S) keys: repeatedly expand the best
 *      not-yet-expanded entry of W, evaluate its unvisited links by ADC
 *      (sum of LUT[s][code[s]]), keep the best ef_eff; stop when every entry
 *      of W has been expanded;
 *   3. short-list = the min(S, |W|) best entries of W.
 * lut:       as written by lc_build_lut (lut_scale for F16, else NULL); an
 *            F16 node key is the float32 sum, in sub-space order, of its
 *            entries times their row scales (each product exact).
 * ef:        i32 [nq] per-query efSearch, or NULL for ef_max everywhere;
 *            a query with ef[q] < 1 or ef[q] > ef_max is not searched and
 *            gets cand_n[q] = -1.
 * cand_ids:  i32 [nq][S] short-list ids in key order, -1 padded.
 * cand_adc:  f32 [nq][S] their ADC distances, +inf padded.
 * cand_n:    i32 [nq] number of valid short-list entries.
 * stats:     i32 [nq][2] = (E, D): level-0 expansions and newly visited
 *            nodes, or NULL.
 * ws:        workspace of at least lc_search_workspace_bytes(ix, nq, ef_max, S). */
int lc_search(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale,
              int64_t nq, const int32_t *ef, int32_t ef_max, int32_t S, int32_t *cand_ids,
              float *cand_adc, int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes,
              void *stream);

/* Launch schedule of the walk.  Every schedule returns exactly the same
 * short-lists, distances and (E, D) counts; only speed changes.
 *   hash_bits     log2 of the per-query LDS table of the visited set, in
 *                 4-byte words (9..14; 0 = automatic: 9 for visited mode 1,
 *                 else the largest table of 2^10..2^12 words that leaves 8
 *                 query slots per compute unit; 2^12 when the query's
 *                 distance table alone leaves fewer than 8; else 2^10).
 *   prefetch      visited mode 0 only: 1 = at the start of every step, load
 *                 the adjacency rows of the two unexpanded entries that follow
 *                 the two being expanded (used at the next step when they
 *                 are still the next two), 0 = load each row when it is
 *                 needed.
 *   waves_per_cu  cap on resident query slots per compute unit (0 = as many as
 *                 LDS allows).
 *   queue         1 = slots take queries from an atomic counter in the
 *                 workspace (load balance for uneven walk lengths), 0 = each
 *                 slot strides over the batch.
 *   visited       0 = the LDS table holds the visited ids: each id has a home
 *                 bucket of 16 bytes and is kept there while the bucket has
 *                 room, else in the slot's bitset in the workspace.  Each
 *                 step expands the best unexpanded entry and, when the
 *                 sequential walk would expand it next, the second one too
 *                 (same results, half the dependent steps).
 *                 1 = the slot's bitset in the workspace is the visited set;
 *                 the LDS table is a direct-mapped cache of recently visited
 *                 ids, and a miss tests-and-sets the bit while the node's
 *                 code is fetched speculatively (less LDS per query, so more
 *                 queries resident).
 *   wide          visited mode 0 only: 1 = the table holds 32-bit ids (four
 *                 per bucket); 0 = 16-bit tags (eight per bucket, twice the
 *                 ids in the same LDS) whenever ids below n fit a tag, which
 *                 is when n <= 2^(hash_bits + 13).
 *   pool          visited mode 0 only: 0 = the pool W lives in registers when
 *                 it has at most 128 entries (max(ef_max, S) <= 128; the scan
 *                 is a ballot, kept keys are merged by bitonic networks) and
 *                 the table is not in registers, in LDS otherwise; 1 = always
 *                 in LDS.
 *   table         visited mode 0 only: where an fp16 table of the one-level
 *                 codec lives during the walk.  1 = LDS; 2 = the wave's
 *                 registers (2m words per lane, four entries per lane,
 *                 m <= 56; read by cross-lane permutes, so that a slot's LDS
 *                 holds only the row scales, the pool and the visited table,
 *                 and a CU keeps up to 8 slots, 12 at m <= 24), with the pool
 *                 in LDS whatever `pool` says; 0 = registers when they keep at
 *                 least 1.3 times the slots per CU of the table in LDS, or as
 *                 many with a larger visited table (m = 24..56, and m = 16
 *                 beyond a pool of 128 entries), else LDS.  Same results
 *                 either way; float32 tables and the 2-level codec's stay in
 *                 LDS.
 *   codes         visited mode 0 only: 0 = each step fetches the codes of all
 *                 the links it probes while the visited table is probed (a
 *                 link found visited reads its code for nothing: more HBM
 *                 traffic, a shorter dependent chain); 1 = only the codes of
 *                 links the table does not hold, once it has answered.
 * The default schedule (sched = NULL, and lc_search) is {0, 1, 0, 1, 0, 0, 0, 0, 0}. */
typedef struct {
  int32_t hash_bits, prefetch, waves_per_cu, queue, visited, wide, pool, table, codes;
} lc_schedule;

/* The walk that lc_search_sched would launch for these sizes, table type and
 * schedule (NULL = default), without launching it or touching the device: a
 * NUL-terminated line "<kernel> grid=<slots> slots_per_cu=<k> hash_bits=<b>
 * lds_bytes=<bytes>" written to buf (len bytes, truncated to fit).  The
 * kernel is named as a profiler lists it, without its namespace (the
 * variant that counts distance evaluations, used when max_evals > 0, ends in
 * "true" instead of "false").  LC_EINVAL for bad sizes, dtype or schedule;
 * LC_ENOTSUP for an m the walk does not take. */
int lc_walk_describe(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, int lut_dtype,
                     const lc_schedule *sched, char *buf, size_t len);

/* Workspace bytes for lc_search_sched with schedule `sched` (NULL = default). */
size_t lc_search_workspace_bytes_sched(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S,
                                       const lc_schedule *sched);

/* lc_search with an explicit schedule (NULL = the default of lc_search) and an
 * optional processing order: order i32 [nq] is a permutation of 0..nq-1 (or
 * NULL for 0..nq-1); slots take queries in that order (e.g. longest ef first),
 * and every output still lands in the query's own row.  An entry outside
 * 0..nq-1 is skipped. */
int lc_search_sched(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale,
                    int64_t nq, const int32_t *ef, int32_t ef_max, int32_t S, const int32_t *order,
                    int32_t *cand_ids, float *cand_adc, int32_t *cand_n, int32_t *stats, void *ws,
                    size_t ws_bytes, const lc_schedule *sched, void *stream);

/* lc_search_sched with the paper's budget T on distance computations (Sec.
 * 3.1: the walk stops once it has compared the query with T nodes):
 * max_evals > 0 ends a query's level-0 walk right after its max_evals-th
 * distance evaluation, so D = min(max_evals, D of the unbounded walk); the
 * links of that last expansion past the budget are not evaluated, and the
 * short-list is the best S of the pool at that point.  Evaluations on the
 * upper levels are not counted.  max_evals = 0: no budget (lc_search_sched);
 * max_evals < 0: LC_EINVAL.  Other arguments, outputs and errors as
 * lc_search_sched. */
int lc_search_budget(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale,
                     int64_t nq, const int32_t *ef, int32_t ef_max, int32_t S, int32_t max_evals,
                     const int32_t *order, int32_t *cand_ids, float *cand_adc, int32_t *cand_n,
                     int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sched, void *stream);

/* lc_search for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops or harnesses that forbid hipMalloc): the same
 * first stage with the default schedule, its workspace being a fixed array of
 * LC_NOALLOC_SCRATCH_BYTES inside the library instead of an argument.  The
 * call allocates nothing; the caller still owns lut, lut_scale, ef and the
 * outputs, which are as for lc_search (identical values).
 *  - Each GPU the library runs on holds its own copy of the array until the
 *    process ends; the call uses the current device's, which must be the
 *    device the index was bound on (else LC_EINVAL).
 *  - The first call on a device zeroes the array with a kernel on `stream`;
 *    every call then zeroes the queue counters at its head the same way, and
 *    a completed walk leaves the rest zero-filled.
 *  - The walk launches only as many resident query slots as the array holds
 *    (each slot needs an n-bit visited bitset and an id list), so for a large
 *    index it runs slower than lc_search with a full workspace; LC_ENOSPC when
 *    not even one slot fits.
 *  - Calls that overlap on one GPU (other streams, other threads) share the
 *    array and race: serialise them.
 * Errors as lc_search. */
#define LC_NOALLOC_SCRATCH_BYTES (128u << 20)
int lc_search_noalloc(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale,
                      int64_t nq, const int32_t *ef, int32_t ef_max, int32_t S, int32_t *cand_ids,
                      float *cand_adc, int32_t *cand_n, int32_t *stats, void *stream);

/* Second stage (Sec. 4.1 "Refinement strategy"; Sec. 4.2 Eq. 5; Sec. 4.3
 * Eq. 7 and Eq. 9).  For each valid short-list id i:
 *   g_0 = i, g_j = adj0[i][j-1] (j = 1..k_reg, -1 -> zero),
 *   block jb of x~ (coordinates [jb w, jb w + w), w = d_pad / m_beta):
 *     x~ = sum_j beta[jb][beta_idx[i][jb]][j] * q(g_j),
 *   d~ = || P y - x~ ||^2,
 * then the K smallest (d~, id) in ascending order.  A short-list id with a
 * codebook byte >= n_beta is treated as no candidate.
 * cand_ids, cand_n: as produced by lc_search (cand_n[q] <= 0 -> no candidates).
 * precision: LC_REFINE_F32 (fp32 throughout) or LC_REFINE_BF16_RESCORE.
 * out_ids i32 [nq][K] (-1 padded), out_d f32 [nq][K] (+inf padded).
 * Requires 1 <= K <= S.  The centroids are staged in LDS when they fit
 * (d_pad x 256 values beside the per-wave buffers), else the float32 kernel
 * reads them from global memory; LC_ENOTSUP for the precision form on a
 * shape without a specialised kernel.  2-level codec: q(g) decodes both
 * levels (the first-level centroid of each half plus the PQ residual), in
 * float32 only (the precision form returns LC_ENOTSUP when its re-score does
 * not cover the whole short-list). */
int lc_refine(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids,
              const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids,
              float *out_d, void *stream);

/* Projected queries for an index with a projection P (required when d_pad > d,
 * e.g. a rotation learned ahead of PQ): qp[i] = P q[i], f32 [nq][d_pad]
 * device, each coordinate summed over the inputs in order (float32).  Without
 * P the rows are copied (d == d_pad).  lc_build_lut_projected and
 * lc_refine_projected then take qp in place of q and skip the projection,
 * which the plain entry points apply per table block and per refined query:
 * projecting a batch once reads P once per block of queries instead of once
 * per query.  Results equal the plain entry points' up to float32 rounding of
 * the projection (a P too large for the LDS of one compute unit together with
 * 32 queries is read from global memory instead; which way depends only on
 * d and d_pad).  Errors: LC_EINVAL (null pointers, nq < 0). */
int lc_project_queries(const lc_index *ix, const float *q, int64_t nq, float *qp, void *stream);
int lc_build_lut_projected(const lc_index *ix, const float *qp, int64_t nq, int lut_dtype, void *lut,
                           float *lut_scale, void *stream);
int lc_refine_projected(const lc_index *ix, const float *qp, int64_t nq, const int32_t *cand_ids,
                        const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids,
                        float *out_d, void *stream);

/* Regression-codebook assignment of database vectors (Sec. 4.3, Eq. 7; one
 * entry per block for the product codebook, Eq. 9) — the step of the index
 * build that touches every vector.  For vectors i = n0 .. n0+count-1 of this
 * index, with G(x_i) = [q(x_i), q(g_1), ..., q(g_k_reg)] (its code and the
 * codes of its first k_reg level-0 links, a -1 link a zero column) and x' =
 * P x_i, block jb's entry is the b minimising
 *   ||x'||^2 - 2 beta^T (G^T x') + beta^T (G^T G) beta,  beta = beta[jb][b],
 * over the block's coordinates [jb w, jb w + w), w = d_pad / m_beta, lowest b
 * on ties.  The arg-min is taken in float64 with every sum in ascending order
 * and no fused multiply-add, so it is the entry a plain sequential float64
 * evaluation picks.
 * x:   f32 [count][d] device, row r is vector n0 + r (raw, before P).
 * out: u8 [count][m_beta] device.
 * Uses the bound index's centroids, codes, adj0, proj and beta (not its
 * beta_idx).  Requires 0 <= n0, 0 <= count, n0 + count <= n (LC_EINVAL). */
int lc_assign_beta(const lc_index *ix, const float *x, int64_t n0, int64_t count, uint8_t *out,
                   void *stream);

/* ---- Index build on the GPU (steps before the search path) -------------- */

/* The projection the builder applies to database vectors: xp[i][r] =
 * float(sum_t double(proj[r][t]) * double(x[i][t])), t ascending in float64 (a
 * copy when proj is NULL, which requires d_pad == d).  x f32 [n][d], xp f32
 * [n][d_pad], device.  Errors: LC_EINVAL. */
int lc_project_exact(const float *x, int64_t n, int d, const float *proj, int d_pad, float *xp, void *stream);

/* Product-quantizer encoding (Sec. 3.3, Sec. 4.1): codes[i][s] = the c
 * minimising ||xp_i^s - C[s][c]||^2, each distance a float32 sum over the
 * sub-space's coordinates in order, the lowest c on ties; bytes m..code_stride-1
 * of a row are zero.  xp f32 [n][d_pad], centroids f32 [m][256][d_pad/m], codes
 * u8 [n][code_stride], device.  Errors: LC_EINVAL; LC_ENOTSUP for d_pad/m > 16. */
int lc_pq_encode(const float *xp, int64_t n, int d_pad, int m, const float *centroids, uint8_t *codes,
                 int code_stride, void *stream);

/* Workspace bytes of lc_graph_insert for batches of at most max_count nodes
 * (0 for bad arguments or ef_construction > 64). */
size_t lc_graph_insert_workspace_bytes(const lc_index *ix, int32_t max_count, int32_t ef_construction);

/* One batch of the graph build (Sec. 5.1: nodes added in batches, each
 * searched against the graph as it stood when the batch began, then linked)
 * for nodes of level 0.  For every node x of nodes[0..count):
 *   1. search: greedy descent from `entry` on the upper levels, then the
 *      level-0 walk of lc_search with ef = S = ef_construction, on the table
 *      ||xp_x^s - C[s][c]||^2 (float32 sums in coordinate order; Sec. 4.1
 *      asymmetric distances from the raw vector);
 *   2. x's list (deg0 entries, -1 padded): over the candidates in (distance,
 *      id) order, the shrinking rule of Sec. 2 keeps e if d(x, e) < d(e, s)
 *      for every link s kept before it, d(e, s) = ||q(e) - q(s)||^2 summed
 *      over the sub-spaces in order; free slots take the nearest rejected
 *      candidates;
 *   3. reverse links: every y in x's list gets x; y's list and its new links,
 *      ordered by (||xp_y - q(.)||^2, id), are kept whole when they fit deg0
 *      and re-shrunk by the rule of step 2 otherwise.
 * With these float orders (no fused multiply-add) the lists are those of the
 * host builder (lcb_graph_build) given the same arrays.
 * ix:    the index being built (its adj0 is adj0; codes, centroids, up_base,
 *        adj_up, entry and max_level as for lc_search; one-level PQ only).
 * adj0:  i32 [n][deg0] device, modified in place; must be the view's adj0.
 * xp:    f32 [n][d_pad] projected database vectors (lc_project_exact).
 * nodes: i32 [count] device, the batch (level-0 nodes not yet linked).
 * ws:    at least lc_graph_insert_workspace_bytes(ix, max_count,
 *        ef_construction) bytes, zero-filled before the first call; every
 *        call leaves it zero-filled where that matters.
 * Requires 0 <= count <= max_count, 1 <= ef_construction <= 64 (LC_ENOTSUP
 * above), d_pad * 1 KB of centroids plus 16 vectors within one compute unit's
 * LDS (LC_ENOTSUP otherwise), coarse_k == 0 (LC_ENOTSUP). */
int lc_graph_insert(const lc_index *ix, int32_t *adj0, const float *xp, const int32_t *nodes, int32_t count,
                    int32_t max_count, int32_t ef_construction, void *ws, size_t ws_bytes, void *stream);

const char *lc_strerror(int code);

/* Identity of the build: a hex sha1 over this header and the library's
 * sources, fixed at compile time, so that a binding can refuse a library
 * built from other sources (e.g. with another layout of lc_index_view). */
const char *lc_build_id(void);

#ifdef __cplusplus
}
#endif
#endif
