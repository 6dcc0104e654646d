// C-ABI of liblc: argument validation and dispatch to the kernel launchers.
#include <new>

#include "lc_internal.h"

namespace {

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

bool supported_dsub(int ds) {
  return ds == 1 || ds == 2 || ds == 3 || ds == 4 || ds == 6 || ds == 8 || ds == 12 || ds == 16;
}

}  // namespace

extern "C" {

#ifndef LC_SOURCE_ID
#define LC_SOURCE_ID "unknown"
#endif

const char *lc_build_id(void) { return LC_SOURCE_ID; }

const char *lc_strerror(int code) {
  switch (code) {
    case LC_OK: return "ok";
    case LC_EINVAL: return "invalid argument";
    case LC_ENOSPC: return "workspace too small";
    case LC_ENOTSUP: return "unsupported shape or mode";
    case LC_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

int lc_index_bind(const lc_index_view *v, lc_index **out) {
  if (!out) return LC_EINVAL;
  *out = nullptr;
  if (!v) return LC_EINVAL;
  if (v->n < 1 || v->d < 1 || v->d_pad < v->d || v->m < 1 || v->ksub != 256) return LC_EINVAL;
  if (v->d_pad % v->m != 0) return LC_EINVAL;
  if (!pow2(v->code_stride) || v->code_stride < v->m || (v->code_stride >> 1) >= v->m) return LC_EINVAL;
  if (v->deg0 < 1 || v->deg_up < 1 || v->k_reg < 1 || v->k_reg > v->deg0) return LC_EINVAL;
  if (v->n_beta < 1 || v->n_beta > 256) return LC_EINVAL;
  if (v->m_beta < 1 || v->m % v->m_beta != 0) return LC_EINVAL;
  if (v->entry < 0 || v->entry >= v->n || v->max_level < 0 || v->n_up_rows < 0) return LC_EINVAL;
  if (v->max_level > 0 && v->n_up_rows < v->max_level) return LC_EINVAL;
  if (!v->centroids || !v->codes || !v->adj0 || !v->up_base || !v->beta || !v->beta_idx) return LC_EINVAL;
  if (v->max_level > 0 && !v->adj_up) return LC_EINVAL;
  if (v->d_pad != v->d && !v->proj) return LC_EINVAL;  // padding needs the projection; a rotation is optional
  if (v->coarse_k < 0 || v->coarse_k > 65536) return LC_EINVAL;
  if (v->coarse_k > 0 && (v->d_pad % 2 != 0 || !v->coarse_cent || !v->coarse_codes || !v->coarse_norm ||
                          (reinterpret_cast<uintptr_t>(v->coarse_codes) & 3) != 0))
    return LC_EINVAL;
  if (v->m % 8 != 0 || v->m > 64 || v->deg0 > 32 || v->deg_up > 32) return LC_ENOTSUP;
  if (!supported_dsub(v->d_pad / v->m)) return LC_ENOTSUP;
  lc_index *ix = new (std::nothrow) lc_index;
  if (!ix) return LC_EINVAL;
  ix->v = *v;
  ix->dsub = v->d_pad / v->m;
  if (hipGetDevice(&ix->device) != hipSuccess) {
    delete ix;
    return LC_EHIP;
  }
  int cus = 0, lds = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ix->device) != hipSuccess ||
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, ix->device) !=
          hipSuccess) {
    delete ix;
    return LC_EHIP;
  }
  ix->num_cus = cus > 0 ? cus : 1;
  ix->lds_per_cu = lds > 0 ? lds : 65536;
  *out = ix;
  return LC_OK;
}

void lc_index_release(lc_index *ix) { delete ix; }

int64_t lc_lut_stride(const lc_index *ix, int lut_dtype) {
  if (!ix || (lut_dtype != LC_LUT_F32 && lut_dtype != LC_LUT_F16)) return 0;
  return lc_lut_row_bytes(ix, lut_dtype) / (lut_dtype == LC_LUT_F16 ? 2 : 4);
}

namespace {
int build_lut(const lc_index *ix, const float *q, int64_t nq, int lut_dtype, void *lut, float *lut_scale,
              bool projected, void *stream) {
  if (!ix || nq < 0) return LC_EINVAL;
  if (lut_dtype != LC_LUT_F32 && lut_dtype != LC_LUT_F16) return LC_EINVAL;
  if (nq == 0) return LC_OK;
  if (!q || !lut) return LC_EINVAL;
  if (reinterpret_cast<uintptr_t>(lut) % 16) return LC_EINVAL;  // rows are written 8 or 16 bytes per lane
  if (lut_dtype == LC_LUT_F16 && !lut_scale) return LC_EINVAL;
  return lc_launch_lut(ix, q, nq, lut_dtype, lut, lut_scale, projected, static_cast<hipStream_t>(stream));
}

int refine(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids, const int32_t *cand_n,
           int32_t S, int32_t K, int precision, int32_t *out_ids, float *out_d, bool projected, void *stream) {
  if (!ix || nq < 0 || S < 1 || K < 1 || K > S) return LC_EINVAL;
  if (S > 4096) return LC_ENOTSUP;
  if (precision != LC_REFINE_F32 && precision != LC_REFINE_BF16_RESCORE) return LC_EINVAL;
  if (nq == 0) return LC_OK;
  if (!q || !cand_ids || !cand_n || !out_ids || !out_d) return LC_EINVAL;
  return lc_launch_refine(ix, q, nq, cand_ids, cand_n, S, K, precision, out_ids, out_d, projected,
                          static_cast<hipStream_t>(stream));
}
}  // namespace

int lc_build_lut(const lc_index *ix, const float *q, int64_t nq, int lut_dtype, void *lut,
                 float *lut_scale, void *stream) {
  return build_lut(ix, q, nq, lut_dtype, lut, lut_scale, false, stream);
}

int lc_build_lut_projected(const lc_index *ix, const float *qp, int64_t nq, int lut_dtype, void *lut,
                           float *lut_scale, void *stream) {
  return build_lut(ix, qp, nq, lut_dtype, lut, lut_scale, true, stream);
}

int lc_project_queries(const lc_index *ix, const float *q, int64_t nq, float *qp, void *stream) {
  if (!ix || nq < 0) return LC_EINVAL;
  if (nq == 0) return LC_OK;
  if (!q || !qp) return LC_EINVAL;
  return lc_launch_project(ix, q, nq, qp, static_cast<hipStream_t>(stream));
}

size_t lc_search_workspace_bytes_sched(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S,
                                       const lc_schedule *sched) {
  if (!ix || nq < 1 || ef_max < 1 || S < 1) return 0;
  return lc_walk_workspace_bytes(ix, nq, ef_max, S, sched);
}

size_t lc_search_workspace_bytes(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S) {
  return lc_search_workspace_bytes_sched(ix, nq, ef_max, S, nullptr);
}

int lc_walk_describe(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, int lut_dtype,
                     const lc_schedule *sched, char *buf, size_t len) {
  if (!ix || nq < 1 || ef_max < 1 || S < 1 || !buf || len < 1) return LC_EINVAL;
  return lc_describe_walk(ix, nq, ef_max, S, lut_dtype, sched, buf, len);
}

int lc_search_budget(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale, int64_t nq,
                     const int32_t *ef, int32_t ef_max, int32_t S, int32_t max_evals, const int32_t *order,
                     int32_t *cand_ids, float *cand_adc, int32_t *cand_n, int32_t *stats, void *ws,
                     size_t ws_bytes, const lc_schedule *sched, void *stream) {
  if (!ix || nq < 0 || ef_max < 1 || S < 1 || max_evals < 0) return LC_EINVAL;
  if (ef_max > 4096 || S > 4096) return LC_ENOTSUP;
  if (lut_dtype != LC_LUT_F32 && lut_dtype != LC_LUT_F16) return LC_EINVAL;
  if (nq == 0) return LC_OK;
  if (nq > int64_t(0x7FFFFFFF)) return LC_EINVAL;
  if (!lut || !cand_ids || !cand_adc || !cand_n || !ws) return LC_EINVAL;
  if (lut_dtype == LC_LUT_F16 && !lut_scale) return LC_EINVAL;
  return lc_launch_walk(ix, lut, lut_dtype, lut_scale, nq, ef, ef_max, S, max_evals, order, cand_ids, cand_adc,
                        cand_n, stats, ws, ws_bytes, sched, static_cast<hipStream_t>(stream));
}

int lc_search_sched(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale, int64_t nq,
                    const int32_t *ef, int32_t ef_max, int32_t S, const int32_t *order, int32_t *cand_ids,
                    float *cand_adc, int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes,
                    const lc_schedule *sched, void *stream) {
  return lc_search_budget(ix, lut, lut_dtype, lut_scale, nq, ef, ef_max, S, 0, order, cand_ids, cand_adc, cand_n,
                          stats, ws, ws_bytes, sched, stream);
}

int lc_search(const lc_index *ix, const void *lut, int lut_dtype, const float *lut_scale, int64_t nq,
              const int32_t *ef, int32_t ef_max, int32_t S, int32_t *cand_ids, float *cand_adc,
              int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, void *stream) {
  return lc_search_sched(ix, lut, lut_dtype, lut_scale, nq, ef, ef_max, S, nullptr, cand_ids, cand_adc, cand_n,
                         stats, ws, ws_bytes, nullptr, stream);
}

int lc_assign_beta(const lc_index *ix, const float *x, int64_t n0, int64_t count, uint8_t *out, void *stream) {
  if (!ix || n0 < 0 || count < 0 || n0 > ix->v.n || count > int64_t(ix->v.n) - n0) return LC_EINVAL;
  if (count == 0) return LC_OK;
  if (!x || !out) return LC_EINVAL;
  return lc_launch_assign(ix, x, n0, count, out, static_cast<hipStream_t>(stream));
}

int lc_refine(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids,
              const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids, float *out_d,
              void *stream) {
  return refine(ix, q, nq, cand_ids, cand_n, S, K, precision, out_ids, out_d, false, stream);
}

int lc_refine_projected(const lc_index *ix, const float *qp, int64_t nq, const int32_t *cand_ids,
                        const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids,
                        float *out_d, void *stream) {
  return refine(ix, qp, nq, cand_ids, cand_n, S, K, precision, out_ids, out_d, true, stream);
}

}  // extern "C"
