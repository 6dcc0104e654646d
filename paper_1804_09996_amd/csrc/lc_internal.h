// Internal declarations shared by the liblc translation units (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc.h"

struct lc_index {
  lc_index_view v;
  int dsub;
  int device;
  int num_cus;
  int lds_per_cu;  // bytes of LDS per compute unit
};

namespace lc {

// A key orders (distance, id) as one unsigned 64-bit integer: the IEEE bits of
// a non-negative float32 distance in the high word, the id in the low word.
// Bit 31 of the low word marks a pool entry as expanded; it is masked off for
// every comparison (ids are < 2^31).
constexpr uint64_t kKeyMax = ~0ull;
constexpr uint64_t kExpanded = 1ull << 31;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t make_key(float d, int32_t id) {
  return (uint64_t(__float_as_uint(d)) << 32) | uint32_t(id);
}
__device__ __forceinline__ uint64_t pure_key(uint64_t k) { return k & ~kExpanded; }
__device__ __forceinline__ int32_t key_id(uint64_t k) { return int32_t(uint32_t(k) & 0x7FFFFFFFu); }
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float(uint32_t(k >> 32)); }

// Non-negative clamp that never produces -0.0 (whose bits would sort last).
__device__ __forceinline__ float clamp0(float x) { return x > 0.f ? x : 0.f; }

// Wave-level ordering of LDS traffic between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl(uint32_t(v), src), hi = __shfl(uint32_t(v >> 32), src);
  return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
  uint32_t lo = __shfl_xor(uint32_t(v), mask), hi = __shfl_xor(uint32_t(v >> 32), mask);
  return (uint64_t(hi) << 32) | lo;
}

// Minimum over the 64 lanes of a wave (every lane receives it).
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

// Bitonic sort of one 64-bit key per lane across groups of 32 lanes
// (ascending by lane index within each group).
__device__ __forceinline__ uint64_t sort32(uint64_t v, int lane) {
  const int l = lane & 31;
  for (int k = 2; k <= 32; k <<= 1) {
    for (int j = k >> 1; j >= 1; j >>= 1) {
      uint64_t o = shfl_xor64(v, j);
      bool up = ((l & k) == 0);
      bool lower = ((l & j) == 0);
      uint64_t mn = o < v ? o : v, mx = o < v ? v : o;
      v = (lower == up) ? mn : mx;
    }
  }
  return v;
}

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

}  // namespace lc

// Bytes of one query's distance-table row: m * 256 entries of 4 (F32) or 2
// (F16) bytes; for the 2-level codec then 2 * coarse_k float32 first-level
// entries, the row padded to a multiple of 256 bytes.
inline int64_t lc_lut_row_bytes(const lc_index *ix, int dtype) {
  const int64_t base = int64_t(ix->v.m) * 256 * (dtype == LC_LUT_F16 ? 2 : 4);
  if (ix->v.coarse_k <= 0) return base;
  return (base + 8 * int64_t(ix->v.coarse_k) + 255) / 256 * 256;
}
// Float32 entries per row (the float32 table).
inline int64_t lc_lut_entries(const lc_index *ix) { return lc_lut_row_bytes(ix, LC_LUT_F32) / 4; }

// Launchers (return LC_* codes).  lc_launch_walk with fit_ws launches no more
// resident query slots than the workspace holds (LC_ENOSPC when not even one
// fits) instead of requiring the workspace of the full grid.
int lc_launch_project(const lc_index *ix, const float *q, int64_t nq, float *out, hipStream_t st);
int lc_launch_lut(const lc_index *ix, const float *q, int64_t nq, int dtype, void *lut, float *scale,
                  bool projected,
                  hipStream_t st);
size_t lc_walk_workspace_bytes(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S,
                               const lc_schedule *sched);
int lc_describe_walk(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, int dtype, const lc_schedule *sched,
                     char *buf, size_t len);
int lc_launch_assign(const lc_index *ix, const float *x, int64_t n0, int64_t count, uint8_t *out, hipStream_t st);
int lc_launch_walk(const lc_index *ix, const void *lut, int dtype, const float *scale, int64_t nq,
                   const int32_t *ef, int32_t ef_max, int32_t S, int32_t max_d, const int32_t *order, int32_t *cand_ids,
                   float *cand_adc,
                   int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sched,
                   hipStream_t st, bool fit_ws = false);
int lc_launch_refine(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids,
                     const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids,
                     float *out_d, bool projected, hipStream_t st);
