// Per-query ADC tables on the matrix cores (Sec. 4.1: asymmetric distances).
//
//   LUT[q][s][c] = || y'^s - C[s][c] ||^2,   y' = P y (or y when P is absent)
//
// computed as ||y'^s - mu_s||^2 + ||C[s][c] - mu_s||^2 - 2 <y'^s - mu_s, C[s][c] - mu_s>
// where mu_s is the mean of the 256 centroids of sub-space s.  The distance is
// translation invariant, and centring both operands keeps the float32
// cancellation of the expansion small.  The cross term for a tile of 16
// queries x 16 centroids is one v_mfma_f32_16x16x4_f32 per 4 sub-dimensions.
//
// One wavefront per (16 queries, sub-space); the write of the table (m*256
// floats per query) dominates, so the kernel is bound by HBM writes.
#include "lc_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int DSUB>
__global__ __launch_bounds__(64) void lut_f32_kernel(const float *__restrict__ q, int64_t nq, int d,
                                                      const float *__restrict__ proj, int m,
                                                      const float *__restrict__ cent,
                                                      float *__restrict__ lut) {
  constexpr int KS = (DSUB + 3) / 4;  // MFMA K steps
  constexpr int DP = KS * 4;          // sub-dimension padded to the MFMA K
  __shared__ float cc[256 * DP];      // centred centroids, zero padded
  __shared__ float nc[256];           // their squared norms
  __shared__ float mu[DP];
  __shared__ float ya[16 * DP];  // centred projected queries
  __shared__ float ny[16];
  const int lane = threadIdx.x;
  const int s = blockIdx.y;
  const int64_t q0 = int64_t(blockIdx.x) * 16;
  const float *cs = cent + size_t(s) * 256 * DSUB;

  if (lane < DP) {
    float acc = 0.f;
    if (lane < DSUB)
      for (int c = 0; c < 256; ++c) acc += cs[c * DSUB + lane];
    mu[lane] = lane < DSUB ? acc * (1.f / 256.f) : 0.f;
  }
  __syncthreads();
  for (int c = lane; c < 256; c += 64) {
    float nrm = 0.f;
#pragma unroll
    for (int t = 0; t < DP; ++t) {
      const float v = t < DSUB ? cs[c * DSUB + t] - mu[t] : 0.f;
      cc[c * DP + t] = v;
      nrm += v * v;
    }
    nc[c] = nrm;
  }
  for (int e = lane; e < 16 * DP; e += 64) {
    const int i = e / DP, t = e % DP;
    const int64_t qi = q0 + i;
    float v = 0.f;
    if (qi < nq && t < DSUB) {
      const int r = s * DSUB + t;
      const float *y = q + qi * d;
      float yp;
      if (proj) {
        const float *pr = proj + size_t(r) * d;
        yp = 0.f;
        for (int u = 0; u < d; ++u) yp += pr[u] * y[u];
      } else {
        yp = y[r];
      }
      v = yp - mu[t];
    }
    ya[e] = v;
  }
  __syncthreads();
  if (lane < 16) {
    float a = 0.f;
#pragma unroll
    for (int t = 0; t < DP; ++t) a += ya[lane * DP + t] * ya[lane * DP + t];
    ny[lane] = a;
  }
  __syncthreads();

  // v_mfma_f32_16x16x4_f32 operand layout: lane l supplies A[l % 16][l / 16]
  // and B[l / 16][l % 16]; it receives D[4 (l / 16) + r][l % 16], r = 0..3.
  const int col = lane & 15, kg = lane >> 4;
  float a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a[ks] = ya[col * DP + ks * 4 + kg];
  for (int tile = 0; tile < 16; ++tile) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const int c = tile * 16 + col;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], cc[c * DP + ks * 4 + kg], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = kg * 4 + r;
      const int64_t qi = q0 + i;
      if (qi < nq) lut[(qi * m + s) * 256 + c] = lc::clamp0(ny[i] + nc[c] - 2.f * acc[r]);
    }
  }
}

template <int DSUB>
hipError_t launch_dsub(const lc_index *ix, const float *q, int64_t nq, float *lut, hipStream_t st) {
  dim3 grid(lc::ceil_div(nq, 16), ix->v.m);
  hipLaunchKernelGGL(lut_f32_kernel<DSUB>, grid, dim3(64), 0, st, q, nq, ix->v.d, ix->v.proj, ix->v.m,
                     ix->v.centroids, lut);
  return hipGetLastError();
}

}  // namespace

int lc_launch_lut(const lc_index *ix, const float *q, int64_t nq, int dtype, void *lut, float *scale,
                  hipStream_t st) {
  (void)scale;
  if (dtype != LC_LUT_F32) return LC_ENOTSUP;
  if (nq > int64_t(65535) * 16 * 1024) return LC_EINVAL;
  hipError_t e;
  switch (ix->dsub) {
    case 1: e = launch_dsub<1>(ix, q, nq, (float *)lut, st); break;
    case 2: e = launch_dsub<2>(ix, q, nq, (float *)lut, st); break;
    case 3: e = launch_dsub<3>(ix, q, nq, (float *)lut, st); break;
    case 4: e = launch_dsub<4>(ix, q, nq, (float *)lut, st); break;
    case 6: e = launch_dsub<6>(ix, q, nq, (float *)lut, st); break;
    case 8: e = launch_dsub<8>(ix, q, nq, (float *)lut, st); break;
    case 12: e = launch_dsub<12>(ix, q, nq, (float *)lut, st); break;
    case 16: e = launch_dsub<16>(ix, q, nq, (float *)lut, st); break;
    default: return LC_ENOTSUP;
  }
  return e == hipSuccess ? LC_OK : LC_EHIP;
}
