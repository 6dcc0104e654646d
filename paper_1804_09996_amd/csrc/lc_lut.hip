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
// One wavefront per (sub-space, a run of 16-query groups); the write of the
// table (m*256 entries per query) dominates, so the kernel is bound by HBM
// writes.
#include <hip/hip_fp16.h>

#include <type_traits>

#include "lc_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// OUT = float: the table itself.  OUT = __half: the table divided by a
// power-of-two scale per (query, sub-space) row that maps the row's largest
// entry to at most 2^15 (scale written to `scale`).  A block stages the
// sub-space's centred centroids once and then takes `groups` consecutive
// groups of 16 queries.
template <int DSUB, typename OUT>
__global__ __launch_bounds__(64) void lut_kernel(const float *__restrict__ q, int64_t nq, int d,
                                                  const float *__restrict__ proj, int m,
                                                  const float *__restrict__ cent, OUT *__restrict__ lut,
                                                  float *__restrict__ scale, int groups) {
  constexpr int KS = (DSUB + 3) / 4;  // MFMA K steps
  constexpr int DP = KS * 4;          // sub-dimension padded to the MFMA K
  __shared__ float cc[256 * DP];      // centred centroids, zero padded
  __shared__ float nc[256];           // their squared norms
  __shared__ float mu[DP];
  __shared__ float ya[16 * DP];  // centred projected queries
  __shared__ float ny[16];
  const int lane = threadIdx.x;
  const int s = blockIdx.y;
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

  // v_mfma_f32_16x16x4_f32 operand layout: lane l supplies A[l % 16][l / 16]
  // and B[l / 16][l % 16]; it receives D[4 (l / 16) + r][l % 16], r = 0..3.
  // A is a tile of 16 centroids, B the 16 queries: lane l holds centroids
  // 4 (l / 16) .. 4 (l / 16) + 3 of the tile for query l % 16, contiguous in
  // that query's table row.
  const int col = lane & 15, kg = lane >> 4;
  for (int g = 0; g < groups; ++g) {
    const int64_t q0 = (int64_t(blockIdx.x) * groups + g) * 16;
    if (q0 >= nq) break;
    __syncthreads();  // the previous group's queries are no longer read
    if (proj) {
      // the sub-space's DSUB rows of P y for the 16 queries: four lanes per query,
      // each over a quarter of the inputs (contiguous runs of the query and of
      // every row of P, the rows shared by all queries), summed over the four
      const int i = lane >> 2, part = lane & 3;
      const int64_t qi = q0 + i;
      const int span = (d + 3) / 4, u0 = part * span, u1 = u0 + span < d ? u0 + span : d;
      float acc[DSUB];
#pragma unroll
      for (int t = 0; t < DSUB; ++t) acc[t] = 0.f;
      if (qi < nq) {
        const float *y = q + qi * d;
        for (int u = u0; u < u1; ++u) {
          const float yu = y[u];
#pragma unroll
          for (int t = 0; t < DSUB; ++t) acc[t] += proj[size_t(s * DSUB + t) * d + u] * yu;
        }
      }
#pragma unroll
      for (int t = 0; t < DSUB; ++t) {
        acc[t] += __shfl_xor(acc[t], 1);
        acc[t] += __shfl_xor(acc[t], 2);
      }
      if (part == 0) {
#pragma unroll
        for (int t = 0; t < DP; ++t) ya[i * DP + t] = qi < nq && t < DSUB ? acc[t < DSUB ? t : 0] - mu[t] : 0.f;
      }
    } else {
      for (int e = lane; e < 16 * DP; e += 64) {
        const int i = e / DP, t = e % DP;
        const int64_t qi = q0 + i;
        float v = 0.f;
        if (qi < nq && t < DSUB) v = q[qi * d + s * DSUB + t] - mu[t];
        ya[e] = v;
      }
    }
    __syncthreads();
    if (lane < 16) {
      float a = 0.f;
#pragma unroll
      for (int t = 0; t < DP; ++t) a += ya[lane * DP + t] * ya[lane * DP + t];
      ny[lane] = a;
    }
    __syncthreads();

    float b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) b[ks] = ya[col * DP + ks * 4 + kg];
    const float nq_ = ny[col];
    const int64_t qi = q0 + col;  // this lane's query
    OUT *row = lut + (qi * m + s) * 256 + 4 * kg;
    float vals[16][4];
    float mx = 0.f;
#pragma unroll
    for (int tile = 0; tile < 16; ++tile) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      const int c = tile * 16 + col;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cc[c * DP + ks * 4 + kg], b[ks], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        vals[tile][r] = lc::clamp0(nq_ + nc[tile * 16 + 4 * kg + r] - 2.f * acc[r]);
        if constexpr (!std::is_same<OUT, float>::value) mx = fmaxf(mx, vals[tile][r]);
      }
      if constexpr (std::is_same<OUT, float>::value) {
        if (qi < nq) *reinterpret_cast<float4 *>(row + tile * 16) = make_float4(vals[tile][0], vals[tile][1],
                                                                                vals[tile][2], vals[tile][3]);
      }
    }
    if constexpr (!std::is_same<OUT, float>::value) {
      // the row maximum across the four lanes that share the query
      mx = fmaxf(mx, __shfl_xor(mx, 16));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      int e = 0;
      if (mx > 0.f) {
        frexpf(mx * (1.f / 32768.f), &e);  // mx / 2^15 = f * 2^e, f in [0.5, 1)
        e = e < -100 ? -100 : (e > 100 ? 100 : e);
      }
      const float inv = ldexpf(1.f, -e);
      if (qi < nq) {
        if (kg == 0) scale[qi * m + s] = ldexpf(1.f, e);
#pragma unroll
        for (int tile = 0; tile < 16; ++tile) {
          const uint32_t h0 = __half_as_ushort(__float2half_rn(vals[tile][0] * inv));
          const uint32_t h1 = __half_as_ushort(__float2half_rn(vals[tile][1] * inv));
          const uint32_t h2 = __half_as_ushort(__float2half_rn(vals[tile][2] * inv));
          const uint32_t h3 = __half_as_ushort(__float2half_rn(vals[tile][3] * inv));
          *reinterpret_cast<uint2 *>(row + tile * 16) = make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
        }
      }
    }
  }
}

// Query groups per block: as many as keep at least 4096 blocks in the grid
// (up to 8), so that the centroid staging is shared without idling CUs; one
// when the kernel projects the queries itself (that projection, not the
// staging, then dominates a group, and more blocks run it in parallel).
inline int lut_groups(int64_t nq, int m, bool projects) {
  if (projects) return 1;
  const int64_t g16 = lc::ceil_div(nq, 16);
  int g = 1;
  while (g < 8 && int64_t(lc::ceil_div(g16, 2 * g)) * m >= 4096) g *= 2;
  return g;
}

template <int DSUB>
hipError_t launch_dsub(const lc_index *ix, const float *q, int64_t nq, int dtype, void *lut, float *scale,
                       bool projected, hipStream_t st) {
  // projected queries [nq][d_pad] need no projection
  const float *proj = projected ? nullptr : ix->v.proj;
  const int groups = lut_groups(nq, ix->v.m, proj != nullptr);
  dim3 grid(lc::ceil_div(lc::ceil_div(nq, 16), groups), ix->v.m);
  const int d = projected ? ix->v.d_pad : ix->v.d;
  if (dtype == LC_LUT_F32)
    hipLaunchKernelGGL((lut_kernel<DSUB, float>), grid, dim3(64), 0, st, q, nq, d, proj, ix->v.m,
                       ix->v.centroids, static_cast<float *>(lut), scale, groups);
  else
    hipLaunchKernelGGL((lut_kernel<DSUB, __half>), grid, dim3(64), 0, st, q, nq, d, proj, ix->v.m,
                       ix->v.centroids, static_cast<__half *>(lut), scale, groups);
  return hipGetLastError();
}

// y' = P y for a batch: a block stages P (rows padded by one word, so that
// the lanes reading different rows at one column hit different banks) and
// kQB queries in LDS, then every thread forms some of the kQB x d_pad outputs,
// each summed over the inputs in order.  Without a projection the rows are
// copied.
constexpr int kQB = 32;

__global__ __launch_bounds__(256) void project_kernel(const float *__restrict__ q, int64_t nq, int d, int d_pad,
                                                      const float *__restrict__ proj, float *__restrict__ out) {
  extern __shared__ float sm[];
  float *P = sm;                       // [d_pad][d + 1]
  float *Y = sm + size_t(d_pad) * (d + 1);  // [kQB][d]
  const int64_t q0 = int64_t(blockIdx.x) * kQB;
  const int nqb = nq - q0 < kQB ? int(nq - q0) : kQB;
  for (int e = threadIdx.x; e < d_pad * d; e += blockDim.x) P[(e / d) * (d + 1) + e % d] = proj[e];
  for (int e = threadIdx.x; e < nqb * d; e += blockDim.x) Y[e] = q[q0 * d + e];
  __syncthreads();
  for (int e = threadIdx.x; e < nqb * d_pad; e += blockDim.x) {
    const int i = e / d_pad, r = e % d_pad;
    const float *pr = P + size_t(r) * (d + 1), *y = Y + size_t(i) * d;
    float v = 0.f;
    for (int u = 0; u < d; ++u) v += pr[u] * y[u];
    out[(q0 + i) * d_pad + r] = v;
  }
}

}  // namespace

// The same without staging, for a P too large for LDS: one wavefront per
// query, each row of P read as a contiguous run (lanes over its columns) and
// summed across the lanes.  Which kernel projects depends only on (d, d_pad),
// so every batch of one index is projected the same way.
namespace {
__global__ __launch_bounds__(256) void project_kernel_global(const float *__restrict__ q, int64_t nq, int d,
                                                             int d_pad, const float *__restrict__ proj,
                                                             float *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= nq) return;  // whole wavefronts leave together
  const float *y = q + i * d;
  for (int r = 0; r < d_pad; ++r) {
    const float *pr = proj + size_t(r) * d;
    float v = 0.f;
    for (int u = lane; u < d; u += 64) v += pr[u] * y[u];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) out[i * d_pad + r] = v;
  }
}
}  // namespace

int lc_launch_project(const lc_index *ix, const float *q, int64_t nq, float *out, hipStream_t st) {
  const int d = ix->v.d, dp = ix->v.d_pad;
  if (!ix->v.proj) {
    // no projection: the rows themselves (d == d_pad)
    return hipMemcpyAsync(out, q, size_t(nq) * d * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess
               ? LC_OK
               : LC_EHIP;
  }
  const size_t lds = (size_t(dp) * (d + 1) + size_t(kQB) * d) * sizeof(float);
  if (lds > size_t(ix->lds_per_cu)) {
    hipLaunchKernelGGL(project_kernel_global, dim3(int(lc::ceil_div(nq, 4))), dim3(256), 0, st, q, nq, d, dp,
                       ix->v.proj, out);
    return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
  }
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&project_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
    return LC_EHIP;
  hipLaunchKernelGGL(project_kernel, dim3(int(lc::ceil_div(nq, kQB))), dim3(256), lds, st, q, nq, d, dp,
                     ix->v.proj, out);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

namespace {

// Tables of the 2-level codec (Sec. 5.1) for kQR queries per block, with
// z = P y: the [m][256] entries -2 <z^s, C[s][c]> and the [2][coarse_k]
// entries ||z^h - C1[h][c]||^2, then zero padding up to the row stride.  One
// thread per table entry, its centroid row read once for the block's queries.
constexpr int kQR = 8;
static_assert(kQR == 8, "the query rows are read as two float4");

struct ResLutArgs {
  const float *q, *proj, *cent, *ccent;
  int64_t nq, row_bytes, row_floats;
  int d, d_pad, m, dsub, k1;
  int coff;         // float offset of the first-level entries in a row
  int f16;          // inner-product entries as fp16 with a power-of-two scale per row
  int skip_coarse;  // the first-level entries are written by coarse_lut_kernel
  unsigned char *lut;
  float *scale;     // [nq][m] (f16)
};

// First-level entries of the 2-level codec on MFMA: ||z - c||^2 =
// ||z||^2 + ||c||^2 - 2 <z, c> for 256 queries (four 16-query tiles per wave) and
// a chunk of 256 centroids of one half, staged once per block by a coalesced
// copy.  z = the query's half (queries already projected, or no projection);
// centroids past k are zero rows, not written.  The halves of unit-norm data
// have squared norms near 1/2, so the cancellation costs about 1e-7 of that.
template <int H>
__global__ __launch_bounds__(256) void coarse_lut_kernel(const float *__restrict__ z, int64_t nq, int zstride,
                                                          const float *__restrict__ ccent, int k1, int64_t stride,
                                                          int off, float *__restrict__ lut) {
  static_assert(H % 4 == 0, "a half of a multiple of 4 coordinates");
  constexpr int KS = H / 4;
  __shared__ float4 cc4[256 * H / 4];  // the chunk's centroids, row stride H
  __shared__ float nc[256];
  __shared__ float ya[4][16 * H];
  __shared__ float ny[4][16];
  const float *cc = reinterpret_cast<const float *>(cc4);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nch = (k1 + 255) / 256;
  const int half = blockIdx.y / nch, c0 = (blockIdx.y % nch) * 256;
  const int nvalid = k1 - c0 < 256 ? k1 - c0 : 256;
  const float4 *cs = reinterpret_cast<const float4 *>(ccent + (size_t(half) * k1 + c0) * H);
  for (int e = tid; e < 256 * H / 4; e += 256)
    cc4[e] = e < nvalid * H / 4 ? cs[e] : make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  {
    float a2 = 0.f;
#pragma unroll
    for (int t = 0; t < H; ++t) a2 += cc[tid * H + t] * cc[tid * H + t];
    nc[tid] = a2;
  }
  __syncthreads();
  float *yw = ya[wave];
  const int col = lane & 15, kg = lane >> 4;
  for (int qt = 0; qt < 4; ++qt) {
    const int64_t q0 = int64_t(blockIdx.x) * 256 + wave * 64 + qt * 16;
    if (q0 >= nq) break;
    for (int e = lane; e < 16 * H; e += 64) {
      const int i = e / H, t = e % H;
      const int64_t qi = q0 + i;
      yw[e] = qi < nq ? z[qi * zstride + half * H + t] : 0.f;
    }
    lc::wave_sync();
    if (lane < 16) {
      float a2 = 0.f;
#pragma unroll
      for (int t = 0; t < H; ++t) a2 += yw[lane * H + t] * yw[lane * H + t];
      ny[wave][lane] = a2;
    }
    lc::wave_sync();
    // v_mfma_f32_16x16x4_f32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
    // and receives D[4 (l / 16) + r][l % 16], r = 0..3
    float a[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = yw[col * H + ks * 4 + kg];
    for (int tile = 0; tile < 16; ++tile) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      const int c = tile * 16 + col;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], cc[c * H + ks * 4 + kg], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t qi = q0 + kg * 4 + r;
        if (qi < nq && c < nvalid)
          lut[qi * stride + off + int64_t(half) * k1 + c0 + c] = lc::clamp0(ny[wave][kg * 4 + r] + nc[c] - 2.f * acc[r]);
      }
    }
    lc::wave_sync();  // yw and ny are rewritten for the next tile
  }
}

template <int H>
int launch_coarse_lut(const ResLutArgs &a, const float *z, int zstride, hipStream_t st) {
  const dim3 grid(lc::ceil_div(a.nq, 256), 2 * ((a.k1 + 255) / 256));
  hipLaunchKernelGGL((coarse_lut_kernel<H>), grid, dim3(256), 0, st, z, a.nq, zstride, a.ccent, a.k1, a.row_floats,
                     a.coff, reinterpret_cast<float *>(a.lut));
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

__global__ __launch_bounds__(256) void lut_res_kernel(ResLutArgs a) {
  // [d_pad][kQR]: the block's queries side by side, so that one coordinate of all
  // of them is two 16-byte reads (every lane reads the same address)
  extern __shared__ float4 zs4[];
  __shared__ float red[4][kQR];
  float *zs = reinterpret_cast<float *>(zs4);
  const int64_t q0 = int64_t(blockIdx.x) * kQR;
  const int nqb = int(a.nq - q0 < kQR ? a.nq - q0 : kQR);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kQR * a.d_pad; e += blockDim.x) {
    const int qi = e % kQR, t = e / kQR;
    float v = 0.f;
    if (qi < nqb) {
      const float *y = a.q + (q0 + qi) * a.d;
      if (a.proj) {
        for (int u = 0; u < a.d; ++u) v += a.proj[int64_t(t) * a.d + u] * y[u];
      } else {
        v = y[t];
      }
    }
    zs[e] = v;
  }
  __syncthreads();
  auto zrow = [&](int t, float (&z)[kQR]) {
    const float4 lo = zs4[t * 2], hi = zs4[t * 2 + 1];
    z[0] = lo.x, z[1] = lo.y, z[2] = lo.z, z[3] = lo.w, z[4] = hi.x, z[5] = hi.y, z[6] = hi.z, z[7] = hi.w;
  };
  auto row = [&](int i) { return a.lut + (q0 + i) * a.row_bytes; };
  // inner-product rows, one row of 256 entries per pass (one entry per thread)
  for (int s = 0; s < a.m; ++s) {
    const int e = s * 256 + tid;
    float acc[kQR];
#pragma unroll
    for (int i = 0; i < kQR; ++i) acc[i] = 0.f;
    const float *c = a.cent + int64_t(e) * a.dsub;
    for (int t = 0; t < a.dsub; ++t) {
      const float cv = c[t];
      float z[kQR];
      zrow(s * a.dsub + t, z);
#pragma unroll
      for (int i = 0; i < kQR; ++i) acc[i] += z[i] * cv;
    }
#pragma unroll
    for (int i = 0; i < kQR; ++i) acc[i] *= -2.f;
    if (!a.f16) {
      for (int i = 0; i < nqb; ++i) reinterpret_cast<float *>(row(i))[e] = acc[i];
      continue;
    }
    // the row's largest magnitude per query: over the wave, then over the four waves
    float mx[kQR];
#pragma unroll
    for (int i = 0; i < kQR; ++i) {
      mx[i] = fabsf(acc[i]);
      for (int o = 32; o >= 1; o >>= 1) mx[i] = fmaxf(mx[i], __shfl_xor(mx[i], o));
    }
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < kQR; ++i) red[wave][i] = mx[i];
    __syncthreads();
    for (int i = 0; i < nqb; ++i) {
      const float m4 = fmaxf(fmaxf(red[0][i], red[1][i]), fmaxf(red[2][i], red[3][i]));
      int ex = 0;
      if (m4 > 0.f) {
        frexpf(m4 * (1.f / 32768.f), &ex);  // m4 / 2^15 = f * 2^ex, f in [0.5, 1)
        ex = ex < -100 ? -100 : (ex > 100 ? 100 : ex);
      }
      reinterpret_cast<__half *>(row(i))[e] = __float2half_rn(acc[i] * ldexpf(1.f, -ex));
      if (tid == 0) a.scale[(q0 + i) * a.m + s] = ldexpf(1.f, ex);
    }
    __syncthreads();  // red is rewritten for the next row
  }
  // first-level entries (unless on MFMA) and the padding, float32
  const int h = a.d_pad / 2;
  for (int e = tid; e < a.row_floats - a.coff; e += blockDim.x) {
    float acc[kQR];
#pragma unroll
    for (int i = 0; i < kQR; ++i) acc[i] = 0.f;
    if (e < 2 * a.k1) {
      if (a.skip_coarse) continue;
      const int half = e / a.k1;
      const float *c = a.ccent + int64_t(e) * h;
      for (int t = 0; t < h; ++t) {
        const float cv = c[t];
        float z[kQR];
        zrow(half * h + t, z);
#pragma unroll
        for (int i = 0; i < kQR; ++i) {
          const float df = z[i] - cv;
          acc[i] += df * df;
        }
      }
    }
    for (int i = 0; i < nqb; ++i) reinterpret_cast<float *>(row(i))[a.coff + e] = acc[i];
  }
}

int launch_res(const lc_index *ix, const float *q, int64_t nq, int dtype, void *lut, float *scale, bool projected,
               hipStream_t st) {
  if (dtype == LC_LUT_F16 && !scale) return LC_EINVAL;
  ResLutArgs a;
  a.q = q;
  a.proj = projected ? nullptr : ix->v.proj;
  a.cent = ix->v.centroids;
  a.ccent = ix->v.coarse_cent;
  a.nq = nq;
  a.row_bytes = lc_lut_row_bytes(ix, dtype);
  a.row_floats = a.row_bytes / 4;
  a.f16 = dtype == LC_LUT_F16;
  a.coff = ix->v.m * 256 * (a.f16 ? 2 : 4) / 4;
  a.scale = scale;
  a.d = projected ? ix->v.d_pad : ix->v.d;
  a.d_pad = ix->v.d_pad;
  a.m = ix->v.m;
  a.dsub = ix->dsub;
  a.k1 = ix->v.coarse_k;
  a.lut = static_cast<unsigned char *>(lut);
  const size_t lds = size_t(kQR) * a.d_pad * 4;
  if (lds > 65536) return LC_ENOTSUP;
  // first-level entries on MFMA when the queries need no projection here and the half has a kernel
  const int h = a.d_pad / 2;
  const bool mfma = !a.proj && (h == 16 || h == 24 || h == 32 || h == 36 || h == 48 || h == 56);
  a.skip_coarse = mfma ? 1 : 0;
  hipLaunchKernelGGL(lut_res_kernel, dim3(lc::ceil_div(nq, kQR)), dim3(256), lds, st, a);
  if (hipGetLastError() != hipSuccess) return LC_EHIP;
  if (!mfma) return LC_OK;
  switch (h) {
    case 16: return launch_coarse_lut<16>(a, q, a.d, st);
    case 24: return launch_coarse_lut<24>(a, q, a.d, st);
    case 32: return launch_coarse_lut<32>(a, q, a.d, st);
    case 36: return launch_coarse_lut<36>(a, q, a.d, st);
    case 48: return launch_coarse_lut<48>(a, q, a.d, st);
    default: return launch_coarse_lut<56>(a, q, a.d, st);
  }
}

}  // namespace

int lc_launch_lut(const lc_index *ix, const float *q, int64_t nq, int dtype, void *lut, float *scale,
                  bool projected, hipStream_t st) {
  if (dtype != LC_LUT_F32 && dtype != LC_LUT_F16) return LC_ENOTSUP;
  if (nq > int64_t(0x7FFFFFFF) * 16) return LC_EINVAL;
  if (ix->v.coarse_k > 0) return launch_res(ix, q, nq, dtype, lut, scale, projected, st);
  hipError_t e;
  switch (ix->dsub) {
#define CASE(DS) \
  case DS: e = launch_dsub<DS>(ix, q, nq, dtype, lut, scale, projected, st); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(6) CASE(8) CASE(12) CASE(16)
#undef CASE
    default: return LC_ENOTSUP;
  }
  return e == hipSuccess ? LC_OK : LC_EHIP;
}
