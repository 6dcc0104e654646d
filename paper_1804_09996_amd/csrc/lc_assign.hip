// Regression-codebook assignment of database vectors (Sec. 4.3, Eq. 7; block
// by block for the product codebook, Eq. 9): for vector i with
// G(x) = [q(x), q(g_1(x)), ..., q(g_k(x))] (a -1 link a zero column), the
// entry b of each block's codebook minimising
//
//   ||x - G beta_b||^2 = ||x||^2 - 2 beta_b^T (G^T x) + beta_b^T (G^T G) beta_b
//
// over the block's coordinates, lowest b on ties.  This is the step of the
// index build that touches every vector; the arg-min is an integer decided by
// floating point, so it is taken in float64 with the sums in ascending order
// and no fused multiply-adds (contraction is off in this file): the same
// arithmetic as a plain sequential loop, hence the same entry.
//
// One wavefront per vector: the k+1 decoded rows go to LDS as float32 (the
// centroids' own values), the projected vector as float64; the lanes share
// the Gram entries, then the codebook entries, and a wave arg-min picks the
// winner.
#include "lc_internal.h"

#pragma clang fp contract(off)

namespace {

using namespace lc;

struct AssignArgs {
  const float *x;  // [count][d] rows of vectors n0 .. n0 + count - 1
  int64_t n0, count;
  int n, d, d_pad, m, dsub, code_stride, deg0, k_reg, n_beta, m_beta, wpb;
  const float *proj, *cent, *beta;
  const uint8_t *codes;
  const int32_t *adj0;
  uint8_t *out;  // [count][m_beta]
  const float *ccent;        // 2-level codec: first-level centroids [2][coarse_k][d_pad/2], or null
  const uint32_t *ccodes;    // (c0 | c1 << 16)
  int coarse_k;
};

// LDS per wave: G [p][d_pad] (float32: the centroids' own values; float64 for
// the 2-level codec, whose rows are sums of two centroids), x' float64
// [d_pad], G^T G [p][p], G^T x [p], ||x'||^2
__host__ __device__ inline size_t wave_lds_bytes(int p, int d_pad, int gbytes) {
  return (size_t(p) * d_pad * gbytes + 7) / 8 * 8 + size_t(d_pad) * 8 + (size_t(p) * p + p + 1) * 8;
}

// ||x||^2 - 2 beta^T c + beta^T A beta for one codebook entry, in the order of
// a sequential loop: for each u, subtract 2 beta_u c_u, then add beta_u times
// the u-th row of A dotted with beta (ascending).  P > 0: the entry held in
// registers (P = k + 1 known at compile time); P = 0: any k, read in place.
template <int P>
__device__ __forceinline__ double entry_loss(const float *be, int p, const double *A, const double *Cv, double xx) {
  double l = xx;
  if constexpr (P > 0) {
    double bv[P];
#pragma unroll
    for (int v = 0; v < P; ++v) bv[v] = double(be[v]);
    // rows of A one at a time (a loop, so that A is not held in registers);
    // beta_u re-read from the cache, the inner product over the registers
#pragma unroll 1
    for (int u = 0; u < P; ++u) {
      const double bu = double(be[u]);
      l -= 2.0 * bu * Cv[u];
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < P; ++v) s += A[u * P + v] * bv[v];
      l += bu * s;
    }
  } else {
    for (int u = 0; u < p; ++u) {
      const double bu = double(be[u]);
      l -= 2.0 * bu * Cv[u];
      double s = 0.0;
      for (int v = 0; v < p; ++v) s += A[u * p + v] * double(be[v]);
      l += bu * s;
    }
  }
  return l;
}

template <int P, typename GT>
__global__ __launch_bounds__(512) void beta_assign_kernel(AssignArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = P > 0 ? P : a.k_reg + 1, dp = a.d_pad;
  unsigned char *base = smem + size_t(wave) * wave_lds_bytes(p, dp, int(sizeof(GT)));
  GT *G = reinterpret_cast<GT *>(base);
  double *xv = reinterpret_cast<double *>(base + (size_t(p) * dp * sizeof(GT) + 7) / 8 * 8);
  double *A = xv + dp;
  double *Cv = A + p * p;
  double *XX = Cv + p;
  const int bw = dp / a.m_beta;
  for (int64_t r = int64_t(blockIdx.x) * a.wpb + wave; r < a.count; r += int64_t(gridDim.x) * a.wpb) {
    const int64_t i = a.n0 + r;
    const float *y = a.x + r * a.d;
    // x' = P x in float64, each coordinate summed over the input in order
    for (int t = lane; t < dp; t += 64) {
      double v;
      if (a.proj) {
        v = 0.0;
        for (int u = 0; u < a.d; ++u) v += double(a.proj[int64_t(t) * a.d + u]) * double(y[u]);
      } else {
        v = double(y[t]);
      }
      xv[t] = v;
    }
    // decoded rows: row j is q(g_j), g_0 = i
    for (int e = lane; e < p * a.m; e += 64) {
      const int j = e / a.m, s = e % a.m;
      const int32_t src = j == 0 ? int32_t(i) : a.adj0[i * a.deg0 + (j - 1)];
      GT *dst = G + j * dp + s * a.dsub;
      if (src < 0 || src >= a.n) {
        for (int t = 0; t < a.dsub; ++t) dst[t] = GT(0);  // a missing link is a zero vector
      } else {
        const float *c = a.cent + (int64_t(s) * 256 + a.codes[int64_t(src) * a.code_stride + s]) * a.dsub;
        for (int t = 0; t < a.dsub; ++t) dst[t] = GT(c[t]);
        if (a.ccent) {  // 2-level codec: plus the first-level centroid's part, summed in float64
          const int half = s >= a.m / 2;
          const uint32_t cc = a.ccodes[src];
          const float *c1 = a.ccent + (int64_t(half) * a.coarse_k + (half ? cc >> 16 : cc & 0xFFFFu)) * (dp / 2) +
                            (s - half * (a.m / 2)) * a.dsub;
          for (int t = 0; t < a.dsub; ++t) dst[t] = GT(double(dst[t]) + double(c1[t]));
        }
      }
    }
    wave_sync();
    for (int jb = 0; jb < a.m_beta; ++jb) {
      const int t0 = jb * bw, t1 = t0 + bw;
      // G^T G, G^T x and ||x||^2 over the block's coordinates
      for (int e = lane; e < p * p + p + 1; e += 64) {
        double s = 0.0;
        if (e < p * p) {
          const GT *ga = G + (e / p) * dp, *gb = G + (e % p) * dp;
          for (int t = t0; t < t1; ++t) s += double(ga[t]) * double(gb[t]);
          A[e] = s;
        } else if (e < p * p + p) {
          const GT *ga = G + (e - p * p) * dp;
          for (int t = t0; t < t1; ++t) s += double(ga[t]) * xv[t];
          Cv[e - p * p] = s;
        } else {
          for (int t = t0; t < t1; ++t) s += xv[t] * xv[t];
          *XX = s;
        }
      }
      wave_sync();
      // every codebook entry of the block, lanes in turn; the best (loss, entry)
      double best = 0.0;
      int bi = -1;
      const float *B = a.beta + int64_t(jb) * a.n_beta * p;
      for (int b = lane; b < a.n_beta; b += 64) {
        const double l = entry_loss<P>(B + int64_t(b) * p, p, A, Cv, *XX);
        if (bi < 0 || l < best) {  // entries of a lane ascend: a tie keeps the lower
          best = l;
          bi = b;
        }
      }
      // wave arg-min: smallest loss, then smallest entry
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        const bool take = oi >= 0 && (bi < 0 || ob < best || (ob == best && oi < bi));
        if (take) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) a.out[r * a.m_beta + jb] = uint8_t(bi);
      wave_sync();  // the Gram of the next block overwrites this one
    }
  }
}

template <int P, typename GT>
int launch_p(const AssignArgs &a, int64_t blocks, size_t lds, hipStream_t st) {
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&beta_assign_kernel<P, GT>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
    return LC_EHIP;
  hipLaunchKernelGGL((beta_assign_kernel<P, GT>), dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

}  // namespace

int lc_launch_assign(const lc_index *ix, const float *x, int64_t n0, int64_t count, uint8_t *out, hipStream_t st) {
  const lc_index_view &v = ix->v;
  AssignArgs a;
  a.x = x;
  a.n0 = n0;
  a.count = count;
  a.n = v.n;
  a.d = v.d;
  a.d_pad = v.d_pad;
  a.m = v.m;
  a.dsub = ix->dsub;
  a.code_stride = v.code_stride;
  a.deg0 = v.deg0;
  a.k_reg = v.k_reg;
  a.n_beta = v.n_beta;
  a.m_beta = v.m_beta;
  a.proj = v.proj;
  a.cent = v.centroids;
  a.beta = v.beta;
  a.codes = v.codes;
  a.adj0 = v.adj0;
  a.out = out;
  a.ccent = v.coarse_k > 0 ? v.coarse_cent : nullptr;
  a.ccodes = reinterpret_cast<const uint32_t *>(v.coarse_codes);
  a.coarse_k = v.coarse_k;
  const bool two = a.ccent != nullptr;
  const size_t per_wave = wave_lds_bytes(v.k_reg + 1, v.d_pad, two ? 8 : 4);
  int wpb = int(size_t(ix->lds_per_cu) / per_wave);
  if (wpb > 8) wpb = 8;
  if (wpb < 1) return LC_ENOTSUP;
  a.wpb = wpb;
  const size_t lds = per_wave * wpb;
  int64_t blocks = (count + wpb - 1) / wpb;
  if (blocks > int64_t(ix->num_cus) * 4) blocks = int64_t(ix->num_cus) * 4;
  const int p = v.k_reg + 1;
  if (two) return launch_p<0, double>(a, blocks, lds, st);
  return p == 9    ? launch_p<9, float>(a, blocks, lds, st)
         : p == 17 ? launch_p<17, float>(a, blocks, lds, st)
         : p == 33 ? launch_p<33, float>(a, blocks, lds, st)
                   : launch_p<0, float>(a, blocks, lds, st);
}
