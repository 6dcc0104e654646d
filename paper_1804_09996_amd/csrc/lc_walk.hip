// First stage of the search (Sec. 2; Sec. 4.1): greedy descent on the upper
// levels, then a best-first walk on level 0 over nodes that hold only PQ codes,
// scored by asymmetric distances from the per-query table.
//
// One wavefront owns one query at a time (grid-stride over queries):
//  * the query's table (m x 256 float32) is staged in LDS;
//  * the pool W (<= ef_eff keys, sorted, "expanded" flag in bit 31) is an LDS
//    array;
//  * the visited set is exact: an LDS open-addressing table of node ids, and
//    once that table is half full, a per-wave bitset in the workspace (cleared
//    again before the next query);
//  * each expansion reads one 32-link row of adj0 (lanes 0..31), tests and
//    marks the links as visited, gathers the codes of the fresh ones (lanes L
//    and L+32 each sum half of the sub-spaces, in a fixed order), and merges
//    the keys that can enter W.
//
// Expanding the best unexpanded entry of W, evaluating all its fresh links,
// and merging them at once leaves W, the expansion count E and the evaluation
// count D exactly as in the textbook two-heap form: keys are unique, keeping
// the best ef_eff of a union is associative, and a candidate that is no longer
// in W is worse than every entry of W, so it would end the two-heap loop.
#include "lc_internal.h"

namespace {

using namespace lc;

struct WalkArgs {
  const uint8_t *codes;
  const int32_t *adj0, *up_base, *adj_up;
  const float *lut;
  const int32_t *ef;
  int32_t ef_max, S;
  int64_t nq, n_up_rows;
  int32_t n, code_stride, deg0, deg_up, entry, max_level;
  int32_t w_cap, hash_bits;
  uint32_t *bits;
  int64_t words;
  int32_t *cand_ids;
  float *cand_adc;
  int32_t *cand_n, *stats;
};

// Sum of LUT[s][code[s]] over one half of the sub-spaces (s ascending).
template <int M>
__device__ __forceinline__ float adc_half(const float *lut, const uint8_t *codes, int cs, int32_t id,
                                          int half) {
  constexpr int HB = M / 2;  // code bytes per half
  const uint8_t *row = codes + size_t(id) * cs + half * HB;
  const float *L = lut + half * HB * 256;
  float acc = 0.f;
  if constexpr (HB % 16 == 0) {
#pragma unroll
    for (int i = 0; i < HB / 16; ++i) {
      const uint4 w = reinterpret_cast<const uint4 *>(row)[i];
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int t = 0; t < 16; ++t) acc += L[(i * 16 + t) * 256 + ((ws[t >> 2] >> (8 * (t & 3))) & 0xFFu)];
    }
  } else if constexpr (HB % 8 == 0) {
#pragma unroll
    for (int i = 0; i < HB / 8; ++i) {
      const uint2 w = reinterpret_cast<const uint2 *>(row)[i];
      const uint32_t ws[2] = {w.x, w.y};
#pragma unroll
      for (int t = 0; t < 8; ++t) acc += L[(i * 8 + t) * 256 + ((ws[t >> 2] >> (8 * (t & 3))) & 0xFFu)];
    }
  } else {
    static_assert(HB % 4 == 0, "m must be a multiple of 8");
#pragma unroll
    for (int i = 0; i < HB / 4; ++i) {
      const uint32_t w = reinterpret_cast<const uint32_t *>(row)[i];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc += L[(i * 4 + t) * 256 + ((w >> (8 * t)) & 0xFFu)];
    }
  }
  return acc;
}

// Key of node `id` (lanes L and L+32 carry the same id and validity).
template <int M>
__device__ __forceinline__ uint64_t eval_key(const float *lut, const uint8_t *codes, int cs, int32_t id,
                                             bool valid, int lane) {
  float part = 0.f;
  if (valid) part = adc_half<M>(lut, codes, cs, id, lane >> 5);
  const float lo = __shfl(part, lane & 31);
  const float hi = __shfl(part, (lane & 31) + 32);
  return valid ? make_key(lo + hi, id) : kKeyMax;
}

// Test-and-set of `id` in the visited set; true when `id` was not there.
__device__ __forceinline__ bool visit(uint32_t *hash, uint32_t hmask, int hshift, int32_t id, bool ovf,
                                      uint32_t *bits) {
  uint32_t h = (uint32_t(id) * 0x9E3779B1u) >> hshift;
  if (!ovf) {
    for (;;) {
      const uint32_t old = atomicCAS(&hash[h], kEmpty, uint32_t(id));
      if (old == kEmpty) return true;
      if (old == uint32_t(id)) return false;
      h = (h + 1) & hmask;
    }
  }
  for (;;) {
    const uint32_t v = hash[h];
    if (v == uint32_t(id)) return false;
    if (v == kEmpty) break;
    h = (h + 1) & hmask;
  }
  const uint32_t bit = 1u << (uint32_t(id) & 31u);
  const uint32_t old = atomicOr(&bits[uint32_t(id) >> 5], bit);
  return (old & bit) == 0;
}

// First index of W[0..n) whose key is >= k.
__device__ __forceinline__ int lower_bound(const uint64_t *W, int n, uint64_t k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pure_key(W[mid]) < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Number of entries of the sorted nk[0..n) smaller than k.
__device__ __forceinline__ int count_less(const uint64_t *nk, int n, uint64_t k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nk[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <int M>
__global__ __launch_bounds__(64) void walk_kernel(WalkArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  float *lut = reinterpret_cast<float *>(smem);
  uint64_t *W = reinterpret_cast<uint64_t *>(smem + M * 256 * 4);
  uint64_t *nk = W + a.w_cap;
  uint32_t *hash = reinterpret_cast<uint32_t *>(nk + 32);
  const int H = 1 << a.hash_bits;
  const uint32_t hmask = uint32_t(H - 1);
  const int hshift = 32 - a.hash_bits;
  const int hlimit = H / 2;
  uint32_t *bits = a.bits + int64_t(blockIdx.x) * a.words;

  for (int64_t q = blockIdx.x; q < a.nq; q += gridDim.x) {
    const int32_t efq = a.ef ? a.ef[q] : a.ef_max;
    if (efq < 1 || efq > a.ef_max) {
      for (int i = lane; i < a.S; i += 64) {
        a.cand_ids[q * a.S + i] = -1;
        a.cand_adc[q * a.S + i] = __builtin_inff();
      }
      if (lane == 0) {
        a.cand_n[q] = -1;
        if (a.stats) {
          a.stats[2 * q] = 0;
          a.stats[2 * q + 1] = 0;
        }
      }
      continue;
    }
    const int efe = efq > a.S ? efq : a.S;

    // stage the table, clear the visited table
    const float4 *src = reinterpret_cast<const float4 *>(a.lut + q * (M * 256));
    for (int i = lane; i < M * 64; i += 64) reinterpret_cast<float4 *>(lut)[i] = src[i];
    for (int i = lane; i < H; i += 64) hash[i] = kEmpty;
    wave_sync();

    // greedy descent on levels max_level .. 1
    int32_t cur = a.entry;
    uint64_t curkey = eval_key<M>(lut, a.codes, a.code_stride, cur, true, lane);
    for (int l = a.max_level; l >= 1; --l) {
      for (;;) {
        const int64_t row = int64_t(a.up_base[cur]) + l - 1;
        int32_t nb = -1;
        if (l32 < a.deg_up && row >= 0 && row < a.n_up_rows) nb = a.adj_up[row * a.deg_up + l32];
        if (nb >= a.n) nb = -1;  // a malformed link is ignored rather than followed
        const uint64_t k = eval_key<M>(lut, a.codes, a.code_stride, nb, nb >= 0, lane);
        const uint64_t mn = wave_min64(k);
        if (mn < curkey) {
          curkey = mn;
          cur = key_id(mn);
        } else {
          break;
        }
      }
    }

    // best-first walk on level 0
    if (lane == 0) {
      W[0] = curkey;
      visit(hash, hmask, hshift, cur, false, bits);
    }
    int nw = 1, fu = 0, E = 0, D = 0, hcount = 1;
    bool ovf = false;
    wave_sync();
    while (fu < nw) {
      const uint64_t ck = W[fu];
      const int32_t c = key_id(ck);
      wave_sync();
      if (lane == 0) W[fu] = ck | kExpanded;
      ++E;
      int32_t nb = l32 < a.deg0 ? a.adj0[int64_t(c) * a.deg0 + l32] : -1;
      if (nb >= a.n) nb = -1;  // a malformed link is ignored rather than followed
      if (!ovf && hcount + a.deg0 > hlimit) ovf = true;
      int fresh = 0;
      if (lane < 32 && nb >= 0) fresh = visit(hash, hmask, hshift, nb, ovf, bits) ? 1 : 0;
      fresh = __shfl(fresh, l32);
      const int nf = __popcll(__ballot(fresh) & 0xFFFFFFFFull);
      D += nf;
      if (!ovf) hcount += nf;
      uint64_t k = eval_key<M>(lut, a.codes, a.code_stride, nb, fresh != 0, lane);
      const uint64_t wmax = (nw == efe) ? pure_key(W[nw - 1]) : kKeyMax;
      if (k >= wmax) k = kKeyMax;
      const int nn = __popcll(__ballot(k != kKeyMax) & 0xFFFFFFFFull);
      int p0 = fu;
      if (nn > 0) {
        k = sort32(k, lane);
        if (lane < nn) nk[lane] = k;
        wave_sync();
        const int pos = lane < nn ? lower_bound(W, nw, k) : 0;
        const int lo = __shfl(pos, 0);
        // move the old entries [lo, nw) up, highest chunk first
        for (int top = nw; top > lo; top -= 64) {
          const int idx = top - 64 + lane;
          uint64_t v = 0;
          int np = -1;
          if (idx >= lo && idx < top) {
            v = W[idx];
            np = idx + count_less(nk, nn, pure_key(v));
          }
          wave_sync();
          if (np >= 0 && np < efe) W[np] = v;
          wave_sync();
        }
        if (lane < nn && pos + lane < efe) W[pos + lane] = k;
        const int fu_new = fu < lo ? fu : fu + count_less(nk, nn, pure_key(ck));
        p0 = fu_new < lo ? fu_new : lo;
        nw = nw + nn < efe ? nw + nn : efe;
        wave_sync();
      }
      wave_sync();
      // first unexpanded entry at or after p0 (everything before it is expanded)
      int nfu = nw;
      for (int base = p0; base < nw; base += 64) {
        const int idx = base + lane;
        const bool un = idx < nw && (W[idx] & kExpanded) == 0;
        const uint64_t bm = __ballot(un);
        if (bm) {
          nfu = base + __ffsll((unsigned long long)bm) - 1;
          break;
        }
      }
      fu = nfu;
    }

    // short-list = the first min(S, |W|) entries of W
    const int ns = a.S < nw ? a.S : nw;
    for (int i = lane; i < a.S; i += 64) {
      if (i < ns) {
        const uint64_t v = W[i];
        a.cand_ids[q * a.S + i] = key_id(v);
        a.cand_adc[q * a.S + i] = key_dist(v);
      } else {
        a.cand_ids[q * a.S + i] = -1;
        a.cand_adc[q * a.S + i] = __builtin_inff();
      }
    }
    if (lane == 0) {
      a.cand_n[q] = ns;
      if (a.stats) {
        a.stats[2 * q] = E;
        a.stats[2 * q + 1] = D;
      }
    }
    if (ovf) {
      for (int64_t i = lane; i < a.words; i += 64) bits[i] = 0u;
      __threadfence();
    }
    wave_sync();
  }
}

struct WalkPlan {
  int w_cap, hash_bits, lds_bytes, grid;
};

template <int M>
int lds_bytes_for(int w_cap, int hash_bits) {
  return M * 256 * 4 + w_cap * 8 + 32 * 8 + (1 << hash_bits) * 4;
}

int pick_hash_bits(int w_cap) {
  // room for about 16 evaluations per pool slot before the bitset takes over
  int want = 16 * w_cap * 2, bits = 10;
  while ((1 << bits) < want && bits < 13) ++bits;
  return bits;
}

template <int M>
WalkPlan plan_for(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S) {
  WalkPlan p;
  int ef_eff = ef_max > S ? ef_max : S;
  p.w_cap = (ef_eff + 63) / 64 * 64;
  p.hash_bits = pick_hash_bits(p.w_cap);
  p.lds_bytes = lds_bytes_for<M>(p.w_cap, p.hash_bits);
  int per_cu = ix->lds_per_cu / p.lds_bytes;
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 32) per_cu = 32;
  int64_t g = int64_t(per_cu) * ix->num_cus;
  if (g > nq) g = nq;
  if (g < 1) g = 1;
  p.grid = int(g);
  return p;
}

template <int M>
size_t ws_bytes_m(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S) {
  WalkPlan p = plan_for<M>(ix, nq, ef_max, S);
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  return size_t(p.grid) * size_t(words) * 4;
}

template <int M>
int launch_m(const lc_index *ix, const float *lut, int64_t nq, const int32_t *ef, int32_t ef_max,
             int32_t S, int32_t *cand_ids, float *cand_adc, int32_t *cand_n, int32_t *stats, void *ws,
             size_t ws_bytes, hipStream_t st) {
  WalkPlan p = plan_for<M>(ix, nq, ef_max, S);
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  if (ws_bytes < size_t(p.grid) * size_t(words) * 4) return LC_ENOSPC;
  if (p.lds_bytes > ix->lds_per_cu) return LC_ENOTSUP;
  WalkArgs a;
  a.codes = ix->v.codes;
  a.adj0 = ix->v.adj0;
  a.up_base = ix->v.up_base;
  a.adj_up = ix->v.adj_up;
  a.lut = lut;
  a.ef = ef;
  a.ef_max = ef_max;
  a.S = S;
  a.nq = nq;
  a.n = ix->v.n;
  a.n_up_rows = ix->v.n_up_rows;
  a.code_stride = ix->v.code_stride;
  a.deg0 = ix->v.deg0;
  a.deg_up = ix->v.deg_up;
  a.entry = ix->v.entry;
  a.max_level = ix->v.max_level;
  a.w_cap = p.w_cap;
  a.hash_bits = p.hash_bits;
  a.bits = static_cast<uint32_t *>(ws);
  a.words = words;
  a.cand_ids = cand_ids;
  a.cand_adc = cand_adc;
  a.cand_n = cand_n;
  a.stats = stats;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&walk_kernel<M>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_bytes) != hipSuccess)
    return LC_EHIP;
  hipLaunchKernelGGL(walk_kernel<M>, dim3(p.grid), dim3(64), p.lds_bytes, st, a);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

}  // namespace

#define LC_FOR_EACH_M(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

size_t lc_walk_workspace_bytes(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S) {
  switch (ix->v.m) {
#define CASE(MM) \
  case MM: return ws_bytes_m<MM>(ix, nq, ef_max, S);
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return 0;
  }
}

int lc_launch_walk(const lc_index *ix, const void *lut, int dtype, const float *scale, int64_t nq,
                   const int32_t *ef, int32_t ef_max, int32_t S, int32_t *cand_ids, float *cand_adc,
                   int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, hipStream_t st) {
  (void)scale;
  if (dtype != LC_LUT_F32) return LC_ENOTSUP;
  switch (ix->v.m) {
#define CASE(MM)                                                                                  \
  case MM:                                                                                        \
    return launch_m<MM>(ix, static_cast<const float *>(lut), nq, ef, ef_max, S, cand_ids, cand_adc, \
                        cand_n, stats, ws, ws_bytes, st);
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return LC_ENOTSUP;
  }
}
