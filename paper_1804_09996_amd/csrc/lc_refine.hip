// Second stage of the search (Sec. 4.1 "Refinement strategy"): every
// short-list entry i is rebuilt from its own code and the codes of its first
// k graph links, weighted by its regression vector (Sec. 4.2 Eq. 5 with the
// codebook entry of Sec. 4.3 Eq. 7):
//
//   x~_i = sum_{j=0..k} beta[b_i][j] * q(g_j(i)),  g_0 = i, g_j = adj0[i][j-1]
//   d~   = || P y - x~_i ||^2
//
// and the K smallest (d~, id) are kept.  With a product regression codebook
// (Sec. 4.3, Eq. 9) the coordinates are cut into m_beta equal blocks of m /
// m_beta whole sub-spaces, and block jb of x~ takes its weights from codebook
// jb at the vector's byte b_i[jb].  A block stages the centroids of all
// sub-spaces in LDS once; each wavefront then owns one query at a time.  L
// lanes share a candidate (L = 2 for m <= 16, else 4), lane part p
// accumulating the sub-spaces s = p mod L in registers; the candidate's
// distance is the sum of the L partial sums in a fixed order.  A candidate's
// rows are dependent gathers (its links, then their codes), so more
// candidates per wavefront (fewer lanes each) means fewer rounds of them.
// The short-list keys are sorted in LDS by a bitonic network and the first K
// written out.
//
// Precision form: the centroids are staged in LDS as bfloat16 and the beta
// weights rounded to bfloat16, products accumulated in float32; the best
// K' = min(S, 2K) candidates of that pass are then re-scored with exactly the
// float32 arithmetic of the plain kernel (float32 centroids read from global
// memory) and re-sorted, so every returned distance is the plain one.
#include "lc_internal.h"

namespace {

using namespace lc;

struct RefineArgs {
  const float *q;
  int64_t nq;
  int d, d_pad;
  const float *proj, *cent;
  const uint8_t *codes;
  int code_stride;
  const int32_t *adj0;
  int n, n_beta, m_beta, deg0, k_reg;
  const float *beta;
  const uint8_t *beta_idx;
  const int32_t *cand_ids, *cand_n;
  int S, K, S_pad, K2, K2_pad, wpb;
  int32_t *out_ids;
  float *out_d;
  // 2-level codec: first-level centroids [2][coarse_k][d_pad/2] and codes (c0 | c1 << 16), or null
  const float *ccent;
  const uint32_t *ccodes;
  int coarse_k;
};

template <int CS>
struct CodeRow {
  uint32_t w[CS >= 16 ? CS / 4 : 2];
  __device__ __forceinline__ void load(const uint8_t *p) {
    if constexpr (CS >= 16) {
#pragma unroll
      for (int i = 0; i < CS / 16; ++i) {
        const uint4 v = reinterpret_cast<const uint4 *>(p)[i];
        w[4 * i] = v.x;
        w[4 * i + 1] = v.y;
        w[4 * i + 2] = v.z;
        w[4 * i + 3] = v.w;
      }
    } else {
      const uint2 v = *reinterpret_cast<const uint2 *>(p);
      w[0] = v.x;
      w[1] = v.y;
    }
  }
  __device__ __forceinline__ uint32_t byte(int s) const { return (w[s >> 2] >> (8 * (s & 3))) & 0xFFu; }
};

// NB consecutive code bytes (NB = 4 or 8, aligned to NB) of one code row.
template <int NB>
struct CodePiece {
  uint32_t w[NB / 4];
  __device__ __forceinline__ void load(const uint8_t *p) {
    if constexpr (NB == 8) {
      const uint2 v = *reinterpret_cast<const uint2 *>(p);
      w[0] = v.x;
      w[NB == 8 ? 1 : 0] = v.y;
    } else {
      static_assert(NB == 4, "code piece");
      w[0] = *reinterpret_cast<const uint32_t *>(p);
    }
  }
  __device__ __forceinline__ uint32_t byte(int u) const { return (w[u >> 2] >> (8 * (u & 3))) & 0xFFu; }
};

// Centroid element as float32: float32 storage, or bfloat16 (top 16 bits).
[[maybe_unused]] __device__ __forceinline__ float cval(const float *C, int i) { return C[i]; }
[[maybe_unused]] __device__ __forceinline__ float cval(const uint16_t *C, int i) { return __uint_as_float(uint32_t(C[i]) << 16); }

// One centroid row (DSUB elements from index base) as float32.  bfloat16 rows
// of an even length are read as 32-bit words, two elements each (a row starts
// at a multiple of DSUB elements, so the words are aligned): half the LDS
// reads of element-wise 16-bit loads.
template <int DSUB>
__device__ __forceinline__ void crow(const float *C, int base, float *out) {
#pragma unroll
  for (int q = 0; q < DSUB; ++q) out[q] = C[base + q];
}
template <int DSUB>
__device__ __forceinline__ void crow(const uint16_t *C, int base, float *out) {
  if constexpr (DSUB % 2 == 0) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(C + base);
#pragma unroll
    for (int h = 0; h < DSUB / 2; ++h) {
      const uint32_t v = w[h];
      out[2 * h] = __uint_as_float(v << 16);
      out[2 * h + 1] = __uint_as_float(v & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int q = 0; q < DSUB; ++q) out[q] = cval(C, base + q);
  }
}

// Round a float32 to the nearest bfloat16 (ties to even), returned as float32.
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// Lanes per candidate: two while the accumulators fit, else four.
template <int M>
constexpr int lanes_per_cand() {
  return M <= 16 ? 2 : 4;
}

// This lane part's share of || y' - x~_id ||^2 over the sub-spaces BlockMap
// gives it: with two lanes [part U, part U + U) (one aligned piece of each
// code row), with four lanes a whole code row is loaded and its bytes picked.
// Which sub-spaces a lane part sums, and the blocks of the product codebook
// they fall in.  MB blocks of SPB = M / MB sub-spaces; accumulator u of part
// p is sub-space sub(u, p): with two lanes the contiguous [p U, p U + U) (one
// aligned piece of each code row), with four lanes s = p + 4u (the whole code
// row is loaded and the word holding byte s is u, known at compile time).
// Sub-space u lies in slot slot(u) of the part's NJ distinct blocks, and slot
// sl is block block(sl, p).
template <int M, int MB>
struct BlockMap {
  static constexpr int L = lanes_per_cand<M>();
  static constexpr int U = M / L;
  static constexpr int SPB = M / MB;
  static_assert(M % MB == 0, "blocks hold whole sub-spaces");
  static constexpr bool kOne = L == 2 ? SPB >= U : MB == 1;
  // four lanes, SPB a multiple of 4: block (p + 4u) / SPB = 4u / SPB for every p
  static constexpr bool kStrideAligned = L == 4 && SPB % 4 == 0;
  static constexpr int NJ = kOne ? 1 : L == 2 ? U / SPB : kStrideAligned ? MB : U;
  static_assert(L == 4 || kOne || U % SPB == 0, "a two-lane part holds whole blocks");
  __device__ static constexpr int sub(int u, int p) { return L == 2 ? p * U + u : p + L * u; }
  __device__ static constexpr int slot(int u) {
    return kOne ? 0 : L == 2 ? u / SPB : kStrideAligned ? (4 * u) / SPB : u;
  }
  __device__ static int block(int sl, int p) {
    if constexpr (kOne) return L == 2 ? (p * U) / SPB : 0;
    else if constexpr (L == 2) return p * NJ + sl;
    else if constexpr (kStrideAligned) return sl;
    else return (p + 4 * sl) / SPB;
  }
};

// A candidate whose code-book bytes are out of range is malformed input.
template <int MB>
__device__ __forceinline__ bool beta_ok(const RefineArgs &a, int32_t id) {
  bool ok = true;
#pragma unroll
  for (int jb = 0; jb < MB; ++jb) ok = ok && a.beta_idx[int64_t(id) * MB + jb] < a.n_beta;
  return ok;
}

// Four consecutive 32-bit words from a 4-byte aligned address: one 16-byte
// load (a global_load_dwordx4), so that four regression rows cost one memory
// request for their links and one per codebook row for their weights.
struct __attribute__((aligned(4))) Words4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ Words4 load4(const void *p) { return *reinterpret_cast<const Words4 *>(p); }

template <int M, int DSUB, int CS, typename CT, bool BF16W, int MB>
__device__ __forceinline__ float part_dist(const RefineArgs &a, const CT *C, const float *yv, int32_t id,
                                           int part) {
  constexpr int L = lanes_per_cand<M>();
  constexpr int U = M / L;
  using BM = BlockMap<M, MB>;
  constexpr int NJ = BM::NJ;
  static_assert(L == 4 || U == 4 || U == 8, "two lanes take 4 or 8 sub-spaces each");
  // The rows are r = 0..k: r = 0 is the vector's own code, r >= 1 its link
  // r-1.  They go in batches of RB rows; with RB >= 4 a group of four rows
  // shares one load of its links and one load per codebook row of weights (a
  // product codebook's rows do not stay in the L1 cache, so this is what
  // bounds its cost).  A part spanning many blocks keeps fewer rows in
  // registers and loads them one by one.  Code rows are fetched SB at a time,
  // then summed.
  constexpr int RB = (CS <= 16 && NJ <= 2) ? 8 : NJ <= 4 ? 4 : NJ <= 8 ? 2 : 1;
  constexpr int SB = RB < 4 ? RB : CS >= 64 ? 2 : 4;
  float acc[U * DSUB];
#pragma unroll
  for (int t = 0; t < U * DSUB; ++t) acc[t] = 0.f;
  // the codebook row of every block this part touches (offsets into beta)
  int bw[NJ];
#pragma unroll
  for (int sl = 0; sl < NJ; ++sl) {
    const int jb = BM::block(sl, part);
    bw[sl] = (jb * a.n_beta + int(a.beta_idx[int64_t(id) * MB + jb])) * (a.k_reg + 1);
  }
  const int k = a.k_reg;
  const int32_t *links = a.adj0 + int64_t(id) * a.deg0;
  for (int r0 = 0; r0 <= k; r0 += RB) {
    int32_t lk[RB];
    float wv[RB][NJ];
    if constexpr (RB >= 4) {
#pragma unroll
      for (int h = 0; h < RB / 4; ++h) {
        const int rb = r0 + 4 * h;
        if (rb >= 1 && rb + 3 <= k) {  // links rb-1 .. rb+2 in one load
          const Words4 v = load4(links + rb - 1);
          lk[4 * h] = int32_t(v.x), lk[4 * h + 1] = int32_t(v.y), lk[4 * h + 2] = int32_t(v.z),
                  lk[4 * h + 3] = int32_t(v.w);
        } else {
          // the first group and the tail: rows clamped into 1..k, so every read is in bounds
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int r = rb + t;
            lk[4 * h + t] = links[(r < 1 ? 1 : r > k ? k : r) - 1];
          }
        }
#pragma unroll
        for (int sl = 0; sl < NJ; ++sl) {
          if (rb + 3 <= k) {  // weights rb .. rb+3 of the block's codebook row in one load
            const Words4 v = load4(a.beta + bw[sl] + rb);
            wv[4 * h][sl] = __uint_as_float(v.x), wv[4 * h + 1][sl] = __uint_as_float(v.y);
            wv[4 * h + 2][sl] = __uint_as_float(v.z), wv[4 * h + 3][sl] = __uint_as_float(v.w);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) wv[4 * h + t][sl] = a.beta[bw[sl] + (rb + t > k ? k : rb + t)];
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < RB; ++t) {
        const int r = r0 + t;
        const int rc = r > k ? k : r;
        lk[t] = links[(rc < 1 ? 1 : rc) - 1];
#pragma unroll
        for (int sl = 0; sl < NJ; ++sl) wv[t][sl] = a.beta[bw[sl] + rc];
      }
    }
    int32_t g[RB];
    float wj[RB][NJ];
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      const int r = r0 + t;
      const int32_t gj = r == 0 ? id : lk[t];
      const bool ok = r <= k && gj >= 0 && gj < a.n;  // a missing link is a zero vector
      g[t] = ok ? gj : id;
#pragma unroll
      for (int sl = 0; sl < NJ; ++sl) wj[t][sl] = ok ? (BF16W ? round_bf16(wv[t][sl]) : wv[t][sl]) : 0.f;
    }
    // a row past k or a missing link has weight 0: it adds exact zeros, and the
    // sums run over the rows in ascending order whatever the batching
#pragma unroll
    for (int t0 = 0; t0 < RB; t0 += SB) {
      if (r0 + t0 > k) break;  // uniform: the rest of the batch lies past row k
      if constexpr (L == 2) {
        CodePiece<U> row[SB];
#pragma unroll
        for (int t = 0; t < SB; ++t) row[t].load(a.codes + size_t(g[t0 + t]) * CS + part * U);
#pragma unroll
        for (int t = 0; t < SB; ++t) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int s = BM::sub(u, part);
            const int base = (s * 256 + int(row[t].byte(u))) * DSUB;
            float cr[DSUB];
            crow<DSUB>(C, base, cr);
#pragma unroll
            for (int q = 0; q < DSUB; ++q) acc[u * DSUB + q] += wj[t0 + t][BM::slot(u)] * cr[q];
          }
        }
      } else {
        CodeRow<CS> row[SB];
#pragma unroll
        for (int t = 0; t < SB; ++t) row[t].load(a.codes + size_t(g[t0 + t]) * CS);
#pragma unroll
        for (int t = 0; t < SB; ++t) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int s = BM::sub(u, part);
            const int base = (s * 256 + int(row[t].byte(s))) * DSUB;
            float cr[DSUB];
            crow<DSUB>(C, base, cr);
#pragma unroll
            for (int q = 0; q < DSUB; ++q) acc[u * DSUB + q] += wj[t0 + t][BM::slot(u)] * cr[q];
          }
        }
      }
    }
  }
  float e = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int s = BM::sub(u, part);
#pragma unroll
    for (int t = 0; t < DSUB; ++t) {
      const float df = yv[s * DSUB + t] - acc[u * DSUB + t];
      e += df * df;
    }
  }
  return e;
}

// p0 + p1, or (p0 + p1) + (p2 + p3), over the L lanes of a candidate group.
template <int L>
__device__ __forceinline__ float group_sum(float e) {
  e += __shfl_xor(e, 1);
  if constexpr (L == 4) e += __shfl_xor(e, 2);
  return e;
}

// Ascending bitonic sort of n (a power of two) keys in LDS by one wavefront.
__device__ __forceinline__ void wave_sort(uint64_t *keys, int n, int lane) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < n; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = keys[i], z = keys[ixj];
          const bool asc = (i & k) == 0;
          if ((x > z) == asc) {
            keys[i] = z;
            keys[ixj] = x;
          }
        }
      }
      wave_sync();
    }
  }
}

// y' = P y for one query into yv: each row of P is read by the wave as one
// contiguous run (lanes over its columns), then summed across the lanes.
__device__ __forceinline__ void project_query(const RefineArgs &a, int64_t q, float *yv, int lane) {
  const float *y = a.q + q * a.d;
  if (!a.proj) {
    for (int r = lane; r < a.d_pad; r += 64) yv[r] = y[r];
    return;
  }
  for (int r = 0; r < a.d_pad; ++r) {
    const float *pr = a.proj + size_t(r) * a.d;
    float v = 0.f;
    for (int u = lane; u < a.d; u += 64) v += pr[u] * y[u];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) yv[r] = v;
  }
}

__device__ __forceinline__ int32_t candidate_id(const RefineArgs &a, int64_t q, int c, int cn) {
  int32_t id = -1;
  if (c < a.S && c < cn) id = a.cand_ids[q * a.S + c];
  return id >= a.n ? -1 : id;
}

template <int MB>
__device__ __forceinline__ int32_t candidate(const RefineArgs &a, int64_t q, int c, int cn) {
  const int32_t id = candidate_id(a, q, c, cn);
  return id >= 0 && !beta_ok<MB>(a, id) ? -1 : id;  // malformed input: no candidate
}

__device__ __forceinline__ void write_topk(const RefineArgs &a, int64_t q, const uint64_t *keys, int lane) {
  for (int r = lane; r < a.K; r += 64) {
    const uint64_t v = keys[r];
    a.out_ids[q * a.K + r] = v == kKeyMax ? -1 : key_id(v);
    a.out_d[q * a.K + r] = v == kKeyMax ? __builtin_inff() : key_dist(v);
  }
}

// CT = float: plain float32 refinement.  CT = uint16_t: bfloat16 first pass
// plus exact float32 re-score of the best K2 candidates.
template <int M, int DSUB, int CS, typename CT, int MB>
__global__ __launch_bounds__(1024) void refine_kernel(RefineArgs a) {
  constexpr int DP = M * DSUB;
  constexpr bool kBF16 = sizeof(CT) == 2;
  extern __shared__ __align__(16) unsigned char smem[];
  CT *C = reinterpret_cast<CT *>(smem);  // [M][256][DSUB]
  constexpr int kCentBytes = (M * 256 * DSUB * int(sizeof(CT)) + 15) / 16 * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char *wbase = smem + kCentBytes + size_t(wave) * (DP * 4 + a.S_pad * 8);
  float *yv = reinterpret_cast<float *>(wbase);
  uint64_t *keys = reinterpret_cast<uint64_t *>(wbase + DP * 4);

  if constexpr (kBF16) {
    for (int i = threadIdx.x; i < M * 256 * DSUB; i += blockDim.x)
      C[i] = uint16_t(__float_as_uint(round_bf16(a.cent[i])) >> 16);
  } else {
    for (int i = threadIdx.x; i < M * 256 * DSUB / 4; i += blockDim.x)
      reinterpret_cast<float4 *>(C)[i] = reinterpret_cast<const float4 *>(a.cent)[i];
  }
  __syncthreads();

  constexpr int L = lanes_per_cand<M>();
  constexpr int G = 64 / L;  // candidates per round
  const int part = lane & (L - 1), grp = lane / L;
  for (int64_t q = int64_t(blockIdx.x) * a.wpb + wave; q < a.nq; q += int64_t(gridDim.x) * a.wpb) {
    project_query(a, q, yv, lane);
    wave_sync();
    const int cn = a.cand_n[q];
    for (int c0 = 0; c0 < a.S_pad; c0 += G) {
      const int c = c0 + grp;
      const int32_t id = c < a.S_pad ? candidate<MB>(a, q, c, cn) : -1;
      float e = 0.f;
      if (id >= 0) e = part_dist<M, DSUB, CS, CT, kBF16, MB>(a, C, yv, id, part);
      e = group_sum<L>(e);
      if (part == 0 && c < a.S_pad) keys[c] = id >= 0 ? make_key(e, id) : kKeyMax;
    }
    wave_sync();
    wave_sort(keys, a.S_pad, lane);
    if constexpr (kBF16) {
      // exact float32 re-score of the best K2, then re-sort those
      for (int c0 = 0; c0 < a.K2_pad; c0 += G) {
        const int c = c0 + grp;
        const uint64_t v = c < a.K2 ? keys[c] : kKeyMax;
        const int32_t id = v == kKeyMax ? -1 : key_id(v);
        float e = 0.f;
        if (id >= 0) e = part_dist<M, DSUB, CS, float, false, MB>(a, a.cent, yv, id, part);
        e = group_sum<L>(e);
        wave_sync();
        if (part == 0 && c < a.K2_pad) keys[c] = id >= 0 ? make_key(e, id) : kKeyMax;
        wave_sync();
      }
      wave_sort(keys, a.K2_pad, lane);
    }
    write_topk(a, q, keys, lane);
    wave_sync();
  }
}

// Any (m, dsub) without a specialised kernel (float32 only): a lane part walks
// its sub-spaces one at a time and re-reads the code byte of each neighbour.
// staged = 0: the centroids do not fit LDS and are read from global memory
// (cached); the arithmetic is the same.
template <bool STAGED>  // the centroids in LDS: read with LDS loads
__global__ __launch_bounds__(1024) void refine_f32_generic(RefineArgs a, int m, int dsub) {
  const int DP = m * dsub;
  extern __shared__ __align__(16) unsigned char smem[];
  const bool staged = STAGED;
  const size_t cent_bytes = staged ? (size_t(m) * 256 * dsub * 4 + 15) / 16 * 16 : 0;
  const float *C = STAGED ? reinterpret_cast<const float *>(smem) : a.cent;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char *wbase = smem + cent_bytes + size_t(wave) * (DP * 4 + a.S_pad * 8);
  float *yv = reinterpret_cast<float *>(wbase);
  uint64_t *keys = reinterpret_cast<uint64_t *>(wbase + DP * 4);
  if (staged)
    for (int i = threadIdx.x; i < m * 256 * dsub; i += blockDim.x) reinterpret_cast<float *>(smem)[i] = a.cent[i];
  __syncthreads();
  const int part = lane & 3, grp = lane >> 2;
  for (int64_t q = int64_t(blockIdx.x) * a.wpb + wave; q < a.nq; q += int64_t(gridDim.x) * a.wpb) {
    project_query(a, q, yv, lane);
    wave_sync();
    const int cn = a.cand_n[q];
    for (int c0 = 0; c0 < a.S_pad; c0 += 16) {
      const int c = c0 + grp;
      int32_t id = candidate_id(a, q, c, cn);
      for (int jb = 0; id >= 0 && jb < a.m_beta; ++jb)
        if (a.beta_idx[int64_t(id) * a.m_beta + jb] >= a.n_beta) id = -1;  // malformed input: no candidate
      float e = 0.f;
      if (id >= 0) {
        const int32_t *links = a.adj0 + int64_t(id) * a.deg0;
        for (int s = part; s < m; s += 4) {
          const int jb = s / (m / a.m_beta);  // block of the product codebook holding sub-space s
          const float *bw =
              a.beta + (size_t(jb) * a.n_beta + a.beta_idx[int64_t(id) * a.m_beta + jb]) * (a.k_reg + 1);
          float acc[16];
          for (int t = 0; t < 16; ++t) acc[t] = 0.f;
          for (int j = 0; j <= a.k_reg; ++j) {
            const int32_t g = j == 0 ? id : links[j - 1];
            if (g < 0 || g >= a.n) continue;
            const float w = bw[j];
            const float *cr = C + (s * 256 + int(a.codes[size_t(g) * a.code_stride + s])) * dsub;
            for (int t = 0; t < dsub; ++t) acc[t] += w * cr[t];
            if (a.ccent) {  // 2-level codec: the first-level centroid's part over sub-space s
              const int half = s >= m / 2;
              const uint32_t cc = a.ccodes[g];
              const float *c1 = a.ccent + (size_t(half) * a.coarse_k + (half ? cc >> 16 : cc & 0xFFFFu)) * (DP / 2) +
                                (s - half * (m / 2)) * dsub;
              for (int t = 0; t < dsub; ++t) acc[t] += w * c1[t];
            }
          }
          for (int t = 0; t < dsub; ++t) {
            const float df = yv[s * dsub + t] - acc[t];
            e += df * df;
          }
        }
      }
      e = group_sum<4>(e);
      if (part == 0) keys[c] = id >= 0 ? make_key(e, id) : kKeyMax;
    }
    wave_sync();
    wave_sort(keys, a.S_pad, lane);
    write_topk(a, q, keys, lane);
    wave_sync();
  }
}

// Refinement for the 2-level codec (float32).  Lane `part` of a candidate's
// four owns the contiguous coordinates [part Q, part Q + Q): Q / DSUB whole
// sub-spaces inside one half of the vector, so each neighbour's first-level
// centroid contributes one contiguous slice of its row.  Neighbours go four at
// a time so that their loads overlap.  Per coordinate the sum runs over the
// neighbours in order, the PQ centroid before the first-level one, as in the
// generic kernel.
// STAGED: the PQ centroids in LDS (a compile-time choice, so that their reads
// are LDS reads rather than generic ones that also wait on global loads).
template <int Q, int DSUB, bool STAGED>
__global__ __launch_bounds__(512) void refine_coarse_kernel(RefineArgs a, int m) {
  constexpr int NS = Q / DSUB;  // sub-spaces per lane
  constexpr int DP = 4 * Q;
  extern __shared__ __align__(16) unsigned char smem[];
  const bool staged = STAGED;
  const size_t cent_bytes = staged ? (size_t(m) * 256 * DSUB * 4 + 15) / 16 * 16 : 0;
  const float *C = STAGED ? reinterpret_cast<const float *>(smem) : a.cent;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char *wbase = smem + cent_bytes + size_t(wave) * (DP * 4 + a.S_pad * 8);
  float *yv = reinterpret_cast<float *>(wbase);
  uint64_t *keys = reinterpret_cast<uint64_t *>(wbase + DP * 4);
  if (staged)
    for (int i = threadIdx.x; i < m * 256 * DSUB; i += blockDim.x) reinterpret_cast<float *>(smem)[i] = a.cent[i];
  __syncthreads();
  const int part = lane & 3, grp = lane >> 2;
  const int s0 = part * NS, half = part >> 1;
  const int spb = m / a.m_beta;  // sub-spaces per codebook block
  for (int64_t q = int64_t(blockIdx.x) * a.wpb + wave; q < a.nq; q += int64_t(gridDim.x) * a.wpb) {
    project_query(a, q, yv, lane);
    wave_sync();
    const int cn = a.cand_n[q];
    for (int c0 = 0; c0 < a.S_pad; c0 += 16) {
      const int c = c0 + grp;
      int32_t id = candidate_id(a, q, c, cn);
      for (int jb = 0; id >= 0 && jb < a.m_beta; ++jb)
        if (a.beta_idx[int64_t(id) * a.m_beta + jb] >= a.n_beta) id = -1;  // malformed input: no candidate
      float e = 0.f;
      if (id >= 0) {
        const int32_t *links = a.adj0 + int64_t(id) * a.deg0;
        uint32_t bo[NS];  // offset of the beta row of each of the lane's sub-spaces
#pragma unroll
        for (int v = 0; v < NS; ++v) {
          const int jb = (s0 + v) / spb;
          bo[v] = (uint32_t(jb) * a.n_beta + a.beta_idx[int64_t(id) * a.m_beta + jb]) * uint32_t(a.k_reg + 1);
        }
        float acc[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] = 0.f;
        for (int j0 = 0; j0 <= a.k_reg; j0 += 4) {
          constexpr int NW = (NS + 3) / 4;
          int32_t g[4];
          uint32_t cc[4];
          uint32_t cd[4][NW];  // the lane's code bytes of each neighbour, four to a word
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int j = j0 + u;
            int32_t x = j > a.k_reg ? -1 : (j == 0 ? id : links[j - 1]);
            g[u] = x < 0 || x >= a.n ? -1 : x;  // a missing link is a zero vector
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            cc[u] = g[u] >= 0 ? a.ccodes[g[u]] : 0u;
#pragma unroll
            for (int i = 0; i < NW; ++i) cd[u][i] = 0u;
#pragma unroll
            for (int v = 0; v < NS; ++v)
              cd[u][v >> 2] |= (g[u] >= 0 ? uint32_t(a.codes[size_t(g[u]) * a.code_stride + s0 + v]) : 0u)
                               << (8 * (v & 3));
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (g[u] < 0) continue;
            const int j = j0 + u;
            const float *c1 = a.ccent + (size_t(half) * a.coarse_k + (half ? cc[u] >> 16 : cc[u] & 0xFFFFu)) * (DP / 2) +
                              (part & 1) * Q;
#pragma unroll
            for (int v = 0; v < NS; ++v) {
              const float w = a.beta[bo[v] + j];
              const float *cr = C + ((s0 + v) * 256 + int((cd[u][v >> 2] >> (8 * (v & 3))) & 0xFFu)) * DSUB;
#pragma unroll
              for (int t = 0; t < DSUB; ++t) acc[v * DSUB + t] += w * cr[t];
#pragma unroll
              for (int t = 0; t < DSUB; ++t) acc[v * DSUB + t] += w * c1[v * DSUB + t];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const float df = yv[part * Q + i] - acc[i];
          e += df * df;
        }
      }
      e = group_sum<4>(e);
      if (part == 0) keys[c] = id >= 0 ? make_key(e, id) : kKeyMax;
    }
    wave_sync();
    wave_sort(keys, a.S_pad, lane);
    write_topk(a, q, keys, lane);
    wave_sync();
  }
}

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

RefineArgs make_args(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids,
                     const int32_t *cand_n, int32_t S, int32_t K, int32_t *out_ids, float *out_d) {
  RefineArgs a;
  a.q = q;
  a.nq = nq;
  a.d = ix->v.d;
  a.d_pad = ix->v.d_pad;
  a.proj = ix->v.proj;
  a.cent = ix->v.centroids;
  a.codes = ix->v.codes;
  a.code_stride = ix->v.code_stride;
  a.adj0 = ix->v.adj0;
  a.n = ix->v.n;
  a.n_beta = ix->v.n_beta;
  a.m_beta = ix->v.m_beta;
  a.ccent = ix->v.coarse_k > 0 ? ix->v.coarse_cent : nullptr;
  a.ccodes = reinterpret_cast<const uint32_t *>(ix->v.coarse_codes);
  a.coarse_k = ix->v.coarse_k;
  a.deg0 = ix->v.deg0;
  a.k_reg = ix->v.k_reg;
  a.beta = ix->v.beta;
  a.beta_idx = ix->v.beta_idx;
  a.cand_ids = cand_ids;
  a.cand_n = cand_n;
  a.S = S;
  a.K = K;
  a.S_pad = next_pow2(S < 16 ? 16 : S);
  a.K2 = 2 * K < S ? 2 * K : S;
  a.K2_pad = next_pow2(a.K2 < 16 ? 16 : a.K2);
  a.out_ids = out_ids;
  a.out_d = out_d;
  a.wpb = 0;
  return a;
}

// Waves per block and LDS bytes for the staged centroids plus per-wave buffers.
bool plan_blocks(const lc_index *ix, RefineArgs &a, int cent_elem_bytes, int *lds, int64_t *blocks,
                 bool stage = true, int max_wpb = 16) {
  const int cent_bytes = stage ? (ix->v.m * 256 * ix->dsub * cent_elem_bytes + 15) / 16 * 16 : 0;
  const int per_wave = ix->v.d_pad * 4 + a.S_pad * 8;
  int wpb = (ix->lds_per_cu - cent_bytes) / per_wave;
  if (wpb > max_wpb) wpb = max_wpb;
  if (wpb < 1) return false;
  a.wpb = wpb;
  *lds = cent_bytes + wpb * per_wave;
  int64_t b = (a.nq + wpb - 1) / wpb;
  if (b > ix->num_cus) b = ix->num_cus;
  *blocks = b < 1 ? 1 : b;
  return true;
}

template <int M, int DSUB, int CS, typename CT, int MB>
int launch_spec(const lc_index *ix, RefineArgs a, hipStream_t st) {
  int lds;
  int64_t blocks;
  if (!plan_blocks(ix, a, int(sizeof(CT)), &lds, &blocks)) return LC_ENOTSUP;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&refine_kernel<M, DSUB, CS, CT, MB>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return LC_EHIP;
  hipLaunchKernelGGL((refine_kernel<M, DSUB, CS, CT, MB>), dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

// The product codebook's block count as a kernel parameter (1, 2, 4 or 8 blocks).
template <int M, int DSUB, int CS, typename CT>
int launch_blocks(const lc_index *ix, const RefineArgs &a, hipStream_t st) {
  switch (a.m_beta) {
    case 1: return launch_spec<M, DSUB, CS, CT, 1>(ix, a, st);
    case 2: return launch_spec<M, DSUB, CS, CT, 2>(ix, a, st);
    case 4: return launch_spec<M, DSUB, CS, CT, 4>(ix, a, st);
    case 8: return launch_spec<M, DSUB, CS, CT, 8>(ix, a, st);
    default: return LC_ENOTSUP;
  }
}

int launch_generic(const lc_index *ix, RefineArgs a, hipStream_t st) {
  int lds;
  int64_t blocks;
  if (ix->dsub > 16) return LC_ENOTSUP;
  // centroids in LDS when they fit beside the per-wave buffers, else read from global memory
  const bool staged = plan_blocks(ix, a, 4, &lds, &blocks);
  if (!staged && !plan_blocks(ix, a, 4, &lds, &blocks, false)) return LC_ENOTSUP;
  const void *fn = staged ? reinterpret_cast<const void *>(&refine_f32_generic<true>)
                          : reinterpret_cast<const void *>(&refine_f32_generic<false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return LC_EHIP;
  if (staged)
    hipLaunchKernelGGL(refine_f32_generic<true>, dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a, ix->v.m, ix->dsub);
  else
    hipLaunchKernelGGL(refine_f32_generic<false>, dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a, ix->v.m, ix->dsub);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

template <int Q, int DSUB>
int launch_coarse_q(const lc_index *ix, RefineArgs a, hipStream_t st) {
  int lds;
  int64_t blocks;
  // 8 waves per block: the kernel is built for 512 threads (256 registers a lane)
  const bool staged = plan_blocks(ix, a, 4, &lds, &blocks, true, 8);
  if (!staged && !plan_blocks(ix, a, 4, &lds, &blocks, false, 8)) return LC_ENOTSUP;
  const void *fn = staged ? reinterpret_cast<const void *>(&refine_coarse_kernel<Q, DSUB, true>)
                          : reinterpret_cast<const void *>(&refine_coarse_kernel<Q, DSUB, false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return LC_EHIP;
  if (staged)
    hipLaunchKernelGGL((refine_coarse_kernel<Q, DSUB, true>), dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a,
                       ix->v.m);
  else
    hipLaunchKernelGGL((refine_coarse_kernel<Q, DSUB, false>), dim3(int(blocks)), dim3(64 * a.wpb), lds, st, a,
                       ix->v.m);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

// 2-level codec: shapes with a quarter of the coordinates per lane (Q = d_pad / 4
// whole sub-spaces) take refine_coarse_kernel, others the generic kernel.
int launch_coarse(const lc_index *ix, const RefineArgs &a, hipStream_t st) {
  const int qd = ix->v.d_pad / 4, ds = ix->dsub;
  if (ix->v.d_pad % 4 == 0 && qd % ds == 0) {
#define QSHAPE(QQ, DS) \
  if (qd == QQ && ds == DS) return launch_coarse_q<QQ, DS>(ix, a, st);
    QSHAPE(8, 2) QSHAPE(8, 4) QSHAPE(12, 2) QSHAPE(16, 4) QSHAPE(24, 6) QSHAPE(24, 12) QSHAPE(28, 2) QSHAPE(32, 4)
#undef QSHAPE
  }
  return launch_generic(ix, a, st);
}

}  // namespace

// Specialised shapes (m, dsub, code stride) with 1, 2, 4 or 8 codebook
// blocks; other shapes and block counts take the generic float32 kernel, and
// the precision form needs a specialised one.
int lc_launch_refine(const lc_index *ix, const float *q, int64_t nq, const int32_t *cand_ids,
                     const int32_t *cand_n, int32_t S, int32_t K, int precision, int32_t *out_ids,
                     float *out_d, bool projected, hipStream_t st) {
  RefineArgs a = make_args(ix, q, nq, cand_ids, cand_n, S, K, out_ids, out_d);
  if (projected) {  // queries already projected: rows of d_pad
    a.proj = nullptr;
    a.d = ix->v.d_pad;
  }
  const int m = ix->v.m, ds = ix->dsub;
  const bool bf = precision == LC_REFINE_BF16_RESCORE;
  // when the re-score covers the whole short-list (2K >= S) the first pass decides nothing: every
  // candidate's distance is the float32 one and all are sorted by it, which is the plain kernel
  const bool bf_pass = bf && a.K2 < S;
  const bool spec_mb = a.m_beta == 1 || a.m_beta == 2 || a.m_beta == 4 || a.m_beta == 8;
  if (a.ccent) return bf_pass ? LC_ENOTSUP : launch_coarse(ix, a, st);  // 2-level codec: float32 kernels
#define SHAPE(MM, DS, CSS)                                                                              \
  if (m == MM && ds == DS && spec_mb)                                                                   \
    return bf_pass ? launch_blocks<MM, DS, CSS, uint16_t>(ix, a, st) : launch_blocks<MM, DS, CSS, float>(ix, a, st);
  SHAPE(8, 2, 8)
  SHAPE(8, 4, 8)
  SHAPE(8, 12, 8)
  SHAPE(16, 6, 16)
  SHAPE(32, 4, 32)
  SHAPE(56, 2, 64)
#undef SHAPE
  if (bf) return LC_ENOTSUP;
  return launch_generic(ix, a, st);
}
