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
#include <hip/hip_fp16.h>

#include "lc_internal.h"

namespace {

using namespace lc;

struct WalkArgs {
  const uint8_t *codes;
  const int32_t *adj0, *up_base, *adj_up;
  const void *lut;
  const float *scale;
  const int32_t *ef;
  const int32_t *order;
  int32_t ef_max, S;
  int64_t nq, n_up_rows;
  int32_t n, code_stride, deg0, deg_up, entry, max_level;
  int32_t w_cap, hash_bits, prefetch, queue, vmode, list_cap;
  uint32_t *counters;  // [0] next query, [1] finished slots (queue mode)
  uint32_t *bits;
  int32_t *vlists;     // [slots][list_cap] ids whose bit is set (visited mode 1)
  int64_t words;
  int32_t *cand_ids;
  float *cand_adc;
  int32_t *cand_n, *stats;
};

// One table entry as float32: the entry itself, or the fp16 entry times its
// row's power-of-two scale (exact).
__device__ __forceinline__ float lut_at(const float *lut, const float *, int s, uint32_t c) {
  return lut[s * 256 + c];
}
__device__ __forceinline__ float lut_at(const __half *lut, const float *sc, int s, uint32_t c) {
  return __half2float(lut[s * 256 + c]) * sc[s];
}

// Sum of LUT[s][code[s]] over all sub-spaces, s ascending (one lane per node).
template <int M, typename T>
__device__ __forceinline__ float adc_full(const T *lut, const float *sc, const uint8_t *codes, int cs,
                                          int32_t id) {
  const uint8_t *row = codes + size_t(id) * cs;
  float acc = 0.f;
  if constexpr (M % 16 == 0) {
#pragma unroll
    for (int i = 0; i < M / 16; ++i) {
      const uint4 w = reinterpret_cast<const uint4 *>(row)[i];
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int t = 0; t < 16; ++t) acc += lut_at(lut, sc, i * 16 + t, (ws[t >> 2] >> (8 * (t & 3))) & 0xFFu);
    }
  } else {
    static_assert(M % 8 == 0, "m must be a multiple of 8");
#pragma unroll
    for (int i = 0; i < M / 8; ++i) {
      const uint2 w = reinterpret_cast<const uint2 *>(row)[i];
      const uint32_t ws[2] = {w.x, w.y};
#pragma unroll
      for (int t = 0; t < 8; ++t) acc += lut_at(lut, sc, i * 8 + t, (ws[t >> 2] >> (8 * (t & 3))) & 0xFFu);
    }
  }
  return acc;
}

// The m code bytes of one node in registers, then its ADC sum from them.
template <int M>
struct CodeRegs {
  uint32_t w[M / 4];
  __device__ __forceinline__ void load(const uint8_t *codes, int cs, int32_t id) {
    const uint8_t *row = codes + size_t(id) * cs;
    if constexpr (M % 16 == 0) {
#pragma unroll
      for (int i = 0; i < M / 16; ++i) {
        const uint4 v = reinterpret_cast<const uint4 *>(row)[i];
        w[4 * i] = v.x;
        w[4 * i + 1] = v.y;
        w[4 * i + 2] = v.z;
        w[4 * i + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < M / 8; ++i) {
        const uint2 v = reinterpret_cast<const uint2 *>(row)[i];
        w[2 * i] = v.x;
        w[2 * i + 1] = v.y;
      }
    }
  }
  template <typename T>
  __device__ __forceinline__ float adc(const T *lut, const float *sc) const {
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < M; ++s) acc += lut_at(lut, sc, s, (w[s >> 2] >> (8 * (s & 3))) & 0xFFu);
    return acc;
  }
};

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l));
  return (uint64_t(hi) << 32) | lo;
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

template <int M, typename T>
__global__ __launch_bounds__(64) void walk_kernel(WalkArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  constexpr int kLutBytes = M * 256 * int(sizeof(T));
  constexpr int kScaleBytes = sizeof(T) == 2 ? (M * 4 + 15) / 16 * 16 : 0;
  T *lut = reinterpret_cast<T *>(smem);
  float *sc = reinterpret_cast<float *>(smem + kLutBytes);
  uint64_t *W = reinterpret_cast<uint64_t *>(smem + kLutBytes + kScaleBytes);
  uint32_t *hash = reinterpret_cast<uint32_t *>(W + a.w_cap);
  const int H = 1 << a.hash_bits;
  const uint32_t hmask = uint32_t(H - 1);
  const int hshift = 32 - a.hash_bits;
  const int hlimit = H / 2;
  uint32_t *bits = a.bits + int64_t(blockIdx.x) * a.words;

  int64_t pos = blockIdx.x;
  if (a.queue) {
    int64_t t = 0;
    if (lane == 0) t = int64_t(atomicAdd(a.counters, 1u));
    pos = __shfl(t, 0);
  }
  while (pos < a.nq) {
    const int64_t q = a.order ? int64_t(a.order[pos]) : pos;
    if (q < 0 || q >= a.nq) {
      // not a query of this batch: nothing to do
    } else {
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
    } else {
      const int efe = efq > a.S ? efq : a.S;

      // stage the table (and its row scales), clear the visited table
      const float4 *src = reinterpret_cast<const float4 *>(static_cast<const T *>(a.lut) + q * (M * 256));
      for (int i = lane; i < kLutBytes / 16; i += 64) reinterpret_cast<float4 *>(lut)[i] = src[i];
      if (sizeof(T) == 2)
        for (int i = lane; i < M; i += 64) sc[i] = a.scale[q * M + i];
      for (int i = lane; i < H; i += 64) hash[i] = kEmpty;
      wave_sync();

      // greedy descent on levels max_level .. 1: the best link while it beats
      // the current key (one lane per link)
      int32_t cur = a.entry;
      uint64_t curkey = make_key(adc_full<M, T>(lut, sc, a.codes, a.code_stride, cur), cur);
      for (int l = a.max_level; l >= 1; --l) {
        for (;;) {
          const int64_t row = int64_t(a.up_base[cur]) + l - 1;
          int32_t nb = -1;
          if (lane < a.deg_up && row >= 0 && row < a.n_up_rows) nb = a.adj_up[row * a.deg_up + lane];
          if (nb >= a.n) nb = -1;  // a malformed link is ignored rather than followed
          const uint64_t k = nb >= 0 ? make_key(adc_full<M, T>(lut, sc, a.codes, a.code_stride, nb), nb) : kKeyMax;
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
      int32_t *vlist = a.vlists + int64_t(blockIdx.x) * a.list_cap;
      if (lane == 0) {
        W[0] = curkey;
        if (a.vmode == 0) {
          visit(hash, hmask, hshift, cur, false, bits);
        } else {
          atomicOr(&bits[uint32_t(cur) >> 5], 1u << (uint32_t(cur) & 31u));
          hash[(uint32_t(cur) * 0x9E3779B1u) >> hshift] = uint32_t(cur);
          vlist[0] = cur;
        }
      }
      int vcount = 1;  // ids recorded in vlist (visited mode 1)
      int nw = 1, fu = 0, E = 0, D = 0, hcount = 1;
      bool ovf = false;
      uint64_t ck = curkey;                            // key of W[fu]
      uint64_t wmax = efe == 1 ? curkey : kKeyMax;     // largest key of W once W is full
      int pidx = -1;                                   // second unexpanded entry (prefetch guess)
      int32_t nb = l32 < a.deg0 ? a.adj0[int64_t(cur) * a.deg0 + l32] : -1;
      wave_sync();
      while (fu < nw) {
        int32_t pred = -1, pnb = -1;
        if (a.prefetch && pidx >= 0) {
          pred = key_id(W[pidx]);
          pnb = l32 < a.deg0 ? a.adj0[int64_t(pred) * a.deg0 + l32] : -1;
        }
        if (lane == 0) W[fu] = ck | kExpanded;
        wave_sync();
        ++E;
        if (nb >= a.n) nb = -1;  // a malformed link is ignored rather than followed
        bool fresh = false;
        uint64_t k = kKeyMax;
        if (a.vmode == 0) {
          if (!ovf && hcount + a.deg0 > hlimit) ovf = true;
          if (lane < 32 && nb >= 0) fresh = visit(hash, hmask, hshift, nb, ovf, bits);
          const int nf = __popcll(__ballot(fresh));
          D += nf;
          if (!ovf) hcount += nf;
          if (fresh) k = make_key(adc_full<M, T>(lut, sc, a.codes, a.code_stride, nb), nb);
        } else {
          // cache hit: visited; miss: test-and-set the bit, fetching the code meanwhile
          CodeRegs<M> row;
          if (lane < 32 && nb >= 0) {
            const uint32_t h = (uint32_t(nb) * 0x9E3779B1u) >> hshift;
            if (hash[h] != uint32_t(nb)) {
              const uint32_t bit = 1u << (uint32_t(nb) & 31u);
              const uint32_t old = atomicOr(&bits[uint32_t(nb) >> 5], bit);
              row.load(a.codes, a.code_stride, nb);
              fresh = (old & bit) == 0;
              hash[h] = uint32_t(nb);
            }
          }
          const uint64_t fm = __ballot(fresh);
          const int nf = __popcll(fm);
          if (fresh) {
            const int at = vcount + __popcll(fm & ((1ull << lane) - 1ull));
            if (at < a.list_cap) vlist[at] = nb;
            k = make_key(row.adc(lut, sc), nb);
          }
          vcount += nf;
          D += nf;
        }
        const bool keep = fresh && k < wmax;
        const uint64_t km = __ballot(keep);
        int p0 = fu;
        if (km) {
          // Merge the kept keys into W without sorting them: every kept key is
          // broadcast in turn; its rank among the kept keys and its count of
          // smaller W entries give its slot, and every W entry moves up by the
          // number of kept keys below it.
          const int nn = __popcll(km);
          uint64_t kmin = kKeyMax;
          int rank = 0, before_ck = 0;
          for (uint64_t mm = km; mm; mm &= mm - 1) {
            const int j = __ffsll((unsigned long long)mm) - 1;
            const uint64_t kj = readlane64(k, j);
            kmin = kj < kmin ? kj : kmin;
            rank += (keep && kj < k) ? 1 : 0;
            before_ck += kj < ck ? 1 : 0;
          }
          int mypos = 0;
          int c = (nw - 1) >> 6;
          for (; c >= 0; --c) {
            const int idx = (c << 6) + lane;
            const bool in = idx < nw;
            const uint64_t v = in ? W[idx] : kKeyMax;
            const uint64_t pv = pure_key(v);
            int cnt = 0;
            for (uint64_t mm = km; mm; mm &= mm - 1) {
              const int j = __ffsll((unsigned long long)mm) - 1;
              const uint64_t kj = readlane64(k, j);
              cnt += (in && kj < pv) ? 1 : 0;
              const int below = __popcll(__ballot(in && pv < kj));
              if (lane == j) mypos += below;
            }
            wave_sync();  // the whole chunk is in registers before anything moves
            if (in && cnt > 0 && idx + cnt < efe) W[idx + cnt] = v;
            wave_sync();
            if (readlane64(pv, 0) < kmin) {  // lower chunks lie entirely below every kept key
              --c;
              break;
            }
          }
          mypos += (c + 1) << 6;
          if (keep && mypos + rank < efe) W[mypos + rank] = k;
          const int jmin = __ffsll((unsigned long long)__ballot(keep && rank == 0)) - 1;
          const int pos_min = __builtin_amdgcn_readlane(mypos, jmin);
          const int fu_new = fu + before_ck;
          p0 = fu_new < pos_min ? fu_new : pos_min;
          nw = nw + nn < efe ? nw + nn : efe;
          wave_sync();
          wmax = nw == efe ? pure_key(W[nw - 1]) : kKeyMax;
        }
        wave_sync();
        // first and second unexpanded entries at or after p0 (all before are expanded)
        int nfu = nw;
        uint64_t nck = 0;
        pidx = -1;
        for (int base = p0; base < nw; base += 64) {
          const int idx = base + lane;
          const uint64_t v = idx < nw ? W[idx] : kExpanded;
          uint64_t bm = __ballot((v & kExpanded) == 0);
          if (bm) {
            const int l0 = __ffsll((unsigned long long)bm) - 1;
            nfu = base + l0;
            nck = readlane64(v, l0);
            bm &= bm - 1;
            if (bm) pidx = base + __ffsll((unsigned long long)bm) - 1;
            break;
          }
        }
        fu = nfu;
        if (fu < nw) {
          ck = nck;
          const int32_t nc = key_id(ck);
          if (nc == pred) nb = pnb;
          else nb = l32 < a.deg0 ? a.adj0[int64_t(nc) * a.deg0 + l32] : -1;
        }
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
      if (a.vmode == 0) {
        if (ovf) {
          for (int64_t i = lane; i < a.words; i += 64) bits[i] = 0u;
          __threadfence();
        }
      } else {
        __threadfence();  // the recorded ids are visible to every lane
        const int nl = vcount < a.list_cap ? vcount : a.list_cap;
        if (vcount > a.list_cap) {
          for (int64_t i = lane; i < a.words; i += 64) bits[i] = 0u;
        } else {
          for (int i = lane; i < nl; i += 64) bits[uint32_t(vlist[i]) >> 5] = 0u;
        }
        __threadfence();
        for (int i = lane; i < nl; i += 64) vlist[i] = 0;  // the workspace is left zero-filled
        __threadfence();
      }
      wave_sync();
    }
    }
    if (a.queue) {
      int64_t t = 0;
      if (lane == 0) t = int64_t(atomicAdd(a.counters, 1u));
      pos = __shfl(t, 0);
    } else {
      pos += gridDim.x;
    }
  }
  if (a.queue && lane == 0) {
    // the last slot to finish leaves both counters at zero for the next launch
    if (atomicAdd(a.counters + 1, 1u) == gridDim.x - 1) {
      atomicExch(a.counters, 0u);
      atomicExch(a.counters + 1, 0u);
    }
  }
}

struct WalkPlan {
  int w_cap, hash_bits, lds_bytes, grid;
};

constexpr size_t kHeaderBytes = 256;  // two queue counters, padded

template <int M>
int lds_bytes_for(int w_cap, int hash_bits, int lut_bytes) {
  const int scale_bytes = lut_bytes == 2 ? (M * 4 + 15) / 16 * 16 : 0;
  return M * 256 * lut_bytes + scale_bytes + w_cap * 8 + (1 << hash_bits) * 4;
}

int auto_hash_bits(int w_cap) {
  // about 8 table slots per pool slot: half of them before the bitset takes over
  int bits = 9;
  while ((1 << bits) < 8 * w_cap && bits < 14) ++bits;
  return bits;
}

template <int M>
WalkPlan plan_for(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, const lc_schedule *sc,
                  int lut_bytes) {
  WalkPlan p;
  int ef_eff = ef_max > S ? ef_max : S;
  p.w_cap = (ef_eff + 63) / 64 * 64;
  // visited mode 1 keeps only a small LDS cache; mode 0 sizes its table from the pool
  p.hash_bits = (sc && sc->hash_bits) ? sc->hash_bits : (sc && sc->visited == 1 ? 9 : auto_hash_bits(p.w_cap));
  p.lds_bytes = lds_bytes_for<M>(p.w_cap, p.hash_bits, lut_bytes);
  int per_cu = ix->lds_per_cu / p.lds_bytes;
  if (sc && sc->waves_per_cu > 0 && sc->waves_per_cu < per_cu) per_cu = sc->waves_per_cu;
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 32) per_cu = 32;
  int64_t g = int64_t(per_cu) * ix->num_cus;
  if (g > nq) g = nq;
  if (g < 1) g = 1;
  p.grid = int(g);
  return p;
}

bool valid_schedule(const lc_schedule *sc) {
  if (!sc) return true;
  if (sc->hash_bits != 0 && (sc->hash_bits < 9 || sc->hash_bits > 14)) return false;
  if (sc->prefetch < 0 || sc->prefetch > 1 || sc->queue < 0 || sc->queue > 1 || sc->waves_per_cu < 0) return false;
  if (sc->visited < 0 || sc->visited > 1) return false;
  return true;
}

const lc_schedule kDefaultSchedule = {0, 0, 0, 1, 1};

int list_cap_for(int w_cap) { return 16 * w_cap > 4096 ? 16 * w_cap : 4096; }

// header, then per slot its bitset, then (visited mode 1) per slot its id list
size_t ws_need(const WalkPlan &p, int64_t words, int vmode) {
  size_t b = kHeaderBytes + size_t(p.grid) * size_t(words) * 4;
  if (vmode == 1) b += size_t(p.grid) * size_t(list_cap_for(p.w_cap)) * 4;
  return b;
}

template <int M>
size_t ws_bytes_m(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, const lc_schedule *sc) {
  // sized for the smaller (fp16) table, which admits the most slots
  WalkPlan p = plan_for<M>(ix, nq, ef_max, S, sc, 2);
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  return ws_need(p, words, sc->visited);
}

template <int M, typename T>
int launch_m(const lc_index *ix, const void *lut, const float *scale, int64_t nq, const int32_t *ef,
             int32_t ef_max, int32_t S, const int32_t *order, int32_t *cand_ids, float *cand_adc, int32_t *cand_n,
             int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sc, hipStream_t st) {
  WalkPlan p = plan_for<M>(ix, nq, ef_max, S, sc, int(sizeof(T)));
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  if (ws_bytes < ws_need(p, words, sc->visited)) return LC_ENOSPC;
  if (p.lds_bytes > ix->lds_per_cu) return LC_ENOTSUP;
  WalkArgs a;
  a.codes = ix->v.codes;
  a.adj0 = ix->v.adj0;
  a.up_base = ix->v.up_base;
  a.adj_up = ix->v.adj_up;
  a.lut = lut;
  a.scale = scale;
  a.ef = ef;
  a.order = order;
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
  a.prefetch = sc->prefetch;
  a.queue = sc->queue;
  a.vmode = sc->visited;
  a.list_cap = list_cap_for(p.w_cap);
  a.counters = static_cast<uint32_t *>(ws);
  a.bits = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + kHeaderBytes);
  a.vlists = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + kHeaderBytes +
                                         size_t(p.grid) * size_t(words) * 4);
  a.words = words;
  a.cand_ids = cand_ids;
  a.cand_adc = cand_adc;
  a.cand_n = cand_n;
  a.stats = stats;
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(&walk_kernel<M, T>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_bytes) != hipSuccess)
    return LC_EHIP;
  hipLaunchKernelGGL((walk_kernel<M, T>), dim3(p.grid), dim3(64), p.lds_bytes, st, a);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

}  // namespace

#define LC_FOR_EACH_M(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

size_t lc_walk_workspace_bytes(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S,
                               const lc_schedule *sched) {
  if (!valid_schedule(sched)) return 0;
  const lc_schedule *sc = sched ? sched : &kDefaultSchedule;
  switch (ix->v.m) {
#define CASE(MM) \
  case MM: return ws_bytes_m<MM>(ix, nq, ef_max, S, sc);
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return 0;
  }
}

int lc_launch_walk(const lc_index *ix, const void *lut, int dtype, const float *scale, int64_t nq,
                   const int32_t *ef, int32_t ef_max, int32_t S, const int32_t *order, int32_t *cand_ids,
                   float *cand_adc,
                   int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sched,
                   hipStream_t st) {
  if (dtype != LC_LUT_F32 && dtype != LC_LUT_F16) return LC_ENOTSUP;
  if (!valid_schedule(sched)) return LC_EINVAL;
  const lc_schedule *sc = sched ? sched : &kDefaultSchedule;
  switch (ix->v.m) {
#define CASE(MM)                                                                                              \
  case MM:                                                                                                    \
    return dtype == LC_LUT_F32 ? launch_m<MM, float>(ix, lut, scale, nq, ef, ef_max, S, order, cand_ids,     \
                                                     cand_adc, cand_n, stats, ws, ws_bytes, sc, st)           \
                               : launch_m<MM, __half>(ix, lut, scale, nq, ef, ef_max, S, order, cand_ids,    \
                                                      cand_adc, cand_n, stats, ws, ws_bytes, sc, st);
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return LC_ENOTSUP;
  }
}
