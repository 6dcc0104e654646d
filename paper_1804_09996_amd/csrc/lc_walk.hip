// First stage of the search (Sec. 2; Sec. 4.1): greedy descent on the upper
// levels, then a best-first walk on level 0 over nodes that hold only PQ codes,
// scored by asymmetric distances from the per-query table.
//
// One wavefront owns one query at a time (slots take queries from an atomic
// counter or stride over the batch):
//  * the query's table (m x 256, float32 or fp16 with per-row scales) is
//    staged in LDS;
//  * the pool W (<= ef_eff keys, sorted, "expanded" flag in bit 31) is an LDS
//    array;
//  * the visited set is exact, in one of two forms (the schedule's choice):
//    an LDS open-addressing table of ids that continues on a per-slot bitset
//    in the workspace once half full (walk_kernel), or the per-slot bitset
//    behind a direct-mapped LDS cache (walk_cache_kernel).
//
// Expanding the best unexpanded entry of W, evaluating all its fresh links,
// and merging them at once leaves W, the expansion count E and the evaluation
// count D exactly as in the textbook two-heap form: keys are unique, keeping
// the best ef_eff of a union is associative, and a candidate that is no longer
// in W is worse than every entry of W, so it would end the two-heap loop.
//
// walk_kernel also expands the second unexpanded entry p of W in the same
// step, on lanes 32..63, whenever that is what the sequential walk would do
// next: after the first expansion c, the next one is p exactly when none of
// c's fresh keys is below key(p).  Both expansions' links are probed against
// the visited table together (p's only looked up), their codes fetched and
// scored together; once every fresh key of c is known to be above key(p), p's
// absent links are inserted for real and the kept keys of both are merged at
// once.  Merging c's keys and then p's keys (each time keeping the best
// ef_eff) equals merging their union, so W, E and D stay those of the
// sequential walk.  The adjacency rows of the two entries that follow p are
// loaded at the start of each step and used at the next one when they are
// still the next two unexpanded entries.
#include <hip/hip_fp16.h>

#include <cstdio>
#include <type_traits>

#include "lc_internal.h"

namespace {

using namespace lc;

constexpr int kMergeScratch = 34;  // keys of merge scratch: up to 32 kept keys and a pad, 16-byte multiple

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
  int32_t tag_bits;    // walk_kernel's table: 16-bit tags of this many bits, 0 = 32-bit ids
  int32_t max_d;       // budget T on distance evaluations (Sec. 3.1), 0 = none
  int32_t late_codes;  // 1: a step fetches only the codes of links the visited table does not hold
  uint32_t *counters;  // [0] next query, [1] finished slots (queue mode)
  uint32_t *bits;
  int32_t *vlists;     // [slots][list_cap] ids whose bit is set (visited mode 1)
  int64_t words;
  int32_t *cand_ids;
  float *cand_adc;
  int32_t *cand_n, *stats;
  // 2-level codec (rfloat tables): first-level codes (c0 | c1 << 16), per-node terms, centroids per half
  const uint32_t *ccodes;
  const float *cnorm;
  int32_t coarse_k;
  int64_t lut_stride;  // table entries per query
};

// One table entry as float32: the entry itself, or the fp16 entry times its
// row's power-of-two scale (exact).
__device__ __forceinline__ float lut_at(const float *lut, const float *, int s, uint32_t c) {
  return lut[s * 256 + c];
}
__device__ __forceinline__ float lut_at(const __half *lut, const float *sc, int s, uint32_t c) {
  return __half2float(lut[s * 256 + c]) * sc[s];
}

// Table of the 2-level codec (Sec. 5.1): its [m][256] part holds
// -2 <z^s, C[s][c]> (rfloat: float32; rhalf: fp16 times its row's power-of-two
// scale); a node's key adds its two first-level entries (float32, read from the
// query's table row in global memory) and its stored term, clamped at 0.
struct rfloat {
  float v;
};
struct rhalf {
  __half v;
};
__device__ __forceinline__ float lut_at(const rfloat *lut, const float *, int s, uint32_t c) {
  return lut[s * 256 + c].v;
}
__device__ __forceinline__ float lut_at(const rhalf *lut, const float *sc, int s, uint32_t c) {
  return __half2float(lut[s * 256 + c].v) * sc[s];
}
template <typename T>
constexpr bool kRes = std::is_same<T, rfloat>::value || std::is_same<T, rhalf>::value;

// Table entries read together before they are summed (m is a multiple of 8).
constexpr int kAdcGroup = 8;

// Where a walk reads the query's table from.  LdsTab: the table staged in LDS,
// one load per entry, on any set of lanes.
template <typename T>
struct LdsTab {
  static constexpr bool kWaveWide = false;
  static constexpr int kGroup = kAdcGroup;  // entries read together
  const T *lut;
  __device__ __forceinline__ float at(const float *sc, int s, uint32_t c) const { return lut_at(lut, sc, s, c); }
};

// RegTab: an fp16 table spread over the wave's registers, 2m words per lane
// (m <= 56): lane l holds entries 4l .. 4l + 3 of every row s, in word 2s
// (entries 4l, 4l + 1 as low and high half) and word 2s + 1 (4l + 2,
// 4l + 3), so that entry c sits at lane c >> 2, at byte 2 (c & 3) of the
// lane's two words.  A read fetches both words from that lane with two
// cross-lane permutes, whose byte address is the code byte itself (the lane
// is the address over 4), and picks the entry with a byte permute whose
// selector comes from the code's two low bits; the four entries of a code
// word share the few operations that form their addresses and selectors.
// Every lane of the wave takes part in each permute, so callers evaluate
// keys on all 64 lanes and discard the ones they do not need.  Each entry's
// value is that of lut_at (the fp16 entry times its row's power-of-two
// scale), so keys are identical to the LDS table's.
template <int M>
struct RegTab {
  static constexpr bool kWaveWide = true;
  static constexpr int kGroup = 4;  // entries read together: one code word
  uint32_t r[2 * M];
  // row s of the table is 64 pairs of words; lane l takes pair l
  __device__ __forceinline__ void load(const __half *row, int lane) {
    const uint2 *w = reinterpret_cast<const uint2 *>(row);
#pragma unroll
    for (int s = 0; s < M; ++s) {
      const uint2 v = w[s * 64 + lane];
      r[2 * s] = v.x;
      r[2 * s + 1] = v.y;
    }
  }
  // acc plus the entries of rows s0 .. s0 + 3 at the four codes of word cw
  // (row s0 in its low byte), added in row order
  __device__ __forceinline__ float sum4(const float *sc, int s0, uint32_t cw, float acc) const {
    // per byte: 2 (c & 3), the entry's first byte within the two words, and the byte after it
    const uint32_t q2 = (cw << 1) & 0x06060606u;
    const uint32_t q2b = q2 | 0x01010101u;
    uint32_t w0[4], w1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int addr = int((cw >> (8 * t)) & 0xFFu);  // byte address 4 (c >> 2) + (c & 3)
      w0[t] = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(r[2 * (s0 + t)])));
      w1[t] = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(r[2 * (s0 + t) + 1])));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // selector: bytes 2q and 2q + 1 of (w1:w0) into the low half (byte values 0-3: w0, 4-7: w1)
      const uint32_t sel = __builtin_amdgcn_perm(q2b, q2, uint32_t(t) | (uint32_t(4 + t) << 8) | 0x0C0C0000u);
      const uint32_t v = __builtin_amdgcn_perm(w1[t], w0[t], sel);
      acc += __half2float(__ushort_as_half((unsigned short)(v & 0xFFFFu))) * sc[s0 + t];
    }
    return acc;
  }
};

// Stage the query's table into LDS, 16 bytes per lane and pass.
template <typename T, int M>
__device__ __forceinline__ void stage_table(T *dst, const T *src, int lane) {
  constexpr int kChunks = M * 256 * int(sizeof(T)) / 16;
  const float4 *s4 = reinterpret_cast<const float4 *>(src);
  float4 *d4 = reinterpret_cast<float4 *>(dst);
  for (int i = lane; i < kChunks; i += 64) d4[i] = s4[i];
}

// First-level entries of node id plus its stored term (2-level codec).
__device__ __forceinline__ float coarse_term(const WalkArgs &a, const float *ctab, int32_t id) {
  const uint32_t c = a.ccodes[id];
  return (ctab[c & 0xFFFFu] + ctab[a.coarse_k + (c >> 16)]) + a.cnorm[id];
}

// Sum of LUT[s][code[s]] over all sub-spaces, s ascending (one lane per node).
template <int M, typename T>
__device__ __forceinline__ float adc_full(const T *lut, const float *sc, const uint8_t *codes, int cs,
                                          int32_t id) {
  static_assert(M % 8 == 0, "m must be a multiple of 8");
  const uint8_t *row = codes + size_t(id) * cs;
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < M / 8; ++i) {
    const uint2 w = reinterpret_cast<const uint2 *>(row)[i];
    const uint32_t ws[2] = {w.x, w.y};
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = lut_at(lut, sc, i * 8 + t, (ws[t >> 2] >> (8 * (t & 3))) & 0xFFu);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc += v[t];
  }
  return acc;
}

// The m code bytes of one node in registers, then its ADC sum from them.
template <int M>
struct CodeRegs {
  uint32_t w[M / 4];
  float extra;  // 2-level codec: the node's first-level entries and term
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
  __device__ __forceinline__ void load_coarse(const WalkArgs &a, const float *ctab, int32_t id) {
    extra = coarse_term(a, ctab, id);
  }
  // the sum of the m entries (sub-space order) from either table view
  // The sum of the m entries (sub-space order) from either table view.  The
  // entries are read in groups of 8 before they are added, so that a group's
  // reads are in flight together rather than one LDS round trip per entry.
  template <typename Tab>
  __device__ __forceinline__ float adc_sum(const Tab &tab, const float *sc) const {
    constexpr int G = Tab::kGroup;
    float acc = 0.f;
    if constexpr (Tab::kWaveWide) {
#pragma unroll
      for (int i = 0; i < M / 4; ++i) acc = tab.sum4(sc, 4 * i, w[i], acc);
    } else {
#pragma unroll
      for (int s0 = 0; s0 < M; s0 += G) {
        float v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = tab.at(sc, s0 + g, (w[(s0 + g) >> 2] >> (8 * ((s0 + g) & 3))) & 0xFFu);
#pragma unroll
        for (int g = 0; g < G; ++g) acc += v[g];
      }
    }
    return acc;
  }
  template <typename T>
  __device__ __forceinline__ float adc(const T *lut, const float *sc) const {
    float acc = adc_sum(LdsTab<T>{lut}, sc);
    if constexpr (kRes<T>) acc = clamp0(acc + extra);
    return acc;
  }
};

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l));
  return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t hash_slot(int32_t id, int hshift) {
  return (uint32_t(id) * 0x9E3779B1u) >> hshift;
}

// Merges the kept keys (one per lane with `keep`, all unique, none in W, each
// below the largest key of W when W is full) into the sorted pool W[0..nw),
// keeping the best efe; nw is updated.  Without sorting the kept keys: each is
// broadcast in turn; its rank among the kept keys plus its count of smaller W
// entries is its slot, and every W entry moves up by the number of kept keys
// below it (chunks of 64 from the top, stopping below the smallest kept key).
// Returns the slot of the smallest kept key; before_ck = kept keys below ck.
__device__ __forceinline__ int merge_kept(uint64_t *W, int &nw, int efe, uint64_t k, bool keep, uint64_t km,
                                          uint64_t ck, int lane, int &before_ck) {
  const int nn = __popcll(km);
  uint64_t kmin = kKeyMax;
  int rank = 0;
  before_ck = 0;
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
  nw = nw + nn < efe ? nw + nn : efe;
  wave_sync();
  return pos_min;
}

// The visited table of walk_kernel: 2^(hash_bits-2) buckets of 16 bytes in
// LDS.  An id has one home bucket; it is stored there while the bucket has a
// free slot, and otherwise in the slot's bitset in the workspace (so an id is
// in exactly one of the two, and only a full bucket sends a look-up on to the
// bitset).  Narrow tables hold eight 16-bit tags per bucket: with
// h = id * 0x9E3779B1 mod 2^id_bits (a bijection), the bucket is the top bits
// of h and the tag the rest, so (bucket, tag) identifies the id.  Wide tables
// hold four ids per bucket (bucket from the top bits of the 32-bit product).
struct VTable {
  uint32_t *t;
  int bshift;       // wide: 32 - bucket bits
  int tbits;        // narrow: tag bits (<= 15)
  uint32_t hmask;   // narrow: 2^id_bits - 1
  bool narrow;
};


__device__ __forceinline__ void vt_locate(const VTable &v, int32_t id, uint32_t &b, uint32_t &tag) {
  const uint32_t p = uint32_t(id) * 0x9E3779B1u;
  if (v.narrow) {
    const uint32_t h = p & v.hmask;
    b = h >> v.tbits;
    tag = h & ((1u << v.tbits) - 1u);
  } else {
    b = p >> v.bshift;
    tag = uint32_t(id);
  }
}

__device__ __forceinline__ uint32_t dword_of(const uint4 &s, int i) {
  return i == 0 ? s.x : i == 1 ? s.y : i == 2 ? s.z : s.w;
}

// Packed unsigned 16-bit minimum and sum of two words, as single instructions
// (the compiler otherwise splits the halves into compares).
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ uint32_t pk_add_u16(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_pk_add_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// hit: the tag is in the bucket; e: its first free slot (-1: full).  Every
// store takes the first free slot of the bucket as read, so the filled slots
// are always a prefix and the first free slot is their count.  Narrow
// buckets are inspected two tags at a time with packed 16-bit arithmetic:
// min(x ^ tag, 1) is 0 exactly where x holds the tag, min(x + 1, 1) is 0
// exactly where x is empty (0xFFFF).
__device__ __forceinline__ void vt_inspect(const VTable &v, const uint4 &s, uint32_t tag, bool &hit, int &e) {
  uint32_t hm, em;
  if (v.narrow) {
    const uint32_t one = 0x00010001u;
    const uint32_t t2 = tag | (tag << 16);
    const uint32_t m0 = pk_min_u16(s.x ^ t2, one), m1 = pk_min_u16(s.y ^ t2, one);
    const uint32_t m2 = pk_min_u16(s.z ^ t2, one), m3 = pk_min_u16(s.w ^ t2, one);
    hit = ((m0 & m1) & (m2 & m3)) != one;
    const uint32_t f0 = pk_min_u16(pk_add_u16(s.x, one), one), f1 = pk_min_u16(pk_add_u16(s.y, one), one);
    const uint32_t f2 = pk_min_u16(pk_add_u16(s.z, one), one), f3 = pk_min_u16(pk_add_u16(s.w, one), one);
    const uint32_t cnt = pk_add_u16(pk_add_u16(f0, f1), pk_add_u16(f2, f3));
    const int filled = int(cnt & 0xFFFFu) + int(cnt >> 16);
    e = filled < 8 ? filled : -1;
    return;
  } else {
    hm = uint32_t(s.x == tag) | (uint32_t(s.y == tag) << 1) | (uint32_t(s.z == tag) << 2) |
         (uint32_t(s.w == tag) << 3);
    em = uint32_t(s.x == kEmpty) | (uint32_t(s.y == kEmpty) << 1) | (uint32_t(s.z == kEmpty) << 2) |
         (uint32_t(s.w == kEmpty) << 3);
  }
  hit = hm != 0u;
  e = em ? __builtin_ctz(em) : -1;
}

// One CAS that stores the tag in free slot e of bucket b, given the bucket as
// read; false when another lane changed that word first.
__device__ __forceinline__ bool vt_try_store(const VTable &v, uint32_t b, int e, uint32_t tag, const uint4 &s) {
  if (v.narrow) {
    const uint32_t seen = dword_of(s, e >> 1);
    const int sh = (e & 1) * 16;
    const uint32_t want = (seen & ~(0xFFFFu << sh)) | (tag << sh);
    return atomicCAS(&v.t[4 * b + (e >> 1)], seen, want) == seen;
  }
  return atomicCAS(&v.t[4 * b + e], kEmpty, tag) == kEmpty;
}

// Test-and-set of the bitset bit of id: true when it was clear.
__device__ __forceinline__ bool bit_set(uint32_t *bits, int32_t id) {
  const uint32_t bit = 1u << (uint32_t(id) & 31u);
  return (atomicOr(&bits[uint32_t(id) >> 5], bit) & bit) == 0u;
}

// Test of the bitset bit of id (device-coherent read): true when it is clear.
__device__ __forceinline__ bool bit_clear(uint32_t *bits, int32_t id) {
  const uint32_t w = __hip_atomic_load(&bits[uint32_t(id) >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (w & (1u << (uint32_t(id) & 31u))) == 0u;
}

// General test-and-set of id: true when id was not visited; set_bit tells
// that it went to the bitset.
__device__ __forceinline__ bool vt_insert(const VTable &v, uint32_t b, uint32_t tag, int32_t id, uint32_t *bits,
                                          bool &set_bit) {
  set_bit = false;
  for (;;) {
    const uint4 s = reinterpret_cast<const uint4 *>(v.t)[b];
    bool hit;
    int e;
    vt_inspect(v, s, tag, hit, e);
    if (hit) return false;
    if (e < 0) {
      const bool f = bit_set(bits, id);
      set_bit = f;
      return f;
    }
    if (vt_try_store(v, b, e, tag, s)) return true;
  }
}

// Lowest set bits of a 128-bit lane mask, one at a time (-1 once empty).
struct Pick2 {
  uint64_t lo, hi;
  __device__ __forceinline__ int next() {
    const bool l = lo != 0;
    const uint64_t m = l ? lo : hi;
    const int r = m ? __ffsll((unsigned long long)m) - 1 + (l ? 0 : 64) : -1;
    const uint64_t m2 = m & (m - 1);
    lo = l ? m2 : lo;
    hi = l ? hi : m2;
    return r;
  }
};

// Insertion of a single kept key k (held by lane j): entries above it move up
// by one, chunk by chunk from the top.  Returns its slot.
__device__ __forceinline__ int merge_one(uint64_t *W, int &nw, int efe, uint64_t k, int j, int lane) {
  const uint64_t kk = readlane64(k, j);
  int pos = 0;
  for (int c = (nw - 1) >> 6; c >= 0; --c) {
    const int idx = (c << 6) + lane;
    const bool in = idx < nw;
    const uint64_t v = in ? W[idx] : kKeyMax;
    const bool up = in && pure_key(v) > kk;
    wave_sync();
    if (up && idx + 1 < efe) W[idx + 1] = v;
    const uint64_t below = __ballot(in && !up);
    if (below) {  // the slot is in this chunk, right above its last entry below kk
      pos = (c << 6) + 64 - __clzll((long long)below);
      break;
    }
  }
  if (lane == 0 && pos < efe) W[pos] = kk;
  nw = nw + 1 < efe ? nw + 1 : efe;
  wave_sync();
  return pos;
}

// v moved up one lane across the whole wave; lane 0 receives `fill`.
__device__ __forceinline__ int shr1(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}

// Merge of 2..32 kept keys (one per lane with `keep` in km, all unique, none
// in W, each below the largest key of W when W is full) into the sorted pool
// W[0..nw), keeping the best efe; nw is updated.  The kept keys are packed
// into Ks in lane order, every lane reads them back and ranks its own key by
// counting the smaller ones, and each key is then stored at its rank, so that
// Ks holds them sorted.  Chunks of 64 entries move
// from the top down: an entry moves up by the number of kept keys below it,
// and the kept keys of ranks [below entry i-1, below entry i) land just
// below entry i (slot nw acts as +inf).  Each chunk's counts come with the
// next-lower chunk read one step ahead, whose top lane gives lane 0 its
// predecessor's count; the walk stops below the smallest kept key.
// Returns the slot of the smallest kept key.
template <bool Ahead>
__device__ __forceinline__ int merge_keys(uint64_t *W, uint64_t *Ks, int &nw, int efe, uint64_t k, bool keep,
                                          uint64_t km, int lane) {
  const int nn = __popcll(km);
  const bool mid = nn > 8, more = nn > 16;
  // packed in lane order (slots past nn keep the largest key, which never counts as smaller)
  const int packed = int(__builtin_amdgcn_mbcnt_hi(uint32_t(km >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(km), 0u)));
  if (lane < 32) Ks[lane] = kKeyMax;
  wave_sync();
  if (keep) Ks[packed] = k;
  wave_sync();
  uint64_t kv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) kv[j] = Ks[j];
  int rank;
  {
    int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
      r0 += kv[j] < k ? 1 : 0;
      r1 += kv[j + 1] < k ? 1 : 0;
      r2 += kv[j + 2] < k ? 1 : 0;
      r3 += kv[j + 3] < k ? 1 : 0;
    }
    if (more) {
#pragma unroll
      for (int j = 16; j < 32; j += 4) {
        r0 += Ks[j] < k ? 1 : 0;
        r1 += Ks[j + 1] < k ? 1 : 0;
        r2 += Ks[j + 2] < k ? 1 : 0;
        r3 += Ks[j + 3] < k ? 1 : 0;
      }
    }
    rank = (r0 + r1) + (r2 + r3);
  }
  wave_sync();  // every read of the packed keys comes before the sorted store
  if (keep) Ks[rank] = k;
  wave_sync();
  // below() counts over kv and, past 16 keys, over Ks[16 .. 32): the two must
  // then be the sorted halves; up to 16 keys kv holds them all in packed order
  if (more) {
#pragma unroll
    for (int j = 0; j < 16; ++j) kv[j] = Ks[j];
  }
  // number of kept keys below x (the padding never counts), in four
  // independent sums so that the compares overlap
  auto below = [&](uint64_t x) {
    int n0 = 0, n1 = 0, n2 = 0, n3 = 0;
#pragma unroll
    for (int j = 0; j < 8; j += 4) {
      n0 += kv[j] < x ? 1 : 0;
      n1 += kv[j + 1] < x ? 1 : 0;
      n2 += kv[j + 2] < x ? 1 : 0;
      n3 += kv[j + 3] < x ? 1 : 0;
    }
    if (mid) {
#pragma unroll
      for (int j = 8; j < 16; j += 4) {
        n0 += kv[j] < x ? 1 : 0;
        n1 += kv[j + 1] < x ? 1 : 0;
        n2 += kv[j + 2] < x ? 1 : 0;
        n3 += kv[j + 3] < x ? 1 : 0;
      }
    }
    if (more) {
#pragma unroll
      for (int j = 16; j < 32; j += 4) {
        n0 += Ks[j] < x ? 1 : 0;
        n1 += Ks[j + 1] < x ? 1 : 0;
        n2 += Ks[j + 2] < x ? 1 : 0;
        n3 += Ks[j + 3] < x ? 1 : 0;
      }
    }
    return (n0 + n1) + (n2 + n3);
  };
  int c = nw >> 6;
  int idx = (c << 6) + lane;
  uint64_t v = idx < nw ? W[idx] : kKeyMax;
  // lower chunks lie wholly below nw and no chunk's writes reach below it, so
  // with Ahead each is read one step before its turn (two more registers)
  uint64_t vl = Ahead && c > 0 ? W[idx - 64] : 0;
  int cnt = idx < nw ? below(pure_key(v)) : nn;
  int pos_min = efe;
  for (; c >= 0; --c) {
    int cl = 0;
    const int il = ((c - 1) << 6) + lane;
    uint64_t vll = 0;
    if constexpr (Ahead) {
      if (c > 1) vll = W[il - 64];
    } else if (c > 0) {
      vl = W[il];
    }
    if (c > 0) cl = below(pure_key(vl));
    const int fill = c > 0 ? __builtin_amdgcn_readlane(cl, 63) : 0;
    const int cprev = shr1(cnt, fill);
    wave_sync();  // reads of this chunk and the one below come before any write
    if (idx < nw && cnt > 0 && idx + cnt < efe) W[idx + cnt] = v;
    for (int t = cprev; t < cnt; ++t)
      if (idx + t < efe) W[idx + t] = Ks[t];
    const uint64_t m0 = __ballot(cprev == 0 && cnt > 0 && idx <= nw);
    wave_sync();
    if (fill == 0) {  // nothing below this chunk moves
      if (m0) pos_min = (c << 6) + __ffsll((unsigned long long)m0) - 1;
      break;
    }
    idx = il;
    v = vl;
    if constexpr (Ahead) vl = vll;
    cnt = cl;
  }
  nw = nw + nn < efe ? nw + nn : efe;
  return pos_min;
}

// Merge of 1..32 kept keys (as merge_keys), a single one by merge_one.
template <bool Ahead>
__device__ __forceinline__ int merge_few(uint64_t *W, uint64_t *Ks, int &nw, int efe, uint64_t k, bool keep,
                                         uint64_t km, int lane) {
  if (__popcll(km) == 1) return merge_one(W, nw, efe, k, __ffsll((unsigned long long)km) - 1, lane);
  return merge_keys<Ahead>(W, Ks, nw, efe, k, keep, km, lane);
}

// ---------------------------------------------------------------------------
// The pool held in registers (pools of up to 64 R entries): lane l of chunk c
// holds entry 64 c + l, and entries at or past nw hold kKeyMax (whose expanded
// flag keeps them out of every scan and whose key sorts last).  Entries
// compare by key without the flag.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_lt(uint64_t a, uint64_t b) { return pure_key(a) < pure_key(b); }
__device__ __forceinline__ uint64_t key_min(uint64_t a, uint64_t b) { return key_lt(b, a) ? b : a; }
__device__ __forceinline__ uint64_t key_max(uint64_t a, uint64_t b) { return key_lt(b, a) ? a : b; }

// The value of lane (lane ^ J), without the LDS crossbar: quad permutes for
// J = 1, 2, row shifts for J = 4, 8, and the half-row / half-wave swaps of
// gfx950 for J = 16, 32.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int lane) {
  if constexpr (J == 1) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xf, 0xf, false));  // quad_perm [1,0,3,2]
  } else if constexpr (J == 2) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xf, 0xf, false));  // quad_perm [2,3,0,1]
  } else if constexpr (J == 4 || J == 8) {
    const uint32_t up = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x100 | J, 0xf, 0xf, false));  // row_shl:J
    const uint32_t dn = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x110 | J, 0xf, 0xf, false));  // row_shr:J
    return (lane & J) ? dn : up;
  } else if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? r[0] : r[1];
  } else {
    static_assert(J == 32, "xor distance");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? r[0] : r[1];
  }
}
template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, int lane) {
  const uint32_t lo = xor_lane<J>(uint32_t(v), lane), hi = xor_lane<J>(uint32_t(v >> 32), lane);
  return (uint64_t(hi) << 32) | lo;
}

// Lane 63 - lane's value: each row of 16 mirrored, then rows r and 3 - r exchanged.
__device__ __forceinline__ uint64_t reverse64(uint64_t v, int lane) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(v)), 0x140, 0xf, 0xf, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(v >> 32)), 0x140, 0xf, 0xf, false));
  return xor_lane64<16>(xor_lane64<32>((uint64_t(hi) << 32) | lo, lane), lane);
}

// Compare-exchange with the lane at xor-distance J: keep the smaller entry
// when keep_min, else the larger.
template <int J>
__device__ __forceinline__ uint64_t cx(uint64_t v, bool keep_min, int lane) {
  const uint64_t o = xor_lane64<J>(v, lane);
  return keep_min == key_lt(o, v) ? o : v;
}

// A bitonic sequence over the 64 lanes, sorted ascending (distances J .. 1).
template <int J = 32>
__device__ __forceinline__ uint64_t bitonic_clean(uint64_t v, int lane) {
  v = cx<J>(v, (lane & J) == 0, lane);
  if constexpr (J > 1) return bitonic_clean<J / 2>(v, lane);
  else return v;
}

// Two bitonic sequences sorted together, stage by stage (independent work).
template <int J = 32>
__device__ __forceinline__ void bitonic_clean2(uint64_t &a, uint64_t &b, int lane) {
  const bool lo = (lane & J) == 0;
  a = cx<J>(a, lo, lane);
  b = cx<J>(b, lo, lane);
  if constexpr (J > 1) bitonic_clean2<J / 2>(a, b, lane);
}

// Any 64 entries sorted ascending across the lanes: merges of sorted runs of
// K / 2 into runs of K, K = 2 .. 64.
template <int K = 2, int J = 1>
__device__ __forceinline__ uint64_t bitonic_sort(uint64_t v, int lane) {
  v = cx<J>(v, ((lane & J) == 0) == ((lane & K) == 0), lane);
  if constexpr (J > 1) return bitonic_sort<K, J / 2>(v, lane);
  else if constexpr (K < 64) return bitonic_sort<K * 2, K>(v, lane);
  else return v;
}

// The pool's chunks as named registers (never an array, so that no access
// can become an indexed one into private memory); R <= 2 are used.
struct Pool {
  uint64_t w0, w1;
};
template <int C>
__device__ __forceinline__ uint64_t &chunk(Pool &p) {
  static_assert(C >= 0 && C < 2, "chunk index");
  if constexpr (C == 0) return p.w0;
  else return p.w1;
}

// f(integral_constant<C>) for C = B, B+1, .., E-1 (ascending) or E-1 .. B (descending).
template <int B, int E, typename F>
__device__ __forceinline__ void for_chunks(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    for_chunks<B + 1, E>(f);
  }
}
template <int B, int E, typename F>
__device__ __forceinline__ void for_chunks_down(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    for_chunks_down<B, E - 1>(f);
  }
}

// Entry i of the pool (i uniform); the chunks come by value, so that the
// choice between them is a choice between values, never between addresses.
template <int R>
__device__ __forceinline__ uint64_t entry_of(uint64_t w0, uint64_t w1, int i) {
  return readlane64(R > 1 && (i >> 6) == 1 ? w1 : w0, i & 63);
}
template <int R>
__device__ __forceinline__ uint64_t entry_at(const Pool &p, int i) {
  return entry_of<R>(p.w0, p.w1, i);
}

// Sets the expanded flag of entry i (i uniform).
template <int R>
__device__ __forceinline__ void mark_expanded(Pool &p, int i, int lane) {
  const bool here = lane == (i & 63);
  for_chunks<0, R>([&](auto C) {
    uint64_t &w = chunk<C>(p);
    w = (here && (i >> 6) == C) ? (w | kExpanded) : w;
  });
}

// Entries at or past efe are dropped.
template <int R>
__device__ __forceinline__ void truncate_pool(Pool &p, int efe, int lane) {
  for_chunks<0, R>([&](auto C) {
    uint64_t &w = chunk<C>(p);
    w = (C << 6) + lane >= efe ? kKeyMax : w;
  });
}

// One kept key kk (not in W, below the largest entry when W is full): the
// entries above it move up one slot.
template <int R>
__device__ __forceinline__ void reg_insert_one(Pool &p, uint64_t kk, int efe, int lane) {
  int pos = 0;
  for_chunks<0, R>([&](auto C) { pos += __popcll(__ballot(key_lt(chunk<C>(p), kk))); });
  for_chunks_down<0, R>([&](auto C) {
    // entry 64 C + lane - 1, from the chunk below for lane 0 (read before that chunk changes)
    uint64_t fill = kKeyMax;
    if constexpr (C > 0) fill = readlane64(chunk<C - 1>(p), 63);
    uint64_t &w = chunk<C>(p);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill)), int(uint32_t(w)), 0x138, 0xf, 0xf,
                                                             false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(fill >> 32)), int(uint32_t(w >> 32)),
                                                             0x138, 0xf, 0xf, false));
    const uint64_t up = (uint64_t(hi) << 32) | lo;
    const int idx = (C << 6) + lane;
    w = idx < pos ? w : (idx == pos ? kk : up);
  });
  truncate_pool<R>(p, efe, lane);
}

// Kept keys, sorted ascending (lane r holds the r-th, the rest kKeyMax),
// merged into the pool: the best 64 R of pool and keys, sorted, of which the
// first efe are kept.  The 64 largest of pool and keys lie in the top chunk
// and the keys, so the keys first meet the top chunk; what is left below
// meets the next chunk down, until a chunk lies wholly below what is left.
template <int R>
__device__ __forceinline__ void reg_merge_sorted(Pool &p, uint64_t kv, int efe, int lane) {
  uint64_t x = bitonic_clean(key_min(chunk<R - 1>(p), reverse64(kv, lane)), lane);
  bool done = false;
  for_chunks_down<0, R - 1>([&](auto C) {
    if (!done) {
      uint64_t &w = chunk<C>(p);
      if (key_lt(readlane64(w, 63), readlane64(x, 0))) {
        chunk<C + 1>(p) = x;  // chunk C and those below stay as they are
        done = true;
      } else {
        const uint64_t rx = reverse64(x, lane);
        uint64_t hi = key_max(w, rx), lo = key_min(w, rx);
        bitonic_clean2(hi, lo, lane);
        chunk<C + 1>(p) = hi;
        x = lo;
      }
    }
  });
  if (!done) p.w0 = x;
  truncate_pool<R>(p, efe, lane);
}

// Greedy descent on levels max_level .. 1 (Sec. 2): from the entry node,
// move to the best link while it beats the current key, one lane per link.
// (Fetching every link's upper row index with its code saves one dependent
// load per move but reads a cache line per link for it: more HBM traffic and
// no measurable time, so the winner's row index is read after the move.)
template <int M, typename T, typename Tab>
__device__ __forceinline__ void greedy_descent(const WalkArgs &a, const Tab &tab, const float *sc, int lane,
                                               int32_t &cur, uint64_t &curkey, const float *ctab) {
  auto dist = [&](int32_t id) {
    float v;
    if constexpr (Tab::kWaveWide) {
      CodeRegs<M> cr;
      cr.load(a.codes, a.code_stride, id);
      v = cr.adc_sum(tab, sc);
    } else {
      v = adc_full<M, T>(tab.lut, sc, a.codes, a.code_stride, id);
    }
    if constexpr (kRes<T>) v = clamp0(v + coarse_term(a, ctab, id));
    return v;
  };
  cur = a.entry;
  curkey = make_key(dist(cur), cur);
  for (int l = a.max_level; l >= 1; --l) {
    for (;;) {
      const int64_t row = int64_t(a.up_base[cur]) + l - 1;
      int32_t nb = -1;
      if (lane < a.deg_up && row >= 0 && row < a.n_up_rows) nb = a.adj_up[row * a.deg_up + lane];
      if (nb >= a.n) nb = -1;  // a malformed link is ignored rather than followed
      uint64_t k;
      if constexpr (Tab::kWaveWide) {  // every lane evaluates (a missing link: the current node's code)
        const float v = dist(nb >= 0 ? nb : cur);
        k = nb >= 0 ? make_key(v, nb) : kKeyMax;
      } else {
        k = nb >= 0 ? make_key(dist(nb), nb) : kKeyMax;
      }
      const uint64_t mn = wave_min64(k);
      if (mn < curkey) {
        curkey = mn;
        cur = key_id(mn);
      } else {
        break;
      }
    }
  }
}

// Links of the expanded entry c (lanes 0..31, nb) and of the next unexpanded
// entry p (lanes 32..63 when `two`): test-and-set against the visited set,
// codes and ADC keys, and whether p's expansion is the sequential walk's next
// step (dual).  D, E and the bitset id list are updated; `fresh` marks the
// keys that enter the merge (subject to the wmax filter).  With a budget T on
// distance evaluations, the evaluation that reaches T is the walk's last: the
// fresh links past it (in link order, c's before p's) are dropped and `stop`
// ends the walk after this step's merge.
struct StepOut {
  uint64_t k;
  bool fresh, dual, stop;
};

// Keep the first `room` lanes of mask m (in lane order) when m has more;
// returns the kept mask and sets stop when the budget is reached.
__device__ __forceinline__ uint64_t budget_cut(uint64_t m, int D, int max_d, bool &stop) {
  if (max_d <= 0) return m;
  const int room = max_d - D;  // >= 1: a walk that reached its budget has stopped
  if (__popcll(m) < room) return m;
  stop = true;
  uint64_t kept = 0;
  for (int i = 0; i < room; ++i) {
    const uint64_t low = m & (~m + 1ull);
    kept |= low;
    m ^= low;
  }
  return kept;
}

template <int M, typename T, bool BUDGET, typename Tab>
__device__ __forceinline__ StepOut expand_links(const WalkArgs &a, const VTable &vt, uint32_t *bits, int32_t *vlist,
                                                const Tab &tab, const float *sc, int32_t nb, int32_t cid,
                                                const float *ctab, bool lo, bool two, uint64_t pk, int lane, int &D,
                                                int &E, int &vcount) {
  // The links' codes: by default every link's, fetched while the visited set
  // is probed (a link that turns out visited reads its code for nothing);
  // with late_codes only those of links the table does not hold, once the
  // probe has answered (the other lanes read the expanded node's own code,
  // one shared line).
  CodeRegs<M> cr;
  const bool late = a.late_codes != 0;
  if (!late) {
    cr.load(a.codes, a.code_stride, nb >= 0 ? nb : cid);
    if constexpr (kRes<T>) cr.load_coarse(a, ctab, nb >= 0 ? nb : cid);
  }
  // lanes 0..31 test-and-set c's links; lanes 32..63 look p's links up.
  // One bucket read and at most one CAS settle almost every link; a full
  // bucket or a lost CAS goes round the general path.
  const bool act = nb >= 0;
  uint32_t b, tag;
  vt_locate(vt, act ? nb : 0, b, tag);
  const uint4 s4 = reinterpret_cast<const uint4 *>(vt.t)[b];
  bool hit;
  int e;
  vt_inspect(vt, s4, tag, hit, e);
  hit = hit & act;
  if (late) {
    const int32_t src = act && !hit ? nb : cid;
    cr.load(a.codes, a.code_stride, src);
    if constexpr (kRes<T>) cr.load_coarse(a, ctab, src);
  }
  const bool ins = act & lo & !hit & (e >= 0);
  bool ok = false;
  if (ins) ok = vt_try_store(vt, b, e, tag, s4);
  bool cand = lo ? ok : (act & !hit & (e >= 0));  // lanes 32..63: absent before this step
  bool set_bit = false;
  const bool rest = act & !hit & ((e < 0) | (ins & !ok));
  if (__ballot(rest)) {
    if (rest) {
      if (lo) cand = vt_insert(vt, b, tag, nb, bits, set_bit);
      else cand = bit_clear(bits, nb);  // the bucket is full: the bitset decides
    }
  }
  StepOut o;
  o.stop = false;
  if constexpr (BUDGET) {
    const uint64_t cm = __ballot(lo && cand);
    const uint64_t kept = budget_cut(cm, D, a.max_d, o.stop);
    if (lo) cand = cand && ((kept >> lane) & 1ull);  // a dropped link stays marked: the walk ends here
    D += __popcll(kept);
  } else {
    D += __popcll(__ballot(lo && cand));
  }

  // ADC keys of both halves' candidates, from the codes loaded at the start of the step
  o.k = kKeyMax;
  if constexpr (Tab::kWaveWide) {  // every lane evaluates, candidates keep theirs
    const float v = cr.adc_sum(tab, sc);
    if (cand) o.k = make_key(v, nb);
  } else {
    if (cand) o.k = make_key(cr.adc(tab.lut, sc), nb);
  }

  // p is the next expansion of the sequential walk iff no fresh key of c is below it
  o.dual = (!BUDGET || !o.stop) && two && __ballot(lo && cand && o.k < pk) == 0ull;
  o.fresh = lo && cand;
  if (o.dual) {
    // p's absent links, inserted for real: one CAS at the slot the look-up
    // saw free, the general path otherwise (a full bucket: the bitset)
    const bool ins2 = !lo & cand & (e >= 0);
    bool ok2 = false;
    if (ins2) ok2 = vt_try_store(vt, b, e, tag, s4);
    if (!lo) o.fresh = ok2;
    const bool rest2 = !lo & cand & !ok2;
    if (__ballot(rest2)) {
      if (rest2) o.fresh = vt_insert(vt, b, tag, nb, bits, set_bit);
    }
    if constexpr (BUDGET) {
      const uint64_t pm = budget_cut(__ballot(!lo && o.fresh), D, a.max_d, o.stop);
      if (!lo) o.fresh = o.fresh && ((pm >> lane) & 1ull);
      D += __popcll(pm);
    } else {
      D += __popcll(__ballot(!lo && o.fresh));
    }
    E += 2;
  } else {
    E += 1;
  }
  // ids that went to the bitset, listed for clearing at the end of the query
  const uint64_t sb = __ballot(set_bit);
  if (sb) {
    const int at = vcount + __popcll(sb & ((1ull << lane) - 1ull));
    if (set_bit && at < a.list_cap) vlist[at] = nb;
    vcount += __popcll(sb);
  }
  return o;
}

// Level-0 walk with the visited set in an LDS table (and the bitset for ids
// whose home bucket is full), two expansions per step when the sequential
// order allows it; the query's table in LDS, or (RL) an fp16 table in
// registers.
template <int M, typename T, bool BUDGET, bool RL>
__device__ __forceinline__ void walk_body(const WalkArgs &a) {
  static_assert(!RL || std::is_same<T, __half>::value, "registers hold fp16 tables only");
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  const bool lo = lane < 32;
  constexpr int kLutBytes = RL ? 0 : M * 256 * int(sizeof(T));
  constexpr int kScaleBytes = sizeof(T) == 2 ? (M * 4 + 15) / 16 * 16 : 0;
  T *lut = reinterpret_cast<T *>(smem);
  float *sc = reinterpret_cast<float *>(smem + kLutBytes);
  uint64_t *W = reinterpret_cast<uint64_t *>(smem + kLutBytes + kScaleBytes);
  uint64_t *Ks = W + a.w_cap;  // merge scratch: the kept keys (compacted, then sorted)
  using Tab = std::conditional_t<RL, RegTab<M>, LdsTab<T>>;
  // the merge's read-ahead, except where its two registers would cost the
  // register-table kernel its third wave per SIMD (m <= 24)
  constexpr bool kAhead = !RL || M > 24;
  Tab tab;
  if constexpr (!RL) tab.lut = lut;
  uint32_t *hash = reinterpret_cast<uint32_t *>(Ks + kMergeScratch);
  const int H = 1 << a.hash_bits;  // table words
  VTable vt;
  vt.t = hash;
  vt.bshift = 32 - (a.hash_bits - 2);
  vt.tbits = a.tag_bits;
  vt.hmask = a.tag_bits ? uint32_t((1ull << (a.tag_bits + a.hash_bits - 2)) - 1ull) : 0u;
  vt.narrow = a.tag_bits != 0;
  uint32_t *bits = a.bits + int64_t(blockIdx.x) * a.words;
  int32_t *vlist = a.vlists + int64_t(blockIdx.x) * a.list_cap;
  // every row load reads a valid column, so that loads need no branch around them
  const int lcol = l32 < a.deg0 ? l32 : a.deg0 - 1;
  const bool col_ok = l32 < a.deg0;

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
      const T *src = static_cast<const T *>(a.lut) + q * a.lut_stride;
      [[maybe_unused]] const float *ctab =
          kRes<T> ? reinterpret_cast<const float *>(static_cast<const T *>(a.lut) + q * a.lut_stride + M * 256)
                  : nullptr;
      if constexpr (RL)
        tab.load(src, lane);
      else
        stage_table<T, M>(lut, src, lane);
      if (sizeof(T) == 2)
        for (int i = lane; i < M; i += 64) sc[i] = a.scale[q * M + i];
      for (int i = lane; i < H; i += 64) hash[i] = kEmpty;
      wave_sync();

      // greedy descent on levels max_level .. 1
      int32_t cur;
      uint64_t curkey;
      greedy_descent<M, T>(a, tab, sc, lane, cur, curkey, ctab);

      // best-first walk on level 0
      if (lane == 0) {
        W[0] = curkey;
        uint32_t b0, t0;
        vt_locate(vt, cur, b0, t0);
        hash[4 * b0] = vt.narrow ? (t0 | 0xFFFF0000u) : t0;
      }
      int nw = 1, fu = 0, pidx = -1, E = 0, D = 0, vcount = 0;
      uint64_t ck = curkey;                         // key of W[fu], the next expansion
      uint64_t pk = kKeyMax;                        // key of W[pidx], the unexpanded entry after it
      uint64_t wmax = efe == 1 ? curkey : kKeyMax;  // largest key of W once W is full
      int32_t pre0 = -1, pre1 = -1;                 // ids whose rows `nxt` holds (lanes 0..31, 32..63)
      int32_t row = a.adj0[int64_t(cur) * a.deg0 + lcol];
      if (row >= a.n) row = -1;  // a malformed link is ignored rather than followed
      wave_sync();
      while (fu < nw) {
        const int32_t cid = key_id(ck);
        // rows of the entries likely to come next; every lane loads, from the
        // expanded node's own row when there is no guess
        int32_t nxt = 0;
        if (a.prefetch) {
          const int32_t g = lo ? pre0 : pre1;
          nxt = a.adj0[int64_t(g >= 0 ? g : cid) * a.deg0 + lcol];
        }
        const bool two = pidx >= 0;
        if (lane == 0) W[fu] = ck | kExpanded;
        const int32_t nb = col_ok && (lo || two) ? row : -1;
        const StepOut o = expand_links<M, T, BUDGET>(a, vt, bits, vlist, tab, sc, nb, cid, ctab, lo, two, pk, lane, D,
                                                     E, vcount);
        const bool dual = o.dual;
        const bool fresh = o.fresh;
        const uint64_t k = o.k;
        if (dual && lane == 0) W[pidx] = pk | kExpanded;
        wave_sync();

        const bool keep = fresh && k < wmax;
        const uint64_t km = __ballot(keep);
        int p0 = fu;
        if (km) {
          const int nn = __popcll(km);
          int pos_min;
          if (nn <= 32) {
            pos_min = merge_few<kAhead>(W, Ks, nw, efe, k, keep, km, lane);
          } else {
            // more than 32 (the first steps of a walk): c's links, then p's, which are filtered
            // again by the pool's largest key once c's have filled it
            pos_min = merge_few<kAhead>(W, Ks, nw, efe, k, keep && lo, km & 0xFFFFFFFFull, lane);
            wave_sync();
            const uint64_t wm = nw == efe ? pure_key(W[nw - 1]) : kKeyMax;
            const bool keep2 = keep && !lo && k < wm;
            const uint64_t km2 = __ballot(keep2);
            if (km2) {
              const int pos2 = merge_few<kAhead>(W, Ks, nw, efe, k, keep2, km2, lane);
              pos_min = pos2 < pos_min ? pos2 : pos_min;
            }
          }
          // unexpanded entries were at or above fu and only move up; new ones sit at or above pos_min
          p0 = fu < pos_min ? fu : pos_min;
          wave_sync();
          wmax = nw == efe ? pure_key(W[nw - 1]) : kKeyMax;
        }
        if (BUDGET && o.stop) break;  // the budget of distance evaluations is spent

        // the first four unexpanded entries at or after p0 (all before are expanded),
        // from two chunks at a time
        int i0 = nw, i1 = -1;
        uint64_t k0 = 0, k1 = kKeyMax;
        int32_t g2 = -1, g3 = -1;
        {
          const int ia = p0 + lane, ib = p0 + 64 + lane;
          const uint64_t va = ia < nw ? W[ia] : kExpanded;
          const uint64_t vb = ib < nw ? W[ib] : kExpanded;
          Pick2 pm;
          pm.lo = __ballot((va & kExpanded) == 0);
          pm.hi = __ballot((vb & kExpanded) == 0);
          const int r0 = pm.next(), r1 = pm.next(), r2 = pm.next(), r3 = pm.next();
          const uint64_t x0 = readlane64(r0 < 64 ? va : vb, r0 & 63);
          const uint64_t x1 = readlane64(r1 < 64 ? va : vb, r1 & 63);
          const int32_t y2 = __builtin_amdgcn_readlane(int(uint32_t(r2 < 64 ? va : vb)), r2 & 63) & 0x7FFFFFFF;
          const int32_t y3 = __builtin_amdgcn_readlane(int(uint32_t(r3 < 64 ? va : vb)), r3 & 63) & 0x7FFFFFFF;
          if (r0 >= 0) {
            i0 = p0 + r0;
            k0 = x0;
          }
          if (r1 >= 0) {
            i1 = p0 + r1;
            k1 = x1;
          }
          g2 = r2 >= 0 ? y2 : -1;
          g3 = r3 >= 0 ? y3 : -1;
          if (r3 < 0 && p0 + 128 < nw) {
            // fewer than four in these two chunks: look further (rare)
            int found = r0 < 0 ? 0 : r1 < 0 ? 1 : r2 < 0 ? 2 : 3;
            for (int base = p0 + 128; base < nw && found < 4; base += 64) {
              const int idx = base + lane;
              const uint64_t v = idx < nw ? W[idx] : kExpanded;
              uint64_t bm = __ballot((v & kExpanded) == 0);
              while (bm && found < 4) {
                const int l = __ffsll((unsigned long long)bm) - 1;
                const uint64_t x = readlane64(v, l);
                if (found == 0) {
                  i0 = base + l;
                  k0 = x;
                } else if (found == 1) {
                  i1 = base + l;
                  k1 = x;
                } else if (found == 2) {
                  g2 = key_id(x);
                } else {
                  g3 = key_id(x);
                }
                ++found;
                bm &= bm - 1;
              }
            }
          }
        }
        fu = i0;
        pidx = i1;
        if (fu < nw) {
          ck = k0;
          pk = k1;
          const int32_t nc = key_id(k0);
          const int32_t np = i1 >= 0 ? key_id(k1) : -1;
          // only a dual step can meet the guess: when p was not expanded, a
          // kept key of c lies below key(p) and comes next
          if (a.prefetch && dual && nc == pre0 && (np < 0 || np == pre1)) {
            row = nxt;  // the guessed pair came next
          } else {
            row = a.adj0[int64_t(lo || np < 0 ? nc : np) * a.deg0 + lcol];
          }
          if (row >= a.n) row = -1;
          pre0 = g2;
          pre1 = g3;
        }
        // nothing is in flight across steps: the next step's loads are the only ones to wait for
        __builtin_amdgcn_s_waitcnt(0);
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
      if (vcount > 0) {
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

template <int M, typename T, bool BUDGET>
__global__ __launch_bounds__(64) void walk_kernel(WalkArgs a) {
  walk_body<M, T, BUDGET, false>(a);
}

// The same walk with the fp16 table in registers (RegTab): a slot's LDS holds
// the row scales, the pool and the visited table only, so that a CU keeps up
// to 8 slots (two waves per SIMD) where the table in LDS keeps it to 3 or 4
// (m >= 48); the register budget is held to 256 for those two waves, and to
// 168 for three at m <= 24 (12 slots; at m = 24 a few registers spill).
template <int M, bool BUDGET>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(M <= 24 ? 3 : 2))) void walk_rl_kernel(
    WalkArgs a) {
  walk_body<M, __half, BUDGET, true>(a);
}

// The same walk with the pool in registers (pools of up to 64 R entries, R <= 2):
// the scan for the next unexpanded entries is a ballot per chunk, one kept key
// moves the entries above it up one lane, and several kept keys are sorted
// and merged by bitonic networks; LDS holds only the table and the visited
// table.
template <int M, typename T, int R, bool BUDGET>
__global__ __launch_bounds__(64) void walk_reg_kernel(WalkArgs a) {
  static_assert(R >= 1 && R <= 2, "pool chunks");
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  const bool lo = lane < 32;
  constexpr int kLutBytes = M * 256 * int(sizeof(T));
  // LDS holds only the table and the visited table (the fp16 row scales live
  // in registers, the sorting permutation goes through ds_permute), so that a
  // slot of m = 16 fp16 with 2^11 table words takes exactly 16 KB
  T *lut = reinterpret_cast<T *>(smem);
  uint32_t *hash = reinterpret_cast<uint32_t *>(smem + kLutBytes);
  const int H = 1 << a.hash_bits;  // table words
  VTable vt;
  vt.t = hash;
  vt.bshift = 32 - (a.hash_bits - 2);
  vt.tbits = a.tag_bits;
  vt.hmask = a.tag_bits ? uint32_t((1ull << (a.tag_bits + a.hash_bits - 2)) - 1ull) : 0u;
  vt.narrow = a.tag_bits != 0;
  uint32_t *bits = a.bits + int64_t(blockIdx.x) * a.words;
  int32_t *vlist = a.vlists + int64_t(blockIdx.x) * a.list_cap;
  // every row load reads a valid column, so that loads need no branch around them
  const int lcol = l32 < a.deg0 ? l32 : a.deg0 - 1;
  const bool col_ok = l32 < a.deg0;

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

      // stage the table, take its row scales into registers, clear the visited table
      const T *src = static_cast<const T *>(a.lut) + q * a.lut_stride;
      [[maybe_unused]] const float *ctab =
          kRes<T> ? reinterpret_cast<const float *>(static_cast<const T *>(a.lut) + q * a.lut_stride + M * 256)
                  : nullptr;
      stage_table<T, M>(lut, src, lane);
      float scr[sizeof(T) == 2 ? M : 1];
#pragma unroll
      for (int i = 0; i < (sizeof(T) == 2 ? M : 1); ++i) scr[i] = sizeof(T) == 2 ? a.scale[q * M + i] : 1.f;
      const float *sc = scr;
      for (int i = lane; i < H; i += 64) hash[i] = kEmpty;
      wave_sync();

      // greedy descent on levels max_level .. 1
      int32_t cur;
      uint64_t curkey;
      greedy_descent<M, T>(a, LdsTab<T>{lut}, sc, lane, cur, curkey, ctab);

      // best-first walk on level 0
      if (lane == 0) {
        uint32_t b0, t0;
        vt_locate(vt, cur, b0, t0);
        hash[4 * b0] = vt.narrow ? (t0 | 0xFFFF0000u) : t0;
      }
      Pool wr = {kKeyMax, kKeyMax};
      if (lane == 0) wr.w0 = curkey;
      int nw = 1, fu = 0, pidx = -1, E = 0, D = 0, vcount = 0;
      uint64_t ck = curkey;                         // key of entry fu, the next expansion
      uint64_t pk = kKeyMax;                        // key of entry pidx, the unexpanded entry after it
      uint64_t wmax = efe == 1 ? curkey : kKeyMax;  // largest key of W once W is full
      int32_t pre0 = -1, pre1 = -1;                 // ids whose rows `nxt` holds (lanes 0..31, 32..63)
      int32_t row = a.adj0[int64_t(cur) * a.deg0 + lcol];
      if (row >= a.n) row = -1;  // a malformed link is ignored rather than followed
      wave_sync();
      while (fu < nw) {
        const int32_t cid = key_id(ck);
        // rows of the entries likely to come next; every lane loads, from the
        // expanded node's own row when there is no guess
        int32_t nxt = 0;
        if (a.prefetch) {
          const int32_t g = lo ? pre0 : pre1;
          nxt = a.adj0[int64_t(g >= 0 ? g : cid) * a.deg0 + lcol];
        }
        const bool two = pidx >= 0;
        mark_expanded<R>(wr, fu, lane);
        const int32_t nb = col_ok && (lo || two) ? row : -1;
        const StepOut o = expand_links<M, T, BUDGET>(a, vt, bits, vlist, LdsTab<T>{lut}, sc, nb, cid, ctab, lo, two,
                                                     pk, lane, D, E, vcount);
        const bool dual = o.dual;
        const uint64_t k = o.k;
        if (dual) mark_expanded<R>(wr, pidx, lane);

        const bool keep = o.fresh && k < wmax;
        const uint64_t km = __ballot(keep);
        if (km) {
          const int nn = __popcll(km);
          if (nn == 1) {
            reg_insert_one<R>(wr, readlane64(k, __ffsll((unsigned long long)km) - 1), efe, lane);
          } else {
            uint64_t kv;
            if (nn <= 12) {
              // rank by broadcast; every lane takes one slot of a permutation
              int rank = 0;
              for (uint64_t mm = km; mm; mm &= mm - 1) {
                const uint64_t kj = readlane64(k, __ffsll((unsigned long long)mm) - 1);
                rank += kj < k ? 1 : 0;
              }
              const int below = __popcll(km & ((1ull << lane) - 1ull));
              const int dst = (keep ? rank : nn + lane - below) * 4;
              const uint64_t v = keep ? k : kKeyMax;
              const uint32_t lo32 = uint32_t(__builtin_amdgcn_ds_permute(dst, int(uint32_t(v))));
              const uint32_t hi32 = uint32_t(__builtin_amdgcn_ds_permute(dst, int(uint32_t(v >> 32))));
              kv = (uint64_t(hi32) << 32) | lo32;
            } else {
              kv = bitonic_sort(keep ? k : kKeyMax, lane);
            }
            reg_merge_sorted<R>(wr, kv, efe, lane);
          }
          nw = nw + nn < efe ? nw + nn : efe;
          wmax = nw == efe ? pure_key(entry_at<R>(wr, efe - 1)) : kKeyMax;
        }
        if (BUDGET && o.stop) break;  // the budget of distance evaluations is spent

        // the first four unexpanded entries
        Pick2 pm;
        pm.lo = __ballot((wr.w0 & kExpanded) == 0);
        pm.hi = R > 1 ? __ballot((wr.w1 & kExpanded) == 0) : 0ull;
        const int f0 = pm.next(), f1 = pm.next(), f2 = pm.next(), f3 = pm.next();
        fu = f0 >= 0 ? f0 : nw;
        pidx = f1;
        if (fu < nw) {
          ck = entry_at<R>(wr, f0);
          pk = f1 >= 0 ? entry_at<R>(wr, f1) : kKeyMax;
          const int32_t g2 = f2 >= 0 ? key_id(entry_at<R>(wr, f2)) : -1;
          const int32_t g3 = f3 >= 0 ? key_id(entry_at<R>(wr, f3)) : -1;
          const int32_t nc = key_id(ck);
          const int32_t np = f1 >= 0 ? key_id(pk) : -1;
          // only a dual step can meet the guess: when p was not expanded, a
          // kept key of c lies below key(p) and comes next
          if (a.prefetch && dual && nc == pre0 && (np < 0 || np == pre1)) {
            row = nxt;  // the guessed pair came next
          } else {
            row = a.adj0[int64_t(lo || np < 0 ? nc : np) * a.deg0 + lcol];
          }
          if (row >= a.n) row = -1;
          pre0 = g2;
          pre1 = g3;
        }
        // nothing is in flight across steps: the next step's loads are the only ones to wait for
        __builtin_amdgcn_s_waitcnt(0);
      }

      // short-list = the first min(S, |W|) entries of W
      const int ns = a.S < nw ? a.S : nw;
      for_chunks<0, R>([&](auto C) {
        const int i = (C << 6) + lane;
        const uint64_t w = chunk<C>(wr);
        if (i < a.S) {
          a.cand_ids[q * a.S + i] = i < ns ? key_id(w) : -1;
          a.cand_adc[q * a.S + i] = i < ns ? key_dist(w) : __builtin_inff();
        }
      });
      if (lane == 0) {
        a.cand_n[q] = ns;
        if (a.stats) {
          a.stats[2 * q] = E;
          a.stats[2 * q + 1] = D;
        }
      }
      if (vcount > 0) {
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

// Level-0 walk with the visited set in the slot's bitset behind a
// direct-mapped LDS cache; one expansion per step.
template <int M, typename T, bool BUDGET>
__global__ __launch_bounds__(64) void walk_cache_kernel(WalkArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  constexpr int kLutBytes = M * 256 * int(sizeof(T));
  constexpr int kScaleBytes = sizeof(T) == 2 ? (M * 4 + 15) / 16 * 16 : 0;
  T *lut = reinterpret_cast<T *>(smem);
  float *sc = reinterpret_cast<float *>(smem + kLutBytes);
  uint64_t *W = reinterpret_cast<uint64_t *>(smem + kLutBytes + kScaleBytes);
  uint32_t *hash = reinterpret_cast<uint32_t *>(W + a.w_cap + kMergeScratch);  // after the merge scratch
  const int H = 1 << a.hash_bits;
  const int hshift = 32 - a.hash_bits;
  uint32_t *bits = a.bits + int64_t(blockIdx.x) * a.words;
  int32_t *vlist = a.vlists + int64_t(blockIdx.x) * a.list_cap;

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

      const T *src = static_cast<const T *>(a.lut) + q * a.lut_stride;
      [[maybe_unused]] const float *ctab =
          kRes<T> ? reinterpret_cast<const float *>(static_cast<const T *>(a.lut) + q * a.lut_stride + M * 256)
                  : nullptr;
      stage_table<T, M>(lut, src, lane);
      if (sizeof(T) == 2)
        for (int i = lane; i < M; i += 64) sc[i] = a.scale[q * M + i];
      for (int i = lane; i < H; i += 64) hash[i] = kEmpty;
      wave_sync();

      // greedy descent on levels max_level .. 1
      int32_t cur;
      uint64_t curkey;
      greedy_descent<M, T>(a, LdsTab<T>{lut}, sc, lane, cur, curkey, ctab);

      if (lane == 0) {
        W[0] = curkey;
        atomicOr(&bits[uint32_t(cur) >> 5], 1u << (uint32_t(cur) & 31u));
        hash[hash_slot(cur, hshift)] = uint32_t(cur);
        vlist[0] = cur;
      }
      int vcount = 1;  // ids recorded in vlist
      int nw = 1, fu = 0, E = 0, D = 0;
      uint64_t ck = curkey;
      uint64_t wmax = efe == 1 ? curkey : kKeyMax;
      int32_t nb = l32 < a.deg0 ? a.adj0[int64_t(cur) * a.deg0 + l32] : -1;
      wave_sync();
      while (fu < nw) {
        if (lane == 0) W[fu] = ck | kExpanded;
        wave_sync();
        ++E;
        if (nb >= a.n) nb = -1;
        bool fresh = false;
        uint64_t k = kKeyMax;
        // cache hit: visited; miss: test-and-set the bit, fetching the code meanwhile
        CodeRegs<M> cr;
        if (lane < 32 && nb >= 0) {
          const uint32_t h = hash_slot(nb, hshift);
          if (hash[h] != uint32_t(nb)) {
            const uint32_t bit = 1u << (uint32_t(nb) & 31u);
            const uint32_t old = atomicOr(&bits[uint32_t(nb) >> 5], bit);
            cr.load(a.codes, a.code_stride, nb);
            if constexpr (kRes<T>) cr.load_coarse(a, ctab, nb);
            fresh = (old & bit) == 0;
            hash[h] = uint32_t(nb);
          }
        }
        const uint64_t fm = __ballot(fresh);
        const int nf = __popcll(fm);
        bool stop = false;
        const uint64_t kept = BUDGET ? budget_cut(fm, D, a.max_d, stop) : fm;  // the evaluations within the budget
        if (fresh) {
          if ((kept >> lane) & 1ull) k = make_key(cr.adc(lut, sc), nb);
          // every bit set is listed for clearing, a dropped link's too
          const int at = vcount + __popcll(fm & ((1ull << lane) - 1ull));
          if (at < a.list_cap) vlist[at] = nb;  // after the scoring, so that nothing waits on this store
          fresh = (kept >> lane) & 1ull;
        }
        vcount += nf;
        D += __popcll(kept);
        const bool keep = fresh && k < wmax;
        const uint64_t km = __ballot(keep);
        int p0 = fu;
        if (km) {
          int before_ck = 0;
          const int pos_min = merge_kept(W, nw, efe, k, keep, km, ck, lane, before_ck);
          const int fu_new = fu + before_ck;
          p0 = fu_new < pos_min ? fu_new : pos_min;
          wmax = nw == efe ? pure_key(W[nw - 1]) : kKeyMax;
        }
        wave_sync();
        if (BUDGET && stop) break;  // the budget of distance evaluations is spent
        int nfu = nw;
        uint64_t nck = 0;
        for (int base = p0; base < nw; base += 64) {
          const int idx = base + lane;
          const uint64_t v = idx < nw ? W[idx] : kExpanded;
          const uint64_t bm = __ballot((v & kExpanded) == 0);
          if (bm) {
            const int l0 = __ffsll((unsigned long long)bm) - 1;
            nfu = base + l0;
            nck = readlane64(v, l0);
            break;
          }
        }
        fu = nfu;
        if (fu < nw) {
          ck = nck;
          nb = l32 < a.deg0 ? a.adj0[int64_t(key_id(ck)) * a.deg0 + l32] : -1;
        }
      }

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
    if (atomicAdd(a.counters + 1, 1u) == gridDim.x - 1) {
      atomicExch(a.counters, 0u);
      atomicExch(a.counters + 1, 0u);
    }
  }
}

struct WalkPlan {
  int w_cap, hash_bits, lds_bytes, grid;
  int reg_chunks;  // > 0: the pool lives in registers, this many chunks of 64 (walk_reg_kernel)
  bool reg_lut;    // the fp16 table lives in registers (walk_rl_kernel)
};

// Slots per CU of walk_rl_kernel when its register count cannot be read: two waves per SIMD (its register
// budget is 256 of a SIMD's 512).
constexpr int kRegLutSlotsPerCu = 8;
// Largest m whose table registers hold within that budget (m = 64 spills).
constexpr int kRegLutMaxM = 56;

// Slots per CU that walk_rl_kernel<M>'s registers allow: four SIMDs times the waves that fit a SIMD's 512
// registers per lane (its register count, either budget variant, rounded up to the allocation granule of 8),
// at most 8 per SIMD.  m = 16 takes 155 registers, so three waves per SIMD; m = 56 takes 243, so two.
template <int M>
int rl_slots_cap() {
  if constexpr (M > kRegLutMaxM) {
    return 0;
  } else {
    static const int cap = [] {
      int regs = 0;
      for (const void *fn : {reinterpret_cast<const void *>(&walk_rl_kernel<M, false>),
                             reinterpret_cast<const void *>(&walk_rl_kernel<M, true>)}) {
        hipFuncAttributes at;
        if (hipFuncGetAttributes(&at, fn) != hipSuccess || at.numRegs <= 0) return kRegLutSlotsPerCu;
        if (at.numRegs > regs) regs = at.numRegs;
      }
      regs = (regs + 7) / 8 * 8;
      int waves = 512 / regs;
      if (waves > 8) waves = 8;
      if (waves < 1) waves = 1;
      return 4 * waves;
    }();
    return cap;
  }
}

// Largest pool held in registers: two chunks (four chunks were measured
// slower than the LDS pool: their merge networks cost more than they save).
constexpr int kRegPoolMax = 128;

constexpr size_t kHeaderBytes = 256;  // two queue counters, padded

template <int M>
int lds_bytes_for(int w_cap, int hash_bits, int lut_bytes, bool reg, bool rl = false) {
  const int scale_bytes = lut_bytes == 2 ? (M * 4 + 15) / 16 * 16 : 0;
  if (reg) return M * 256 * lut_bytes + (1 << hash_bits) * 4;  // table and visited table only
  const int table = rl ? 0 : M * 256 * lut_bytes;                // rl: the table is in registers
  return table + scale_bytes + w_cap * 8 + kMergeScratch * 8 + (1 << hash_bits) * 4;
}

// Tag width of a narrow visited table with 2^(hash_bits-2) buckets for ids
// below n, or 0 when 16-bit tags cannot tell every id apart.
int table_tag_bits(int32_t n, int hash_bits) {
  int id_bits = 0;
  while (id_bits < 31 && (int64_t(1) << id_bits) < int64_t(n)) ++id_bits;
  const int bb = hash_bits - 2;
  const int t = id_bits > bb ? id_bits - bb : 1;
  return t <= 15 ? t : 0;
}

// The visited table is sized by LDS: the largest narrow table of 2^10..2^12
// words that leaves 8 query slots per CU (a full bucket sends ids to the
// global bitset, which the longest walks pay for at every step, so capacity
// beats residency down to about 8 slots).  When the query's table alone keeps
// a CU below 8 slots (m * 256 entries of 28 KB and more), the largest table,
// 2^12 words: one slot fewer per CU costs less than the overflow (measured on
// the 20M-vector, 56-sub-space workload: 3.66 ms per 10k queries with 2^12
// words and 3 slots per CU, 4.30 ms with 2^10 words and 4).
template <int M>
int auto_hash_bits(int w_cap, int32_t n, int lut_bytes, int lds_per_cu, bool reg, bool rl) {
  for (int hb = 12; hb >= 10; --hb)
    if (table_tag_bits(n, hb) && lds_per_cu / lds_bytes_for<M>(w_cap, hb, lut_bytes, reg, rl) >= 8) return hb;
  if (lds_per_cu / lds_bytes_for<M>(w_cap, 10, lut_bytes, reg, rl) < 8) return 12;
  return table_tag_bits(n, 10) || !table_tag_bits(n, 11) ? 10 : 11;
}

// The visited table of the walk with its table in registers: the largest that
// keeps every slot its registers allow (12 per CU at m <= 24, 8 beyond), else
// the rule above.  At m = 16 the larger register budget outweighs a larger
// table: on 1M vectors, pools of 192 and 256, 1.91 and 2.44 ms per 10k
// queries with 2^11 words and 12 slots per CU, against 2.10 and 2.66 with
// 2^12 words and 8 (and 1.07 against 1.17 at a pool of 128).
template <int M>
int rl_hash_bits(int w_cap, int32_t n, int lut_bytes, int lds_per_cu) {
  const int cap = rl_slots_cap<M>();
  for (int hb = 12; hb >= 10; --hb)
    if (table_tag_bits(n, hb) && lds_per_cu / lds_bytes_for<M>(w_cap, hb, lut_bytes, false, true) >= cap) return hb;
  return auto_hash_bits<M>(w_cap, n, lut_bytes, lds_per_cu, false, true);
}

// plain_f16: the table is the one-level codec's fp16 table (the only one registers can hold)
template <int M>
WalkPlan plan_for(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, const lc_schedule *sc,
                  int lut_bytes, bool plain_f16) {
  WalkPlan p;
  int ef_eff = ef_max > S ? ef_max : S;
  p.w_cap = (ef_eff + 63) / 64 * 64;
  // The table in registers (fp16 tables of the walk with the visited table): when asked for, or (auto) when
  // it keeps at least 1.3 times the slots per CU of the table in LDS (a slot's step costs more with the table
  // in registers: two permutes per entry), or as many slots with a larger visited table (the LDS the table
  // no longer takes; a full bucket sends ids to the global bitset).  That walk keeps its pool in LDS: at
  // m = 56 it beats the register pool with the table in LDS at every pool size (8 slots per CU against 3;
  // measured on the 20M-vector, 56-sub-space workload: 1.36 against 1.82 ms at ef 64, 2.22 against 2.83 at
  // ef 128, per 10k queries); at m = 32 and a pool of 128 both keep 8 slots, with 2^12 visited words against
  // 2^10 (1M 128-d integer vectors, ef 144 and 128, short-list 128: 3.44M against 2.54M queries/s).
  const bool rl_ok = plain_f16 && sc->visited == 0 && M <= kRegLutMaxM;
  const int32_t n_tags = sc->wide ? INT32_MAX : ix->v.n;
  if (rl_ok && sc->table == 0) {
    const bool reg_alt = sc->pool == 0 && p.w_cap <= kRegPoolMax;  // the kernel the table in LDS would take
    const int hb_alt = sc->hash_bits ? sc->hash_bits
                                     : auto_hash_bits<M>(p.w_cap, n_tags, lut_bytes, ix->lds_per_cu, reg_alt, false);
    const int slots_alt = ix->lds_per_cu / lds_bytes_for<M>(p.w_cap, hb_alt, lut_bytes, reg_alt, false);
    const int hb_rl = sc->hash_bits ? sc->hash_bits
                                    : auto_hash_bits<M>(p.w_cap, n_tags, lut_bytes, ix->lds_per_cu, false, true);
    int slots_rl = ix->lds_per_cu / lds_bytes_for<M>(p.w_cap, hb_rl, lut_bytes, false, true);
    if (slots_rl > rl_slots_cap<M>()) slots_rl = rl_slots_cap<M>();
    p.reg_lut = 10 * slots_rl >= 13 * slots_alt || (slots_rl >= slots_alt && hb_rl > hb_alt);
  } else {
    p.reg_lut = rl_ok && sc->table == 2;
  }
  const bool reg = !p.reg_lut && sc->visited == 0 && sc->pool == 0 && p.w_cap <= kRegPoolMax;
  p.reg_chunks = reg ? 2 : 0;
  // visited mode 1 keeps only a small LDS cache; mode 0 sizes its table from the pool
  // (the choice above compares the register table at its largest visited table leaving 8 slots; once
  // taken, it gets the table that keeps all the slots its registers allow)
  p.hash_bits = sc->hash_bits ? sc->hash_bits
              : sc->visited == 1 ? 9
              : p.reg_lut        ? rl_hash_bits<M>(p.w_cap, n_tags, lut_bytes, ix->lds_per_cu)
                                 : auto_hash_bits<M>(p.w_cap, n_tags, lut_bytes, ix->lds_per_cu, reg, false);
  p.lds_bytes = lds_bytes_for<M>(p.w_cap, p.hash_bits, lut_bytes, reg, p.reg_lut);
  int per_cu = ix->lds_per_cu / p.lds_bytes;
  if (p.reg_lut && per_cu > rl_slots_cap<M>()) per_cu = rl_slots_cap<M>();
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
  if (sc->visited < 0 || sc->visited > 1 || sc->wide < 0 || sc->wide > 1 || sc->pool < 0 || sc->pool > 1)
    return false;
  if (sc->table < 0 || sc->table > 2 || sc->codes < 0 || sc->codes > 1) return false;
  return true;
}

const lc_schedule kDefaultSchedule = {0, 1, 0, 1, 0, 0, 0, 0, 0};

int list_cap_for(int w_cap) { return 16 * w_cap > 4096 ? 16 * w_cap : 4096; }

// header, then per slot its bitset, then per slot its id list
size_t ws_need(const WalkPlan &p, int64_t words) {
  return kHeaderBytes + size_t(p.grid) * size_t(words) * 4 + size_t(p.grid) * size_t(list_cap_for(p.w_cap)) * 4;
}

template <int M>
size_t ws_bytes_m(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, const lc_schedule *sc) {
  // enough for either table type
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  const size_t a = ws_need(plan_for<M>(ix, nq, ef_max, S, sc, 2, true), words);
  const size_t b = ws_need(plan_for<M>(ix, nq, ef_max, S, sc, 4, false), words);
  const size_t c = ws_need(plan_for<M>(ix, nq, ef_max, S, sc, 2, false), words);
  const size_t ab = a > b ? a : b;
  return ab > c ? ab : c;
}

// The kernel the plan picks; with a budget on distance evaluations, its
// variant that counts them (the kernels without one carry no such test).
template <int M, typename T, bool BUDGET>
int launch_kernel(const WalkPlan &p, const lc_schedule *sc, const WalkArgs &a, hipStream_t st) {
  if constexpr (std::is_same<T, __half>::value && M <= kRegLutMaxM) {
    if (p.reg_lut) {
      const void *fr = reinterpret_cast<const void *>(&walk_rl_kernel<M, BUDGET>);
      if (hipFuncSetAttribute(fr, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_bytes) != hipSuccess)
        return LC_EHIP;
      hipLaunchKernelGGL((walk_rl_kernel<M, BUDGET>), dim3(p.grid), dim3(64), p.lds_bytes, st, a);
      return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
    }
  }
  if (p.reg_lut) return LC_EINVAL;  // the plan gives registers fp16 tables only
  const void *fn = sc->visited == 1 ? reinterpret_cast<const void *>(&walk_cache_kernel<M, T, BUDGET>)
                   : p.reg_chunks  ? reinterpret_cast<const void *>(&walk_reg_kernel<M, T, 2, BUDGET>)
                                   : reinterpret_cast<const void *>(&walk_kernel<M, T, BUDGET>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds_bytes) != hipSuccess)
    return LC_EHIP;
  if (sc->visited == 1)
    hipLaunchKernelGGL((walk_cache_kernel<M, T, BUDGET>), dim3(p.grid), dim3(64), p.lds_bytes, st, a);
  else if (p.reg_chunks)
    hipLaunchKernelGGL((walk_reg_kernel<M, T, 2, BUDGET>), dim3(p.grid), dim3(64), p.lds_bytes, st, a);
  else
    hipLaunchKernelGGL((walk_kernel<M, T, BUDGET>), dim3(p.grid), dim3(64), p.lds_bytes, st, a);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

template <int M, typename T>
int launch_m(const lc_index *ix, const void *lut, const float *scale, int64_t nq, const int32_t *ef,
             int32_t ef_max, int32_t S, int32_t max_d, const int32_t *order, int32_t *cand_ids, float *cand_adc,
             int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sc, hipStream_t st,
             bool fit_ws) {
  WalkPlan p = plan_for<M>(ix, nq, ef_max, S, sc, int(sizeof(T)), std::is_same<T, __half>::value);
  const int64_t words = (int64_t(ix->v.n) + 31) / 32;
  if (fit_ws) {
    // as many resident slots as the workspace holds (results do not depend on the slot count)
    const size_t per_slot = size_t(words) * 4 + size_t(list_cap_for(p.w_cap)) * 4;
    const size_t fit = ws_bytes > kHeaderBytes ? (ws_bytes - kHeaderBytes) / per_slot : 0;
    if (fit < 1) return LC_ENOSPC;
    if (size_t(p.grid) > fit) p.grid = int(fit);
  }
  if (ws_bytes < ws_need(p, words)) return LC_ENOSPC;
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
  a.max_d = max_d;
  a.late_codes = sc->codes;
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
  a.tag_bits = sc->wide ? 0 : table_tag_bits(ix->v.n, p.hash_bits);
  a.counters = static_cast<uint32_t *>(ws);
  a.bits = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + kHeaderBytes);
  a.vlists = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + kHeaderBytes +
                                         size_t(p.grid) * size_t(words) * 4);
  a.words = words;
  a.cand_ids = cand_ids;
  a.cand_adc = cand_adc;
  a.cand_n = cand_n;
  a.stats = stats;
  a.ccodes = reinterpret_cast<const uint32_t *>(ix->v.coarse_codes);
  a.cnorm = ix->v.coarse_norm;
  a.coarse_k = ix->v.coarse_k;
  a.lut_stride = lc_lut_row_bytes(ix, sizeof(T) == 2 ? LC_LUT_F16 : LC_LUT_F32) / int64_t(sizeof(T));
  return max_d > 0 ? launch_kernel<M, T, true>(p, sc, a, st) : launch_kernel<M, T, false>(p, sc, a, st);
}


// The kernel and plan launch_m would use (lc_walk_describe).
template <int M, typename T>
int describe_m(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, const lc_schedule *sc, char *buf,
               size_t len) {
  const WalkPlan p = plan_for<M>(ix, nq, ef_max, S, sc, int(sizeof(T)), std::is_same<T, __half>::value);
  const char *t = std::is_same<T, float>::value ? "float" : std::is_same<T, __half>::value ? "__half"
                  : std::is_same<T, rfloat>::value ? "rfloat" : "rhalf";
  char kname[96];
  if (p.reg_lut)
    snprintf(kname, sizeof kname, "walk_rl_kernel<%d, %s>", M, "false");
  else if (sc->visited == 1)
    snprintf(kname, sizeof kname, "walk_cache_kernel<%d, %s, %s>", M, t, "false");
  else if (p.reg_chunks)
    snprintf(kname, sizeof kname, "walk_reg_kernel<%d, %s, 2, %s>", M, t, "false");
  else
    snprintf(kname, sizeof kname, "walk_kernel<%d, %s, %s>", M, t, "false");
  const int slots = int((p.grid + ix->num_cus - 1) / ix->num_cus);
  snprintf(buf, len, "%s grid=%d slots_per_cu=%d hash_bits=%d lds_bytes=%d", kname, p.grid, slots, p.hash_bits,
           p.lds_bytes);
  return LC_OK;
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
                   const int32_t *ef, int32_t ef_max, int32_t S, int32_t max_d, const int32_t *order,
                   int32_t *cand_ids, float *cand_adc,
                   int32_t *cand_n, int32_t *stats, void *ws, size_t ws_bytes, const lc_schedule *sched,
                   hipStream_t st, bool fit_ws) {
  if (dtype != LC_LUT_F32 && dtype != LC_LUT_F16) return LC_ENOTSUP;
  if (!valid_schedule(sched)) return LC_EINVAL;
  const lc_schedule *sc = sched ? sched : &kDefaultSchedule;
  if (ix->v.coarse_k > 0) {  // 2-level codec
    switch (ix->v.m) {
#define CASE(MM)                                                                                              \
  case MM:                                                                                                    \
    return dtype == LC_LUT_F32 ? launch_m<MM, rfloat>(ix, lut, scale, nq, ef, ef_max, S, max_d, order,       \
                                                      cand_ids, cand_adc, cand_n, stats, ws, ws_bytes, sc, st, fit_ws) \
                               : launch_m<MM, rhalf>(ix, lut, scale, nq, ef, ef_max, S, max_d, order,        \
                                                     cand_ids, cand_adc, cand_n, stats, ws, ws_bytes, sc, st, fit_ws);
      LC_FOR_EACH_M(CASE)
#undef CASE
      default: return LC_ENOTSUP;
    }
  }
  switch (ix->v.m) {
#define CASE(MM)                                                                                              \
  case MM:                                                                                                    \
    return dtype == LC_LUT_F32 ? launch_m<MM, float>(ix, lut, scale, nq, ef, ef_max, S, max_d, order,        \
                                                     cand_ids, cand_adc, cand_n, stats, ws, ws_bytes, sc, st, fit_ws) \
                               : launch_m<MM, __half>(ix, lut, scale, nq, ef, ef_max, S, max_d, order,       \
                                                      cand_ids, cand_adc, cand_n, stats, ws, ws_bytes, sc, st, fit_ws);
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return LC_ENOTSUP;
  }
}

int lc_describe_walk(const lc_index *ix, int64_t nq, int32_t ef_max, int32_t S, int dtype, const lc_schedule *sched,
                     char *buf, size_t len) {
  if (dtype != LC_LUT_F32 && dtype != LC_LUT_F16) return LC_EINVAL;
  if (!valid_schedule(sched)) return LC_EINVAL;
  const lc_schedule *sc = sched ? sched : &kDefaultSchedule;
  const bool f32 = dtype == LC_LUT_F32, res = ix->v.coarse_k > 0;
  switch (ix->v.m) {
#define CASE(MM)                                                                                    \
  case MM:                                                                                          \
    return res ? (f32 ? describe_m<MM, rfloat>(ix, nq, ef_max, S, sc, buf, len)                    \
                      : describe_m<MM, rhalf>(ix, nq, ef_max, S, sc, buf, len))                    \
               : (f32 ? describe_m<MM, float>(ix, nq, ef_max, S, sc, buf, len)                     \
                      : describe_m<MM, __half>(ix, nq, ef_max, S, sc, buf, len));
    LC_FOR_EACH_M(CASE)
#undef CASE
    default: return LC_ENOTSUP;
  }
}
