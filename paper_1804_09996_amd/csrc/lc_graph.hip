// Index build steps on the GPU: the exact projection and PQ encoding of the
// database, and the insertion of level-0 nodes into the graph by batches.
//
// Sec. 5.1 adds vectors to the graph in batches: every node of a batch is
// searched against the graph as it stood when the batch began, then the batch
// is linked.  For a node x (Sec. 2, Sec. 4.1):
//   1. greedy descent from the entry point on the upper levels, then a
//      best-first search of level 0 with a pool of ef_construction entries,
//      scored by the asymmetric distance ||x - q(y)||^2 of x's raw vector to
//      the codes (a per-node table, summed over the sub-spaces);
//   2. x's list: the shrinking rule over the candidates in (distance, id)
//      order keeps a candidate e only if d(x, e) < d(e, s) for every link s
//      kept before it, d(e, s) = ||q(e) - q(s)||^2 between reconstructions;
//      free slots then take the nearest rejected candidates;
//   3. every node y that x picked gets x as a reverse link: y's list plus
//      its new links, ordered by the distance from y's own raw vector to their
//      reconstructions, re-shrunk by the same rule when it overflows.
//
// Step 1 is the search path's own walk (lc_launch_walk, ef = S =
// ef_construction) on a float32 table written here.  Every float here is
// taken the way a plain sequential loop takes it (contraction off: no fused
// multiply-add; sums in ascending index order, starting from zero), so the
// lists are the ones such a loop builds: bit for bit those of the host
// builder with the same inputs.
//
// Reverse links are grouped by target on the device (an atomic count per
// node, one group per target, a range of the link list per group taken by
// atomics, a scatter); a group's candidates are
// ordered by their keys, so the order in which its links arrive does not
// matter.  A group of at most 64 candidates is handled in registers (one per
// lane), a larger one in LDS.
#include "lc_internal.h"

#pragma clang fp contract(off)

namespace {

using namespace lc;

constexpr int kCounters = 256;  // [0] groups, [1] overflowing groups, [2] links placed

__device__ __forceinline__ uint32_t byte_of(const uint32_t *w, int s) { return (w[s >> 2] >> (8 * (s & 3))) & 0xFFu; }

// ||C[s][a] - C[s][b]||^2 as a sequential float loop.  DSUB > 0: the
// sub-vector length known at compile time (the loops unrolled, so a
// candidate's independent look-ups issue back to back); 0: dsub at run time.
template <int DSUB>
__device__ __forceinline__ float cent_dist(const float *cent, int dsub, int s, uint32_t a, uint32_t b) {
  constexpr int kUnrollU = DSUB > 0 ? DSUB : 1;
  const int ds = DSUB > 0 ? DSUB : dsub;
  const float *ca = cent + (size_t(s) * 256 + a) * ds;
  const float *cb = cent + (size_t(s) * 256 + b) * ds;
  float e = 0.f;
#pragma unroll kUnrollU
  for (int u = 0; u < (DSUB > 0 ? DSUB : dsub); ++u) {
    const float df = ca[u] - cb[u];
    e += df * df;
  }
  return e;
}

// d(e, s) = sum over sub-spaces of ||C[t][e_t] - C[t][s_t]||^2, ascending t:
// the terms are independent (eight at a time, their look-ups issued
// together), only their sum runs in order.
template <int M, int DSUB>
__device__ __forceinline__ float rec_rec(const float *cent, int dsub, const uint32_t *ca, const uint32_t *cb) {
  constexpr int CH = DSUB > 0 ? 8 : 1;  // a run-time dsub keeps one term in flight (registers)
  float acc = 0.f;
#pragma unroll
  for (int s0 = 0; s0 < M; s0 += CH) {
    float e[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) e[j] = cent_dist<DSUB>(cent, dsub, s0 + j, byte_of(ca, s0 + j), byte_of(cb, s0 + j));
#pragma unroll
    for (int j = 0; j < CH; ++j) acc += e[j];
  }
  return acc;
}

// ||v - q(y)||^2 over all coordinates in order (v the raw projected vector).
template <int M, int DSUB>
__device__ __forceinline__ float raw_rec(const float *v, const float *cent, int dsub, const uint32_t *cy) {
  constexpr int kUnrollS = DSUB > 0 ? M : 1, kUnrollU = DSUB > 0 ? DSUB : 1;
  const int ds = DSUB > 0 ? DSUB : dsub;
  float acc = 0.f;
#pragma unroll kUnrollS
  for (int s = 0; s < M; ++s) {
    const float *c = cent + (size_t(s) * 256 + byte_of(cy, s)) * ds;
#pragma unroll kUnrollU
    for (int u = 0; u < (DSUB > 0 ? DSUB : dsub); ++u) {
      const float df = v[s * ds + u] - c[u];
      acc += df * df;
    }
  }
  return acc;
}

template <int M>
__device__ __forceinline__ void load_codes(const uint8_t *codes, int cs, int32_t id, uint32_t *w) {
  if (id < 0) {
#pragma unroll
    for (int k = 0; k < M / 4; ++k) w[k] = 0u;
    return;
  }
  const uint32_t *row = reinterpret_cast<const uint32_t *>(codes + size_t(id) * cs);
#pragma unroll
  for (int k = 0; k < M / 4; ++k) w[k] = row[k];
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Every test of the shrinking rule for candidates held one per lane in key
// order (lanes 0..nc-1, nc <= 64): lane i returns the lanes s < i whose link
// candidate i does not beat, d(x, i) >= d(i, s).  Whether i beats s does not
// depend on which links end up kept, so the nc (nc - 1) / 2 pairs are spread
// over the lanes, 64 at a time (pair p = i (i - 1) / 2 + s on lane p mod 64),
// each lane fetching both candidates' codes from their lanes and summing
// d(i, s) exactly as rec_rec does; the lanes of one candidate's pairs are
// contiguous, so its mask is a slice of the round's ballot.
template <int M, int DSUB>
__device__ uint64_t pair_fails(float dist, const uint32_t *code, int nc, const float *cent, int dsub, int lane) {
  uint64_t fails = 0;
  const int np = nc * (nc - 1) / 2;
  const int first = lane * (lane - 1) / 2;  // this lane's pairs as candidate i: [first, first + lane)
  for (int p0 = 0; p0 < np; p0 += 64) {
    const int p = p0 + lane;
    const bool act = p < np;
    // i = floor((1 + sqrt(1 + 8p)) / 2): exact in float for p < 2016, checked anyway
    int i = act ? int((1.f + __builtin_sqrtf(float(1 + 8 * p))) * 0.5f) : 1;
    if (act) {
      if (i * (i - 1) / 2 > p) --i;
      if (i * (i + 1) / 2 <= p) ++i;
    }
    const int sidx = act ? p - i * (i - 1) / 2 : 0;
    uint32_t ci[M / 4], cs[M / 4];
#pragma unroll
    for (int k = 0; k < M / 4; ++k) {
      ci[k] = uint32_t(__builtin_amdgcn_ds_bpermute(i << 2, int(code[k])));
      cs[k] = uint32_t(__builtin_amdgcn_ds_bpermute(sidx << 2, int(code[k])));
    }
    const float di = __int_as_float(__builtin_amdgcn_ds_bpermute(i << 2, __float_as_int(dist)));
    const bool fail = act && !(di < rec_rec<M, DSUB>(cent, dsub, ci, cs));
    const uint64_t b = __ballot(fail);
    // this lane's pairs that fall in the round
    const int lo = first > p0 ? first : p0;
    const int hi = first + lane < p0 + 64 ? first + lane : p0 + 64;
    if (lo < hi) {
      const int len = hi - lo;
      const uint64_t bits = (b >> (lo - p0)) & (len >= 64 ? ~0ull : ((1ull << len) - 1ull));
      fails |= bits << (lo - first);
    }
  }
  return fails;
}

// The shrinking rule over candidates held one per lane in key order (lanes
// 0..nc-1, nc <= 64): returns the lanes of the kept links and of the filled
// slots (at most cap).  Candidate i is kept when d(x, i) < d(i, s) for every
// link s kept before it, candidates taken in order until cap are kept; when
// fewer are, the nearest rejected ones fill the free slots.
template <int M, int DSUB>
__device__ uint64_t shrink_lanes(float dist, const uint32_t *code, int nc, int cap, const float *cent, int dsub,
                                 int lane) {
  const uint64_t fails = pair_fails<M, DSUB>(dist, code, nc, cent, dsub, lane);
  uint64_t kept = 0;
  int nk = 0;
  for (int i = 0; i < nc && nk < cap; ++i) {
    const uint64_t f = (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(fails >> 32)), i))) << 32) |
                       uint32_t(__builtin_amdgcn_readlane(int(uint32_t(fails)), i));
    if ((f & kept) == 0ull) {
      kept |= 1ull << i;
      ++nk;
    }
  }
  uint64_t out = kept;
  if (nk < cap) {  // every candidate was tested: fill with the nearest rejected ones
    uint64_t rej = (nc >= 64 ? ~0ull : ((1ull << nc) - 1)) & ~kept;
    for (int f = nk; f < cap && rej; ++f) {
      out |= rej & (~rej + 1);
      rej &= rej - 1;
    }
  }
  return out;
}

// Ascending bitonic sort of one key per lane over the whole wave.
__device__ __forceinline__ uint64_t sort64(uint64_t v, int lane) {
  for (int k = 2; k <= 64; k <<= 1) {
    for (int j = k >> 1; j >= 1; j >>= 1) {
      const uint64_t o = shfl_xor64(v, j);
      const bool up = (lane & k) == 0 || k == 64;
      const bool lower = (lane & j) == 0;
      const uint64_t mn = o < v ? o : v, mx = o < v ? v : o;
      v = (lower == up) ? mn : mx;
    }
  }
  return v;
}

struct InsertArgs {
  const float *xp;        // [n][d_pad] projected raw vectors
  const float *cent;      // [m][256][dsub]
  const uint8_t *codes;   // [n][cs]
  int32_t *adj0;          // [n][deg0]
  const int32_t *nodes;   // [count] the batch
  int32_t count, efc, deg0, cs, m, dsub, d_pad;
  const int32_t *cand_ids;  // [count][efc] the walk's short-lists (key order)
  const float *cand_adc;
  const int32_t *cand_n;
  int32_t *req_tgt;     // [count][deg0] targets of the reverse links (-1: none)
  int32_t *inbox;       // [n] reverse links per target in this batch (zero between batches)
  int32_t *gid_of;      // [n] group of a target
  int32_t *group_tgt, *group_cnt, *group_off, *group_fill, *srcs, *ovf;
  uint32_t *counters;
};

// Centroids staged in LDS by all waves of a block.
__device__ __forceinline__ void stage_cent(float *lds, const float *cent, int nfl) {
  for (int i = threadIdx.x; i < nfl; i += blockDim.x) lds[i] = cent[i];
  __syncthreads();
}

// 1. Tables: tab[b][s][c] = ||xp^s - C[s][c]||^2 for the batch's nodes.
__global__ __launch_bounds__(256) void table_kernel(InsertArgs a, float *tab) {
  extern __shared__ float v[];
  const int b = blockIdx.x;
  const float *row = a.xp + size_t(a.nodes[b]) * a.d_pad;
  for (int t = threadIdx.x; t < a.d_pad; t += blockDim.x) v[t] = row[t];
  __syncthreads();
  const int c = threadIdx.x;
  for (int s = 0; s < a.m; ++s) {
    const float *cc = a.cent + (size_t(s) * 256 + c) * a.dsub;
    float e = 0.f;
    for (int u = 0; u < a.dsub; ++u) {
      const float df = v[s * a.dsub + u] - cc[u];
      e += df * df;
    }
    tab[(size_t(b) * a.m + s) * 256 + c] = e;
  }
}

// Records a reverse link x -> tgt: counts it on the target and opens the
// target's group on its first link.
__device__ __forceinline__ void note_link(const InsertArgs &a, int32_t tgt) {
  if (atomicAdd(a.inbox + tgt, 1) == 0) {
    const int g = int(atomicAdd(a.counters, 1u));
    a.gid_of[tgt] = g;
    a.group_tgt[g] = tgt;
  }
}

// 2. Each new node's own list from its short-list, and its reverse links.
template <int M, int DSUB>
__global__ __launch_bounds__(1024) void select_kernel(InsertArgs a) {
  extern __shared__ float lcent[];
  stage_cent(lcent, a.cent, a.m * 256 * a.dsub);
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= a.count) return;
  const int32_t x = a.nodes[b];
  const int nc = a.cand_n[b] < 0 ? 0 : (a.cand_n[b] > a.efc ? a.efc : a.cand_n[b]);
  const int32_t id = lane < nc ? a.cand_ids[size_t(b) * a.efc + lane] : -1;
  const float dist = lane < nc ? a.cand_adc[size_t(b) * a.efc + lane] : 0.f;
  uint32_t code[M / 4];
  load_codes<M>(a.codes, a.cs, id, code);
  const uint64_t out = shrink_lanes<M, DSUB>(dist, code, nc, a.deg0, lcent, a.dsub, lane);
  const bool mine = (out >> lane) & 1ull;
  const int pos = __builtin_amdgcn_mbcnt_hi(uint32_t(out >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(out), 0u));
  const int w = __popcll(out);
  int32_t *row = a.adj0 + size_t(x) * a.deg0;
  int32_t *req = a.req_tgt + size_t(b) * a.deg0;
  if (mine) {
    row[pos] = id;
    req[pos] = id;
    note_link(a, id);
  }
  if (lane >= w && lane < a.deg0) {
    row[lane] = -1;
    req[lane] = -1;
  }
}

// 3. Each group's range of the link list: a wave sums its groups' counts and
// takes its ranges with one atomic add.  Groups are independent and a group's
// links are ordered by key before they are used, so where a range lies does
// not change the graph.
__global__ __launch_bounds__(256) void offsets_kernel(InsertArgs a) {
  const int ng = int(a.counters[0]);
  const int lane = threadIdx.x & 63;
  for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < ng; base += gridDim.x * blockDim.x) {
    const int g = base + lane;
    const int32_t c = g < ng ? a.inbox[a.group_tgt[g]] : 0;
    int32_t incl = c;  // inclusive sum over the wave's lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    int32_t start = 0;
    if (lane == 63) start = int32_t(atomicAdd(a.counters + 2, uint32_t(incl)));
    start = __shfl(start, 63);
    if (g < ng) {
      a.group_cnt[g] = c;
      a.group_off[g] = start + incl - c;
    }
  }
}

// 4. Each reverse link into its target's list (any order inside a group).
__global__ __launch_bounds__(256) void scatter_kernel(InsertArgs a) {
  const int total = a.count * a.deg0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < total; r += gridDim.x * blockDim.x) {
    const int32_t tgt = a.req_tgt[r];
    if (tgt < 0) continue;
    const int g = a.gid_of[tgt];
    const int p = atomicAdd(a.group_fill + g, 1);
    a.srcs[a.group_off[g] + p] = a.nodes[r / a.deg0];
  }
}

__device__ __forceinline__ void close_group(const InsertArgs &a, int g, int32_t tgt, int lane) {
  if (lane == 0) {
    a.inbox[tgt] = 0;
    a.group_fill[g] = 0;
  }
}

// 5. A target's merge when its list and new links fit one wave (<= 64).
template <int M, int DSUB>
__global__ __launch_bounds__(1024) void merge_kernel(InsertArgs a) {
  extern __shared__ float lds[];
  float *lcent = lds;
  const int waves = blockDim.x >> 6;
  float *vbuf = lds + a.m * 256 * a.dsub + (threadIdx.x >> 6) * a.d_pad;
  stage_cent(lcent, a.cent, a.m * 256 * a.dsub);
  const int lane = threadIdx.x & 63;
  const int ng = int(a.counters[0]);
  for (int g = blockIdx.x * waves + (threadIdx.x >> 6); g < ng; g += gridDim.x * waves) {
    const int32_t tgt = a.group_tgt[g];
    int32_t *row = a.adj0 + size_t(tgt) * a.deg0;
    const int32_t r = lane < a.deg0 ? row[lane] : -1;
    const int have = __popcll(__ballot(r >= 0));
    const int ns = a.group_cnt[g];
    const int nc = have + ns;
    if (nc > 64) {  // the LDS kernel takes it
      if (lane == 0) a.ovf[atomicAdd(a.counters + 1, 1u)] = g;
      continue;
    }
    for (int t = lane; t < a.d_pad; t += 64) vbuf[t] = a.xp[size_t(tgt) * a.d_pad + t];
    wave_sync();
    const int32_t id = lane < have ? r : (lane < nc ? a.srcs[a.group_off[g] + lane - have] : -1);
    uint32_t code[M / 4];
    load_codes<M>(a.codes, a.cs, id, code);
    const float dist = id >= 0 ? raw_rec<M, DSUB>(vbuf, lcent, a.dsub, code) : 0.f;
    uint64_t key = id >= 0 ? make_key(dist, id) : kKeyMax;
    key = sort64(key, lane);
    const int32_t sid = key == kKeyMax ? -1 : key_id(key);
    if (nc <= a.deg0) {
      if (lane < a.deg0) row[lane] = lane < nc ? sid : -1;
    } else {
      load_codes<M>(a.codes, a.cs, sid, code);
      const uint64_t out = shrink_lanes<M, DSUB>(key_dist(key), code, nc, a.deg0, lcent, a.dsub, lane);
      const int pos = __builtin_amdgcn_mbcnt_hi(uint32_t(out >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(out), 0u));
      const int w = __popcll(out);
      if ((out >> lane) & 1ull) row[pos] = sid;
      if (lane >= w && lane < a.deg0) row[lane] = -1;
    }
    wave_sync();
    close_group(a, g, tgt, lane);
  }
}

// 6. A target with more than 64 candidates: keys sorted in LDS, the rule run
// over them with the kept links' codes in lanes 0..deg0-1.
template <int M, int DSUB>
__global__ __launch_bounds__(64) void merge_large_kernel(InsertArgs a, int kcap) {
  extern __shared__ uint64_t keys[];  // [kcap], then kcap flag bytes, then d_pad floats
  uint8_t *flag = reinterpret_cast<uint8_t *>(keys + kcap);
  float *vbuf = reinterpret_cast<float *>(flag + kcap);
  const int lane = threadIdx.x;
  const int no = int(a.counters[1]);
  for (int k = blockIdx.x; k < no; k += gridDim.x) {
    const int g = a.ovf[k];
    const int32_t tgt = a.group_tgt[g];
    int32_t *row = a.adj0 + size_t(tgt) * a.deg0;
    const int32_t r = lane < a.deg0 ? row[lane] : -1;
    const int have = __popcll(__ballot(r >= 0));
    const int nc = have + a.group_cnt[g];
    int p2 = 64;
    while (p2 < nc) p2 <<= 1;
    for (int t = lane; t < a.d_pad; t += 64) vbuf[t] = a.xp[size_t(tgt) * a.d_pad + t];
    wave_sync();
    for (int j = lane; j < p2; j += 64) {
      uint64_t key = kKeyMax;
      if (j < nc) {
        const int32_t id = j < have ? row[j] : a.srcs[a.group_off[g] + j - have];
        uint32_t code[M / 4];
        load_codes<M>(a.codes, a.cs, id, code);
        key = make_key(raw_rec<M, DSUB>(vbuf, a.cent, a.dsub, code), id);
      }
      keys[j] = key;
      flag[j] = 0;
    }
    wave_sync();
    for (int kk = 2; kk <= p2; kk <<= 1) {  // bitonic sort of keys[0..p2)
      for (int jj = kk >> 1; jj >= 1; jj >>= 1) {
        for (int i = lane; i < p2; i += 64) {
          const int o = i ^ jj;
          if (o > i) {
            const uint64_t x = keys[i], y = keys[o];
            const bool up = (i & kk) == 0;
            if ((x > y) == up) {
              keys[i] = y;
              keys[o] = x;
            }
          }
        }
        wave_sync();
      }
    }
    // the rule, candidate by candidate; lane t < nk holds kept link t's codes
    uint32_t mine[M / 4];
#pragma unroll
    for (int q = 0; q < M / 4; ++q) mine[q] = 0u;
    int nk = 0;
    for (int i = 0; i < nc && nk < a.deg0; ++i) {
      const uint64_t ki = keys[i];
      const int32_t id = key_id(ki);
      uint32_t ci[M / 4];
      load_codes<M>(a.codes, a.cs, id, ci);
      bool fail = false;
      if (lane < nk) fail = !(key_dist(ki) < rec_rec<M, DSUB>(a.cent, a.dsub, ci, mine));
      if (__ballot(fail) == 0ull) {
        if (lane == nk) {
#pragma unroll
          for (int q = 0; q < M / 4; ++q) mine[q] = ci[q];
          flag[i] = 1;
        }
        ++nk;
      }
    }
    wave_sync();
    if (nk < a.deg0) {  // fill with the nearest rejected candidates
      if (lane == 0) {
        for (int i = 0; i < nc && nk < a.deg0; ++i)
          if (!flag[i]) {
            flag[i] = 2;
            ++nk;
          }
      }
      wave_sync();
    }
    // write the chosen ones in key order
    int w = 0;
    for (int base = 0; base < nc; base += 64) {
      const int i = base + lane;
      const bool take = i < nc && flag[i] != 0;
      const uint64_t bal = __ballot(take);
      const int pos = w + __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
      if (take) row[pos] = key_id(keys[i]);
      w += __popcll(bal);
    }
    if (lane >= w && lane < a.deg0) row[lane] = -1;
    wave_sync();
    close_group(a, g, tgt, lane);
  }
}

__global__ void reset_kernel(uint32_t *counters) {
  if (threadIdx.x < 3) counters[threadIdx.x] = 0u;
}

// -- projection and encoding ------------------------------------------------

// xp[i][r] = float(sum_t double(P[r][t]) * double(x[i][t])), t ascending.
__global__ __launch_bounds__(256) void project_exact_kernel(const float *x, int64_t n, int d, const float *P,
                                                             int d_pad, float *xp) {
  const int64_t total = n * d_pad;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < total; k += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = k / d_pad;
    const int r = int(k - i * d_pad);
    const float *xr = x + i * d;
    const float *pr = P + size_t(r) * d;
    double s = 0.0;
    for (int t = 0; t < d; ++t) s += double(pr[t]) * double(xr[t]);
    xp[k] = float(s);
  }
}

// codes[i][s] = argmin_c ||xp^s - C[s][c]||^2 (lowest c on ties); bytes
// m..cs-1 of a row are zero.
__global__ __launch_bounds__(256) void pq_encode_kernel(const float *xp, int64_t n, int d_pad, int m, int dsub,
                                                         const float *cent, uint8_t *codes, int cs) {
  __shared__ float cc[256 * 16];
  const int s = blockIdx.y;
  if (s >= m) {  // the padding bytes
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
      for (int t = m; t < cs; ++t) codes[i * cs + t] = 0;
    return;
  }
  for (int k = threadIdx.x; k < 256 * dsub; k += blockDim.x) cc[k] = cent[size_t(s) * 256 * dsub + k];
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    float v[16];
    for (int t = 0; t < dsub; ++t) v[t] = xp[i * d_pad + s * dsub + t];
    float best = 3.402823466e+38f;
    int bj = 0;
    for (int c = 0; c < 256; ++c) {
      float e = 0.f;
      for (int t = 0; t < dsub; ++t) {
        const float df = v[t] - cc[c * dsub + t];
        e += df * df;
      }
      if (e < best) {
        best = e;
        bj = c;
      }
    }
    codes[i * cs + s] = uint8_t(bj);
  }
}

// -- workspace ----------------------------------------------------------------

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct InsertLayout {
  size_t walk, tab, cand_ids, cand_adc, cand_n, req, inbox, gid, gt, gc, go, gf, srcs, ovf, total;
};

InsertLayout insert_layout(const lc_index *ix, int32_t max_count, int32_t efc) {
  InsertLayout L;
  const size_t B = size_t(max_count), links = B * ix->v.deg0, n = size_t(ix->v.n);
  size_t o = kCounters;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.walk = take(lc_walk_workspace_bytes(ix, max_count, efc, efc, nullptr));
  L.tab = take(B * ix->v.m * 256 * 4);
  L.cand_ids = take(B * efc * 4);
  L.cand_adc = take(B * efc * 4);
  L.cand_n = take(B * 4);
  L.req = take(links * 4);
  L.inbox = take(n * 4);
  L.gid = take(n * 4);
  L.gt = take(links * 4);
  L.gc = take(links * 4);
  L.go = take(links * 4);
  L.gf = take(links * 4);
  L.srcs = take(links * 4);
  L.ovf = take(links * 4);
  L.total = o;
  return L;
}

template <int M, int DSUB>
int insert_m(const lc_index *ix, InsertArgs &a, const InsertLayout &L, char *ws, int32_t max_count,
             hipStream_t st) {
  const int cent_bytes = a.m * 256 * a.dsub * 4;
  // tables, then the walk on them (ef = S = ef_construction)
  float *tab = reinterpret_cast<float *>(ws + L.tab);
  hipLaunchKernelGGL(table_kernel, dim3(a.count), dim3(256), a.d_pad * 4, st, a, tab);
  if (hipGetLastError() != hipSuccess) return LC_EHIP;
  int rc = lc_launch_walk(ix, tab, LC_LUT_F32, nullptr, a.count, nullptr, a.efc, a.efc, 0, nullptr,
                          const_cast<int32_t *>(a.cand_ids), const_cast<float *>(a.cand_adc),
                          const_cast<int32_t *>(a.cand_n), nullptr, ws + L.walk,
                          lc_walk_workspace_bytes(ix, max_count, a.efc, a.efc, nullptr), nullptr, st);
  if (rc != LC_OK) return rc;
  const int wpb = 16;  // waves per block sharing the staged centroids
  const void *sel = reinterpret_cast<const void *>(&select_kernel<M, DSUB>);
  if (hipFuncSetAttribute(sel, hipFuncAttributeMaxDynamicSharedMemorySize, cent_bytes) != hipSuccess) return LC_EHIP;
  hipLaunchKernelGGL((select_kernel<M, DSUB>), dim3(ceil_div(a.count, wpb)), dim3(64 * wpb), cent_bytes, st, a);
  hipLaunchKernelGGL(offsets_kernel, dim3(ceil_div(int64_t(a.count) * a.deg0, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(scatter_kernel, dim3(ceil_div(int64_t(a.count) * a.deg0, 256)), dim3(256), 0, st, a);
  const int merge_lds = cent_bytes + wpb * a.d_pad * 4;
  const void *mk = reinterpret_cast<const void *>(&merge_kernel<M, DSUB>);
  if (hipFuncSetAttribute(mk, hipFuncAttributeMaxDynamicSharedMemorySize, merge_lds) != hipSuccess) return LC_EHIP;
  // groups are at most count * deg0; a grid of a block per compute unit loops over them
  hipLaunchKernelGGL((merge_kernel<M, DSUB>), dim3(ix->num_cus), dim3(64 * wpb), merge_lds, st, a);
  int kcap = 64;
  while (kcap < a.deg0 + max_count) kcap <<= 1;
  const int large_lds = kcap * 9 + a.d_pad * 4;
  const void *lk = reinterpret_cast<const void *>(&merge_large_kernel<M, DSUB>);
  if (hipFuncSetAttribute(lk, hipFuncAttributeMaxDynamicSharedMemorySize, large_lds) != hipSuccess) return LC_EHIP;
  hipLaunchKernelGGL((merge_large_kernel<M, DSUB>), dim3(ix->num_cus), dim3(64), large_lds, st, a, kcap);
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, a.counters);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

}  // namespace

extern "C" {

int lc_project_exact(const float *x, int64_t n, int d, const float *proj, int d_pad, float *xp, void *stream) {
  if (n < 0 || d < 1 || d_pad < d) return LC_EINVAL;
  if (n == 0) return LC_OK;
  if (!x || !xp || (!proj && d_pad != d)) return LC_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!proj) {
    if (hipMemcpyAsync(xp, x, size_t(n) * d * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) return LC_EHIP;
    return LC_OK;
  }
  const int64_t total = n * d_pad;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(project_exact_kernel, dim3(unsigned(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, x, n,
                     d, proj, d_pad, xp);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

int lc_pq_encode(const float *xp, int64_t n, int d_pad, int m, const float *centroids, uint8_t *codes,
                 int code_stride, void *stream) {
  if (n < 0 || m < 1 || d_pad < m || d_pad % m || code_stride < m) return LC_EINVAL;
  if (d_pad / m > 16) return LC_ENOTSUP;
  if (n == 0) return LC_OK;
  if (!xp || !centroids || !codes) return LC_EINVAL;
  const int64_t blocks = (n + 255) / 256;
  dim3 grid(unsigned(blocks < 8192 ? blocks : 8192), unsigned(m + (code_stride > m ? 1 : 0)));
  hipLaunchKernelGGL(pq_encode_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), xp, n, d_pad, m,
                     d_pad / m, centroids, codes, code_stride);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_EHIP;
}

size_t lc_graph_insert_workspace_bytes(const lc_index *ix, int32_t max_count, int32_t ef_construction) {
  if (!ix || max_count < 1 || ef_construction < 1 || ef_construction > 64) return 0;
  return insert_layout(ix, max_count, ef_construction).total;
}

int lc_graph_insert(const lc_index *ix, int32_t *adj0, const float *xp, const int32_t *nodes, int32_t count,
                    int32_t max_count, int32_t ef_construction, void *ws, size_t ws_bytes, void *stream) {
  if (!ix || count < 0 || max_count < 1 || count > max_count || ef_construction < 1) return LC_EINVAL;
  if (ef_construction > 64) return LC_ENOTSUP;
  if (count == 0) return LC_OK;
  if (!adj0 || !xp || !nodes || !ws || adj0 != ix->v.adj0) return LC_EINVAL;
  if (ix->v.coarse_k > 0) return LC_ENOTSUP;
  const int cent_bytes = ix->v.d_pad * 256 * 4;
  if (cent_bytes + 16 * ix->v.d_pad * 4 > ix->lds_per_cu) return LC_ENOTSUP;
  const InsertLayout L = insert_layout(ix, max_count, ef_construction);
  if (ws_bytes < L.total) return LC_ENOSPC;
  char *w = static_cast<char *>(ws);
  InsertArgs a;
  a.xp = xp;
  a.cent = ix->v.centroids;
  a.codes = ix->v.codes;
  a.adj0 = adj0;
  a.nodes = nodes;
  a.count = count;
  a.efc = ef_construction;
  a.deg0 = ix->v.deg0;
  a.cs = ix->v.code_stride;
  a.m = ix->v.m;
  a.dsub = ix->dsub;
  a.d_pad = ix->v.d_pad;
  a.cand_ids = reinterpret_cast<int32_t *>(w + L.cand_ids);
  a.cand_adc = reinterpret_cast<float *>(w + L.cand_adc);
  a.cand_n = reinterpret_cast<int32_t *>(w + L.cand_n);
  a.req_tgt = reinterpret_cast<int32_t *>(w + L.req);
  a.inbox = reinterpret_cast<int32_t *>(w + L.inbox);
  a.gid_of = reinterpret_cast<int32_t *>(w + L.gid);
  a.group_tgt = reinterpret_cast<int32_t *>(w + L.gt);
  a.group_cnt = reinterpret_cast<int32_t *>(w + L.gc);
  a.group_off = reinterpret_cast<int32_t *>(w + L.go);
  a.group_fill = reinterpret_cast<int32_t *>(w + L.gf);
  a.srcs = reinterpret_cast<int32_t *>(w + L.srcs);
  a.ovf = reinterpret_cast<int32_t *>(w + L.ovf);
  a.counters = reinterpret_cast<uint32_t *>(w);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // sub-vector lengths of the usual shapes unrolled at compile time, any other at run time
#define CASE_D(MM)                                                  \
  case MM:                                                          \
    switch (a.dsub) {                                               \
      case 2: return insert_m<MM, 2>(ix, a, L, w, max_count, st);   \
      case 4: return insert_m<MM, 4>(ix, a, L, w, max_count, st);   \
      case 6: return insert_m<MM, 6>(ix, a, L, w, max_count, st);   \
      default: return insert_m<MM, 0>(ix, a, L, w, max_count, st);  \
    }
  switch (ix->v.m) {
    CASE_D(8) CASE_D(16) CASE_D(24) CASE_D(32) CASE_D(40) CASE_D(48) CASE_D(56) CASE_D(64)
    default: return LC_ENOTSUP;
  }
#undef CASE_D
}

}  // extern "C"
