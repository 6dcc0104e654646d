// Host-side index construction (include/lc_build.h).  Float32 distances with
// per-sub-space tables; float64 for the regression least squares.  Work is
// split over threads only where items are independent (vectors of a batch,
// reverse-link owners, codebook clusters), so results never depend on the
// thread count.
#include "lc_build.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

namespace {

// Progress lines on stderr every ~15 s when LCB_PROGRESS is set (long builds).
struct Progress {
  const char *what;
  bool on;
  std::chrono::steady_clock::time_point last, start;
  explicit Progress(const char *w) : what(w), on(std::getenv("LCB_PROGRESS") != nullptr) {
    last = start = std::chrono::steady_clock::now();
  }
  void tick(int64_t done, int64_t total) {
    if (!on) return;
    auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - last).count() < 15.0) return;
    last = now;
    std::fprintf(stderr, "[lc_build] %s: %lld / %lld (%.0f s)\n", what, (long long)done, (long long)total,
                 std::chrono::duration<double>(now - start).count());
    std::fflush(stderr);
  }
};

// ---------------------------------------------------------------------------
// threads
// ---------------------------------------------------------------------------
void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int)> &fn, int64_t grain = 1) {
  if (n <= 0) return;
  if (nthreads < 1) nthreads = 1;
  if (nthreads == 1 || n <= grain) {
    for (int64_t i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  int nt = int(std::min<int64_t>(nthreads, (n + grain - 1) / grain));
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (;;) {
        int64_t i0 = next.fetch_add(grain);
        if (i0 >= n) break;
        int64_t i1 = std::min(n, i0 + grain);
        for (int64_t i = i0; i < i1; ++i) fn(i, t);
      }
    });
  for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
struct Space {
  int d, d_pad, m, dsub;
  const float *proj;
  const float *cent;           // [m][256][dsub]
  const float *rec = nullptr;  // [n][d_pad] reconstructions of a 2-level codec, else decoded from the codes
  void project(const float *x, float *out) const {
    if (!proj) {
      std::memcpy(out, x, sizeof(float) * d);
      return;
    }
    for (int r = 0; r < d_pad; ++r) {
      double s = 0;
      const float *pr = proj + int64_t(r) * d;
      for (int t = 0; t < d; ++t) s += double(pr[t]) * x[t];
      out[r] = float(s);
    }
  }
  // table[s][c] = ||v^s - C[s][c]||^2; with reconstructions given, v itself
  void table(const float *v, float *tab) const {
    if (rec) {
      std::memcpy(tab, v, sizeof(float) * d_pad);
      return;
    }
    for (int s = 0; s < m; ++s) {
      const float *vs = v + s * dsub;
      const float *cs = cent + int64_t(s) * 256 * dsub;
      for (int c = 0; c < 256; ++c) {
        float e = 0;
        for (int t = 0; t < dsub; ++t) {
          float df = vs[t] - cs[c * dsub + t];
          e += df * df;
        }
        tab[s * 256 + c] = e;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// k-means (float32 distances, float64 sums)
// ---------------------------------------------------------------------------
// init: seed rows of x, or NULL to start from the centroids already in cent
void kmeans_f32(const float *x, int64_t n, int dim, int k, const int64_t *init, int iters, int nthreads,
                float *cent) {
  if (init)
    for (int j = 0; j < k; ++j) std::memcpy(cent + int64_t(j) * dim, x + init[j] * dim, sizeof(float) * dim);
  std::vector<int32_t> as(n);
  std::vector<float> err(n);
  std::vector<double> sum(size_t(k) * dim);
  std::vector<int64_t> cnt(k);
  for (int it = 0; it < iters; ++it) {
    parallel_for(
        n, nthreads,
        [&](int64_t i, int) {
          const float *xi = x + i * dim;
          float best = FLT_MAX;
          int bj = 0;
          for (int j = 0; j < k; ++j) {
            const float *cj = cent + int64_t(j) * dim;
            float e = 0;
            for (int t = 0; t < dim; ++t) {
              float df = xi[t] - cj[t];
              e += df * df;
            }
            if (e < best) {
              best = e;
              bj = j;
            }
          }
          as[i] = bj;
          err[i] = best;
        },
        1024);
    std::fill(sum.begin(), sum.end(), 0.0);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = 0; i < n; ++i) {
      cnt[as[i]]++;
      for (int t = 0; t < dim; ++t) sum[size_t(as[i]) * dim + t] += x[i * dim + t];
    }
    for (int j = 0; j < k; ++j) {
      if (cnt[j] > 0) {
        for (int t = 0; t < dim; ++t) cent[int64_t(j) * dim + t] = float(sum[size_t(j) * dim + t] / cnt[j]);
      } else {
        int64_t bi = int64_t(std::max_element(err.begin(), err.end()) - err.begin());
        std::memcpy(cent + int64_t(j) * dim, x + bi * dim, sizeof(float) * dim);
        err[bi] = -1.f;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// least squares (float64): Cholesky, else eigen pseudo-inverse
// ---------------------------------------------------------------------------
void eig_sym(std::vector<double> a, int p, std::vector<double> &w, std::vector<double> &v) {
  v.assign(size_t(p) * p, 0.0);
  for (int i = 0; i < p; ++i) v[i * p + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < p * p; ++i) tot += a[i] * a[i];
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j)
        if (i != j) off += a[i * p + j] * a[i * p + j];
    if (off == 0 || off <= 1e-30 * tot) break;
    for (int r = 0; r < p; ++r)
      for (int c = r + 1; c < p; ++c) {
        double arc = a[r * p + c];
        if (arc == 0) continue;
        double th = (a[c * p + c] - a[r * p + r]) / (2 * arc);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
        for (int k = 0; k < p; ++k) {
          double x = a[k * p + r], y = a[k * p + c];
          a[k * p + r] = cs * x - sn * y;
          a[k * p + c] = sn * x + cs * y;
        }
        for (int k = 0; k < p; ++k) {
          double x = a[r * p + k], y = a[c * p + k];
          a[r * p + k] = cs * x - sn * y;
          a[c * p + k] = sn * x + cs * y;
        }
        for (int k = 0; k < p; ++k) {
          double x = v[k * p + r], y = v[k * p + c];
          v[k * p + r] = cs * x - sn * y;
          v[k * p + c] = sn * x + cs * y;
        }
      }
  }
  w.resize(p);
  for (int i = 0; i < p; ++i) w[i] = a[i * p + i];
}

void lsq(const double *a, const double *c, int p, double *beta) {
  std::vector<double> L(size_t(p) * p, 0.0);
  double amax = 0;
  for (int i = 0; i < p; ++i) amax = std::max(amax, a[i * p + i]);
  bool ok = amax > 0;
  for (int j = 0; j < p && ok; ++j) {
    double s = a[j * p + j];
    for (int k = 0; k < j; ++k) s -= L[j * p + k] * L[j * p + k];
    if (!(s > 1e-12 * amax)) {
      ok = false;
      break;
    }
    L[j * p + j] = std::sqrt(s);
    for (int i = j + 1; i < p; ++i) {
      double t = a[i * p + j];
      for (int k = 0; k < j; ++k) t -= L[i * p + k] * L[j * p + k];
      L[i * p + j] = t / L[j * p + j];
    }
  }
  if (ok) {
    std::vector<double> z(p);
    for (int i = 0; i < p; ++i) {
      double t = c[i];
      for (int k = 0; k < i; ++k) t -= L[i * p + k] * z[k];
      z[i] = t / L[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
      double t = z[i];
      for (int k = i + 1; k < p; ++k) t -= L[k * p + i] * beta[k];
      beta[i] = t / L[i * p + i];
    }
    return;
  }
  std::vector<double> w, v;
  eig_sym(std::vector<double>(a, a + size_t(p) * p), p, w, v);
  double wmax = 0;
  for (double x : w) wmax = std::max(wmax, x);
  for (int i = 0; i < p; ++i) beta[i] = 0;
  if (wmax <= 0) return;
  for (int e = 0; e < p; ++e) {
    if (!(w[e] > 1e-12 * wmax)) continue;
    double pr = 0;
    for (int i = 0; i < p; ++i) pr += v[i * p + e] * c[i];
    for (int i = 0; i < p; ++i) beta[i] += v[i * p + e] * pr / w[e];
  }
}

// ---------------------------------------------------------------------------
// graph
// ---------------------------------------------------------------------------
struct Cand {
  float d;
  int32_t id;
  bool operator<(const Cand &o) const { return d < o.d || (d == o.d && id < o.id); }
};

struct Builder {
  int64_t n;
  Space sp;
  const float *xp;  // [n][d_pad] projected raw vectors
  const uint8_t *codes;
  int cs;
  const int8_t *level;
  int deg0, deg_up, efc;
  int32_t *adj0, *up_base, *adj_up;
  int32_t entry = 0, max_level = 0;
  std::vector<float> sdc;  // [m][256][256] distances between centroids

  int cap(int l) const { return l == 0 ? deg0 : deg_up; }
  int32_t *row(int l, int32_t i) const {
    return l == 0 ? adj0 + int64_t(i) * deg0 : adj_up + (int64_t(up_base[i]) + l - 1) * deg_up;
  }
  static float dist2(const float *a, const float *b, int n) {
    float s = 0;
    for (int u = 0; u < n; ++u) {
      float df = a[u] - b[u];
      s += df * df;
    }
    return s;
  }
  float adc(const float *tab, int32_t i) const {
    if (sp.rec) return dist2(tab, sp.rec + int64_t(i) * sp.d_pad, sp.d_pad);
    const uint8_t *c = codes + int64_t(i) * cs;
    float s = 0;
    for (int t = 0; t < sp.m; ++t) s += tab[t * 256 + c[t]];
    return s;
  }
  float rec_rec(int32_t a, int32_t b) const {
    if (sp.rec) return dist2(sp.rec + int64_t(a) * sp.d_pad, sp.rec + int64_t(b) * sp.d_pad, sp.d_pad);
    const uint8_t *ca = codes + int64_t(a) * cs, *cb = codes + int64_t(b) * cs;
    float s = 0;
    for (int t = 0; t < sp.m; ++t) s += sdc[(size_t(t) * 256 + ca[t]) * 256 + cb[t]];
    return s;
  }
  float raw_rec(const float *v, int32_t j) const {
    if (sp.rec) return dist2(v, sp.rec + int64_t(j) * sp.d_pad, sp.d_pad);
    const uint8_t *c = codes + int64_t(j) * cs;
    float s = 0;
    for (int t = 0; t < sp.m; ++t) {
      const float *cr = sp.cent + (int64_t(t) * 256 + c[t]) * sp.dsub;
      for (int u = 0; u < sp.dsub; ++u) {
        float df = v[t * sp.dsub + u] - cr[u];
        s += df * df;
      }
    }
    return s;
  }

  struct Scratch {
    std::vector<uint32_t> stamp;
    uint32_t sv = 0;
    std::vector<float> tab;
    std::vector<Cand> C, W, tmp;
  };

  // best-first search on level l from ep, pool bounded by ef; W sorted out
  void layer_search(const float *tab, int l, int32_t ep, int ef, Scratch &S, std::vector<Cand> &out) const {
    if (++S.sv == 0) {
      std::fill(S.stamp.begin(), S.stamp.end(), 0u);
      S.sv = 1;
    }
    auto &C = S.C;
    auto &W = S.W;
    C.clear();
    W.clear();
    Cand e{adc(tab, ep), ep};
    S.stamp[ep] = S.sv;
    auto minf = [](const Cand &a, const Cand &b) { return b < a; };  // min-heap
    C.push_back(e);
    W.push_back(e);
    const int cp = cap(l);
    while (!C.empty()) {
      std::pop_heap(C.begin(), C.end(), minf);
      Cand c = C.back();
      C.pop_back();
      if (int(W.size()) >= ef && W.front() < c) break;
      const int32_t *r = row(l, c.id);
      for (int j = 0; j < cp; ++j) {
        int32_t nb = r[j];
        if (nb < 0) break;
        if (S.stamp[nb] == S.sv) continue;
        S.stamp[nb] = S.sv;
        Cand k{adc(tab, nb), nb};
        if (int(W.size()) < ef || k < W.front()) {
          C.push_back(k);
          std::push_heap(C.begin(), C.end(), minf);
          W.push_back(k);
          std::push_heap(W.begin(), W.end());
          if (int(W.size()) > ef) {
            std::pop_heap(W.begin(), W.end());
            W.pop_back();
          }
        }
      }
    }
    out.assign(W.begin(), W.end());
    std::sort(out.begin(), out.end());
  }

  // shrinking heuristic + fill; cand sorted by (distance to owner, id)
  int select(const std::vector<Cand> &cand, int cp, int32_t *out) const {
    int nk = 0;
    std::vector<char> kept(cand.size(), 0);
    int32_t kid[64];
    for (size_t i = 0; i < cand.size() && nk < cp; ++i) {
      bool good = true;
      for (int t = 0; t < nk && good; ++t)
        if (!(cand[i].d < rec_rec(cand[i].id, kid[t]))) good = false;
      if (good) {
        kept[i] = 1;
        kid[nk++] = cand[i].id;
      }
    }
    for (size_t i = 0; i < cand.size() && nk < cp; ++i)
      if (!kept[i]) {
        kept[i] = 1;
        ++nk;
      }
    int w = 0;
    for (size_t i = 0; i < cand.size(); ++i)
      if (kept[i]) out[w++] = cand[i].id;
    for (int i = w; i < cp; ++i) out[i] = -1;
    return w;
  }
};

}  // namespace

extern "C" {

int lcb_pq_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int m,
                 const int64_t *init, int iters, int nthreads, float *centroids) {
  if (n < 256 || m < 1 || d_pad % m || d_pad < d) return -1;
  const int dsub = d_pad / m;
  Space sp{d, d_pad, m, dsub, proj, nullptr};
  std::vector<float> xp(size_t(n) * d_pad);
  parallel_for(n, nthreads, [&](int64_t i, int) { sp.project(train + i * d, xp.data() + i * d_pad); }, 4096);
  std::vector<float> sub(size_t(n) * dsub);
  for (int s = 0; s < m; ++s) {
    for (int64_t i = 0; i < n; ++i)
      for (int t = 0; t < dsub; ++t) sub[size_t(i) * dsub + t] = xp[size_t(i) * d_pad + s * dsub + t];
    kmeans_f32(sub.data(), n, dsub, 256, init + int64_t(s) * 256, iters, nthreads,
               centroids + int64_t(s) * 256 * dsub);
  }
  return 0;
}

int lcb_pq_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                  const float *centroids, int nthreads, uint8_t *codes, int code_stride) {
  if (m < 1 || d_pad % m || code_stride < m) return -1;
  Space sp{d, d_pad, m, d_pad / m, proj, centroids};
  parallel_for(
      n, nthreads,
      [&](int64_t i, int) {
        float v[1024];
        sp.project(x + i * d, v);
        uint8_t *c = codes + i * code_stride;
        for (int s = 0; s < m; ++s) {
          const float *cs = centroids + int64_t(s) * 256 * sp.dsub;
          float best = FLT_MAX;
          int bj = 0;
          for (int j = 0; j < 256; ++j) {
            float e = 0;
            for (int t = 0; t < sp.dsub; ++t) {
              float df = v[s * sp.dsub + t] - cs[j * sp.dsub + t];
              e += df * df;
            }
            if (e < best) {
              best = e;
              bj = j;
            }
          }
          c[s] = uint8_t(bj);
        }
        for (int s = m; s < code_stride; ++s) c[s] = 0;
      },
      1024);
  return 0;
}

int lcb_coarse_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int k, const int64_t *init,
                     int iters, int nthreads, float *cent) {
  if (k < 1 || k > 65536 || n < k || d_pad % 2 || d_pad < d || d_pad > 1024) return -1;
  const int h = d_pad / 2;
  Space sp{d, d_pad, 2, h, proj, nullptr};
  std::vector<float> xp(size_t(n) * d_pad), sub(size_t(n) * h);
  parallel_for(n, nthreads, [&](int64_t i, int) { sp.project(train + i * d, xp.data() + i * d_pad); }, 4096);
  for (int half = 0; half < 2; ++half) {
    for (int64_t i = 0; i < n; ++i)
      for (int t = 0; t < h; ++t) sub[size_t(i) * h + t] = xp[size_t(i) * d_pad + half * h + t];
    kmeans_f32(sub.data(), n, h, k, init + int64_t(half) * k, iters, nthreads, cent + int64_t(half) * k * h);
  }
  return 0;
}

int lcb_coarse_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int k, const float *cent,
                      int nthreads, uint16_t *codes, float *resid) {
  if (k < 1 || k > 65536 || d_pad % 2 || d_pad < d || d_pad > 1024) return -1;
  const int h = d_pad / 2;
  Space sp{d, d_pad, 2, h, proj, nullptr};
  parallel_for(
      n, nthreads,
      [&](int64_t i, int) {
        float v[1024];
        sp.project(x + i * d, v);
        for (int half = 0; half < 2; ++half) {
          const float *ch = cent + int64_t(half) * k * h;
          float best = FLT_MAX;
          int bj = 0;
          for (int j = 0; j < k; ++j) {
            float e = 0;
            for (int t = 0; t < h; ++t) {
              float df = v[half * h + t] - ch[int64_t(j) * h + t];
              e += df * df;
            }
            if (e < best) {
              best = e;
              bj = j;
            }
          }
          codes[i * 2 + half] = uint16_t(bj);
          for (int t = 0; t < h; ++t) resid[i * d_pad + half * h + t] = v[half * h + t] - ch[int64_t(bj) * h + t];
        }
      },
      256);
  return 0;
}

int lcb_coarse_decode(int64_t n, int d_pad, int m, const float *centroids, const uint8_t *codes, int code_stride,
                      int k, const float *cent, const uint16_t *ccodes, int nthreads, float *rec, float *norm) {
  if (m < 1 || d_pad % m || d_pad % 2 || k < 1 || code_stride < m) return -1;
  const int h = d_pad / 2, dsub = d_pad / m;
  parallel_for(
      n, nthreads,
      [&](int64_t i, int) {
        double cc = 0, qq = 0;
        for (int t = 0; t < d_pad; ++t) {
          const int half = t / h, s = t / dsub;
          const float c = cent[(int64_t(half) * k + ccodes[i * 2 + half]) * h + (t - half * h)];
          const float r = centroids[(int64_t(s) * 256 + codes[i * code_stride + s]) * dsub + (t - s * dsub)];
          const double q = double(c) + double(r);
          if (rec) rec[i * d_pad + t] = float(q);
          cc += double(c) * c;
          qq += q * q;
        }
        if (norm) norm[i] = float(qq - cc);
      },
      4096);
  return 0;
}

int64_t lcb_levels(const double *u, int64_t n, int ratio, int cap, int8_t *level) {
  int64_t rows = 0;
  const double lr = std::log(double(ratio));
  for (int64_t i = 0; i < n; ++i) {
    double v = std::floor(-std::log(u[i]) / lr);
    int l = v > cap ? cap : int(v);
    if (l < 0) l = 0;
    level[i] = int8_t(l);
    rows += l;
  }
  return rows;
}

int lcb_graph_build(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                    const float *centroids, const uint8_t *codes, int code_stride, const int8_t *level,
                    int deg0, int deg_up, int ef_construction, int nthreads, int32_t *adj0, int32_t *up_base,
                    int32_t *adj_up, int32_t *entry, int32_t *max_level, const float *rec) {
  return lcb_graph_build_part(x, n, d, proj, d_pad, m, centroids, codes, code_stride, level, deg0, deg_up,
                              ef_construction, nthreads, adj0, up_base, adj_up, entry, max_level, rec, 0, nullptr);
}

int lcb_graph_build_part(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                         const float *centroids, const uint8_t *codes, int code_stride, const int8_t *level,
                         int deg0, int deg_up, int ef_construction, int nthreads, int32_t *adj0, int32_t *up_base,
                         int32_t *adj_up, int32_t *entry, int32_t *max_level, const float *rec, int upper_only,
                         int64_t *next_pos) {
  if (n < 1 || m < 1 || d_pad % m || deg0 < 1 || deg0 > 64 || deg_up < 1 || deg_up > 64 || ef_construction < 1)
    return -1;
  if (nthreads < 1) nthreads = 1;
  Builder B;
  B.n = n;
  B.sp = Space{d, d_pad, m, d_pad / m, proj, centroids, rec};
  B.codes = codes;
  B.cs = code_stride;
  B.level = level;
  B.deg0 = deg0;
  B.deg_up = deg_up;
  B.efc = ef_construction;
  B.adj0 = adj0;
  B.up_base = up_base;
  B.adj_up = adj_up;
  std::vector<float> xpv;
  if (proj) {
    xpv.resize(size_t(n) * d_pad);
    parallel_for(n, nthreads, [&](int64_t i, int) { B.sp.project(x + i * d, xpv.data() + i * d_pad); }, 4096);
    B.xp = xpv.data();
  } else {
    B.xp = x;
  }
  const int dsub = B.sp.dsub;
  if (!rec) B.sdc.resize(size_t(m) * 256 * 256);
  if (!rec) parallel_for(m * 256, nthreads, [&](int64_t sa, int) {
    const int s = int(sa / 256), a = int(sa % 256);
    const float *ca = centroids + (int64_t(s) * 256 + a) * dsub;
    for (int b = 0; b < 256; ++b) {
      const float *cb = centroids + (int64_t(s) * 256 + b) * dsub;
      float e = 0;
      for (int t = 0; t < dsub; ++t) {
        float df = ca[t] - cb[t];
        e += df * df;
      }
      B.sdc[size_t(sa) * 256 + b] = e;
    }
  });

  int64_t rows = 0;
  for (int64_t i = 0; i < n; ++i) {
    up_base[i] = level[i] > 0 ? int32_t(rows) : -1;
    rows += level[i];
  }
  std::fill(adj0, adj0 + n * deg0, -1);
  std::fill(adj_up, adj_up + rows * deg_up, -1);
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = int32_t(i);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return level[a] > level[b]; });
  B.entry = order[0];
  B.max_level = level[order[0]];

  std::vector<Builder::Scratch> scratch(nthreads);
  for (auto &S : scratch) {
    S.stamp.assign(n, 0u);
    S.tab.resize(size_t(m) * 256);
  }
  const int capmax = std::max(deg0, deg_up);
  const int64_t bmax = 4096;
  const int L1 = B.max_level + 1;
  std::vector<int32_t> sel(size_t(bmax) * L1 * capmax);
  std::vector<int32_t> seln(size_t(bmax) * L1);
  struct RL {
    int32_t lvl, tgt, src;
  };
  std::vector<RL> rl;
  std::vector<int64_t> goff;

  Progress prog("graph");
  int64_t pos = 1;
  while (pos < n) {
    if (upper_only && level[order[pos]] == 0) break;  // the rest are level-0 nodes
    prog.tick(pos, n);
    int64_t bs = std::max<int64_t>(1, std::min<int64_t>(bmax, pos / 16));
    if (pos + bs > n) bs = n - pos;
    const int32_t *batch = order.data() + pos;
    // 1. search every new node against the frozen graph
    parallel_for(bs, nthreads, [&](int64_t bi, int tid) {
      auto &S = scratch[tid];
      const int32_t xn = batch[bi];
      const float *v = B.xp + int64_t(xn) * d_pad;
      B.sp.table(v, S.tab.data());
      const int lx = level[xn];
      int32_t cur = B.entry;
      Cand curc{B.adc(S.tab.data(), cur), cur};
      for (int l = B.max_level; l > lx; --l) {
        for (;;) {
          const int32_t *r = B.row(l, cur);
          Cand best = curc;
          for (int j = 0; j < deg_up && r[j] >= 0; ++j) {
            Cand k{B.adc(S.tab.data(), r[j]), r[j]};
            if (k < best) best = k;
          }
          if (best.id == cur) break;
          cur = best.id;
          curc = best;
        }
      }
      const int top = std::min(lx, B.max_level);
      std::vector<Cand> W;
      for (int l = top; l >= 0; --l) {
        B.layer_search(S.tab.data(), l, cur, ef_construction, S, W);
        seln[size_t(bi) * L1 + l] = B.select(W, B.cap(l), sel.data() + (size_t(bi) * L1 + l) * capmax);
        cur = W[0].id;
      }
    });
    // 2. the new nodes' own lists and the reverse links they ask for
    rl.clear();
    for (int64_t bi = 0; bi < bs; ++bi) {
      const int32_t xn = batch[bi];
      const int top = std::min<int>(level[xn], B.max_level);
      for (int l = 0; l <= top; ++l) {
        const int32_t *s = sel.data() + (size_t(bi) * L1 + l) * capmax;
        std::memcpy(B.row(l, xn), s, sizeof(int32_t) * B.cap(l));
        for (int j = 0; j < seln[size_t(bi) * L1 + l]; ++j) rl.push_back({l, s[j], xn});
      }
    }
    std::sort(rl.begin(), rl.end(), [](const RL &a, const RL &b) {
      if (a.lvl != b.lvl) return a.lvl < b.lvl;
      if (a.tgt != b.tgt) return a.tgt < b.tgt;
      return a.src < b.src;
    });
    goff.clear();
    for (size_t i = 0; i < rl.size(); ++i)
      if (i == 0 || rl[i].lvl != rl[i - 1].lvl || rl[i].tgt != rl[i - 1].tgt) goff.push_back(int64_t(i));
    goff.push_back(int64_t(rl.size()));
    // 3. every target merges its incoming links (re-shrinking a full list)
    parallel_for(int64_t(goff.size()) - 1, nthreads, [&](int64_t g, int) {
      const int l = rl[goff[g]].lvl;
      const int32_t e = rl[goff[g]].tgt;
      const int cp = B.cap(l);
      int32_t *r = B.row(l, e);
      const float *v = B.xp + int64_t(e) * d_pad;
      std::vector<Cand> cand;
      for (int j = 0; j < cp && r[j] >= 0; ++j) cand.push_back({B.raw_rec(v, r[j]), r[j]});
      for (int64_t i = goff[g]; i < goff[g + 1]; ++i) cand.push_back({B.raw_rec(v, rl[i].src), rl[i].src});
      std::sort(cand.begin(), cand.end());
      if (int(cand.size()) <= cp) {
        for (int j = 0; j < cp; ++j) r[j] = j < int(cand.size()) ? cand[j].id : -1;
      } else {
        int32_t tmp[64];
        B.select(cand, cp, tmp);
        std::memcpy(r, tmp, sizeof(int32_t) * cp);
      }
    });
    pos += bs;
  }
  *entry = B.entry;
  *max_level = B.max_level;
  if (next_pos) *next_pos = pos;
  return 0;
}

// ---------------------------------------------------------------------------
// regression codebook
// ---------------------------------------------------------------------------
namespace {

struct Gram {
  int p, dp;
  std::vector<double> A, C, XX;  // [n][p][p], [n][p], [n]
};

// Grams of G(x) and x restricted to the coordinates [t0, t1) (a block of the
// product codebook, Sec. 4.3 Eq. 9; the whole vector is [0, d_pad)).
void build_grams(const float *x, const int64_t *ids, int64_t n_sub, const Space &sp, const uint8_t *codes,
                 int cs, const int32_t *adj0, int deg0, int k_reg, int nthreads, int t0, int t1, Gram &g) {
  const int p = k_reg + 1, dp = sp.d_pad;
  g.p = p;
  g.dp = dp;
  g.A.assign(size_t(n_sub) * p * p, 0.0);
  g.C.assign(size_t(n_sub) * p, 0.0);
  g.XX.assign(size_t(n_sub), 0.0);
  parallel_for(
      n_sub, nthreads,
      [&](int64_t r, int) {
        const int64_t i = ids ? ids[r] : r;
        std::vector<double> G(size_t(p) * dp, 0.0);
        std::vector<float> v(dp);
        sp.project(x + i * sp.d, v.data());
        for (int j = 0; j < p; ++j) {
          const int64_t src = j == 0 ? i : adj0[i * deg0 + (j - 1)];
          if (src < 0) continue;
          if (sp.rec) {
            for (int t = t0; t < t1; ++t) G[size_t(j) * dp + t] = sp.rec[src * dp + t];
            continue;
          }
          const uint8_t *c = codes + src * cs;
          for (int s = t0 / sp.dsub; s < t1 / sp.dsub; ++s) {
            const float *cr = sp.cent + (int64_t(s) * 256 + c[s]) * sp.dsub;
            for (int t = 0; t < sp.dsub; ++t) G[size_t(j) * dp + s * sp.dsub + t] = cr[t];
          }
        }
        double *A = g.A.data() + size_t(r) * p * p;
        double *C = g.C.data() + size_t(r) * p;
        for (int a = 0; a < p; ++a) {
          for (int b = a; b < p; ++b) {
            double s = 0;
            for (int t = t0; t < t1; ++t) s += G[size_t(a) * dp + t] * G[size_t(b) * dp + t];
            A[a * p + b] = A[b * p + a] = s;
          }
          double s = 0;
          for (int t = t0; t < t1; ++t) s += G[size_t(a) * dp + t] * double(v[t]);
          C[a] = s;
        }
        double s = 0;
        for (int t = t0; t < t1; ++t) s += double(v[t]) * v[t];
        g.XX[r] = s;
      },
      256);
}

// index of the codebook entry minimising ||x - G beta||^2 (lowest on ties)
int best_beta(const Gram &g, int64_t r, const double *B, int nb, double *loss) {
  const int p = g.p;
  const double *A = g.A.data() + size_t(r) * p * p;
  const double *C = g.C.data() + size_t(r) * p;
  double best = DBL_MAX;
  int bi = 0;
  for (int b = 0; b < nb; ++b) {
    const double *be = B + size_t(b) * p;
    double l = g.XX[r];
    for (int a = 0; a < p; ++a) {
      double s = 0;
      for (int c = 0; c < p; ++c) s += A[a * p + c] * be[c];
      l += be[a] * (s - 2 * C[a]);
    }
    if (l < best) {
      best = l;
      bi = b;
    }
  }
  if (loss) *loss = best;
  return bi;
}

}  // namespace

}  // extern "C"

namespace {

// One codebook on the Grams of one block: per-vector optimum, k-means on it,
// then EM (assignment Eq. 7, per-cluster least squares Eq. 8).
void train_block(const Gram &g, int64_t n_sub, int k_reg, int n_beta, const int64_t *init, int km_iters,
                 int em_iters, int nthreads, float *beta, double *loss_hist) {
  const int p = k_reg + 1;
  // per-vector optimum, then k-means on it (float64)
  std::vector<double> bx(size_t(n_sub) * p);
  parallel_for(n_sub, nthreads,
               [&](int64_t r, int) { lsq(g.A.data() + size_t(r) * p * p, g.C.data() + size_t(r) * p, p,
                                         bx.data() + size_t(r) * p); },
               1024);
  std::vector<double> B(size_t(n_beta) * p);
  for (int b = 0; b < n_beta; ++b) std::memcpy(&B[size_t(b) * p], &bx[size_t(init[b]) * p], sizeof(double) * p);
  std::vector<int32_t> as(n_sub);
  std::vector<double> err(n_sub);
  for (int it = 0; it < km_iters; ++it) {
    parallel_for(
        n_sub, nthreads,
        [&](int64_t r, int) {
          double best = DBL_MAX;
          int bj = 0;
          for (int b = 0; b < n_beta; ++b) {
            double e = 0;
            for (int t = 0; t < p; ++t) {
              double df = bx[size_t(r) * p + t] - B[size_t(b) * p + t];
              e += df * df;
            }
            if (e < best) {
              best = e;
              bj = b;
            }
          }
          as[r] = bj;
          err[r] = best;
        },
        1024);
    std::vector<double> sum(size_t(n_beta) * p, 0.0);
    std::vector<int64_t> cnt(n_beta, 0);
    for (int64_t r = 0; r < n_sub; ++r) {
      cnt[as[r]]++;
      for (int t = 0; t < p; ++t) sum[size_t(as[r]) * p + t] += bx[size_t(r) * p + t];
    }
    for (int b = 0; b < n_beta; ++b) {
      if (cnt[b] > 0) {
        for (int t = 0; t < p; ++t) B[size_t(b) * p + t] = sum[size_t(b) * p + t] / cnt[b];
      } else {
        int64_t bi = int64_t(std::max_element(err.begin(), err.end()) - err.begin());
        std::memcpy(&B[size_t(b) * p], &bx[size_t(bi) * p], sizeof(double) * p);
        err[bi] = -1.0;
      }
    }
  }
  // EM: assignment (Eq. 7), per-cluster least squares (Eq. 8)
  std::vector<double> ls(n_sub);
  Progress prog("beta EM");
  for (int it = 0;; ++it) {
    prog.tick(it, em_iters);
    parallel_for(n_sub, nthreads, [&](int64_t r, int) { as[r] = best_beta(g, r, B.data(), n_beta, &ls[r]); },
                 256);
    if (loss_hist) {
      double s = 0;
      for (double v : ls) s += v;
      loss_hist[it] = s;
    }
    if (it == em_iters) break;
    std::vector<std::vector<int64_t>> members(n_beta);
    for (int64_t r = 0; r < n_sub; ++r) members[as[r]].push_back(r);
    parallel_for(n_beta, nthreads, [&](int64_t b, int) {
      if (members[b].empty()) return;
      std::vector<double> SA(size_t(p) * p, 0.0), SC(p, 0.0);
      for (int64_t r : members[b]) {
        for (int t = 0; t < p * p; ++t) SA[t] += g.A[size_t(r) * p * p + t];
        for (int t = 0; t < p; ++t) SC[t] += g.C[size_t(r) * p + t];
      }
      lsq(SA.data(), SC.data(), p, &B[size_t(b) * p]);
    });
  }
  for (size_t t = 0; t < B.size(); ++t) beta[t] = float(B[t]);
}

}  // namespace

extern "C" {

int lcb_beta_train(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj, int d_pad, int m,
                   const float *centroids, const uint8_t *codes, int code_stride, const int32_t *adj0, int deg0,
                   int k_reg, int n_beta, int m_beta, const int64_t *init, int km_iters, int em_iters, int nthreads,
                   float *beta, double *loss_hist, const float *rec) {
  if (k_reg < 1 || k_reg > deg0 || n_beta < 1 || n_beta > n_sub || d_pad % m || m_beta < 1 || m % m_beta)
    return -1;
  Space sp{d, d_pad, m, d_pad / m, proj, centroids, rec};
  const int p = k_reg + 1, bw = d_pad / m_beta;
  // product codebook (Eq. 9): block jb covers coordinates [jb bw, jb bw + bw), m / m_beta whole sub-spaces
  for (int jb = 0; jb < m_beta; ++jb) {
    Gram g;
    build_grams(x, ids, n_sub, sp, codes, code_stride, adj0, deg0, k_reg, nthreads, jb * bw, jb * bw + bw, g);
    train_block(g, n_sub, k_reg, n_beta, init, km_iters, em_iters, nthreads, beta + size_t(jb) * n_beta * p,
                loss_hist ? loss_hist + size_t(jb) * (em_iters + 1) : nullptr);
  }
  return 0;
}

int lcb_beta_assign(const float *x, int64_t n, int d, const float *proj, int d_pad, int m, const float *centroids,
                    const uint8_t *codes, int code_stride, const int32_t *adj0, int deg0, int k_reg, int n_beta,
                    int m_beta, const float *beta, int nthreads, uint8_t *beta_idx, const float *rec) {
  if (k_reg < 1 || k_reg > deg0 || n_beta < 1 || n_beta > 256 || d_pad % m || m_beta < 1 || m % m_beta) return -1;
  Space sp{d, d_pad, m, d_pad / m, proj, centroids, rec};
  const int p = k_reg + 1, bw = d_pad / m_beta;
  std::vector<double> B(size_t(m_beta) * n_beta * p);
  for (size_t t = 0; t < B.size(); ++t) B[t] = beta[t];
  const int64_t chunk = 1 << 17;
  std::vector<int64_t> ids(chunk);
  Progress prog("beta assignment");
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    prog.tick(c0, n);
    const int64_t c1 = std::min(n, c0 + chunk);
    for (int64_t i = c0; i < c1; ++i) ids[i - c0] = i;
    for (int jb = 0; jb < m_beta; ++jb) {
      Gram g;
      build_grams(x, ids.data(), c1 - c0, sp, codes, code_stride, adj0, deg0, k_reg, nthreads, jb * bw,
                  jb * bw + bw, g);
      const double *Bj = B.data() + size_t(jb) * n_beta * p;
      parallel_for(c1 - c0, nthreads,
                   [&](int64_t r, int) {
                     beta_idx[(c0 + r) * m_beta + jb] = uint8_t(best_beta(g, r, Bj, n_beta, nullptr));
                   },
                   256);
    }
  }
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned rotation ahead of the product quantizer (OPQ, the codec of Sec. 4.1
// and Sec. 5.1): alternate PQ training on the rotated vectors with the
// rotation that best maps the vectors onto their reconstructions
// ---------------------------------------------------------------------------
namespace {

// P = S^T (S S^T)^(-1/2) for S [d][D] of full row rank: the D x d matrix with
// orthonormal columns maximising tr(P S) (orthogonal Procrustes; with
// S = U Sigma V^T it is V U^T).
bool procrustes(const std::vector<double> &S, int d, int D, std::vector<double> &P) {
  std::vector<double> SS(size_t(d) * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0;
      for (int t = 0; t < D; ++t) s += S[size_t(i) * D + t] * S[size_t(j) * D + t];
      SS[size_t(i) * d + j] = s;
    }
  std::vector<double> w, v;
  eig_sym(SS, d, w, v);
  double wmax = 0;
  for (double x : w) wmax = std::max(wmax, x);
  // (S S^T)^(-1/2) = V diag(w^-1/2) V^T
  std::vector<double> inv(size_t(d) * d, 0.0);
  for (int e = 0; e < d; ++e) {
    if (!(w[e] > 1e-24 * wmax)) return false;  // S is rank deficient
    const double f = 1.0 / std::sqrt(w[e]);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) inv[size_t(i) * d + j] += v[size_t(i) * d + e] * f * v[size_t(j) * d + e];
  }
  P.assign(size_t(D) * d, 0.0);
  for (int r = 0; r < D; ++r)
    for (int j = 0; j < d; ++j) {
      double s = 0;
      for (int i = 0; i < d; ++i) s += S[size_t(i) * D + r] * inv[size_t(i) * d + j];
      P[size_t(r) * d + j] = s;
    }
  return true;
}

}  // namespace

extern "C" {

int lcb_procrustes(const double *S, int d, int D, double *P) {
  if (d < 1 || D < d) return -1;
  std::vector<double> s(S, S + size_t(d) * D), p;
  if (!procrustes(s, d, D, p)) return 1;
  std::memcpy(P, p.data(), sizeof(double) * p.size());
  return 0;
}

int lcb_opq_train(const float *train, int64_t n, int d, int d_pad, int m, const float *init_proj,
                  const int64_t *init, int opq_iters, int km_iters, int nthreads, float *proj_out,
                  double *mse_hist) {
  if (n < 256 || m < 1 || d_pad % m || d_pad < d || opq_iters < 0 || km_iters < 1) return -1;
  if (!init_proj && d_pad != d) return -1;
  const int dsub = d_pad / m;
  std::vector<float> P(size_t(d_pad) * d, 0.f);
  if (init_proj) std::memcpy(P.data(), init_proj, sizeof(float) * P.size());
  else
    for (int i = 0; i < d; ++i) P[size_t(i) * d + i] = 1.f;
  std::vector<float> cent(size_t(m) * 256 * dsub), y(size_t(n) * d_pad), sub(size_t(n) * dsub),
      rec(size_t(n) * d_pad);
  const int64_t chunk = 4096;  // fixed reduction chunks: the result does not depend on the thread count
  const int64_t nch = (n + chunk - 1) / chunk;
  for (int it = 0;; ++it) {
    Space sp{d, d_pad, m, dsub, P.data(), nullptr};
    parallel_for(n, nthreads, [&](int64_t i, int) { sp.project(train + i * d, y.data() + i * d_pad); }, 4096);
    // PQ on the rotated vectors: from the seeds the first time, from the last centroids after
    for (int s = 0; s < m; ++s) {
      for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < dsub; ++t) sub[size_t(i) * dsub + t] = y[size_t(i) * d_pad + s * dsub + t];
      kmeans_f32(sub.data(), n, dsub, 256, it == 0 ? init + int64_t(s) * 256 : nullptr, km_iters, nthreads,
                 cent.data() + int64_t(s) * 256 * dsub);
    }
    // reconstructions and the distortion ||y - q(y)||^2 (mean over the training vectors)
    std::vector<double> part(nch, 0.0);
    parallel_for(nch, nthreads, [&](int64_t c, int) {
      double acc = 0;
      for (int64_t i = c * chunk; i < std::min(n, (c + 1) * chunk); ++i) {
        const float *yi = y.data() + i * d_pad;
        float *ri = rec.data() + i * d_pad;
        for (int s = 0; s < m; ++s) {
          const float *cs = cent.data() + int64_t(s) * 256 * dsub;
          float best = FLT_MAX;
          int bj = 0;
          for (int j = 0; j < 256; ++j) {
            float e = 0;
            for (int t = 0; t < dsub; ++t) {
              float df = yi[s * dsub + t] - cs[j * dsub + t];
              e += df * df;
            }
            if (e < best) {
              best = e;
              bj = j;
            }
          }
          for (int t = 0; t < dsub; ++t) ri[s * dsub + t] = cs[bj * dsub + t];
          acc += best;
        }
      }
      part[c] = acc;
    });
    double mse = 0;
    for (double x : part) mse += x;
    if (mse_hist) mse_hist[it] = mse / double(n);
    if (it == opq_iters) break;
    // S = X^T Yhat [d][d_pad], summed chunk by chunk in order
    std::vector<std::vector<double>> ps(nch);
    parallel_for(nch, nthreads, [&](int64_t c, int) {
      std::vector<double> acc(size_t(d) * d_pad, 0.0);
      for (int64_t i = c * chunk; i < std::min(n, (c + 1) * chunk); ++i) {
        const float *xi = train + i * d;
        const float *ri = rec.data() + i * d_pad;
        for (int a = 0; a < d; ++a) {
          const double xa = xi[a];
          double *row = acc.data() + size_t(a) * d_pad;
          for (int t = 0; t < d_pad; ++t) row[t] += xa * ri[t];
        }
      }
      ps[c] = std::move(acc);
    });
    std::vector<double> S(size_t(d) * d_pad, 0.0);
    for (int64_t c = 0; c < nch; ++c)
      for (size_t t = 0; t < S.size(); ++t) S[t] += ps[c][t];
    std::vector<double> Pd;
    if (!procrustes(S, d, d_pad, Pd)) return 2;
    for (size_t t = 0; t < P.size(); ++t) P[t] = float(Pd[t]);
  }
  std::memcpy(proj_out, P.data(), sizeof(float) * P.size());
  return 0;
}

}  // extern "C"
