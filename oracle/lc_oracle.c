/*
 * Link & Code reference oracle — TEST INFRASTRUCTURE ONLY (see lc_oracle.h).
 *
 * Plain float64 C.  Loops follow the paper's definitions directly; the only
 * concession to speed is a parallel-for over independent items (queries,
 * vectors of one build batch), which never changes a result.
 */
#include "lc_oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* parallel-for over independent indices                                     */
/* ------------------------------------------------------------------------ */
typedef void (*orc_body)(int64_t i, int tid, void *ctx);

typedef struct {
  int64_t n;
  int64_t next;
  pthread_mutex_t mu;
  orc_body fn;
  void *ctx;
} orc_pool;
typedef struct {
  orc_pool *pool;
  int tid;
} orc_worker;

static void *orc_run(void *arg) {
  orc_worker *w = (orc_worker *)arg;
  orc_pool *p = w->pool;
  for (;;) {
    int64_t i;
    pthread_mutex_lock(&p->mu);
    i = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (i >= p->n) break;
    p->fn(i, w->tid, p->ctx);
  }
  return NULL;
}

static void orc_parallel_for(int64_t n, int nthreads, orc_body fn, void *ctx) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads == 1 || n < 2) {
    for (int64_t i = 0; i < n; i++) fn(i, 0, ctx);
    return;
  }
  if (nthreads > 256) nthreads = 256;
  orc_pool pool;
  pool.n = n;
  pool.next = 0;
  pool.fn = fn;
  pool.ctx = ctx;
  pthread_mutex_init(&pool.mu, NULL);
  pthread_t th[256];
  orc_worker wk[256];
  for (int t = 0; t < nthreads; t++) {
    wk[t].pool = &pool;
    wk[t].tid = t;
    pthread_create(&th[t], NULL, orc_run, &wk[t]);
  }
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&pool.mu);
}

/* ------------------------------------------------------------------------ */
/* (distance, id) keys: the total order used everywhere                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  double d;
  int32_t id;
} okey;

static int okey_lt(okey a, okey b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }
static int okey_cmp(const void *pa, const void *pb) {
  okey a = *(const okey *)pa, b = *(const okey *)pb;
  if (okey_lt(a, b)) return -1;
  if (okey_lt(b, a)) return 1;
  return 0;
}

/* binary heaps of okey: min-heap (sign=+1) or max-heap (sign=-1) */
typedef struct {
  okey *a;
  int n, cap, max_heap;
} oheap;

static int oh_before(const oheap *h, okey x, okey y) { return h->max_heap ? okey_lt(y, x) : okey_lt(x, y); }
static void oh_push(oheap *h, okey k) {
  int i = h->n++;
  h->a[i] = k;
  while (i > 0) {
    int p = (i - 1) / 2;
    if (!oh_before(h, h->a[i], h->a[p])) break;
    okey t = h->a[i];
    h->a[i] = h->a[p];
    h->a[p] = t;
    i = p;
  }
}
static okey oh_pop(oheap *h) {
  okey top = h->a[0];
  h->a[0] = h->a[--h->n];
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, b = i;
    if (l < h->n && oh_before(h, h->a[l], h->a[b])) b = l;
    if (r < h->n && oh_before(h, h->a[r], h->a[b])) b = r;
    if (b == i) break;
    okey t = h->a[i];
    h->a[i] = h->a[b];
    h->a[b] = t;
    i = b;
  }
  return top;
}

/* ------------------------------------------------------------------------ */
/* k-means (Sec. 3.3 PQ training; Sec. 4.3 codebook initialisation)          */
/* ------------------------------------------------------------------------ */
typedef struct {
  const double *x, *cent;
  int dim, k;
  int32_t *assign;
  double *err;
} km_ctx;

static void km_assign_one(int64_t i, int tid, void *vctx) {
  (void)tid;
  km_ctx *c = (km_ctx *)vctx;
  const double *xi = c->x + i * c->dim;
  double best = DBL_MAX;
  int32_t bi = 0;
  for (int j = 0; j < c->k; j++) {
    const double *cj = c->cent + (int64_t)j * c->dim;
    double s = 0;
    for (int t = 0; t < c->dim; t++) {
      double df = xi[t] - cj[t];
      s += df * df;
    }
    if (s < best) { /* strict: lowest index wins ties */
      best = s;
      bi = j;
    }
  }
  c->assign[i] = bi;
  c->err[i] = best;
}

int orc_kmeans(const double *x, int64_t n, int dim, int k, const int64_t *init, int iters,
               int nthreads, double *cent, int32_t *assign, double *sse_hist) {
  if (n < 1 || dim < 1 || k < 1 || k > n) return -1;
  double *err = (double *)malloc(sizeof(double) * n);
  double *sum = (double *)malloc(sizeof(double) * (size_t)k * dim);
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * k);
  if (!err || !sum || !cnt) return -2;
  for (int j = 0; j < k; j++) memcpy(cent + (int64_t)j * dim, x + init[j] * dim, sizeof(double) * dim);
  km_ctx ctx = {x, cent, dim, k, assign, err};
  for (int it = 0;; it++) {
    orc_parallel_for(n, nthreads, km_assign_one, &ctx);
    if (sse_hist) {
      double s = 0;
      for (int64_t i = 0; i < n; i++) s += err[i];
      sse_hist[it] = s;
    }
    if (it == iters) break;
    /* update: each centroid becomes the mean of its members */
    memset(sum, 0, sizeof(double) * (size_t)k * dim);
    memset(cnt, 0, sizeof(int64_t) * k);
    for (int64_t i = 0; i < n; i++) {
      cnt[assign[i]]++;
      for (int t = 0; t < dim; t++) sum[(int64_t)assign[i] * dim + t] += x[i * dim + t];
    }
    for (int j = 0; j < k; j++) {
      if (cnt[j] > 0) {
        for (int t = 0; t < dim; t++) cent[(int64_t)j * dim + t] = sum[(int64_t)j * dim + t] / (double)cnt[j];
      } else {
        /* empty cluster: re-seed with the point of largest current error,
         * lowest index on ties; that point's error is then taken as zero */
        int64_t bi = 0;
        for (int64_t i = 1; i < n; i++)
          if (err[i] > err[bi]) bi = i;
        memcpy(cent + (int64_t)j * dim, x + bi * dim, sizeof(double) * dim);
        err[bi] = -1.0;
      }
    }
  }
  free(err);
  free(sum);
  free(cnt);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* projection and PQ (Sec. 3.3, Sec. 4.1)                                     */
/* ------------------------------------------------------------------------ */
void orc_project(const float *proj, int d_pad, int d, const float *y, double *out) {
  if (!proj) {
    for (int t = 0; t < d; t++) out[t] = (double)y[t];
    return;
  }
  for (int r = 0; r < d_pad; r++) {
    double s = 0;
    for (int t = 0; t < d; t++) s += (double)proj[(int64_t)r * d + t] * (double)y[t];
    out[r] = s;
  }
}

int orc_pq_train(const float *train, int64_t n, int d, const float *proj, int d_pad, int m,
                 int ksub, const int64_t *init, int iters, int nthreads, float *cent,
                 double *sse_hist) {
  if (d_pad % m) return -1;
  int dsub = d_pad / m;
  double *xp = (double *)malloc(sizeof(double) * (size_t)n * d_pad);
  double *sub = (double *)malloc(sizeof(double) * (size_t)n * dsub);
  double *c = (double *)malloc(sizeof(double) * (size_t)ksub * dsub);
  int32_t *as = (int32_t *)malloc(sizeof(int32_t) * n);
  if (!xp || !sub || !c || !as) return -2;
  for (int64_t i = 0; i < n; i++) orc_project(proj, d_pad, d, train + i * d, xp + i * d_pad);
  int rc = 0;
  for (int s = 0; s < m && rc == 0; s++) {
    for (int64_t i = 0; i < n; i++)
      for (int t = 0; t < dsub; t++) sub[i * dsub + t] = xp[i * d_pad + s * dsub + t];
    rc = orc_kmeans(sub, n, dsub, ksub, init + (int64_t)s * ksub, iters, nthreads, c, as,
                    sse_hist ? sse_hist + (int64_t)s * (iters + 1) : NULL);
    for (int j = 0; j < ksub * dsub; j++) cent[(int64_t)s * ksub * dsub + j] = (float)c[j];
  }
  free(xp);
  free(sub);
  free(c);
  free(as);
  return rc;
}

typedef struct {
  const float *x, *proj, *cent;
  int d, d_pad, m, ksub, code_stride;
  uint8_t *codes;
} enc_ctx;

static void enc_one(int64_t i, int tid, void *vctx) {
  (void)tid;
  enc_ctx *c = (enc_ctx *)vctx;
  double xp[4096];
  int dsub = c->d_pad / c->m;
  orc_project(c->proj, c->d_pad, c->d, c->x + i * c->d, xp);
  for (int s = 0; s < c->m; s++) {
    double best = DBL_MAX;
    int bj = 0;
    for (int j = 0; j < c->ksub; j++) {
      const float *cj = c->cent + ((int64_t)s * c->ksub + j) * dsub;
      double e = 0;
      for (int t = 0; t < dsub; t++) {
        double df = xp[s * dsub + t] - (double)cj[t];
        e += df * df;
      }
      if (e < best) {
        best = e;
        bj = j;
      }
    }
    c->codes[i * c->code_stride + s] = (uint8_t)bj;
  }
  for (int s = c->m; s < c->code_stride; s++) c->codes[i * c->code_stride + s] = 0;
}

int orc_pq_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                  int ksub, const float *cent, int nthreads, uint8_t *codes, int code_stride) {
  if (d_pad % m || d_pad > 4096 || ksub > 256 || code_stride < m) return -1;
  enc_ctx c = {x, proj, cent, d, d_pad, m, ksub, code_stride, codes};
  orc_parallel_for(n, nthreads, enc_one, &c);
  return 0;
}

/* 2-level residual codec (Sec. 3.3, Sec. 5.1): nearest first-level centroid
 * of each half, and the residual that the second level encodes */
typedef struct {
  const float *x, *proj, *cent;
  int d, d_pad, k;
  uint16_t *codes;
  float *resid;
} cenc_ctx;

static void cenc_one(int64_t i, int tid, void *vctx) {
  (void)tid;
  cenc_ctx *c = (cenc_ctx *)vctx;
  double xp[4096];
  int h = c->d_pad / 2;
  orc_project(c->proj, c->d_pad, c->d, c->x + i * c->d, xp);
  for (int half = 0; half < 2; half++) {
    double best = DBL_MAX;
    int bj = 0;
    for (int j = 0; j < c->k; j++) {
      const float *cj = c->cent + ((int64_t)half * c->k + j) * h;
      double e = 0;
      for (int t = 0; t < h; t++) {
        double df = xp[half * h + t] - (double)cj[t];
        e += df * df;
      }
      if (e < best) {
        best = e;
        bj = j;
      }
    }
    c->codes[i * 2 + half] = (uint16_t)bj;
    if (c->resid) {
      const float *cj = c->cent + ((int64_t)half * c->k + bj) * h;
      for (int t = 0; t < h; t++) c->resid[i * c->d_pad + half * h + t] = (float)(xp[half * h + t] - (double)cj[t]);
    }
  }
}

int orc_coarse_encode(const float *x, int64_t n, int d, const float *proj, int d_pad, int k,
                      const float *cent, int nthreads, uint16_t *codes, float *resid) {
  if (d_pad % 2 || d_pad > 4096 || k < 1 || k > 65536) return -1;
  cenc_ctx c = {x, proj, cent, d, d_pad, k, codes, resid};
  orc_parallel_for(n, nthreads, cenc_one, &c);
  return 0;
}

/* Levels (Sec. 2: geometric layer sizes; Sec. 4.1: ratio 30 between levels). */
int64_t orc_levels(const double *u, int64_t n, int ratio, int cap, int8_t *level) {
  int64_t rows = 0;
  for (int64_t i = 0; i < n; i++) {
    double v = floor(-log(u[i]) / log((double)ratio));
    int l = v > cap ? cap : (int)v;
    if (l < 0) l = 0;
    level[i] = (int8_t)l;
    rows += l;
  }
  return rows;
}

/* decode q(i) (its reconstruction) into out[d_pad]: the PQ reconstruction,
 * plus, for a 2-level codec, the first-level centroid of each half */
static void decode(const float *cent, const uint8_t *codes, int code_stride, int m, int ksub,
                   int dsub, const orc_coarse *cq, int64_t i, double *out) {
  for (int s = 0; s < m; s++) {
    const float *c = cent + ((int64_t)s * ksub + codes[i * code_stride + s]) * dsub;
    for (int t = 0; t < dsub; t++) out[s * dsub + t] = (double)c[t];
  }
  if (cq && cq->k > 0) {
    int h = m * dsub / 2;
    for (int half = 0; half < 2; half++) {
      const float *c = cq->cent + ((int64_t)half * cq->k + cq->codes[i * 2 + half]) * h;
      for (int t = 0; t < h; t++) out[half * h + t] += (double)c[t];
    }
  }
}

static double sqdist(const double *a, const double *b, int n) {
  double s = 0;
  for (int t = 0; t < n; t++) {
    double df = a[t] - b[t];
    s += df * df;
  }
  return s;
}

int orc_coarse_norms(const orc_index *ix, float *norm) {
  int dp = ix->d_pad, h = dp / 2;
  if (ix->coarse.k < 1 || dp % 2 || dp > 4096) return -1;
  double rec[4096];
  for (int64_t i = 0; i < ix->n; i++) {
    decode(ix->centroids, ix->codes, ix->code_stride, ix->m, ix->ksub, dp / ix->m, &ix->coarse, i, rec);
    double cc = 0, qq = 0;
    for (int half = 0; half < 2; half++) {
      const float *c = ix->coarse.cent + ((int64_t)half * ix->coarse.k + ix->coarse.codes[i * 2 + half]) * h;
      for (int t = 0; t < h; t++) cc += (double)c[t] * (double)c[t];
    }
    for (int t = 0; t < dp; t++) qq += rec[t] * rec[t];
    norm[i] = (float)(qq - cc);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* graph build (Sec. 2; Sec. 4.1 "Graph-based structure"; Sec. 5.1)           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int d, d_pad, m, ksub, dsub, code_stride;
  const float *x, *proj, *cent;
  const uint8_t *codes;
  const int8_t *level;
  const orc_coarse *cq;
  int deg0, deg_up, efc;
  double *xp;    /* [n][d_pad] projected raw vectors        */
  double *rec;   /* [n][d_pad] PQ reconstructions q(i)      */
  int32_t *adj0; /* [n][deg0]                               */
  int32_t *up_base, *adj_up;
  int32_t entry, max_level;
  /* per-batch scratch */
  const int32_t *batch;
  int64_t nb;
  int32_t **sel;   /* [nb][(max_level+1)*cap] new node's lists  */
  int32_t **seln;  /* [nb][max_level+1] counts                  */
  /* per-thread scratch */
  int32_t **stamp;
  int32_t *stamp_val;
  /* reverse-link commit */
  int64_t *tgt_off;  /* offsets into tgt_src for each (level,target) group */
  int32_t *tgt_lvl, *tgt_node, *tgt_src;
  int64_t ntgt;
} gb;

static int32_t *nbr_row(gb *g, int l, int32_t i) {
  if (l == 0) return g->adj0 + (int64_t)i * g->deg0;
  return g->adj_up + ((int64_t)g->up_base[i] + l - 1) * g->deg_up;
}
static int cap_of(gb *g, int l) { return l == 0 ? g->deg0 : g->deg_up; }
static int row_len(gb *g, int l, int32_t i) {
  int32_t *r = nbr_row(g, l, i);
  int c = cap_of(g, l), k = 0;
  while (k < c && r[k] >= 0) k++;
  return k;
}

/* squared distance from a raw (projected) vector to q(j) */
static double dist_raw_rec(gb *g, const double *v, int32_t j) { return sqdist(v, g->rec + (int64_t)j * g->d_pad, g->d_pad); }

/* Textbook best-first search on level l (Sec. 2), bounded by ef, from a single
 * entry.  Returns W sorted ascending in out (<= ef entries). */
static int layer_search(gb *g, const double *v, int l, int32_t ep, int ef, int tid, okey *out) {
  int32_t *stamp = g->stamp[tid];
  int32_t sv = ++g->stamp_val[tid];
  int cap = cap_of(g, l);
  oheap C = {(okey *)malloc(sizeof(okey) * (size_t)(g->n + 1)), 0, (int)g->n + 1, 0};
  oheap W = {(okey *)malloc(sizeof(okey) * (size_t)(ef + 2)), 0, ef + 2, 1};
  okey e = {dist_raw_rec(g, v, ep), ep};
  stamp[ep] = sv;
  oh_push(&C, e);
  oh_push(&W, e);
  while (C.n > 0) {
    okey c = oh_pop(&C);
    if (W.n >= ef && okey_lt(W.a[0], c)) break;
    int32_t *r = nbr_row(g, l, c.id);
    for (int j = 0; j < cap; j++) {
      int32_t nb = r[j];
      if (nb < 0) break;
      if (stamp[nb] == sv) continue;
      stamp[nb] = sv;
      okey k = {dist_raw_rec(g, v, nb), nb};
      if (W.n < ef || okey_lt(k, W.a[0])) {
        oh_push(&C, k);
        oh_push(&W, k);
        if (W.n > ef) oh_pop(&W);
      }
    }
  }
  int nw = W.n;
  for (int i = nw - 1; i >= 0; i--) out[i] = oh_pop(&W);
  free(C.a);
  free(W.a);
  return nw;
}

/* Optional record of every list update of the graph build (test
 * infrastructure, see lc_oracle.h): appended under a mutex, in execution
 * order (one thread gives the sequential order). */
static pthread_mutex_t g_trace_mu = PTHREAD_MUTEX_INITIALIZER;
static int32_t *g_trace = NULL;
static int64_t g_trace_cap = 0, g_trace_used = 0;

void orc_build_trace(int32_t *buf, int64_t cap) {
  pthread_mutex_lock(&g_trace_mu);
  g_trace = buf;
  g_trace_cap = buf ? cap : 0;
  g_trace_used = 0;
  pthread_mutex_unlock(&g_trace_mu);
}

int64_t orc_build_trace_used(void) { return g_trace_used; }

/* record [kind, level, owner, nc, nout, cand[nc], out[nout], kept[nout]] */
static void trace_put(int kind, int level, int32_t owner, const int32_t *cand, int nc, const int32_t *out,
                      const char *kept, int nout) {
  pthread_mutex_lock(&g_trace_mu);
  if (g_trace && g_trace_used >= 0) {
    int64_t need = 5 + (int64_t)nc + 2 * (int64_t)nout;
    if (g_trace_used + need > g_trace_cap) {
      g_trace_used = -1;
    } else {
      int32_t *r = g_trace + g_trace_used;
      r[0] = kind;
      r[1] = level;
      r[2] = owner;
      r[3] = nc;
      r[4] = nout;
      for (int i = 0; i < nc; i++) r[5 + i] = cand[i];
      for (int i = 0; i < nout; i++) {
        r[5 + nc + i] = out[i];
        r[5 + nc + nout + i] = kept ? kept[i] : 0;
      }
      g_trace_used += need;
    }
  }
  pthread_mutex_unlock(&g_trace_mu);
}

/* Neighbour selection (Sec. 2 "shrinking" operator): walk the candidates in
 * (distance to owner, id) order and keep one only if it is closer to the
 * owner than to every already-kept link (distances between reconstructions);
 * then fill the remaining slots with the nearest rejected candidates.  The
 * result is written sorted by (distance to owner, id). */
static int select_links(gb *g, const double *owner, const int32_t *cand, int nc, int cap,
                        int32_t *out, char *by_test) {
  okey *ks = (okey *)malloc(sizeof(okey) * (size_t)(nc > 0 ? nc : 1));
  char *kept = (char *)calloc((size_t)(nc > 0 ? nc : 1), 1);
  int32_t *kid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  for (int i = 0; i < nc; i++) {
    ks[i].id = cand[i];
    ks[i].d = dist_raw_rec(g, owner, cand[i]);
  }
  qsort(ks, (size_t)nc, sizeof(okey), okey_cmp);
  int nk = 0;
  for (int i = 0; i < nc && nk < cap; i++) {
    int good = 1;
    for (int t = 0; t < nk && good; t++) {
      double dcs = sqdist(g->rec + (int64_t)ks[i].id * g->d_pad, g->rec + (int64_t)kid[t] * g->d_pad, g->d_pad);
      if (!(ks[i].d < dcs)) good = 0;
    }
    if (good) {
      kept[i] = 1;
      kid[nk++] = ks[i].id;
    }
  }
  for (int i = 0; i < nc && nk < cap; i++)
    if (!kept[i]) {
      kept[i] = 2; /* filled: the nearest candidates the test rejected */
      nk++;
    }
  int w = 0;
  for (int i = 0; i < nc; i++)
    if (kept[i]) {
      if (by_test) by_test[w] = kept[i] == 1;
      out[w++] = ks[i].id;
    }
  for (int i = w; i < cap; i++) out[i] = -1;
  free(ks);
  free(kept);
  free(kid);
  return w;
}

/* Search phase of one new node against the graph frozen at batch start. */
static void gb_search_one(int64_t bi, int tid, void *vctx) {
  gb *g = (gb *)vctx;
  int32_t x = g->batch[bi];
  const double *v = g->xp + (int64_t)x * g->d_pad;
  int lx = g->level[x];
  int32_t cur = g->entry;
  double curd = dist_raw_rec(g, v, cur);
  /* greedy descent above the node's own level: move to the best neighbour
   * while it is strictly better (key order) */
  for (int l = g->max_level; l > lx; l--) {
    for (;;) {
      int32_t *r = nbr_row(g, l, cur);
      okey best = {curd, cur};
      for (int j = 0; j < g->deg_up && r[j] >= 0; j++) {
        okey k = {dist_raw_rec(g, v, r[j]), r[j]};
        if (okey_lt(k, best)) best = k;
      }
      if (best.id == cur) break;
      cur = best.id;
      curd = best.d;
    }
  }
  okey *W = (okey *)malloc(sizeof(okey) * (size_t)(g->efc + 2));
  int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->efc + 2));
  int top = lx < g->max_level ? lx : g->max_level;
  for (int l = top; l >= 0; l--) {
    int nw = layer_search(g, v, l, cur, g->efc, tid, W);
    for (int i = 0; i < nw; i++) ids[i] = W[i].id;
    int cap = cap_of(g, l);
    int32_t *o = g->sel[bi] + (int64_t)l * (g->deg0 > g->deg_up ? g->deg0 : g->deg_up);
    char *by_test = (char *)malloc((size_t)cap);
    g->seln[bi][l] = select_links(g, v, ids, nw, cap, o, by_test);
    trace_put(0, l, x, ids, nw, o, by_test, g->seln[bi][l]);
    free(by_test);
    cur = W[0].id;
  }
  free(W);
  free(ids);
}

/* Commit of the reverse links for one (level, target) group. */
static void gb_reverse_one(int64_t gi, int tid, void *vctx) {
  (void)tid;
  gb *g = (gb *)vctx;
  int l = g->tgt_lvl[gi];
  int32_t e = g->tgt_node[gi];
  int cap = cap_of(g, l);
  int64_t s0 = g->tgt_off[gi], s1 = g->tgt_off[gi + 1];
  int32_t *row = nbr_row(g, l, e);
  int have = row_len(g, l, e);
  int nc = have + (int)(s1 - s0);
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  for (int i = 0; i < have; i++) cand[i] = row[i];
  for (int64_t i = s0; i < s1; i++) cand[have + (i - s0)] = g->tgt_src[i];
  const double *v = g->xp + (int64_t)e * g->d_pad;
  if (nc <= cap) {
    okey *ks = (okey *)malloc(sizeof(okey) * (size_t)nc);
    for (int i = 0; i < nc; i++) {
      ks[i].id = cand[i];
      ks[i].d = dist_raw_rec(g, v, cand[i]);
    }
    qsort(ks, (size_t)nc, sizeof(okey), okey_cmp);
    for (int i = 0; i < cap; i++) row[i] = i < nc ? ks[i].id : -1;
    free(ks);
    trace_put(2, l, e, cand, nc, row, NULL, nc);
  } else {
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    char *by_test = (char *)malloc((size_t)cap);
    int w = select_links(g, v, cand, nc, cap, tmp, by_test);
    memcpy(row, tmp, sizeof(int32_t) * (size_t)cap);
    trace_put(1, l, e, cand, nc, tmp, by_test, w);
    free(by_test);
    free(tmp);
  }
  free(cand);
}

typedef struct {
  int32_t lvl, tgt, src;
} rlink;
static int rlink_cmp(const void *pa, const void *pb) {
  const rlink *a = (const rlink *)pa, *b = (const rlink *)pb;
  if (a->lvl != b->lvl) return a->lvl < b->lvl ? -1 : 1;
  if (a->tgt != b->tgt) return a->tgt < b->tgt ? -1 : 1;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  return 0;
}

static const int8_t *g_ord_level; /* qsort has no context argument */
static int ord_cmp(const void *pa, const void *pb) {
  int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
  if (g_ord_level[a] != g_ord_level[b]) return g_ord_level[a] > g_ord_level[b] ? -1 : 1;
  return a < b ? -1 : (a > b);
}
static pthread_mutex_t g_ord_mu = PTHREAD_MUTEX_INITIALIZER;

static void prep_one(int64_t i, int tid, void *vctx) {
  (void)tid;
  gb *g = (gb *)vctx;
  orc_project(g->proj, g->d_pad, g->d, g->x + i * g->d, g->xp + i * g->d_pad);
  decode(g->cent, g->codes, g->code_stride, g->m, g->ksub, g->dsub, g->cq, i, g->rec + i * g->d_pad);
}

int orc_hnsw_build(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                   int ksub, const float *cent, const uint8_t *codes, int code_stride,
                   const int8_t *level, int deg0, int deg_up, int ef_construction, int nthreads,
                   int32_t *adj0, int32_t *up_base, int32_t *adj_up, int32_t *entry,
                   int32_t *max_level, const orc_coarse *cq) {
  if (n < 1 || d_pad % m || deg0 < 1 || deg_up < 1 || ef_construction < 1) return -1;
  if (cq && cq->k > 0 && d_pad % 2) return -1;
  if (nthreads < 1) nthreads = 1;
  gb G;
  memset(&G, 0, sizeof(G));
  gb *g = &G;
  g->n = n;
  g->d = d;
  g->d_pad = d_pad;
  g->m = m;
  g->ksub = ksub;
  g->dsub = d_pad / m;
  g->code_stride = code_stride;
  g->x = x;
  g->proj = proj;
  g->cent = cent;
  g->codes = codes;
  g->level = level;
  g->cq = cq;
  g->deg0 = deg0;
  g->deg_up = deg_up;
  g->efc = ef_construction;
  g->adj0 = adj0;
  g->up_base = up_base;
  g->adj_up = adj_up;
  g->xp = (double *)malloc(sizeof(double) * (size_t)n * d_pad);
  g->rec = (double *)malloc(sizeof(double) * (size_t)n * d_pad);
  if (!g->xp || !g->rec) return -2;
  orc_parallel_for(n, nthreads, prep_one, g);

  /* storage layout of the upper rows: node i owns rows up_base[i] .. +level-1 */
  int64_t rows = 0;
  for (int64_t i = 0; i < n; i++) {
    up_base[i] = level[i] > 0 ? (int32_t)rows : -1;
    rows += level[i];
  }
  for (int64_t i = 0; i < n * deg0; i++) adj0[i] = -1;
  for (int64_t i = 0; i < rows * deg_up; i++) adj_up[i] = -1;

  /* insertion order: level descending, then id ascending (layer by layer) */
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) order[i] = (int32_t)i;
  pthread_mutex_lock(&g_ord_mu);
  g_ord_level = level;
  qsort(order, (size_t)n, sizeof(int32_t), ord_cmp);
  pthread_mutex_unlock(&g_ord_mu);
  g->entry = order[0];
  g->max_level = level[order[0]];

  g->stamp = (int32_t **)malloc(sizeof(int32_t *) * nthreads);
  g->stamp_val = (int32_t *)calloc((size_t)nthreads, sizeof(int32_t));
  for (int t = 0; t < nthreads; t++) g->stamp[t] = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  int capmax = deg0 > deg_up ? deg0 : deg_up;
  int64_t bmax = 4096;
  g->sel = (int32_t **)malloc(sizeof(int32_t *) * bmax);
  g->seln = (int32_t **)malloc(sizeof(int32_t *) * bmax);
  for (int64_t b = 0; b < bmax; b++) {
    g->sel[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->max_level + 1) * capmax);
    g->seln[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->max_level + 1));
  }
  rlink *rl = (rlink *)malloc(sizeof(rlink) * (size_t)bmax * (g->max_level + 1) * capmax);
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)bmax * (g->max_level + 1) * capmax + 1));
  int32_t *tl = (int32_t *)malloc(sizeof(int32_t) * (size_t)bmax * (g->max_level + 1) * capmax);
  int32_t *tn = (int32_t *)malloc(sizeof(int32_t) * (size_t)bmax * (g->max_level + 1) * capmax);
  int32_t *ts = (int32_t *)malloc(sizeof(int32_t) * (size_t)bmax * (g->max_level + 1) * capmax);

  /* batches (Sec. 5.1: vectors are added by batches): each batch is searched
   * against the graph as it stood at the start of the batch, then linked.
   * Batch size = clamp(inserted / 16, 1, 4096). */
  int64_t pos = 1;
  while (pos < n) {
    int64_t bs = pos / 16;
    if (bs < 1) bs = 1;
    if (bs > bmax) bs = bmax;
    if (pos + bs > n) bs = n - pos;
    g->batch = order + pos;
    g->nb = bs;
    trace_put(3, 0, (int32_t)bs, g->batch, (int)bs, NULL, NULL, 0);
    orc_parallel_for(bs, nthreads, gb_search_one, g);
    /* the new nodes' own lists */
    int64_t nr = 0;
    for (int64_t b = 0; b < bs; b++) {
      int32_t xnode = g->batch[b];
      int top = level[xnode] < g->max_level ? level[xnode] : g->max_level;
      for (int l = 0; l <= top; l++) {
        int32_t *row = nbr_row(g, l, xnode);
        int cap = cap_of(g, l);
        int32_t *s = g->sel[b] + (int64_t)l * capmax;
        for (int j = 0; j < cap; j++) row[j] = s[j];
        for (int j = 0; j < g->seln[b][l]; j++) {
          rl[nr].lvl = l;
          rl[nr].tgt = s[j];
          rl[nr].src = xnode;
          nr++;
        }
      }
    }
    /* reverse links grouped by (level, target) */
    qsort(rl, (size_t)nr, sizeof(rlink), rlink_cmp);
    int64_t ng = 0;
    for (int64_t i = 0; i < nr; i++) {
      if (i == 0 || rl[i].lvl != rl[i - 1].lvl || rl[i].tgt != rl[i - 1].tgt) {
        off[ng] = i;
        tl[ng] = rl[i].lvl;
        tn[ng] = rl[i].tgt;
        ng++;
      }
      ts[i] = rl[i].src;
    }
    off[ng] = nr;
    g->tgt_off = off;
    g->tgt_lvl = tl;
    g->tgt_node = tn;
    g->tgt_src = ts;
    g->ntgt = ng;
    orc_parallel_for(ng, nthreads, gb_reverse_one, g);
    pos += bs;
  }
  *entry = g->entry;
  *max_level = g->max_level;

  for (int64_t b = 0; b < bmax; b++) {
    free(g->sel[b]);
    free(g->seln[b]);
  }
  free(g->sel);
  free(g->seln);
  for (int t = 0; t < nthreads; t++) free(g->stamp[t]);
  free(g->stamp);
  free(g->stamp_val);
  free(rl);
  free(off);
  free(tl);
  free(tn);
  free(ts);
  free(order);
  free(g->xp);
  free(g->rec);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* least squares (Sec. 4.2, Eq. 4: beta* = Y^+ X)                             */
/* ------------------------------------------------------------------------ */
/* Symmetric eigen-decomposition by cyclic Jacobi rotations. */
static void jacobi_eig(const double *a_in, int p, double *w, double *v) {
  double *a = (double *)malloc(sizeof(double) * (size_t)p * p);
  memcpy(a, a_in, sizeof(double) * (size_t)p * p);
  for (int i = 0; i < p; i++)
    for (int j = 0; j < p; j++) v[i * p + j] = (i == j);
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0, tot = 0;
    for (int i = 0; i < p; i++)
      for (int j = 0; j < p; j++) {
        tot += a[i * p + j] * a[i * p + j];
        if (i != j) off += a[i * p + j] * a[i * p + j];
      }
    if (off <= 1e-30 * tot || off == 0) break;
    for (int r = 0; r < p; r++)
      for (int c = r + 1; c < p; c++) {
        double arc = a[r * p + c];
        if (arc == 0) continue;
        double theta = (a[c * p + c] - a[r * p + r]) / (2 * arc);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
        double cs = 1 / sqrt(t * t + 1), sn = t * cs;
        for (int k = 0; k < p; k++) {
          double akr = a[k * p + r], akc = a[k * p + c];
          a[k * p + r] = cs * akr - sn * akc;
          a[k * p + c] = sn * akr + cs * akc;
        }
        for (int k = 0; k < p; k++) {
          double ark = a[r * p + k], ack = a[c * p + k];
          a[r * p + k] = cs * ark - sn * ack;
          a[c * p + k] = sn * ark + cs * ack;
        }
        for (int k = 0; k < p; k++) {
          double vkr = v[k * p + r], vkc = v[k * p + c];
          v[k * p + r] = cs * vkr - sn * vkc;
          v[k * p + c] = sn * vkr + cs * vkc;
        }
      }
  }
  for (int i = 0; i < p; i++) w[i] = a[i * p + i];
  free(a);
}

int orc_lsq_solve(const double *a, const double *c, int p, double *beta) {
  /* Cholesky A = L L^T; accepted only if every pivot is clearly positive */
  double *L = (double *)calloc((size_t)p * p, sizeof(double));
  double amax = 0;
  for (int i = 0; i < p; i++)
    if (a[i * p + i] > amax) amax = a[i * p + i];
  int ok = amax > 0;
  for (int j = 0; j < p && ok; j++) {
    double s = a[j * p + j];
    for (int k = 0; k < j; k++) s -= L[j * p + k] * L[j * p + k];
    if (!(s > 1e-12 * amax)) {
      ok = 0;
      break;
    }
    L[j * p + j] = sqrt(s);
    for (int i = j + 1; i < p; i++) {
      double t = a[i * p + j];
      for (int k = 0; k < j; k++) t -= L[i * p + k] * L[j * p + k];
      L[i * p + j] = t / L[j * p + j];
    }
  }
  if (ok) {
    double *z = (double *)malloc(sizeof(double) * p);
    for (int i = 0; i < p; i++) {
      double t = c[i];
      for (int k = 0; k < i; k++) t -= L[i * p + k] * z[k];
      z[i] = t / L[i * p + i];
    }
    for (int i = p - 1; i >= 0; i--) {
      double t = z[i];
      for (int k = i + 1; k < p; k++) t -= L[k * p + i] * beta[k];
      beta[i] = t / L[i * p + i];
    }
    free(z);
    free(L);
    return 0;
  }
  free(L);
  /* Moore-Penrose solution through the eigen-decomposition of A = G^T G:
   * eigenvalues below 1e-12 * max (singular values of G below 1e-6 * max)
   * are treated as zero. */
  double *w = (double *)malloc(sizeof(double) * p);
  double *v = (double *)malloc(sizeof(double) * (size_t)p * p);
  jacobi_eig(a, p, w, v);
  double wmax = 0;
  for (int i = 0; i < p; i++)
    if (w[i] > wmax) wmax = w[i];
  for (int i = 0; i < p; i++) beta[i] = 0;
  for (int e = 0; e < p; e++) {
    if (!(w[e] > 1e-12 * wmax) || wmax <= 0) continue;
    double proj = 0;
    for (int i = 0; i < p; i++) proj += v[i * p + e] * c[i];
    for (int i = 0; i < p; i++) beta[i] += v[i * p + e] * proj / w[e];
  }
  free(w);
  free(v);
  return 1;
}

/* ------------------------------------------------------------------------ */
/* regression codebook (Sec. 4.3, Eq. 6-8)                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  const float *x, *proj, *cent;
  const uint8_t *codes;
  const int32_t *adj0;
  const int64_t *ids;
  int d, d_pad, m, ksub, dsub, code_stride, deg0, p;
  int t0, t1; /* coordinates of the block the Gram covers (Sec. 4.3, product codebook) */
  double *A;  /* [n][p][p] G^T G      */
  double *C;  /* [n][p]    G^T x      */
  double *XX; /* [n]       ||x||^2    */
  const orc_coarse *cq;
} gram_ctx;

/* G(x) = [q(x), q(g_1(x)), ..., q(g_k(x))] (Sec. 4.2), a -1 link being a zero column;
 * the products are taken over the coordinates [t0, t1) only, which is G^j(x) and
 * x^j of the product codebook (Sec. 4.3, Eq. 9); [0, d_pad) is the whole vector */
static void gram_one(int64_t r, int tid, void *vctx) {
  (void)tid;
  gram_ctx *g = (gram_ctx *)vctx;
  int64_t i = g->ids ? g->ids[r] : r;
  int p = g->p, dp = g->d_pad;
  double *G = (double *)malloc(sizeof(double) * (size_t)p * dp);
  double *xp = (double *)malloc(sizeof(double) * dp);
  orc_project(g->proj, dp, g->d, g->x + i * g->d, xp);
  for (int j = 0; j < p; j++) {
    int64_t src = j == 0 ? i : g->adj0[i * g->deg0 + (j - 1)];
    if (src < 0)
      for (int t = 0; t < dp; t++) G[j * dp + t] = 0;
    else
      decode(g->cent, g->codes, g->code_stride, g->m, g->ksub, g->dsub, g->cq, src, G + (int64_t)j * dp);
  }
  double *A = g->A + r * p * p, *C = g->C + r * p;
  for (int a = 0; a < p; a++) {
    for (int b = 0; b < p; b++) {
      double s = 0;
      for (int t = g->t0; t < g->t1; t++) s += G[a * dp + t] * G[b * dp + t];
      A[a * p + b] = s;
    }
    double s = 0;
    for (int t = g->t0; t < g->t1; t++) s += G[a * dp + t] * xp[t];
    C[a] = s;
  }
  double s = 0;
  for (int t = g->t0; t < g->t1; t++) s += xp[t] * xp[t];
  g->XX[r] = s;
  free(G);
  free(xp);
}

/* ||x - G beta||^2 = ||x||^2 - 2 beta^T (G^T x) + beta^T (G^T G) beta */
static double reg_loss(const double *A, const double *C, double xx, const double *beta, int p) {
  double l = xx;
  for (int a = 0; a < p; a++) {
    l -= 2 * beta[a] * C[a];
    double s = 0;
    for (int b = 0; b < p; b++) s += A[a * p + b] * beta[b];
    l += beta[a] * s;
  }
  return l;
}

typedef struct {
  gram_ctx *g;
  const double *B;
  int nb;
  int32_t *assign;
  double *loss;
} asg_ctx;

static void assign_one(int64_t r, int tid, void *vctx) {
  (void)tid;
  asg_ctx *c = (asg_ctx *)vctx;
  int p = c->g->p;
  double best = DBL_MAX;
  int32_t bi = 0;
  for (int b = 0; b < c->nb; b++) {
    double l = reg_loss(c->g->A + r * p * p, c->g->C + r * p, c->g->XX[r], c->B + (int64_t)b * p, p);
    if (l < best) {
      best = l;
      bi = b;
    }
  }
  c->assign[r] = bi;
  c->loss[r] = best;
}

static int gram_alloc(gram_ctx *g, int64_t n) {
  g->A = (double *)malloc(sizeof(double) * (size_t)n * g->p * g->p);
  g->C = (double *)malloc(sizeof(double) * (size_t)n * g->p);
  g->XX = (double *)malloc(sizeof(double) * (size_t)n);
  return g->A && g->C && g->XX ? 0 : -2;
}
static void gram_free(gram_ctx *g) {
  free(g->A);
  free(g->C);
  free(g->XX);
}

/* One codebook (Sec. 4.3): per-vector optimum, k-means on it, then EM over
 * assignment (Eq. 7) and per-cluster least squares (Eq. 8), on the Grams of
 * one block of coordinates. */
static void beta_train_block(gram_ctx *g, int64_t n_sub, int n_beta, const int64_t *init, int km_iters,
                             int em_iters, int nthreads, float *beta, double *loss_hist) {
  int p = g->p;
  orc_parallel_for(n_sub, nthreads, gram_one, g);
  /* per-vector optimum beta(x) (Eq. 2 with G(x) for N(x)) seeds a k-means */
  double *bx = (double *)malloc(sizeof(double) * (size_t)n_sub * p);
  for (int64_t r = 0; r < n_sub; r++) orc_lsq_solve(g->A + r * p * p, g->C + r * p, p, bx + r * p);
  double *B = (double *)malloc(sizeof(double) * (size_t)n_beta * p);
  int32_t *as = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_sub);
  double *ls = (double *)malloc(sizeof(double) * (size_t)n_sub);
  orc_kmeans(bx, n_sub, p, n_beta, init, km_iters, nthreads, B, as, NULL);
  double *SA = (double *)malloc(sizeof(double) * (size_t)p * p);
  double *SC = (double *)malloc(sizeof(double) * (size_t)p);
  asg_ctx ac = {g, B, n_beta, as, ls};
  for (int it = 0;; it++) {
    /* assignment step (Eq. 7) */
    orc_parallel_for(n_sub, nthreads, assign_one, &ac);
    if (loss_hist) {
      double s = 0;
      for (int64_t r = 0; r < n_sub; r++) s += ls[r];
      loss_hist[it] = s;
    }
    if (it == em_iters) break;
    /* update step (Eq. 8): per-cluster least squares; empty clusters keep beta */
    for (int b = 0; b < n_beta; b++) {
      memset(SA, 0, sizeof(double) * (size_t)p * p);
      memset(SC, 0, sizeof(double) * (size_t)p);
      int64_t cnt = 0;
      for (int64_t r = 0; r < n_sub; r++) {
        if (as[r] != b) continue;
        cnt++;
        for (int t = 0; t < p * p; t++) SA[t] += g->A[r * p * p + t];
        for (int t = 0; t < p; t++) SC[t] += g->C[r * p + t];
      }
      if (cnt > 0) orc_lsq_solve(SA, SC, p, B + (int64_t)b * p);
    }
  }
  for (int64_t t = 0; t < (int64_t)n_beta * p; t++) beta[t] = (float)B[t];
  free(bx);
  free(B);
  free(as);
  free(ls);
  free(SA);
  free(SC);
}

int orc_beta_train(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj,
                   int d_pad, int m, int ksub, const float *cent, const uint8_t *codes,
                   int code_stride, const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta,
                   const int64_t *init, int km_iters, int em_iters, int nthreads, float *beta,
                   double *loss_hist, const orc_coarse *cq) {
  if (k_reg > deg0 || n_beta > n_sub || n_sub < 1 || m_beta < 1 || m % m_beta) return -1;
  int p = k_reg + 1;
  gram_ctx g = {x, proj, cent, codes, adj0, ids, d, d_pad, m, ksub, d_pad / m, code_stride, deg0, p, 0, d_pad, 0, 0, 0, cq};
  if (gram_alloc(&g, n_sub)) return -2;
  /* product codebook (Sec. 4.3, Eq. 9): block j is the coordinates
   * [j d_pad / m_beta, (j+1) d_pad / m_beta), m / m_beta whole sub-quantizers;
   * each block trains its own codebook from the same seeds */
  for (int jb = 0; jb < m_beta; jb++) {
    g.t0 = jb * (d_pad / m_beta);
    g.t1 = g.t0 + d_pad / m_beta;
    beta_train_block(&g, n_sub, n_beta, init, km_iters, em_iters, nthreads, beta + (int64_t)jb * n_beta * p,
                     loss_hist ? loss_hist + (int64_t)jb * (em_iters + 1) : NULL);
  }
  gram_free(&g);
  return 0;
}

int orc_beta_shared(const float *x, const int64_t *ids, int64_t n_sub, int d, const float *proj,
                    int d_pad, int m, int ksub, const float *cent, const uint8_t *codes,
                    int code_stride, const int32_t *adj0, int deg0, int k_reg, double *beta,
                    const orc_coarse *cq) {
  if (k_reg > deg0 || n_sub < 1) return -1;
  int p = k_reg + 1;
  gram_ctx g = {x, proj, cent, codes, adj0, ids, d, d_pad, m, ksub, d_pad / m, code_stride, deg0, p, 0, d_pad, 0, 0, 0, cq};
  if (gram_alloc(&g, n_sub)) return -2;
  orc_parallel_for(n_sub, 1, gram_one, &g);
  double *SA = (double *)calloc((size_t)p * p, sizeof(double));
  double *SC = (double *)calloc((size_t)p, sizeof(double));
  for (int64_t r = 0; r < n_sub; r++) {
    for (int t = 0; t < p * p; t++) SA[t] += g.A[r * p * p + t];
    for (int t = 0; t < p; t++) SC[t] += g.C[r * p + t];
  }
  orc_lsq_solve(SA, SC, p, beta);
  free(SA);
  free(SC);
  gram_free(&g);
  return 0;
}

int orc_beta_assign(const float *x, int64_t n, int d, const float *proj, int d_pad, int m,
                    int ksub, const float *cent, const uint8_t *codes, int code_stride,
                    const int32_t *adj0, int deg0, int k_reg, int n_beta, int m_beta, const float *beta,
                    int nthreads, uint8_t *beta_idx, const orc_coarse *cq) {
  if (k_reg > deg0 || n_beta > 256 || m_beta < 1 || m % m_beta) return -1;
  int p = k_reg + 1;
  double *B = (double *)malloc(sizeof(double) * (size_t)m_beta * n_beta * p);
  for (int64_t t = 0; t < (int64_t)m_beta * n_beta * p; t++) B[t] = (double)beta[t];
  int64_t chunk = 65536;
  int32_t *as = (int32_t *)malloc(sizeof(int32_t) * (size_t)chunk);
  double *ls = (double *)malloc(sizeof(double) * (size_t)chunk);
  int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)chunk);
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    for (int64_t i = c0; i < c1; i++) ids[i - c0] = i;
    gram_ctx g = {x, proj, cent, codes, adj0, ids, d, d_pad, m, ksub, d_pad / m, code_stride, deg0, p, 0, d_pad, 0, 0, 0, cq};
    if (gram_alloc(&g, c1 - c0)) return -2;
    /* each block of the product codebook picks its own entry (Eq. 7 on x^j, G^j) */
    for (int jb = 0; jb < m_beta; jb++) {
      g.t0 = jb * (d_pad / m_beta);
      g.t1 = g.t0 + d_pad / m_beta;
      orc_parallel_for(c1 - c0, nthreads, gram_one, &g);
      asg_ctx ac = {&g, B + (int64_t)jb * n_beta * p, n_beta, as, ls};
      orc_parallel_for(c1 - c0, nthreads, assign_one, &ac);
      for (int64_t i = c0; i < c1; i++) beta_idx[i * m_beta + jb] = (uint8_t)as[i - c0];
    }
    gram_free(&g);
  }
  free(B);
  free(as);
  free(ls);
  free(ids);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* search (Sec. 2 walk; Sec. 4.1 two-stage search; Eq. 5 / Eq. 7 refinement)  */
/* ------------------------------------------------------------------------ */
void orc_lut(const orc_index *ix, const float *y, double *lut) {
  int dsub = ix->d_pad / ix->m;
  double *yp = (double *)malloc(sizeof(double) * ix->d_pad);
  orc_project(ix->proj, ix->d_pad, ix->d, y, yp);
  if (ix->coarse.k > 0) { /* 2-level codec: the distance is taken from y' directly */
    for (int t = 0; t < ix->d_pad; t++) lut[t] = yp[t];
    free(yp);
    return;
  }
  for (int s = 0; s < ix->m; s++)
    for (int c = 0; c < ix->ksub; c++) {
      const float *cc = ix->centroids + ((int64_t)s * ix->ksub + c) * dsub;
      double e = 0;
      for (int t = 0; t < dsub; t++) {
        double df = yp[s * dsub + t] - (double)cc[t];
        e += df * df;
      }
      lut[s * ix->ksub + c] = e;
    }
  free(yp);
}

static double adc(const orc_index *ix, const double *lut, int32_t i) {
  if (ix->coarse.k > 0) { /* ||y' - q(x_i)||^2, q = first level + residual PQ */
    double rec[4096];
    decode(ix->centroids, ix->codes, ix->code_stride, ix->m, ix->ksub, ix->d_pad / ix->m, &ix->coarse, i, rec);
    return sqdist(lut, rec, ix->d_pad);
  }
  double s = 0;
  for (int t = 0; t < ix->m; t++) s += lut[t * ix->ksub + ix->codes[(int64_t)i * ix->code_stride + t]];
  return s;
}

double orc_refined_distance(const orc_index *ix, const float *y, int32_t i) {
  int dp = ix->d_pad, dsub = dp / ix->m, p = ix->k_reg + 1;
  double *yp = (double *)malloc(sizeof(double) * dp);
  double *xr = (double *)calloc((size_t)dp, sizeof(double));
  double *q = (double *)malloc(sizeof(double) * dp);
  orc_project(ix->proj, dp, ix->d, y, yp);
  /* block jb of x~ uses its own codebook entry (Sec. 4.3, Eq. 9); one block is Eq. 5 */
  int mb = ix->m_beta, bw = dp / mb;
  for (int j = 0; j < p; j++) {
    int32_t g = j == 0 ? i : ix->adj0[(int64_t)i * ix->deg0 + (j - 1)];
    if (g < 0) continue; /* a missing link is a zero vector */
    decode(ix->centroids, ix->codes, ix->code_stride, ix->m, ix->ksub, dsub, &ix->coarse, g, q);
    for (int t = 0; t < dp; t++) {
      int jb = t / bw;
      const float *b = ix->beta + ((int64_t)jb * ix->n_beta + ix->beta_idx[(int64_t)i * mb + jb]) * p;
      xr[t] += (double)b[j] * q[t];
    }
  }
  double e = sqdist(yp, xr, dp);
  free(yp);
  free(xr);
  free(q);
  return e;
}

/* greedy descent on the upper levels: from the entry, move to the neighbour
 * with the smallest key while it is strictly smaller than the current key */
static okey greedy_upper(const orc_index *ix, const double *lut) {
  okey cur = {adc(ix, lut, ix->entry), ix->entry};
  for (int l = ix->max_level; l >= 1; l--) {
    for (;;) {
      const int32_t *r = ix->adj_up + ((int64_t)ix->up_base[cur.id] + l - 1) * ix->deg_up;
      okey best = cur;
      for (int j = 0; j < ix->deg_up; j++) {
        if (r[j] < 0) break;
        okey k = {adc(ix, lut, r[j]), r[j]};
        if (okey_lt(k, best)) best = k;
      }
      if (best.id == cur.id) break;
      cur = best;
    }
  }
  return cur;
}

/* level-0 best-first walk, textbook form with two heaps: C (candidates,
 * min-heap) and W (results, max-heap bounded by ef).  Returns |W| and writes W
 * sorted ascending; E counts expansions and D newly visited nodes (distance
 * evaluations).  max_d > 0 is the paper's budget T on the number of distance
 * computations (Sec. 3.1): the walk stops right after evaluation number max_d,
 * leaving the rest of that expansion's links unvisited. */
static int walk0(const orc_index *ix, const double *lut, okey ep, int ef, int32_t *stamp,
                 int32_t sv, okey *out, int32_t *E, int32_t *D, int32_t *trace, int32_t tcap,
                 int32_t *tn, int32_t max_d) {
  oheap C = {(okey *)malloc(sizeof(okey) * ((size_t)ix->n + 1)), 0, ix->n + 1, 0};
  oheap W = {(okey *)malloc(sizeof(okey) * (size_t)(ef + 2)), 0, ef + 2, 1};
  int32_t e = 0, dd = 0, nt = 0;
  stamp[ep.id] = sv;
  oh_push(&C, ep);
  oh_push(&W, ep);
  while (C.n > 0) {
    okey c = oh_pop(&C);
    if (W.n >= ef && okey_lt(W.a[0], c)) break;
    e++;
    if (trace && nt < tcap) trace[nt] = c.id;
    nt++;
    const int32_t *r = ix->adj0 + (int64_t)c.id * ix->deg0;
    for (int j = 0; j < ix->deg0; j++) {
      int32_t nb = r[j];
      if (nb < 0) continue;
      if (stamp[nb] == sv) continue;
      stamp[nb] = sv;
      dd++;
      okey k = {adc(ix, lut, nb), nb};
      if (W.n < ef || okey_lt(k, W.a[0])) {
        oh_push(&C, k);
        oh_push(&W, k);
        if (W.n > ef) oh_pop(&W);
      }
      if (max_d > 0 && dd >= max_d) goto done;
    }
  }
done:;
  int nw = W.n;
  for (int i = nw - 1; i >= 0; i--) out[i] = oh_pop(&W);
  free(C.a);
  free(W.a);
  *E = e;
  *D = dd;
  if (tn) *tn = nt;
  return nw;
}

typedef struct {
  const orc_index *ix;
  const float *q;
  const int32_t *ef;
  int32_t S, K, max_d;
  int32_t *out_ids, *cand_ids, *cand_n, *stats;
  double *out_d, *cand_adc;
  int32_t **stamp;
  int32_t *sv;
} srch_ctx;

static void search_one(int64_t qi, int tid, void *vctx) {
  srch_ctx *c = (srch_ctx *)vctx;
  const orc_index *ix = c->ix;
  const float *y = c->q + qi * ix->d;
  double *lut = (double *)malloc(sizeof(double) * (size_t)ix->m * ix->ksub);
  orc_lut(ix, y, lut);
  okey ep = greedy_upper(ix, lut);
  int ef = c->ef[qi] > c->S ? c->ef[qi] : c->S;
  okey *W = (okey *)malloc(sizeof(okey) * (size_t)(ef + 2));
  int32_t E, D;
  int nw = walk0(ix, lut, ep, ef, c->stamp[tid], ++c->sv[tid], W, &E, &D, NULL, 0, NULL, c->max_d);
  int ns = nw < c->S ? nw : c->S;
  if (c->cand_ids)
    for (int i = 0; i < c->S; i++) c->cand_ids[qi * c->S + i] = i < ns ? W[i].id : -1;
  if (c->cand_adc)
    for (int i = 0; i < c->S; i++) c->cand_adc[qi * c->S + i] = i < ns ? W[i].d : INFINITY;
  if (c->cand_n) c->cand_n[qi] = ns;
  if (c->stats) {
    c->stats[qi * 2] = E;
    c->stats[qi * 2 + 1] = D;
  }
  /* second stage: refined distances of the short-list, then top-K */
  okey *R = (okey *)malloc(sizeof(okey) * (size_t)(ns > 0 ? ns : 1));
  for (int i = 0; i < ns; i++) {
    R[i].id = W[i].id;
    R[i].d = orc_refined_distance(ix, y, W[i].id);
  }
  qsort(R, (size_t)ns, sizeof(okey), okey_cmp);
  for (int i = 0; i < c->K; i++) {
    if (c->out_ids) c->out_ids[qi * c->K + i] = i < ns ? R[i].id : -1;
    if (c->out_d) c->out_d[qi * c->K + i] = i < ns ? R[i].d : INFINITY;
  }
  free(R);
  free(W);
  free(lut);
}

int orc_search_capped(const orc_index *ix, const float *q, int64_t nq, const int32_t *ef, int32_t S,
                      int32_t K, int32_t max_d, int nthreads, int32_t *out_ids, double *out_d,
                      int32_t *cand_ids, double *cand_adc, int32_t *cand_n, int32_t *stats) {
  if (nq < 0 || S < 1 || K < 0 || ix->n < 1 || max_d < 0) return -1;
  if (nthreads < 1) nthreads = 1;
  srch_ctx c = {ix, q, ef, S, K, max_d, out_ids, cand_ids, cand_n, stats, out_d, cand_adc, NULL, NULL};
  c.stamp = (int32_t **)malloc(sizeof(int32_t *) * nthreads);
  c.sv = (int32_t *)calloc((size_t)nthreads, sizeof(int32_t));
  for (int t = 0; t < nthreads; t++) c.stamp[t] = (int32_t *)calloc((size_t)ix->n, sizeof(int32_t));
  orc_parallel_for(nq, nthreads, search_one, &c);
  for (int t = 0; t < nthreads; t++) free(c.stamp[t]);
  free(c.stamp);
  free(c.sv);
  return 0;
}

typedef struct {
  const orc_index *ix;
  const double *tables;
  const int32_t *ef;
  int32_t S;
  int32_t *cand_ids, *cand_n, *stats;
  double *cand_adc;
  int32_t **stamp;
  int32_t *sv;
} wt_ctx;

static void walk_tables_one(int64_t qi, int tid, void *vctx) {
  wt_ctx *c = (wt_ctx *)vctx;
  const orc_index *ix = c->ix;
  const double *lut = c->tables + qi * (int64_t)ix->m * ix->ksub;
  okey ep = greedy_upper(ix, lut);
  int ef = c->ef[qi] > c->S ? c->ef[qi] : c->S;
  okey *W = (okey *)malloc(sizeof(okey) * (size_t)(ef + 2));
  int32_t E, D;
  int nw = walk0(ix, lut, ep, ef, c->stamp[tid], ++c->sv[tid], W, &E, &D, NULL, 0, NULL, 0);
  int ns = nw < c->S ? nw : c->S;
  for (int i = 0; i < c->S; i++) {
    if (c->cand_ids) c->cand_ids[qi * c->S + i] = i < ns ? W[i].id : -1;
    if (c->cand_adc) c->cand_adc[qi * c->S + i] = i < ns ? W[i].d : INFINITY;
  }
  if (c->cand_n) c->cand_n[qi] = ns;
  if (c->stats) {
    c->stats[qi * 2] = E;
    c->stats[qi * 2 + 1] = D;
  }
  free(W);
}

int orc_walk_tables(const orc_index *ix, const double *tables, int64_t nq, const int32_t *ef, int32_t S,
                    int nthreads, int32_t *cand_ids, double *cand_adc, int32_t *cand_n, int32_t *stats) {
  if (nq < 0 || S < 1 || ix->n < 1 || ix->coarse.k > 0 || !tables) return -1;
  if (nthreads < 1) nthreads = 1;
  wt_ctx c = {ix, tables, ef, S, cand_ids, cand_n, stats, cand_adc, NULL, NULL};
  c.stamp = (int32_t **)malloc(sizeof(int32_t *) * nthreads);
  c.sv = (int32_t *)calloc((size_t)nthreads, sizeof(int32_t));
  for (int t = 0; t < nthreads; t++) c.stamp[t] = (int32_t *)calloc((size_t)ix->n, sizeof(int32_t));
  orc_parallel_for(nq, nthreads, walk_tables_one, &c);
  for (int t = 0; t < nthreads; t++) free(c.stamp[t]);
  free(c.stamp);
  free(c.sv);
  return 0;
}

int orc_search(const orc_index *ix, const float *q, int64_t nq, const int32_t *ef, int32_t S,
               int32_t K, int nthreads, int32_t *out_ids, double *out_d, int32_t *cand_ids,
               double *cand_adc, int32_t *cand_n, int32_t *stats) {
  return orc_search_capped(ix, q, nq, ef, S, K, 0, nthreads, out_ids, out_d, cand_ids, cand_adc, cand_n,
                           stats);
}

int32_t orc_walk_trace(const orc_index *ix, const float *y, int32_t ef_eff, int32_t *trace,
                       int32_t cap) {
  double *lut = (double *)malloc(sizeof(double) * (size_t)ix->m * ix->ksub);
  orc_lut(ix, y, lut);
  okey ep = greedy_upper(ix, lut);
  int32_t *stamp = (int32_t *)calloc((size_t)ix->n, sizeof(int32_t));
  okey *W = (okey *)malloc(sizeof(okey) * (size_t)(ef_eff + 2));
  int32_t E, D, nt;
  walk0(ix, lut, ep, ef_eff, stamp, 1, W, &E, &D, trace, cap, &nt, 0);
  free(stamp);
  free(W);
  free(lut);
  return nt < cap ? nt : cap;
}
