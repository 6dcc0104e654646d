"""Pins of the reference oracle against closed forms, brute force, library
routines and invariants (CPU only).

Each test names the passage of the paper it pins.  Nothing here calls the GPU
library: the oracle must be trusted before it is used to judge the kernels.
"""
import itertools

import numpy as np
import pytest

import datagen
import oracle


# ---------------------------------------------------------------------------
# helpers (plain numpy, independent of the oracle's C code)
# ---------------------------------------------------------------------------
def decode_all(ix) -> np.ndarray:
    dsub = ix.d_pad // ix.m
    rec = np.empty((ix.n, ix.d_pad), np.float64)
    for s in range(ix.m):
        rec[:, s * dsub:(s + 1) * dsub] = ix.centroids[s][ix.codes[:, s]]
    return rec


def proj_np(ix, y):
    y = np.asarray(y, np.float64)
    return y if ix.proj is None else ix.proj.astype(np.float64) @ y


def adc_seq(lut, codes_row, m):
    s = 0.0
    for t in range(m):  # same order as the sequential sum in the oracle
        s += lut[t, codes_row[t]]
    return s


def make_index(n, d, m, ksub, centroids, codes, adj0, beta, beta_idx, k_reg, level=None, up_base=None,
               adj_up=None, entry=0, max_level=0, deg_up=32, proj=None, d_pad=None):
    level = np.zeros(n, np.int8) if level is None else level
    up_base = np.full(n, -1, np.int32) if up_base is None else up_base
    adj_up = np.zeros((0, deg_up), np.int32) if adj_up is None else adj_up
    return oracle.Index(n=n, d=d, d_pad=d_pad or d, m=m, deg0=adj0.shape[1], deg_up=deg_up, k_reg=k_reg,
                        n_beta=beta.shape[0], entry=entry, max_level=max_level, proj=proj,
                        centroids=np.ascontiguousarray(centroids, np.float32),
                        codes=np.ascontiguousarray(codes, np.uint8), adj0=np.ascontiguousarray(adj0, np.int32),
                        level=level, up_base=up_base, adj_up=adj_up, beta=np.ascontiguousarray(beta, np.float32),
                        beta_idx=np.ascontiguousarray(beta_idx, np.uint8), ksub=ksub)


# ---------------------------------------------------------------------------
# k-means and PQ (Sec. 3.3; Sec. 4.1 "Vector approximation")
# ---------------------------------------------------------------------------
def test_kmeans_hand_example():
    # 1-d points {0, 1, 10, 11}, seeds at 0 and 1: the fixed point is {0.5, 10.5}, SSE 1
    x = np.array([[0.0], [1.0], [10.0], [11.0]])
    cent, assign, hist = oracle.kmeans(x, 2, np.array([0, 1]), 5)
    np.testing.assert_allclose(cent[:, 0], [0.5, 10.5])
    assert assign.tolist() == [0, 0, 1, 1]
    assert hist[-1] == pytest.approx(1.0)
    # first assignment: 0 | 1, 10, 11 -> SSE 0 + 0 + 81 + 100
    assert hist[0] == pytest.approx(181.0)


def test_kmeans_empty_cluster_reseeds_largest_error():
    # both seeds at 0: cluster 1 starts empty and is re-seeded with the worst point (10)
    x = np.array([[0.0], [0.0], [4.0], [10.0]])
    cent, assign, hist = oracle.kmeans(x, 2, np.array([0, 1]), 3)
    np.testing.assert_allclose(sorted(cent[:, 0]), [4.0 / 3.0, 10.0])
    assert np.all(np.diff(hist) <= 1e-12)


def test_kmeans_monotone_and_final_argmin():
    rs = np.random.default_rng(0)
    x = rs.standard_normal((500, 3))
    cent, assign, hist = oracle.kmeans(x, 16, rs.permutation(500)[:16], 12, nthreads=4)
    assert np.all(np.diff(hist) <= 1e-9 * hist[0])
    d = ((x[:, None, :] - cent[None]) ** 2).sum(-1)
    np.testing.assert_array_equal(assign, d.argmin(1))
    assert hist[-1] == pytest.approx(d.min(1).sum(), rel=1e-12)


def test_pq_encode_is_best_code_exhaustive():
    # m=2, 4 centroids each: the chosen code has the smallest reconstruction
    # error among all 16 codes
    rs = np.random.default_rng(1)
    train = rs.standard_normal((64, 6)).astype(np.float32)
    init = np.stack([rs.permutation(64)[:4] for _ in range(2)])
    cent, hist = oracle.pq_train(train, None, 6, 2, init, 6, ksub=4)
    assert np.all(np.diff(hist, axis=1) <= 1e-9)
    x = rs.standard_normal((40, 6)).astype(np.float32)
    codes = oracle.pq_encode(x, None, 6, cent)
    for i in range(40):
        errs = {}
        for a, b in itertools.product(range(4), range(4)):
            rec = np.concatenate([cent[0][a], cent[1][b]]).astype(np.float64)
            errs[(a, b)] = ((rec - x[i]) ** 2).sum()
        best = min(errs.values())
        assert errs[(codes[i, 0], codes[i, 1])] == pytest.approx(best, rel=1e-12, abs=1e-15)


def test_levels_formula_and_ratio():
    u = np.array([1.0, 0.5, 1e-3, 1e-30, 0.02])
    lv, rows = oracle.levels(u, 30, 16)
    # floor(-ln U / ln 30): 0, 0, 2.03 -> 2, 20.3 -> capped 16, 1.15 -> 1
    assert lv.tolist() == [0, 0, 2, 16, 1]
    assert rows == 19
    big = 1.0 - np.random.default_rng(2).random(300_000)
    lv, _ = oracle.levels(big, 30, 16)
    frac = (lv >= 1).mean()  # geometric layer sizes, ratio 30 (Sec. 4.1)
    assert abs(frac - 1 / 30) < 5 * np.sqrt((1 / 30) * (29 / 30) / big.size)


# ---------------------------------------------------------------------------
# ADC (Sec. 4.1: asymmetric distances through per-query tables)
# ---------------------------------------------------------------------------
def test_adc_equals_reconstruction_distance(tiny_build):
    w, ix, db, q = tiny_build
    rec = decode_all(ix)
    for y in q[:6]:
        lut = ix.lut(y)
        adc = lut[np.arange(ix.m)[None, :], ix.codes[:, :ix.m]].sum(1)
        direct = ((proj_np(ix, y)[None, :] - rec) ** 2).sum(1)
        np.testing.assert_allclose(adc, direct, rtol=1e-12, atol=1e-15)


def test_projection_is_an_isometry_and_adc_holds():
    w = datagen.small(name="proj", n=600, d=20, m=6, d_pad=24, n_train=1024, nq=4, n_beta=8, n_beta_train=600)
    P = datagen.projection(w)
    assert P.shape == (24, 20)
    rs = np.random.default_rng(3)
    a, b = rs.standard_normal(20).astype(np.float32), rs.standard_normal(20).astype(np.float32)
    pa, pb = oracle.project(P, a, 24), oracle.project(P, b, 24)
    assert ((pa - pb) ** 2).sum() == pytest.approx(((a.astype(np.float64) - b) ** 2).sum(), rel=1e-6)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    rec = decode_all(ix)
    lut = ix.lut(q[0])
    adc = lut[np.arange(ix.m)[None, :], ix.codes[:, :ix.m]].sum(1)
    np.testing.assert_allclose(adc, ((oracle.project(P, q[0], 24)[None] - rec) ** 2).sum(1), rtol=1e-12)


# ---------------------------------------------------------------------------
# graph (Sec. 2; Sec. 4.1 "Graph-based structure"; Sec. 4.2 link order)
# ---------------------------------------------------------------------------
def _check_graph(ix, db):
    rec = decode_all(ix)
    xp = np.stack([proj_np(ix, v) for v in db]) if ix.proj is not None else db.astype(np.float64)
    n = ix.n
    for i in range(n):
        row = ix.adj0[i]
        k = int((row >= 0).sum())
        assert np.all(row[:k] >= 0) and np.all(row[k:] == -1), "padding must be trailing"
        r = row[:k]
        assert i not in r and len(set(r.tolist())) == k
        dist = ((xp[i][None] - rec[r]) ** 2).sum(1)
        assert np.all(np.diff(dist) >= -1e-12), "level-0 lists sorted by increasing distance"
    lmax = int(ix.level.max())
    assert ix.max_level == lmax
    assert ix.entry == int(np.flatnonzero(ix.level == lmax)[0])
    for i in range(n):
        if ix.level[i] == 0:
            assert ix.up_base[i] == -1
            continue
        for l in range(1, ix.level[i] + 1):
            row = ix.adj_up[ix.up_base[i] + l - 1]
            r = row[row >= 0]
            assert i not in r and len(set(r.tolist())) == len(r)
            assert np.all(ix.level[r] >= l), "upper links stay within their level"
    # level-0 reachability from the entry point
    seen = np.zeros(n, bool)
    stack = [ix.entry]
    seen[ix.entry] = True
    while stack:
        c = stack.pop()
        for nb in ix.adj0[c]:
            if nb >= 0 and not seen[nb]:
                seen[nb] = True
                stack.append(nb)
    return seen.mean()


def test_graph_invariants_tiny(tiny_build):
    w, ix, db, q = tiny_build
    assert _check_graph(ix, db) == 1.0
    assert (ix.adj0 >= 0).sum(1).min() == w.deg0  # lists are filled to the degree


def test_graph_invariants_c1(c1_build, capsys):
    # Re-shrinking a full reverse list can drop a node's last incoming link, so
    # a few nodes may become unreachable; that is a property of the graph, not
    # an error, and it is reported rather than required to be zero.
    w, ix, db, q = c1_build
    reach = _check_graph(ix, db)
    print(f"level-0 reachability from the entry: {reach:.4f}")
    assert reach >= 0.995


def test_small_graph_is_complete_and_walk_exact():
    # N <= deg0 + 1 with one node per batch: every level-0 list holds all other nodes
    w = datagen.small(name="complete", n=30, nq=8, ef=4, shortlist=4, topk=4, n_beta=4, n_beta_train=30)
    ix, db, q = oracle.build_workload(w, nthreads=2)
    for i in range(ix.n):
        assert sorted(ix.adj0[i][ix.adj0[i] >= 0].tolist()) == [j for j in range(ix.n) if j != i]
    r = ix.search(q, 4, 4, 4)
    for qi, y in enumerate(q):
        lut = ix.lut(y)
        keys = sorted((adc_seq(lut, ix.codes[i], ix.m), i) for i in range(ix.n))
        assert r["cand_ids"][qi].tolist() == [k[1] for k in keys[:4]]


# ---------------------------------------------------------------------------
# walk (Sec. 2: greedy descent, then best-first on the base layer)
# ---------------------------------------------------------------------------
def walk_sorted_pool(ix, lut, ef, T=0):
    """The same walk written as one sorted pool with 'expanded' flags: pick the
    first unexpanded entry, evaluate its unvisited links, keep the best ef;
    with T > 0 stop right after the T-th evaluation (Sec. 3.1)."""
    def key(i):
        return (adc_seq(lut, ix.codes[i], ix.m), int(i))

    cur = key(ix.entry)
    for l in range(ix.max_level, 0, -1):
        while True:
            row = ix.adj_up[ix.up_base[cur[1]] + l - 1]
            cands = [key(j) for j in row if j >= 0]
            best = min(cands + [cur])
            if best == cur:
                break
            cur = best
    pool = [[cur, False]]
    visited = {cur[1]}
    E = D = 0
    trace = []
    stop = False
    while not stop:
        idx = next((t for t, e in enumerate(pool) if not e[1]), None)
        if idx is None:
            break
        pool[idx][1] = True
        E += 1
        c = pool[idx][0][1]
        trace.append(c)
        for nb in ix.adj0[c]:
            if nb < 0 or nb in visited:
                continue
            visited.add(int(nb))
            D += 1
            pool.append([key(nb), False])
            if T and D >= T:
                stop = True
                break
        pool.sort(key=lambda e: e[0])
        pool = pool[:ef]
    return [e[0][1] for e in pool], E, D, trace


def test_walk_matches_sorted_pool_form(tiny_build):
    w, ix, db, q = tiny_build
    for ef in (1, 5, w.ef, 40):
        S = min(ef, 16)
        r = ix.search(q, ef, S, 3)
        for qi, y in enumerate(q):
            ids, E, D, trace = walk_sorted_pool(ix, ix.lut(y), max(ef, S))
            assert r["stats"][qi].tolist() == [E, D]
            assert r["cand_ids"][qi][: r["cand_n"][qi]].tolist() == ids[:S]
            if ef == w.ef:
                assert ix.walk_trace(y, max(ef, S)).tolist() == trace


def test_walk_budget_matches_sorted_pool_form(tiny_build):
    # the budget T on distance evaluations (Sec. 3.1), from the sorted-pool form
    w, ix, db, q = tiny_build
    free = ix.search(q, 40, 16, 3)
    for T in (1, 7, 32, 33, 100, 250):
        r = ix.search(q, 40, 16, 3, max_evals=T)
        for qi, y in enumerate(q):
            ids, E, D, _ = walk_sorted_pool(ix, ix.lut(y), 40, T=T)
            assert r["stats"][qi].tolist() == [E, D]
            assert D == min(T, free["stats"][qi][1])
            assert r["cand_ids"][qi][: r["cand_n"][qi]].tolist() == ids[:16]
    # a budget at or above every query's unbounded D changes nothing
    big = ix.search(q, 40, 16, 3, max_evals=int(free["stats"][:, 1].max()))
    for k in ("ids", "d", "cand_ids", "stats"):
        assert np.array_equal(big[k], free[k]), k


def test_walk_with_ef_at_least_n_is_exhaustive(tiny_build):
    w, ix, db, q = tiny_build
    n = ix.n
    r = ix.search(q[:3], n, n, 5, nthreads=3)
    for qi in range(3):
        lut = ix.lut(q[qi])
        adc = lut[np.arange(ix.m)[None, :], ix.codes[:, :ix.m]].sum(1)
        order = np.lexsort((np.arange(n), adc))
        assert r["cand_n"][qi] == n
        assert r["stats"][qi][1] == n - 1  # D = |visited| - 1 on a connected graph
        assert set(r["cand_ids"][qi].tolist()) == set(range(n))
        np.testing.assert_allclose(r["cand_adc"][qi], adc[r["cand_ids"][qi]], rtol=1e-12)
        assert np.all(np.diff(r["cand_adc"][qi]) >= 0)
        # equal to brute force up to ties closer than rounding
        np.testing.assert_allclose(adc[order], r["cand_adc"][qi], rtol=1e-12)


def test_walk_on_given_tables(tiny_build):
    # the first stage on caller-given tables (used to hold the fp16 walks to the paper's walk on their own
    # table values): (i) the queries' own tables give the search's first stage; (ii) tables scaled by a power
    # of two give the same walk with keys scaled exactly; (iii) on a Hamming table (entry 0 where the code
    # equals a target node's, else 1) the exhaustive walk's short-list is the brute-force order of
    # (Hamming distance to the target's code, id)
    w, ix, db, q = tiny_build
    n, m = ix.n, ix.m
    tabs = np.stack([ix.lut(y) for y in q[:6]]).reshape(6, m, 256)
    r = ix.search(q[:6], w.ef, w.shortlist, 5, nthreads=3)
    t = ix.walk_tables(tabs, w.ef, w.shortlist, nthreads=3)
    for k in ("cand_ids", "cand_adc", "cand_n", "stats"):
        assert np.array_equal(t[k], r[k]), k
    t4 = ix.walk_tables(tabs * 4.0, w.ef, w.shortlist, nthreads=3)
    assert np.array_equal(t4["cand_ids"], t["cand_ids"]) and np.array_equal(t4["stats"], t["stats"])
    assert np.array_equal(t4["cand_adc"], t["cand_adc"] * 4.0)
    codes = np.asarray(ix.codes)[:, :m]
    rng = np.random.default_rng(3)
    targets = rng.choice(n, 4, replace=False)
    ham = np.ones((4, m, 256))
    for j, tg in enumerate(targets):
        ham[j, np.arange(m), codes[tg]] = 0.0
    th = ix.walk_tables(ham, n, n, nthreads=2)
    for j, tg in enumerate(targets):
        hd = (codes != codes[tg][None, :]).sum(1)
        order = np.lexsort((np.arange(n), hd))
        assert th["cand_n"][j] == n and th["stats"][j][1] == n - 1
        assert np.array_equal(th["cand_ids"][j], order)
        assert np.array_equal(th["cand_adc"][j], hd[order].astype(np.float64))


def test_search_outputs_consistent(tiny_build):
    w, ix, db, q = tiny_build
    r = ix.search(q, w.ef, w.shortlist, w.shortlist + 3)
    for qi, y in enumerate(q):
        n = r["cand_n"][qi]
        cands = r["cand_ids"][qi][:n]
        ckeys = list(zip(r["cand_adc"][qi][:n].tolist(), cands.tolist()))
        assert ckeys == sorted(ckeys) and len(set(cands.tolist())) == n  # (distance, id) order, no duplicates
        top = r["ids"][qi][:n]
        assert sorted(top.tolist()) == sorted(cands.tolist())
        assert np.all(r["ids"][qi][n:] == -1) and np.all(np.isinf(r["d"][qi][n:]))
        for t in range(n):
            assert r["d"][qi][t] == ix.refined_distance(y, top[t])
        keys = [(r["d"][qi][t], top[t]) for t in range(n)]
        assert keys == sorted(keys)


def test_single_node_and_empty_batch():
    rs = np.random.default_rng(4)
    cent = rs.standard_normal((2, 256, 3))
    ix = make_index(1, 6, 2, 256, cent, np.array([[5, 7]]), np.full((1, 4), -1), np.array([[1.0, 0, 0]]),
                    np.zeros(1), 2)
    q = rs.standard_normal((2, 6)).astype(np.float32)
    r = ix.search(q, 8, 4, 3)
    assert r["cand_n"].tolist() == [1, 1]
    assert r["stats"].tolist() == [[1, 0], [1, 0]]
    assert r["ids"][:, 0].tolist() == [0, 0] and np.all(r["ids"][:, 1:] == -1)
    r0 = ix.search(np.zeros((0, 6), np.float32), 8, 4, 3)
    assert r0["ids"].shape == (0, 3)


# ---------------------------------------------------------------------------
# exact kNN special case (lossless codes, beta = e0, ef >= N)
# ---------------------------------------------------------------------------
def test_lossless_special_case_returns_exact_knn():
    rs = np.random.default_rng(5)
    n, d, m = 256, 8, 2
    db = rs.standard_normal((n, d)).astype(np.float32)
    init = np.stack([rs.permutation(n) for _ in range(m)])
    cent, _ = oracle.pq_train(db, None, d, m, init, 3)
    codes = oracle.pq_encode(db, None, d, cent)
    idx = oracle.Index(n=n, d=d, d_pad=d, m=m, deg0=32, deg_up=32, k_reg=4, n_beta=1, entry=0, max_level=0,
                       proj=None, centroids=cent, codes=codes, adj0=None, level=None, up_base=None, adj_up=None,
                       beta=np.array([[1, 0, 0, 0, 0]], np.float32), beta_idx=np.zeros(n, np.uint8))
    assert np.all(decode_all(idx) == db)  # every point is its own centroid: zero quantisation error
    lv, _ = oracle.levels(1.0 - rs.random(n))
    adj0, up_base, adj_up, entry, maxl = oracle.hnsw_build(db, None, d, cent, codes, lv, 32, 32, 64)
    idx.adj0, idx.level, idx.up_base, idx.adj_up, idx.entry, idx.max_level = adj0, lv, up_base, adj_up, entry, maxl
    q = rs.standard_normal((10, d)).astype(np.float32)
    r = idx.search(q, n, n, 10)
    dd = ((q[:, None, :].astype(np.float64) - db[None]) ** 2).sum(-1)
    for qi in range(10):
        order = np.lexsort((np.arange(n), dd[qi]))[:10]
        assert r["ids"][qi].tolist() == order.tolist()
        np.testing.assert_allclose(r["d"][qi], dd[qi][order], rtol=1e-12)


# ---------------------------------------------------------------------------
# refinement (Sec. 4.2 Eq. 5; Sec. 4.3 Eq. 7)
# ---------------------------------------------------------------------------
def _with_beta(ix, beta, beta_idx):
    import dataclasses
    return dataclasses.replace(ix, beta=np.ascontiguousarray(beta, np.float32),
                               beta_idx=np.ascontiguousarray(beta_idx, np.uint8), n_beta=beta.shape[0])


def test_refine_with_e0_is_the_adc_distance(tiny_build):
    w, ix, db, q = tiny_build
    e0 = np.zeros((1, w.k_reg + 1))
    e0[0, 0] = 1
    ix0 = _with_beta(ix, e0, np.zeros(ix.n))
    for y in q[:4]:
        lut = ix0.lut(y)
        for i in range(0, ix.n, 97):
            assert ix0.refined_distance(y, i) == pytest.approx(adc_seq(lut, ix.codes[i], ix.m), rel=1e-12)


def test_refine_random_beta_bruteforce(tiny_build):
    w, ix, db, q = tiny_build
    rs = np.random.default_rng(6)
    B = rs.standard_normal((5, w.k_reg + 1))
    bi = rs.integers(0, 5, ix.n)
    ixr = _with_beta(ix, B, bi)
    rec = decode_all(ix)
    Bf = B.astype(np.float32).astype(np.float64)
    for y in q[:3]:
        yp = proj_np(ix, y)
        for i in range(0, ix.n, 131):
            xt = Bf[bi[i], 0] * rec[i]
            for j in range(1, w.k_reg + 1):
                g = ix.adj0[i, j - 1]
                if g >= 0:
                    xt = xt + Bf[bi[i], j] * rec[g]
            assert ixr.refined_distance(y, i) == pytest.approx(((yp - xt) ** 2).sum(), rel=1e-12)


# ---------------------------------------------------------------------------
# least squares and the regression codebook (Sec. 4.2 Eq. 3-4; Sec. 4.3 Eq. 6-8)
# ---------------------------------------------------------------------------
def test_lsq_matches_numpy():
    rs = np.random.default_rng(7)
    G = rs.standard_normal((24, 5))
    x = rs.standard_normal(24)
    beta, rc = oracle.lsq_solve(G.T @ G, G.T @ x)
    assert rc == 0
    ref = np.linalg.lstsq(G, x, rcond=None)[0]
    np.testing.assert_allclose(beta, ref, rtol=1e-10)
    # rank-deficient: a duplicated column and a zero column (a missing link)
    G2 = np.concatenate([G, G[:, :1], np.zeros((24, 1))], 1)
    beta2, rc2 = oracle.lsq_solve(G2.T @ G2, G2.T @ x)
    assert rc2 == 1
    np.testing.assert_allclose(beta2, np.linalg.pinv(G2, rcond=1e-6) @ x, rtol=1e-8, atol=1e-10)


def _stack_Y(ix, db, ids, k_reg):
    rec = decode_all(ix)
    rows, xs = [], []
    for i in ids:
        cols = [rec[i]] + [rec[g] if g >= 0 else np.zeros(ix.d_pad) for g in ix.adj0[i, :k_reg]]
        rows.append(np.stack(cols, 1))
        xs.append(proj_np(ix, db[i]))
    return np.concatenate(rows, 0), np.concatenate(xs, 0)


def test_shared_beta_closed_form(tiny_build):
    w, ix, db, q = tiny_build
    ids = np.arange(0, ix.n, 3)
    beta = oracle.beta_shared(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg)
    Y, X = _stack_Y(ix, db, ids, w.k_reg)
    ref = np.linalg.lstsq(Y, X, rcond=None)[0]  # beta* = Y^+ X (Eq. 4)
    np.testing.assert_allclose(beta, ref, rtol=1e-9, atol=1e-12)
    e0 = np.zeros_like(beta)
    e0[0] = 1
    assert ((X - Y @ beta) ** 2).sum() <= ((X - Y @ e0) ** 2).sum()  # L(beta*) <= L(e0)


def test_per_cluster_lsq_is_the_em_update(tiny_build):
    # For one cluster, Eq. 8 is Eq. 4 restricted to the members
    w, ix, db, q = tiny_build
    members = np.flatnonzero(ix.beta_idx == np.bincount(ix.beta_idx).argmax())[:200]
    beta = oracle.beta_shared(db, members, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg)
    Y, X = _stack_Y(ix, db, members, w.k_reg)
    np.testing.assert_allclose(beta, np.linalg.lstsq(Y, X, rcond=None)[0], rtol=1e-9, atol=1e-12)


def test_em_loss_never_increases(tiny_build):
    w, ix, db, q = tiny_build
    ids = datagen.beta_train_ids(w)
    init = datagen.beta_init_ids(w, ids.size)
    beta, hist = oracle.beta_train(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg,
                                   w.n_beta, init, w.beta_kmeans_iters, 6, nthreads=4)
    assert np.all(np.diff(hist) <= 1e-9 * hist[0])
    # and the trained codebook beats the plain code q(x) (beta = e0) on the training set
    Y, X = _stack_Y(ix, db, ids[:300], w.k_reg)
    e0 = np.zeros(w.k_reg + 1)
    e0[0] = 1
    assert hist[-1] / ids.size < ((X - Y @ e0) ** 2).sum() / 300 * 1.5


def test_beta_assignment_is_bruteforce_argmin(tiny_build):
    w, ix, db, q = tiny_build
    rec = decode_all(ix)
    Bf = ix.beta.astype(np.float64)
    for i in range(0, ix.n, 37):
        G = np.stack([rec[i]] + [rec[g] if g >= 0 else np.zeros(ix.d_pad) for g in ix.adj0[i, :w.k_reg]], 1)
        losses = (((proj_np(ix, db[i])[:, None] - G @ Bf.T)) ** 2).sum(0)
        assert losses[ix.beta_idx[i]] <= losses.min() * (1 + 1e-10) + 1e-15


def test_beta_first_weight_soft_check(tiny_build, capsys):
    # Sec. 4.2 reports the q(x) weight of the shared beta between about 0.5
    # (coarse codes) and 0.9; reported, not enforced.
    w, ix, db, q = tiny_build
    beta = oracle.beta_shared(db, np.arange(ix.n), ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg)
    assert np.all(np.isfinite(beta))
    print(f"shared beta_0 = {beta[0]:.3f}")


# ---------------------------------------------------------------------------
# product regression codebook (Sec. 4.3, Eq. 9): one codebook per block of
# d_pad / m_beta coordinates, one byte per block and vector
# ---------------------------------------------------------------------------
def _block(ix, m_beta, jb):
    bw = ix.d_pad // m_beta
    return slice(jb * bw, (jb + 1) * bw)


def _G(ix, rec, i, k_reg):
    return np.stack([rec[i]] + [rec[g] if g >= 0 else np.zeros(ix.d_pad) for g in ix.adj0[i, :k_reg]], 1)


def test_product_refine_bruteforce(tiny_build):
    # x~ = [beta^1 G^1(x), ..., beta^M G^M(x)] with each block's own entry
    import dataclasses
    w, ix, db, q = tiny_build
    rs = np.random.default_rng(11)
    for mb in (2, 4):
        B = rs.standard_normal((mb, 5, w.k_reg + 1)).astype(np.float32)
        bi = rs.integers(0, 5, (ix.n, mb)).astype(np.uint8)
        ixp = dataclasses.replace(ix, beta=B, beta_idx=bi, n_beta=5, m_beta=mb)
        rec = decode_all(ix)
        for y in q[:3]:
            yp = proj_np(ix, y)
            for i in range(0, ix.n, 113):
                G = _G(ix, rec, i, w.k_reg)
                xt = np.concatenate([G[_block(ix, mb, jb)] @ B[jb, bi[i, jb]].astype(np.float64) for jb in range(mb)])
                assert ixp.refined_distance(y, i) == pytest.approx(((yp - xt) ** 2).sum(), rel=1e-12)


def test_product_codebook_of_one_entry_is_blockwise_least_squares(tiny_build):
    # With one entry per block, EM ends on Eq. 4 restricted to each block's
    # coordinates: beta^j = argmin sum_x ||x^j - G^j(x) beta||^2 (numpy lstsq)
    w, ix, db, q = tiny_build
    ids = np.arange(0, ix.n, 5)
    rec = decode_all(ix)
    for mb in (2, 4):
        beta, hist = oracle.beta_train(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg, 1,
                                       np.zeros(1, np.int64), 2, 2, nthreads=2, m_beta=mb)
        assert beta.shape == (mb, 1, w.k_reg + 1) and hist.shape == (mb, 3)
        for jb in range(mb):
            bl = _block(ix, mb, jb)
            Y = np.concatenate([_G(ix, rec, i, w.k_reg)[bl] for i in ids], 0)
            X = np.concatenate([proj_np(ix, db[i])[bl] for i in ids], 0)
            ref = np.linalg.lstsq(Y, X, rcond=None)[0]
            np.testing.assert_allclose(beta[jb, 0], ref, rtol=2e-6, atol=1e-6)  # stored as float32
            assert hist[jb, -1] == pytest.approx(((X - Y @ ref) ** 2).sum(), rel=1e-9)


def test_product_loss_at_most_single_codebook_loss(tiny_build):
    # A block-diagonal estimator contains the single one (same beta in every
    # block), so with one entry the product's training loss cannot be larger
    w, ix, db, q = tiny_build
    ids = np.arange(0, ix.n, 3)
    args = (db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg, 1, np.zeros(1, np.int64), 2, 2)
    _, h1 = oracle.beta_train(*args, nthreads=2)
    _, h4 = oracle.beta_train(*args, nthreads=2, m_beta=4)
    assert h4[:, -1].sum() <= h1[-1] * (1 + 1e-12)
    assert h4[:, -1].sum() < h1[-1]  # and strictly better on this data


def test_product_em_loss_never_increases(tiny_build):
    w, ix, db, q = tiny_build
    ids = datagen.beta_train_ids(w)
    init = datagen.beta_init_ids(w, ids.size)
    beta, hist = oracle.beta_train(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg,
                                   w.n_beta, init, w.beta_kmeans_iters, 5, nthreads=4, m_beta=2)
    assert beta.shape == (2, w.n_beta, w.k_reg + 1)
    assert np.all(np.diff(hist, axis=1) <= 1e-9 * hist[:, :1])


def test_product_assignment_is_blockwise_bruteforce_argmin(tiny_build):
    w, ix, db, q = tiny_build
    rs = np.random.default_rng(12)
    mb = 2
    B = rs.standard_normal((mb, 7, w.k_reg + 1)).astype(np.float32)
    B[:, :, 0] += 1.0  # keep the entries near q(x) so that the argmins differ between blocks
    bidx = oracle.beta_assign(db, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg, B, nthreads=2)
    assert bidx.shape == (ix.n, mb)
    rec = decode_all(ix)
    differ = 0
    for i in range(0, ix.n, 29):
        G = _G(ix, rec, i, w.k_reg)
        x = proj_np(ix, db[i])
        for jb in range(mb):
            bl = _block(ix, mb, jb)
            losses = ((x[bl][:, None] - G[bl] @ B[jb].astype(np.float64).T) ** 2).sum(0)
            assert losses[bidx[i, jb]] <= losses.min() * (1 + 1e-10) + 1e-15
        differ += int(bidx[i, 0] != bidx[i, 1])
    assert differ > 0


def test_product_search_uses_blockwise_refinement(tiny_build):
    # the search's returned distances are the product refined distances
    w, ix, db, q = tiny_build
    ids = datagen.beta_train_ids(w)
    init = datagen.beta_init_ids(w, ids.size)
    beta, _ = oracle.beta_train(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg,
                                w.n_beta, init, w.beta_kmeans_iters, 3, nthreads=4, m_beta=4)
    bidx = oracle.beta_assign(db, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, w.k_reg, beta, nthreads=4)
    import dataclasses
    ixp = dataclasses.replace(ix, beta=beta, beta_idx=bidx, m_beta=4)
    r = ixp.search(q[:6], w.ef, w.shortlist, w.topk)
    for qi in range(6):
        cand = r["cand_ids"][qi, :r["cand_n"][qi]]
        dd = np.array([ixp.refined_distance(q[qi], int(i)) for i in cand])
        order = np.lexsort((cand, dd))[:w.topk]
        assert r["ids"][qi].tolist() == cand[order].tolist()
        np.testing.assert_array_equal(r["d"][qi], dd[order])


# ---------------------------------------------------------------------------
# frozen outputs (tests/golden/tiny_search.json, written by make_golden.py)
# ---------------------------------------------------------------------------
def test_golden_fixture_reproduced():
    import json
    import os
    from tests.golden import make_golden
    g = json.load(open(os.path.join(os.path.dirname(make_golden.__file__), "tiny_search.json")))
    ix, db, q = make_golden.build()
    w = make_golden.W
    r = ix.search(q, w.ef, w.shortlist, w.topk, nthreads=3)
    assert (ix.entry, ix.max_level) == (g["entry"], g["max_level"])
    assert ix.codes[:4].tolist() == g["codes_head"] and ix.beta_idx[:32].tolist() == g["beta_idx_head"]
    for k in ("ids", "cand_ids", "cand_n", "stats"):
        assert r[k].tolist() == g[k], k
    assert [[float(x).hex() for x in row] for row in r["d"]] == g["d"]
