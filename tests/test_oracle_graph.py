"""Pins of the oracle's graph build (Sec. 2 nested graph with the shrinking of
neighbour lists; Sec. 4.1 distances from the raw vector to codes; Sec. 5.1
vectors added by batches), CPU only.

The build runs on one thread with its trace on (oracle/lc_oracle.h): one
record per list update.  The test replays the records from an empty graph and
checks each one against what the method defines, with distances taken here in
numpy from the raw vectors and from reconstructions decoded here:

* every new node's candidate list is what a best-first search (written here as
  one sorted pool) finds on the graph as it stood at the start of the node's
  batch, level by level from the greedy descent's end point;
* every selection keeps a candidate e by the shrinking test only if e is
  closer to the owner than to every earlier kept link s (d(x, e) < d(e, s),
  reconstruction to reconstruction), rejects a candidate only when some
  earlier kept link fails that test, and fills the free slots with the
  nearest rejected candidates in (distance, id) order;
* every reverse-link merge takes the target's list as it stood plus the new
  nodes that chose it, in id order; a merge that fits is that set sorted by the
  distance from the target's own (raw) vector, one that overflows is the
  selection above run from the target's raw vector;
* replaying the records gives the final lists.
"""
import numpy as np
import pytest

import datagen
import oracle



def _setup(n=360, d=16, m=4, deg0=6, deg_up=4, efc=10, ratio=4, seed=5, proj_pad=0):
    w = datagen.small(name=f"graph-pin-{seed}", n=n, nq=4, d=d, m=m, n_train=1024, seed=seed)
    db = datagen.vectors(w, "db")
    train = datagen.vectors(w, "train")
    proj = None
    d_pad = d
    if proj_pad:
        d_pad = d + proj_pad
        w = datagen.small(name=f"graph-pin-{seed}", n=n, nq=4, d=d, m=m, d_pad=d_pad, n_train=1024, seed=seed)
        proj = datagen.projection(w)
    init = datagen.pq_init_ids(w, train.shape[0])
    cent, _ = oracle.pq_train(train, proj, d_pad, m, init, 6)
    codes = oracle.pq_encode(db, proj, d_pad, cent)
    lv, _ = oracle.levels(datagen.level_uniforms(w), ratio=ratio)
    adj0, up_base, adj_up, entry, maxl, recs = oracle.hnsw_build_traced(db, proj, d_pad, cent, codes, lv, deg0,
                                                                         deg_up, efc)
    dsub = d_pad // m
    rec = np.empty((n, d_pad))
    for s in range(m):
        rec[:, s * dsub:(s + 1) * dsub] = cent[s][codes[:, s]]
    xp = db.astype(np.float64) if proj is None else db.astype(np.float64) @ proj.astype(np.float64).T
    # float64 summation-order slack for comparisons of distances
    return dict(rel=1e-12, n=n, deg0=deg0, deg_up=deg_up, efc=efc, lv=lv, adj0=adj0, up_base=up_base, adj_up=adj_up,
                entry=entry, maxl=maxl, recs=recs, rec=rec, xp=xp)


class Graph:
    """Lists rebuilt from the trace, one dict per level."""

    def __init__(self, g):
        self.g = g
        self.rows = {}

    def cap(self, l):
        return self.g["deg0"] if l == 0 else self.g["deg_up"]

    def row(self, l, i):
        return list(self.rows.get((l, int(i)), []))

    def put(self, l, i, ids):
        assert len(ids) <= self.cap(l)
        self.rows[(l, int(i))] = [int(x) for x in ids]


def _dist(a, b):
    return float(((a - b) ** 2).sum())


def _search(G, v, x_level):
    """Greedy descent above the node's level, then a best-first search with a
    sorted pool of at most efc entries on each level from min(level, top)
    down to 0, each from the best entry of the level above: the candidate
    list of each level."""
    g = G.g
    rec = g["rec"]

    def key(j):
        return (_dist(v, rec[j]), int(j))

    cur = key(g["entry"])
    for l in range(g["maxl"], x_level, -1):
        while True:
            best = min([key(j) for j in G.row(l, cur[1])] + [cur])
            if best == cur:
                break
            cur = best
    out = {}
    for l in range(min(x_level, g["maxl"]), -1, -1):
        pool = [[cur, False]]
        seen = {cur[1]}
        while True:
            idx = next((t for t, e in enumerate(pool) if not e[1]), None)
            if idx is None:
                break
            pool[idx][1] = True
            for nb in G.row(l, pool[idx][0][1]):
                if nb not in seen:
                    seen.add(nb)
                    pool.append([key(nb), False])
            pool.sort(key=lambda e: e[0])
            pool = pool[:g["efc"]]
        out[l] = [e[0][1] for e in pool]
        cur = pool[0][0]
    return out


def _check_selection(g, owner_vec, cand, out, by_test, cap):
    """The defining properties of the shrinking selection, pair by pair."""
    rec = g["rec"]
    REL = g.get("rel", 1e-12)
    cand = [int(c) for c in cand]
    keys = {c: (_dist(owner_vec, rec[c]), c) for c in cand}
    order = sorted(cand, key=lambda c: keys[c])
    out = [int(c) for c in out]
    assert out == sorted(out, key=lambda c: keys[c]), "list sorted by distance from the owner"
    assert len(out) == min(len(cand), cap), "free slots are filled while candidates remain"
    assert set(out) <= set(cand) and len(set(out)) == len(out)
    kept = [c for c, t in zip(out, by_test) if t]
    filled = [c for c, t in zip(out, by_test) if not t]
    kept_set = set(kept)
    # (a) each kept link is closer to the owner than to every kept link before it
    for e in kept:
        for s in kept:
            if keys[s] < keys[e]:
                assert keys[e][0] < _dist(rec[e], rec[s]) * (1 + REL), (e, s)
    # (b) each rejected candidate met, before the kept list was full, a kept link closer to it than the owner
    last = keys[kept[-1]] if len(kept) == cap else None
    rejected = []
    for c in order:
        if c in kept_set:
            continue
        if last is not None and keys[c] > last:
            break  # the kept list was full before c came up
        rejected.append(c)
        assert any(keys[s] < keys[c] and not (keys[c][0] < _dist(rec[c], rec[s]) * (1 - REL)) for s in kept), c
    # (c) the free slots hold the nearest rejected candidates in (distance, id) order
    assert filled == rejected[:cap - len(kept)] if len(kept) < cap else filled == []


def _replay_and_check(g):
    G = Graph(g)
    recs = g["recs"]
    assert recs[0]["kind"] == 3
    i = 0
    batches = 0
    while i < len(recs):
        r = recs[i]
        assert r["kind"] == 3, "every batch starts with its marker"
        batch = [int(x) for x in r["cand"]]
        i += 1
        # searches against the graph frozen at the start of the batch
        frozen = {x: _search(G, g["xp"][x], int(g["lv"][x])) for x in batch}
        chosen = {}
        writes = []
        for x in batch:
            top = min(int(g["lv"][x]), g["maxl"])
            for l in range(top, -1, -1):
                f = recs[i]
                i += 1
                assert (f["kind"], f["owner"], f["level"]) == (0, x, l)
                assert f["cand"].tolist() == frozen[x][l], (x, l)
                _check_selection(g, g["xp"][x], f["cand"], f["out"], f["by_test"], G.cap(l))
                writes.append((l, x, f["out"]))
                for t in f["out"]:
                    chosen.setdefault((l, int(t)), []).append(x)
        for l, x, o in writes:
            G.put(l, x, o)
        # reverse links, one merge per (level, target) in that order
        groups = sorted(chosen)
        for l, t in groups:
            f = recs[i]
            i += 1
            assert f["kind"] in (1, 2) and (f["level"], f["owner"]) == (l, t)
            expect = G.row(l, t) + sorted(chosen[(l, t)])
            assert f["cand"].tolist() == expect, (l, t)
            v = g["xp"][t]
            if f["kind"] == 2:
                assert len(expect) <= G.cap(l)
                keys = sorted((_dist(v, g["rec"][c]), c) for c in expect)
                assert f["out"].tolist() == [c for _, c in keys]
            else:
                assert len(expect) > G.cap(l)
                _check_selection(g, v, f["cand"], f["out"], f["by_test"], G.cap(l))
            G.put(l, t, f["out"])
        batches += 1
    # the replayed lists are the build's lists
    for x in range(g["n"]):
        row0 = g["adj0"][x]
        assert row0[row0 >= 0].tolist() == G.row(0, x)
        for l in range(1, int(g["lv"][x]) + 1):
            ru = g["adj_up"][g["up_base"][x] + l - 1]
            assert ru[ru >= 0].tolist() == G.row(l, x)
    return batches


@pytest.mark.parametrize("kw", [dict(), dict(deg0=4, deg_up=3, efc=7, seed=6), dict(proj_pad=4, seed=7)])
def test_graph_build_trace_matches_the_definition(kw):
    g = _setup(**kw)
    kinds = [r["kind"] for r in g["recs"]]
    # the cases the pin is about all occur: selections that reject, fills, overflowing merges, upper levels
    assert kinds.count(1) > 50 and kinds.count(2) > 20
    assert any(r["kind"] in (0, 1) and not r["by_test"].all() for r in g["recs"])
    assert any(r["kind"] in (0, 1) and len(r["out"]) < len(r["cand"]) for r in g["recs"])
    assert any(r["level"] > 0 for r in g["recs"] if r["kind"] == 0)
    batches = _replay_and_check(g)
    assert batches > 20


def test_trace_does_not_change_the_build():
    w = datagen.small(name="graph-pin-same", n=300, nq=4, d=16, m=4, n_train=1024)
    db, train = datagen.vectors(w, "db"), datagen.vectors(w, "train")
    cent, _ = oracle.pq_train(train, None, 16, 4, datagen.pq_init_ids(w, train.shape[0]), 4)
    codes = oracle.pq_encode(db, None, 16, cent)
    lv, _ = oracle.levels(datagen.level_uniforms(w), ratio=5)
    a = oracle.hnsw_build(db, None, 16, cent, codes, lv, 6, 4, 10, nthreads=3)
    b = oracle.hnsw_build_traced(db, None, 16, cent, codes, lv, 6, 4, 10)
    for x, y in zip(a, b[:5]):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_shrinking_rule_on_exact_ties():
    # integer points that are their own centroids: every distance is an exact integer in both the oracle and
    # numpy, and many comparisons d(x, e) vs d(e, s) tie exactly; the rule keeps e only when d(x, e) < d(e, s)
    # strictly, so the checks run without slack
    rs = np.random.default_rng(8)
    pts = np.array([(a, b) for a in range(7) for b in range(7)], np.float32)
    pts = pts[rs.permutation(len(pts))][:40]
    n = pts.shape[0]
    cent = pts.reshape(1, n, 2).copy()
    codes = np.arange(n, dtype=np.uint8).reshape(n, 1)
    lv, _ = oracle.levels(1.0 - rs.random(n), ratio=3)
    adj0, up_base, adj_up, entry, maxl, recs = oracle.hnsw_build_traced(pts, None, 2, cent, codes, lv, 3, 2, 6)
    g = dict(rel=0.0, n=n, deg0=3, deg_up=2, efc=6, lv=lv, adj0=adj0, up_base=up_base, adj_up=adj_up, entry=entry,
             maxl=maxl, recs=recs, rec=pts.astype(np.float64), xp=pts.astype(np.float64))
    ties = 0
    for r in recs:
        if r["kind"] in (0, 1):
            v = g["xp"][r["owner"]]
            c = sorted(int(x) for x in r["cand"])
            ties += sum(_dist(v, g["rec"][e]) == _dist(g["rec"][e], g["rec"][t]) for e in c for t in c if t != e)
    assert ties > 10
    _replay_and_check(g)
