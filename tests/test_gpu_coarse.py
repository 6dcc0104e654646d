"""2-level residual codec (Sec. 3.3 residual codecs; Sec. 5.1 two-level
encodings) on the GPU against the oracle, through the C-ABI.

The oracle takes the walk's asymmetric distance by its definition,
||P y - (c + r)||^2 in float64 with both levels decoded; the GPU sums the
decomposed form in float32 (the [m][256] inner-product table, the node's two
first-level entries and its stored term, clamped at 0).  Bars: the short-lists,
E and D of the float32 walk equal the oracle's on every query, every
short-list distance within the rounding bound of the decomposed float32 sum
(_walk_distance_bound: its terms cancel, so 1e-5 relative is not what float32
guarantees there), top-K EXACT against
the oracle's refinement of the GPU's short-list, every returned distance
within 1e-5 relative, and the codebook assignment identical on every vector.
The fp16 tables are an approximation by design: their walk is held to a
short-list overlap with float32's, and its refinement to the oracle's bars.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


_built = {}


def _build(m, d, d_pad=None, k=32):
    key = (m, d, d_pad, k)
    if key not in _built:
        kw = {} if d_pad is None else {"d_pad": d_pad}
        w = datagen.small(name=f"coarse-{m}-{d}", n=1500, nq=24, d=d, m=m, n_train=1024, n_beta=8,
                          n_beta_train=1500, k_reg=6, ef=40, shortlist=48, topk=10, coarse_k=k, **kw)
        ix, db, q = oracle.build_workload(w, nthreads=4)
        _built[key] = (w, ix, db, q)
    return _built[key]


def _walk_distance_bound(ix, y, ids):
    """Rounding bound of the float32 walk's decomposed distance (R33)
    ||z^0 - c^0||^2 + ||z^1 - c^1||^2 - 2 <z, r> + (||c + r||^2 - ||c||^2) against
    its float64 value ||z - (c + r)||^2: the m + 3 additions of the sum each
    round by at most 2^-24 of the running magnitude (at most the sum of the
    terms' magnitudes), and each term is itself a float32 value computed from
    float32 inputs (the first-level entries as ||z||^2 + ||c||^2 - 2 <z, c>,
    the inner-product entries per sub-space, the stored term rounded once).
    The terms cancel down to distances of a few 1e-2 on unit-norm data, so
    this bound, not 1e-5 relative, is what float32 arithmetic guarantees."""
    eps = 2.0 ** -24
    z = y.astype(np.float64) if ix.proj is None else ix.proj.astype(np.float64) @ y.astype(np.float64)
    h, ds = ix.d_pad // 2, ix.d_pad // ix.m
    out = []
    for j in ids:
        j = int(j)
        c = np.concatenate([ix.coarse_cent[t][ix.coarse_codes[j, t]].astype(np.float64) for t in range(2)])
        r = np.concatenate([ix.centroids[s][ix.codes[j, s]].astype(np.float64) for s in range(ix.m)])
        t12 = ((z - c) ** 2).sum()
        t3 = np.abs(-2.0 * (z * r).reshape(ix.m, ds).sum(1)).sum()
        t4 = abs(float(ix.coarse_norm[j]))
        s_abs = t12 + t3 + t4
        inputs = (z * z).sum() + (c * c).sum() + 2.0 * np.abs(z * c).sum() + 2.0 * np.abs(z * r).sum()
        out.append((ix.m + 8) * eps * s_abs + 4 * eps * inputs)
    return np.array(out)


def _oracle_topk(ix, q, cand_ids, cand_n, K):
    ids = np.full((q.shape[0], K), -1, np.int32)
    d = np.full((q.shape[0], K), np.inf)
    for i in range(q.shape[0]):
        c = cand_ids[i, :max(int(cand_n[i]), 0)]
        dd = np.array([ix.refined_distance(q[i], int(x)) for x in c])
        order = np.lexsort((c, dd))[:K]
        ids[i, :order.size] = c[order]
        d[i, :order.size] = dd[order]
    return {"ids": ids, "d": d}


# quarter-vector kernel shapes (d_pad / 4, dsub): (8, 4), (24, 6), (32, 4), (28, 2); m 24 with d 72 has
# no such kernel (18, 3) and takes the generic float32 refinement
@pytest.mark.parametrize("m,d,d_pad", [(8, 32, None), (16, 96, None), (8, 28, 32), (32, 128, None), (56, 112, None),
                                       (24, 72, None)])
def test_two_level_search_matches_oracle(torch, m, d, d_pad):
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(m, d, d_pad)
    assert ix.coarse_k == 32 and (d_pad is None or ix.proj is not None)
    print(f"case m {m} d {d} d_pad {w.d_pad}", flush=True)
    gix = lc.Index.from_index(ix)
    assert gix.coarse_k == 32 and gix.lut_stride == (m * 256 + 64 + 63) // 64 * 64
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    ids, dist, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    cand, cn = r.cand_ids.cpu().numpy(), r.cand_n.cpu().numpy()
    adc = r.cand_adc.cpu().numpy()
    same = [np.array_equal(cand[i], o["cand_ids"][i]) for i in range(q.shape[0])]
    assert np.mean(same) == 1.0, np.mean(same)
    for i in np.flatnonzero(same):
        n = int(cn[i])
        err = np.abs(adc[i, :n].astype(np.float64) - o["cand_adc"][i, :n])
        assert np.all(err <= _walk_distance_bound(ix, q[i], cand[i, :n])), (i, float(err.max()))
        assert np.array_equal(r.stats.cpu().numpy()[i], o["stats"][i])
    ref = _oracle_topk(ix, q, cand, cn, w.topk)
    s = parity.summarize(ix, q, ids.cpu().numpy(), dist.cpu().numpy(), ref)
    print(f"m {m}: walk {np.mean(same):.2f} EXACT {s['exact_frac']:.3f} max rel err {s['max_rel_err']:.1e}")
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()


# (m, d, d_pad, queries projected first): the first-level entries on the VALU with the projection applied
# in the kernel, else on MFMA (halves of 16 and 48; 32 centroids, one partial chunk of 256)
@pytest.mark.parametrize("m,d,d_pad,pre", [(8, 28, 32, False), (8, 28, 32, True), (16, 96, None, False)])
def test_two_level_tables_layout(torch, m, d, d_pad, pre):
    # row q: [m][256] entries -2 <z^s, C[s][c]>, then [2][k] entries ||z^h - C1[h][c]||^2, then zeros
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(m, d, d_pad)
    gix = lc.Index.from_index(ix)
    qt = torch.from_numpy(q)
    lut, scale = gix.build_lut(gix.project(qt), projected=True) if pre else gix.build_lut(qt)
    assert scale is None and tuple(lut.shape) == (q.shape[0], gix.lut_stride)
    lut = lut.cpu().numpy().astype(np.float64)
    h, ds, k = w.d_pad // 2, w.d_pad // w.m, ix.coarse_k
    for i in range(q.shape[0]):
        z = q[i].astype(np.float64) if ix.proj is None else ix.proj.astype(np.float64) @ q[i].astype(np.float64)
        ip = np.concatenate([-2.0 * (ix.centroids[s].astype(np.float64) @ z[s * ds:(s + 1) * ds]) for s in range(w.m)])
        ct = np.concatenate([((z[None, j * h:(j + 1) * h] - ix.coarse_cent[j].astype(np.float64)) ** 2).sum(1)
                             for j in range(2)])
        np.testing.assert_allclose(lut[i, :w.m * 256], ip, rtol=0, atol=1e-5 * np.abs(ip).max())
        np.testing.assert_allclose(lut[i, w.m * 256:w.m * 256 + 2 * k], ct, rtol=1e-5, atol=1e-6)
        assert (lut[i, w.m * 256 + 2 * k:] == 0).all()
    # fp16 form: the inner-product entries times their row's power-of-two scale within fp16 rounding of the
    # row's largest magnitude, the first-level entries float32 after them (byte offset m * 512)
    q16 = gix.project(qt) if pre else qt
    l16, sc = gix.build_lut(q16, lut_dtype=lc.LC_LUT_F16, projected=pre)
    assert tuple(l16.shape) == (q.shape[0], gix.lut_stride_f16) and tuple(sc.shape) == (q.shape[0], w.m)
    raw = l16.cpu().numpy().view(np.uint8)
    sc = sc.cpu().numpy().astype(np.float64)
    assert np.all(np.log2(sc) == np.round(np.log2(sc)))
    for i in range(q.shape[0]):
        ip16 = raw[i, :w.m * 512].view(np.float16).astype(np.float64).reshape(w.m, 256) * sc[i][:, None]
        ref = lut[i, :w.m * 256].reshape(w.m, 256)
        for s in range(w.m):
            assert np.abs(ip16[s] - ref[s]).max() <= 2.0 ** -10 * np.abs(ref[s]).max() + 1e-6
        ct16 = raw[i, w.m * 512:w.m * 512 + 8 * k].view(np.float32).astype(np.float64)
        np.testing.assert_array_equal(ct16, lut[i, w.m * 256:w.m * 256 + 2 * k])
    gix.close()


def test_two_level_budget_matches_oracle(torch):
    # the budget T on distance evaluations (Sec. 3.1) on the 2-level walk
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(16, 96)
    gix = lc.Index.from_index(ix)
    for T in (20, 75):
        o = ix.search(q, w.ef, w.shortlist, w.topk, max_evals=T)
        ids, dist, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True,
                                 max_evals=T)
        st = r.stats.cpu().numpy()
        assert (st[:, 1] <= T).all()
        same = [np.array_equal(r.cand_ids.cpu().numpy()[i], o["cand_ids"][i]) for i in range(q.shape[0])]
        assert np.mean(same) == 1.0
        for i in np.flatnonzero(same):
            assert np.array_equal(st[i], o["stats"][i])
    gix.close()


@pytest.mark.parametrize("m,d,d_pad", [(16, 96, None), (8, 28, 32)])
def test_two_level_assignment_is_identical(torch, m, d, d_pad):
    # the float64 arg-min of Eq. 7 with the 2-level decoding: the oracle's entry on every vector
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(m, d, d_pad)
    gix = lc.Index.from_index(ix)
    got = gix.assign_beta(torch.from_numpy(db)).cpu().numpy()
    assert np.array_equal(got[:, 0], ix.beta_idx), int((got[:, 0] != ix.beta_idx).sum())
    gix.close()


def test_zero_first_level_gives_the_one_level_results(torch):
    # one first-level centroid at the origin: same codes, same graph, the one-level search
    import dataclasses
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(16, 96)
    one = dataclasses.replace(ix, coarse_cent=None, coarse_codes=None, coarse_norm=None)
    zero = dataclasses.replace(ix, coarse_cent=np.zeros((2, 1, w.d_pad // 2), np.float32),
                               coarse_codes=np.zeros((ix.n, 2), np.uint16))
    zero.coarse_norm = zero.coarse_norms()
    a, b = lc.Index.from_index(one), lc.Index.from_index(zero)
    ia, da, ra = a.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    ib, dbb, rb = b.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    # both GPU forms against the oracle's one-level search of the same codes (EXACT on every query)
    o = one.search(q, w.ef, w.shortlist, w.topk)
    for ids_, d_ in ((ia, da), (ib, dbb)):
        s = parity.summarize(one, q, ids_.cpu().numpy(), d_.cpu().numpy(), o)
        assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    np.testing.assert_allclose(dbb.cpu().numpy(), da.cpu().numpy(), rtol=1e-5)
    a.close()
    b.close()


def test_two_level_batched_form_matches_query(torch):
    # the batched form (per-query ef, captured step) on a 2-level index: per query the bits of Index.query
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd.batched import BatchedSearcher
    w, ix, db, q = _build(8, 28, 32)
    gix = lc.Index.from_index(ix)
    ef = np.where(np.arange(q.shape[0]) % 3 == 0, 48, 16).astype(np.int32)
    bs = BatchedSearcher(gix, q.shape[0], 48, 16, 5, precision="f32")
    bs.set_inputs(q, ef)
    ids, d = bs.run()
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    for e in (16, 48):
        sel = np.flatnonzero(ef == e)
        ri, rd, _ = gix.query(torch.from_numpy(q[sel]), ef=e, ef_max=48, S=16, K=5)
        assert np.array_equal(ids[sel], ri.cpu().numpy())
        assert np.array_equal(d[sel].view(np.uint32), rd.cpu().numpy().view(np.uint32))
    bs.capture()
    for _ in range(3):
        gi, gd = bs.run()
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), ids)
        assert np.array_equal(gd.cpu().numpy().view(np.uint32), d.view(np.uint32))
        gix.query(torch.from_numpy(q[:7]), ef=16, ef_max=48, S=16, K=5)
        torch.cuda.synchronize()
    gix.close()


def test_two_level_serving_same_alone_and_in_the_mix(torch):
    # the serving loop on a 2-level index (float32 tables of lut_stride entries): a request's results do not
    # depend on the batch it rides in
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import serve
    w, ix, db, q = _build(8, 28, 32)
    gix = lc.Index.from_index(ix)
    S, K, ef_max = 16, 5, 64
    reqs = serve.poisson_requests(w.d, q, rate_rps=4000.0, n_requests=20, seed=5, efs=(16, 64), max_batch=8)
    eng = serve.GpuEngine(gix, n_slots=3, slot_queries=32, ef_max=ef_max, S=S, K=K, precision="f32")
    bpq = serve.query_bytes(w.m, S, K, w.d, lut_bytes=4, d_proj=w.d_pad, lut_entries=gix.lut_stride)
    stats = serve.serve(eng, serve.Scheduler(3, 32, mem_budget=64 * bpq, bytes_per_query=bpq), reqs)
    torch.cuda.synchronize()
    assert stats["requests"] == 20
    for r in reqs:
        ids, d, _ = gix.query(torch.from_numpy(r.queries), ef=r.ef, ef_max=ef_max, S=S, K=K)
        assert np.array_equal(r.ids, ids.cpu().numpy()), r.rid
        assert np.array_equal(r.dist.view(np.uint32), d.cpu().numpy().view(np.uint32)), r.rid
    gix.close()


def test_two_level_two_chunks_of_first_level_centroids(torch):
    # k = 300: the MFMA first-level tables in two chunks (256 and 44 centroids); values and search
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(16, 96, None, k=300)
    assert ix.coarse_k == 300
    gix = lc.Index.from_index(ix)
    lut, _ = gix.build_lut(torch.from_numpy(q))
    lut = lut.cpu().numpy().astype(np.float64)
    h, base = w.d_pad // 2, w.m * 256
    for i in range(q.shape[0]):
        z = q[i].astype(np.float64)
        ct = np.concatenate([((z[None, j * h:(j + 1) * h] - ix.coarse_cent[j].astype(np.float64)) ** 2).sum(1)
                             for j in range(2)])
        np.testing.assert_allclose(lut[i, base:base + 600], ct, rtol=1e-5, atol=1e-6)
        assert (lut[i, base + 600:] == 0).all()
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    ids, dist, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    cand = r.cand_ids.cpu().numpy()
    assert np.mean([np.array_equal(cand[i], o["cand_ids"][i]) for i in range(q.shape[0])]) == 1.0
    ref = _oracle_topk(ix, q, cand, r.cand_n.cpu().numpy(), w.topk)
    s = parity.summarize(ix, q, ids.cpu().numpy(), dist.cpu().numpy(), ref)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()


@pytest.mark.parametrize("m,d,d_pad", [(16, 96, None), (8, 28, 32)])
def test_two_level_fp16_tables(torch, m, d, d_pad):
    # fp16 inner-product entries (the precision form on the 2-level codec): the walk takes its own
    # short-list; its refinement is the oracle's to the same bars, and the short-lists stay close to float32's
    import paper_1804_09996_amd as lc
    w, ix, db, q = _build(m, d, d_pad)
    gix = lc.Index.from_index(ix)
    i32, d32, r32 = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    ids, dist, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, precision="f16")
    cand, cn = r.cand_ids.cpu().numpy(), r.cand_n.cpu().numpy()
    c32 = r32.cand_ids.cpu().numpy()
    overlap = np.mean([np.intersect1d(cand[i][cand[i] >= 0], c32[i][c32[i] >= 0]).size / max(1, int(cn[i]))
                       for i in range(q.shape[0])])
    assert overlap >= 0.9, overlap
    ref = _oracle_topk(ix, q, cand, cn, w.topk)
    s = parity.summarize(ix, q, ids.cpu().numpy(), dist.cpu().numpy(), ref)
    print(f"m {m} fp16: short-list overlap with float32 {overlap:.3f} EXACT {s['exact_frac']:.3f}")
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()
