"""GPU path against the oracle, element by element, through the C-ABI.

Indexes here are built by the oracle from seeded inputs; the GPU library only
searches them.  Bars: integer outputs (ids, E, D, short-list) bit-exact;
float32 distances within 1e-5 relative of the oracle's float64 values; top-K
ids EXACT in the sense of tests/parity.py on every query.
"""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle
from tests import parity

pytestmark = pytest.mark.gpu

F32_EPS = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def c1(c1_build, torch):
    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    return w, ix, lc.Index.from_index(ix), db, q


@pytest.fixture(scope="module")
def c1_oracle(c1):
    w, ix, gix, db, q = c1
    return ix.search(q, w.ef, w.shortlist, w.topk)


def _lut_bound(ix, q):
    dsub = ix.d_pad // ix.m
    mu = ix.centroids.astype(np.float64).mean(1)  # [m][dsub]
    nc = ((ix.centroids.astype(np.float64) - mu[:, None, :]) ** 2).sum(-1)  # [m][256]
    out = []
    for y in q:
        yp = oracle.project(ix.proj, y, ix.d_pad).reshape(ix.m, dsub)
        ny = ((yp - mu) ** 2).sum(-1)
        out.append(16 * F32_EPS * (ny[:, None] + nc) + 1e-30)
    return np.stack(out)


def test_lut_matches_oracle_within_bound(c1, torch):
    w, ix, gix, db, q = c1
    lut, _ = gix.build_lut(torch.from_numpy(q))
    got = lut.cpu().numpy().astype(np.float64)
    ref = np.stack([ix.lut(y) for y in q])
    bound = _lut_bound(ix, q)
    assert got.shape == ref.shape
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))
    assert np.all(got >= 0) and not np.any(np.signbit(got))


def test_walk_matches_oracle(c1, c1_oracle, torch):
    w, ix, gix, db, q = c1
    lut, _ = gix.build_lut(torch.from_numpy(q))
    r = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist)
    ids = r.cand_ids.cpu().numpy()
    adc = r.cand_adc.cpu().numpy()
    n = r.cand_n.cpu().numpy()
    st = r.stats.cpu().numpy()
    o = c1_oracle
    same = [(np.array_equal(ids[i], o["cand_ids"][i]) and n[i] == o["cand_n"][i]
             and np.array_equal(st[i], o["stats"][i])) for i in range(w.nq)]
    print(f"walk identical (short-list, E, D) on {sum(same)}/{w.nq} queries")
    assert np.mean(same) == 1.0
    for i in np.flatnonzero(same):
        k = n[i]
        np.testing.assert_allclose(adc[i, :k], o["cand_adc"][i, :k], rtol=1e-5)
        assert np.all(ids[i, k:] == -1) and np.all(np.isinf(adc[i, k:]))


def test_full_path_parity(c1, c1_oracle, torch):
    w, ix, gix, db, q = c1
    ids, d, _ = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    s = parity.summarize(ix, q, ids, d, c1_oracle)
    print(f"EXACT {s['exact_frac']:.4f} strict {s['strict_frac']:.4f} max rel err {s['max_rel_err']:.2e}")
    assert s["exact_frac"] == 1.0
    assert s["max_rel_err"] <= 1e-5


def test_per_query_ef_and_rejected_queries(c1, torch):
    w, ix, gix, db, q = c1
    qq = q[:9]
    ef = np.array([1, 5, 16, 64, 0, 65, 33, 2, 64], np.int32)
    lut, _ = gix.build_lut(torch.from_numpy(qq))
    r = gix.search(lut, ef=torch.from_numpy(ef), ef_max=64, S=8)
    ids, n, st = r.cand_ids.cpu().numpy(), r.cand_n.cpu().numpy(), r.stats.cpu().numpy()
    for i in range(9):
        if ef[i] < 1 or ef[i] > 64:
            assert n[i] == -1 and np.all(ids[i] == -1)
            continue
        o = ix.search(qq[i:i + 1], int(ef[i]), 8, 1)
        assert np.array_equal(ids[i], o["cand_ids"][0]) and n[i] == o["cand_n"][0]
        assert np.array_equal(st[i], o["stats"][0])


def test_ragged_batches_and_batch_independence(c1, torch):
    w, ix, gix, db, q = c1
    full_ids, full_d, full_r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk,
                                         stats=True)
    full_ids, full_d = full_ids.cpu().numpy(), full_d.cpu().numpy()
    for lo, hi in ((0, 1), (3, 20), (37, 100)):
        ids, d, _ = gix.query(torch.from_numpy(q[lo:hi]), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
        assert np.array_equal(ids.cpu().numpy(), full_ids[lo:hi])
        assert np.array_equal(d.cpu().numpy().view(np.uint32), full_d[lo:hi].view(np.uint32))
    again_ids, again_d, _ = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    assert np.array_equal(again_ids.cpu().numpy(), full_ids)
    assert np.array_equal(again_d.cpu().numpy().view(np.uint32), full_d.view(np.uint32))
    # the empty batch is a no-op
    e_ids, e_d, _ = gix.query(torch.zeros((0, w.d)), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    assert e_ids.shape == (0, w.topk)


def test_exhaustive_walk_and_short_graph(torch):
    # ef >= N makes the walk visit the whole (connected) graph; S > |W| pads
    import paper_1804_09996_amd as lc
    w = datagen.small(name="gpu-small", n=600, nq=21, d=32, m=8, n_train=1024, n_beta=16, n_beta_train=600, k_reg=8)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    gix = lc.Index.from_index(ix)
    for ef, S, K in ((600, 640, 640), (17, 9, 9), (3, 40, 7)):
        o = ix.search(q, ef, S, K)
        ids, d, r = gix.query(torch.from_numpy(q), ef=ef, ef_max=ef, S=S, K=K, stats=True)
        assert np.array_equal(r.cand_ids.cpu().numpy(), o["cand_ids"])
        assert np.array_equal(r.stats.cpu().numpy(), o["stats"])
        s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
        assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5


def test_lossless_case_returns_exact_knn(torch):
    import paper_1804_09996_amd as lc
    rs = np.random.default_rng(11)
    n, d, m = 256, 16, 8
    db = rs.standard_normal((n, d)).astype(np.float32)
    cent, _ = oracle.pq_train(db, None, d, m, np.stack([rs.permutation(n) for _ in range(m)]), 2)
    codes = oracle.pq_encode(db, None, d, cent)
    lv, _ = oracle.levels(1.0 - rs.random(n))
    adj0, up_base, adj_up, entry, maxl = oracle.hnsw_build(db, None, d, cent, codes, lv, 32, 32, 64)
    beta = np.zeros((1, 5), np.float32)
    beta[0, 0] = 1
    ix = oracle.Index(n=n, d=d, d_pad=d, m=m, deg0=32, deg_up=32, k_reg=4, n_beta=1, entry=entry, max_level=maxl,
                      proj=None, centroids=cent, codes=codes, adj0=adj0, level=lv, up_base=up_base, adj_up=adj_up,
                      beta=beta, beta_idx=np.zeros(n, np.uint8))
    gix = lc.Index.from_index(ix)
    q = rs.standard_normal((33, d)).astype(np.float32)
    ids, dist, _ = gix.query(torch.from_numpy(q), ef=n, ef_max=n, S=n, K=10)
    dd = ((q[:, None, :].astype(np.float64) - db[None]) ** 2).sum(-1)
    gt = np.argsort(dd, axis=1, kind="stable")[:, :10]
    ids = ids.cpu().numpy()
    for i in range(33):
        for r in range(10):
            assert ids[i, r] == gt[i, r] or abs(dd[i, ids[i, r]] - dd[i, gt[i, r]]) <= 1e-5 * dd[i, gt[i, r]]
    np.testing.assert_allclose(dist.cpu().numpy(), np.take_along_axis(dd, ids.astype(np.int64), 1), rtol=1e-5)


def test_single_node_index(torch):
    import paper_1804_09996_amd as lc
    rs = np.random.default_rng(12)
    cent = rs.standard_normal((8, 256, 2)).astype(np.float32)
    ix = oracle.Index(n=1, d=16, d_pad=16, m=8, deg0=32, deg_up=32, k_reg=2, n_beta=1, entry=0, max_level=0,
                      proj=None, centroids=cent, codes=rs.integers(0, 256, (1, 8)).astype(np.uint8),
                      adj0=np.full((1, 32), -1, np.int32), level=np.zeros(1, np.int8),
                      up_base=np.full(1, -1, np.int32), adj_up=np.zeros((0, 32), np.int32),
                      beta=np.array([[0.9, 0.1, 0.2]], np.float32), beta_idx=np.zeros(1, np.uint8))
    gix = lc.Index.from_index(ix)
    q = rs.standard_normal((3, 16)).astype(np.float32)
    ids, d, r = gix.query(torch.from_numpy(q), ef=4, ef_max=4, S=4, K=3, stats=True)
    o = ix.search(q, 4, 4, 3)
    assert np.array_equal(ids.cpu().numpy(), o["ids"])
    assert np.array_equal(r.stats.cpu().numpy(), o["stats"])
    np.testing.assert_allclose(d.cpu().numpy()[:, 0], o["d"][:, 0], rtol=1e-5)


SCHEDULES = [dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=0, visited=0),   # small table: full buckets
             dict(hash_bits=9, prefetch=1, waves_per_cu=1, queue=1, visited=0, wide=1),
             dict(hash_bits=14, prefetch=1, waves_per_cu=0, queue=1, visited=0),
             dict(hash_bits=0, prefetch=0, waves_per_cu=2, queue=1, visited=0),
             dict(hash_bits=11, prefetch=1, waves_per_cu=0, queue=0, visited=0, wide=1),
             dict(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, pool=1),   # pool in LDS
             dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=0, visited=0, pool=1),
             dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=1, visited=1),   # bitset + LDS cache
             dict(hash_bits=10, prefetch=1, waves_per_cu=0, queue=0, visited=1),
             dict(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, codes=1),   # codes after the probe
             dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=1, visited=0, pool=1, codes=1)]


def test_every_schedule_gives_identical_results(c1, c1_oracle, torch):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    lut, _ = gix.build_lut(torch.from_numpy(q))
    ref = None
    for sd in SCHEDULES:
        sc = lc.schedule(**sd)
        for _ in range(2):  # twice: the workspace must come back clean
            r = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist, sched=sc)
            got = (r.cand_ids.cpu().numpy(), r.cand_adc.cpu().numpy().view(np.uint32), r.cand_n.cpu().numpy(),
                   r.stats.cpu().numpy())
            if ref is None:
                ref = got
                assert np.array_equal(got[0], c1_oracle["cand_ids"]) and np.array_equal(got[3], c1_oracle["stats"])
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), sd
            ws = gix.workspace(q.shape[0], w.ef, w.shortlist, sc)
            assert int(ws.count_nonzero().item()) == 0, f"workspace not left zeroed: {sd}"


def test_overflow_path_with_large_pool(torch):
    # ef = N on a graph of 2400 nodes with a 512-slot table: most of the walk
    # runs on the workspace bitset
    import paper_1804_09996_amd as lc
    w = datagen.small(name="ovf", n=2400, nq=12, d=32, m=8, n_train=1024, n_beta=16, n_beta_train=2400, k_reg=8)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    gix = lc.Index.from_index(ix)
    o = ix.search(q, 2400, 64, 10)
    for sd in (dict(hash_bits=9, prefetch=1, waves_per_cu=0, queue=1, visited=0),
               dict(hash_bits=9, prefetch=1, waves_per_cu=0, queue=1, visited=0, wide=1),
               dict(hash_bits=14, prefetch=0, waves_per_cu=0, queue=0, visited=0),
               dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=1, visited=1)):
        sc = lc.schedule(**sd)
        ids, d, r = gix.query(torch.from_numpy(q), ef=2400, ef_max=2400, S=64, K=10, stats=True, sched=sc)
        assert np.array_equal(r.cand_ids.cpu().numpy(), o["cand_ids"])
        assert np.array_equal(r.stats.cpu().numpy(), o["stats"])
        assert np.all(r.stats.cpu().numpy()[:, 1] == 2399)
        assert int(gix.workspace(12, 2400, 64, sc).count_nonzero().item()) == 0


def test_register_pool_sizes(torch):
    # pools of 1..256 entries across the chunk boundaries (in registers up to
    # 128 entries, in LDS beyond), against the oracle and the LDS pool
    import paper_1804_09996_amd as lc
    w = datagen.small(name="regpool", n=2400, nq=12, d=32, m=8, n_train=1024, n_beta=16, n_beta_train=2400, k_reg=8)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    gix = lc.Index.from_index(ix)
    lut, _ = gix.build_lut(torch.from_numpy(q))
    for ef, S in ((1, 1), (2, 1), (63, 8), (64, 64), (65, 10), (127, 16), (128, 128), (129, 32), (200, 100),
                  (255, 255), (256, 64), (40, 256)):
        o = ix.search(q, ef, S, 1)
        got = []
        for sd in (dict(), dict(pool=1), dict(hash_bits=9, prefetch=0)):
            sc = lc.schedule(**sd)
            r = gix.search(lut, ef=ef, ef_max=ef, S=S, sched=sc)
            got.append((r.cand_ids.cpu().numpy(), r.cand_adc.cpu().numpy().view(np.uint32), r.cand_n.cpu().numpy(),
                        r.stats.cpu().numpy()))
            assert int(gix.workspace(12, ef, S, sc).count_nonzero().item()) == 0
        assert np.array_equal(got[0][0], o["cand_ids"]), (ef, S)
        assert np.array_equal(got[0][3], o["stats"]), (ef, S)
        for g in got[1:]:
            for a_, b_ in zip(got[0], g):
                assert np.array_equal(a_, b_), (ef, S)


# ---------------------------------------------------------------------------
# precision form: fp16 tables, bf16 refinement, exact fp32 re-score
# ---------------------------------------------------------------------------
def test_fp16_lut_is_the_scaled_table(c1, torch):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    h = lut.cpu().numpy().astype(np.float64)
    sc = sc.cpu().numpy().astype(np.float64)
    ref = np.stack([ix.lut(y) for y in q])
    mant, _ = np.frexp(sc)
    assert np.all(mant == 0.5), "scales are powers of two"
    assert np.all(h.max(-1) <= 32768.0)
    got = h * sc[:, :, None]
    # fp16 rounding of LUT/scale (half an ulp, at most 2^-11 relative) plus the fp32 table bound
    bound = 2.0 ** -11 * np.abs(ref) + 2.0 ** -24 * sc[:, :, None] + _lut_bound(ix, q)
    assert np.all(np.abs(got - ref) <= bound)


def test_precision_refine_rescores_exactly(c1, torch):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    qt = torch.from_numpy(q)
    lut, _ = gix.build_lut(qt)
    r = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist)
    ids32, d32 = gix.refine(qt, r.cand_ids, r.cand_n, w.topk, lc.LC_REFINE_F32)
    ids16, d16 = gix.refine(qt, r.cand_ids, r.cand_n, w.topk, lc.LC_REFINE_BF16_RESCORE)
    ids32, d32, ids16, d16 = (t.cpu().numpy() for t in (ids32, d32, ids16, d16))
    same = 0
    for i in range(w.nq):
        plain = {int(a): float(b) for a, b in zip(ids32[i], d32[i]) if a >= 0}
        for a, b in zip(ids16[i], d16[i]):
            if a in plain:
                assert np.float32(b).view(np.uint32) == np.float32(plain[a]).view(np.uint32)
        same += np.array_equal(ids16[i], ids32[i])
        keys = list(zip(d16[i].tolist(), ids16[i].tolist()))
        assert keys == sorted(keys)
    print(f"bf16+rescore top-{w.topk} identical to fp32 on {same}/{w.nq} queries")
    assert same >= 0.95 * w.nq


@pytest.mark.parametrize("precision", ["f16", "f16+bf16"])
def test_precision_path_recall_close_to_plain(c1, torch, precision):
    w, ix, gix, db, q = c1
    qt = torch.from_numpy(q)
    gt = np.argmin(((q[:, None, :].astype(np.float64) - db[None].astype(np.float64)) ** 2).sum(-1), 1)
    i32, _, _ = gix.query(qt, ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    i16, d16, _ = gix.query(qt, ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, precision=precision)
    r32 = parity.recall_at(i32.cpu().numpy(), gt, 10)
    r16 = parity.recall_at(i16.cpu().numpy(), gt, 10)
    print(f"R@10 fp32 {r32:.3f} fp16/bf16 {r16:.3f}")
    assert r16 >= r32 - 0.03
    err = parity.distance_errors(ix, q, i16.cpu().numpy(), d16.cpu().numpy())
    assert np.nanmax(err) <= 1e-5  # every returned distance is an exact fp32 re-score


# ---------------------------------------------------------------------------
# batched form: per-query ef, longest-first order, graph replay
# ---------------------------------------------------------------------------
def test_processing_order_does_not_change_results(c1, torch):
    w, ix, gix, db, q = c1
    ef = np.random.default_rng(21).integers(8, 65, w.nq).astype(np.int32)
    lut, _ = gix.build_lut(torch.from_numpy(q))
    a = gix.search(lut, ef=torch.from_numpy(ef), ef_max=64, S=16)
    perm = np.argsort(-ef, kind="stable").astype(np.int32)
    b = gix.search(lut, ef=torch.from_numpy(ef), ef_max=64, S=16, order=torch.from_numpy(perm).cuda())
    for x, y in ((a.cand_ids, b.cand_ids), (a.cand_n, b.cand_n), (a.stats, b.stats)):
        assert torch.equal(x, y)
    o = ix.search(q, ef, 16, 10)
    assert np.array_equal(b.cand_ids.cpu().numpy(), o["cand_ids"])
    assert np.array_equal(b.stats.cpu().numpy(), o["stats"])


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_graph_replays_match_eager(c1, torch, precision):
    from paper_1804_09996_amd.batched import BatchedSearcher
    w, ix, gix, db, q = c1
    ef = np.random.default_rng(22).integers(8, 65, w.nq).astype(np.int32)
    bs = BatchedSearcher(gix, w.nq, ef_max=64, S=32, K=10, precision=precision)
    bs.set_inputs(q, ef)
    eager_ids, eager_d = (t.clone() for t in bs.run())
    bs.capture()
    for rep in range(4):
        # other eager work between replays, on the same device
        gix.query(torch.from_numpy(q[:7]), ef=16, ef_max=16, S=16, K=5)
        torch.cuda.synchronize()
        ids, d = bs.run()
        torch.cuda.synchronize()
        assert torch.equal(ids, eager_ids), rep
        assert torch.equal(d.view(torch.int32), eager_d.view(torch.int32)), rep
        for ws in bs.ws:
            assert int(ws.count_nonzero().item()) == 0
    # a new batch through the same graph
    q2 = np.ascontiguousarray(q[::-1])
    bs.set_inputs(q2, ef[::-1].copy())
    ids2, d2 = bs.run()
    ref_ids, ref_d, _ = gix.query(torch.from_numpy(q2), ef=torch.from_numpy(ef[::-1].copy()), ef_max=64, S=32, K=10,
                                  precision=precision)
    assert torch.equal(ids2, ref_ids)


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_ef_classes_give_the_same_results(c1, torch, precision):
    # the batch split into ef classes (one concurrent walk launch each, rows
    # permuted by class and back): every query as alone, eager and replayed
    from paper_1804_09996_amd.batched import BatchedSearcher, class_limits_options
    w, ix, gix, db, q = c1
    ef = np.random.default_rng(24).integers(8, 301, w.nq).astype(np.int32)
    assert class_limits_options(300, 32) == [[320], [128, 320], [128, 256, 320]]
    bs = BatchedSearcher(gix, w.nq, ef_max=300, S=32, K=10, precision=precision)
    bs.set_inputs(q, ef)
    ref_ids, ref_d, _ = gix.query(torch.from_numpy(q), ef=torch.from_numpy(ef), ef_max=300, S=32, K=10,
                                  precision=precision)
    for limits in ([320], [128, 320], [128, 256, 320], [64, 128, 192, 256, 320]):
        bs.set_classes(limits)
        assert sum(r1 - r0 for r0, r1, _ in bs.ranges) == w.nq
        ids, d = bs.run()
        assert torch.equal(ids, ref_ids), limits
        assert torch.equal(d.view(torch.int32), ref_d.view(torch.int32)), limits
    bs.capture()
    for rep in range(3):
        gix.query(torch.from_numpy(q[:5]), ef=16, ef_max=16, S=16, K=5)
        torch.cuda.synchronize()
        ids, d = bs.run()
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_ids), rep
        for ws in bs.ws:
            assert int(ws.count_nonzero().item()) == 0


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_captured_step_takes_a_batch_with_other_classes(c1, torch, precision):
    # a captured step, then a batch whose largest ef is higher and whose class rows differ: the step is
    # recorded again for it (no query beyond its launch's pool, no freed workspace), and every query gets
    # what Index.query gives it alone; then back to a batch like the first
    from paper_1804_09996_amd.batched import BatchedSearcher
    w, ix, gix, db, q = c1
    rs = np.random.default_rng(25)
    bs = BatchedSearcher(gix, w.nq, ef_max=300, S=32, K=10, precision=precision)
    bs.set_classes([128, 320])
    batches = [rs.integers(8, 100, w.nq).astype(np.int32),       # one class, pools <= 128
               rs.integers(8, 301, w.nq).astype(np.int32),       # two classes, a larger top pool
               np.full(w.nq, 300, np.int32),                     # every query in the top class
               rs.integers(8, 100, w.nq).astype(np.int32)]
    for k, ef in enumerate(batches):
        qk = np.ascontiguousarray(q[::-1] if k % 2 else q)
        bs.set_inputs(qk, ef)
        if k == 0:
            bs.capture()
        assert bs.graph is not None
        ref_ids, ref_d, _ = gix.query(torch.from_numpy(qk), ef=torch.from_numpy(ef), ef_max=300, S=32, K=10,
                                      precision=precision)
        for rep in range(2):
            ids, d = bs.run()
            torch.cuda.synchronize()
            assert torch.equal(ids, ref_ids), (k, rep)
            assert torch.equal(d.view(torch.int32), ref_d.view(torch.int32)), (k, rep)
        for ws in bs.ws:
            assert int(ws.count_nonzero().item()) == 0


def test_golden_fixture_on_gpu(torch):
    # the frozen oracle outputs of tests/golden/tiny_search.json, from the GPU path
    import json
    import os
    import paper_1804_09996_amd as lc
    from tests.golden import make_golden
    g = json.load(open(os.path.join(os.path.dirname(make_golden.__file__), "tiny_search.json")))
    ix, db, q = make_golden.build()
    w = make_golden.W
    gix = lc.Index.from_index(ix)
    ids, d, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    assert r.cand_ids.cpu().numpy().tolist() == g["cand_ids"]
    assert r.stats.cpu().numpy().tolist() == g["stats"]
    gold = {"ids": np.array(g["ids"]), "d": np.array([[float.fromhex(x) for x in row] for row in g["d"]])}
    s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), gold)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()


def test_learned_rotation_index(torch):
    # a rotation with d_pad == d (learned ahead of PQ by the builder) is applied by the tables and the
    # refinement exactly as the oracle applies it
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import builder
    w = datagen.small(name="gpu-opq", n=1500, nq=24, d=32, m=8, n_train=2048, n_beta=8, n_beta_train=1500,
                      opq_iters=3, ef=32, shortlist=32, topk=10)
    bix, db, q = builder.build_workload(w, nthreads=4)
    ix = oracle.build_index(w, db, datagen.vectors(w, "train"), bix.proj, datagen.level_uniforms(w),
                            datagen.pq_init_ids(w, w.n_train), datagen.beta_train_ids(w),
                            datagen.beta_init_ids(w, min(w.n, w.n_beta_train)), 4)
    assert ix.proj is not None and ix.d_pad == ix.d
    gix = lc.Index.from_index(ix)
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    lut, _ = gix.build_lut(torch.from_numpy(q))
    got = lut.cpu().numpy().astype(np.float64)
    ref = np.stack([ix.lut(y) for y in q])
    assert np.all(np.abs(got - ref) <= _lut_bound(ix, q))
    ids, d, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    assert np.array_equal(r.cand_ids.cpu().numpy(), o["cand_ids"]) and np.array_equal(r.stats.cpu().numpy(), o["stats"])
    s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    _projected_entry_points(ix, gix, q, w, o, torch)
    gix.close()


def _projected_entry_points(ix, gix, q, w, o, torch):
    # the batch projected once (lc_project_queries) and the *_projected entry points, against the oracle and
    # against the entry points that project by themselves
    import paper_1804_09996_amd as lc
    qt = torch.from_numpy(q)
    qp = gix.project(qt)
    ref = np.stack([oracle.project(ix.proj, y, ix.d_pad) for y in q])
    np.testing.assert_allclose(qp.cpu().numpy(), ref, rtol=0, atol=1e-5 * np.abs(ref).max())
    lut_p, _ = gix.build_lut(qp, projected=True)
    assert np.all(np.abs(lut_p.cpu().numpy() - np.stack([ix.lut(y) for y in q])) <= _lut_bound(ix, q))
    r = gix.search(lut_p, ef=w.ef, ef_max=w.ef, S=w.shortlist)
    for prec in (lc.LC_REFINE_F32, lc.LC_REFINE_BF16_RESCORE):
        i_p, d_p = gix.refine(qp, r.cand_ids, r.cand_n, w.topk, prec, projected=True)
        i_q, d_q = gix.refine(qt, r.cand_ids, r.cand_n, w.topk, prec)
        err = parity.distance_errors(ix, q, i_p.cpu().numpy(), d_p.cpu().numpy())
        assert np.nanmax(err) <= 1e-5
        np.testing.assert_allclose(d_p.cpu().numpy(), d_q.cpu().numpy(), rtol=1e-5)
    i_f, d_f = gix.refine(qp, r.cand_ids, r.cand_n, w.topk, projected=True)
    s = parity.summarize(ix, q, i_f.cpu().numpy(), d_f.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0


def test_padded_projection_index(torch):
    # d 28 -> d_pad 32 through the seeded projection (required), the batch projected once by query()
    import paper_1804_09996_amd as lc
    w = datagen.small(name="gpu-pad", n=1500, nq=24, d=28, m=8, n_train=2048, n_beta=8, n_beta_train=1500,
                      ef=32, shortlist=32, topk=10)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    assert ix.proj is not None and ix.proj.shape == (32, 28)
    gix = lc.Index.from_index(ix)
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    ids, d, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    same = np.mean([np.array_equal(r.cand_ids.cpu().numpy()[i], o["cand_ids"][i]) for i in range(w.nq)])
    assert same == 1.0
    s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    _projected_entry_points(ix, gix, q, w, o, torch)
    gix.close()


def test_batched_form_on_projected_index(torch):
    # the batched form projects its batch once too: per query the same bits as Index.query
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd.batched import BatchedSearcher
    w = datagen.small(name="batch-pad", n=1500, nq=64, d=28, m=8, n_train=2048, n_beta=8, n_beta_train=1500)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    gix = lc.Index.from_index(ix)
    ef = np.where(np.arange(w.nq) % 3 == 0, 48, 16).astype(np.int32)
    bs = BatchedSearcher(gix, w.nq, 48, 16, 5, precision="f32")
    bs.set_inputs(q, ef)
    ids, d = bs.run()
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    for e in (16, 48):
        sel = np.flatnonzero(ef == e)
        ri, rd, _ = gix.query(torch.from_numpy(q[sel]), ef=e, ef_max=48, S=16, K=5)
        assert np.array_equal(ids[sel], ri.cpu().numpy())
        assert np.array_equal(d[sel].view(np.uint32), rd.cpu().numpy().view(np.uint32))
    # the captured step (the projection included) replays to the same bits, with eager work between replays
    bs.capture()
    for _ in range(3):
        gi, gd = bs.run()
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), ids)
        assert np.array_equal(gd.cpu().numpy().view(np.uint32), d.view(np.uint32))
        gix.query(torch.from_numpy(q[:7]), ef=16, ef_max=48, S=16, K=5)
        torch.cuda.synchronize()
    gix.close()


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_autotuned_batched_form(c1, torch, precision):
    # the autotuner times schedules and ef-class splits on the batch (fp16 tables with their row scales);
    # whatever it picks, the results are the untuned ones
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd.batched import BatchedSearcher
    w, ix, gix, db, q = c1
    ef = np.where(np.arange(w.nq) % 4 == 0, 200, 24).astype(np.int32)
    bs = BatchedSearcher(gix, w.nq, 200, 32, 10, precision=precision)
    bs.set_inputs(q, ef)
    ref_ids, ref_d = (t.cpu().numpy() for t in bs.run())
    cands = [lc.schedule(), lc.schedule(hash_bits=9, prefetch=0), lc.schedule(pool=1)]
    bs.tune(cands=cands, reps=1, cache_path=None)
    assert len(bs.table) >= len(cands)
    bs.capture()
    for _ in range(2):
        ids, d = bs.run()
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), ref_ids)
        assert np.array_equal(d.cpu().numpy().view(np.uint32), ref_d.view(np.uint32))


def test_large_projection_reads_P_from_global(torch):
    # d 200 -> d_pad 256: P (256 x 200) and a block of queries exceed one CU's LDS, so the batch projection
    # reads P from global memory, and the refinement its centroids; the path is still the oracle's
    import paper_1804_09996_amd as lc
    w = datagen.small(name="gpu-bigp", n=1200, nq=16, d=200, m=16, d_pad=256, n_train=1024, n_beta=8,
                      n_beta_train=1200, ef=32, shortlist=32, topk=10)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    assert ix.proj.shape == (256, 200)
    gix = lc.Index.from_index(ix)
    qp = gix.project(torch.from_numpy(q)).cpu().numpy()
    ref = np.stack([oracle.project(ix.proj, y, ix.d_pad) for y in q])
    np.testing.assert_allclose(qp, ref, rtol=0, atol=1e-5 * np.abs(ref).max())
    # tables from the projected batch and the walk: the oracle's short-lists
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    lut, _ = gix.build_lut(torch.from_numpy(qp), projected=True)
    assert np.all(np.abs(lut.cpu().numpy() - np.stack([ix.lut(y) for y in q])) <= _lut_bound(ix, q))
    r = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist)
    same = np.mean([np.array_equal(r.cand_ids.cpu().numpy()[i], o["cand_ids"][i]) for i in range(w.nq)])
    assert same == 1.0
    # the centroids (d_pad x 256 floats = 256 KB) do not fit LDS: the refinement reads them from global memory
    ids, d, _ = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()
