"""The walk with the query's fp16 table in the wave's registers (schedule
table = 2, walk_rl_kernel) against the same walk with the table in LDS
(table = 1): every output bit for bit (short-lists, their ADC keys, lengths,
E and D), on the pool sizes, sub-space counts, per-query ef, budgets and
overflow cases of the LDS-pool walk, with the workspace left zero-filled;
also with the codes fetched after the visited probe (codes = 1); the fp16
keys against their definition; the fp16 walks against the oracle's walk on
the same table values; the plan lc_walk_describe reports."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


_BUILT = {}


def _index(m, n=3000, d=None, **kw):
    from paper_1804_09996_amd import builder
    key = (m, n, d)
    if key not in _BUILT:
        dd = d or (96 if m in (16, 32, 48) else 112 if m == 56 else 32)
        w = datagen.small(name=f"rl-m{m}-{n}", n=n, nq=40, d=dd, m=m, k_reg=8, n_beta=16, n_train=4096,
                          n_beta_train=min(n, 3000), pq_iters=5, beta_kmeans_iters=3, em_iters=2, **kw)
        ix, db, q = builder.build_workload(w, nthreads=8)
        _BUILT[key] = (w, ix, q)
    return _BUILT[key]


def _run(gix, lut, sc, ef, ef_max, S, sched, max_evals=0):
    r = gix.search(lut, sc, ef=ef, ef_max=ef_max, S=S, sched=sched, max_evals=max_evals)
    return (r.cand_ids.cpu().numpy(), r.cand_adc.cpu().numpy().view(np.uint32), r.cand_n.cpu().numpy(),
            r.stats.cpu().numpy())


def _same(a, b, what):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), what


@pytest.mark.parametrize("m", [8, 16, 32, 56])
def test_register_table_equals_lds_table(torch, m):
    import paper_1804_09996_amd as lc
    w, ix, q = _index(m)
    gix = lc.Index.from_index(ix)
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    rng = np.random.default_rng(m)
    per_q = torch.from_numpy(rng.integers(1, 301, q.shape[0]).astype(np.int32))
    cases = [(1, 1, 1), (16, 16, 16), (64, 64, 8), (129, 129, 32), (200, 200, 100), (256, 256, 64),
             (300, 300, 300), (per_q, 300, 32)]
    for ef, ef_max, S in cases:
        for extra in (dict(), dict(hash_bits=9, prefetch=0), dict(queue=0, hash_bits=12), dict(codes=1),
                      dict(hash_bits=9, codes=1)):
            a = _run(gix, lut, sc, ef, ef_max, S, lc.schedule(pool=1, table=1, **extra))
            b = _run(gix, lut, sc, ef, ef_max, S, lc.schedule(pool=1, table=2, **extra))
            _same(a, b, (m, ef_max, S, extra))
            for t in (1, 2):
                sch = lc.schedule(pool=1, table=t, **extra)
                assert int(gix.workspace(q.shape[0], ef_max, S, sch).count_nonzero().item()) == 0
    # the automatic choice (registers at m = 56 with an LDS pool) and the register pool give the same walks
    for ef, S in ((200, 32), (100, 16)):
        _same(_run(gix, lut, sc, ef, ef, S, lc.schedule(pool=1, table=1)),
              _run(gix, lut, sc, ef, ef, S, lc.schedule()), (m, ef, S, "auto"))
    gix.close()


@pytest.mark.parametrize("max_evals", [1, 2, 31, 33, 100, 517])
def test_register_table_with_a_budget(torch, max_evals):
    import paper_1804_09996_amd as lc
    w, ix, q = _index(56)
    gix = lc.Index.from_index(ix)
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    a = _run(gix, lut, sc, 256, 256, 64, lc.schedule(pool=1, table=1), max_evals)
    b = _run(gix, lut, sc, 256, 256, 64, lc.schedule(pool=1, table=2), max_evals)
    _same(a, b, max_evals)
    _same(a, _run(gix, lut, sc, 256, 256, 64, lc.schedule(pool=1, table=2, codes=1), max_evals), max_evals)
    assert np.all(b[3][:, 1] <= max_evals)
    gix.close()


def test_register_table_overflow_and_exhaustive(torch):
    # ef = N on a graph of 2400 nodes with a 512-word visited table: most of the walk runs on the bitset
    import paper_1804_09996_amd as lc
    w, ix, q = _index(56, n=2400)
    gix = lc.Index.from_index(ix)
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    for extra in (dict(hash_bits=9), dict(hash_bits=9, wide=1), dict(hash_bits=9, codes=1)):
        a = _run(gix, lut, sc, 2400, 2400, 64, lc.schedule(pool=1, table=1, **extra))
        b = _run(gix, lut, sc, 2400, 2400, 64, lc.schedule(pool=1, table=2, **extra))
        _same(a, b, extra)
        assert np.all(b[3][:, 1] == 2399)
        assert int(gix.workspace(q.shape[0], 2400, 64, lc.schedule(pool=1, table=2, **extra))
                   .count_nonzero().item()) == 0
    gix.close()


def test_register_table_on_a_float32_table_is_the_lds_walk(torch):
    # the register form holds fp16 tables only: a float32 table with table = 2 walks as with table = 1
    import paper_1804_09996_amd as lc
    w, ix, q = _index(56)
    gix = lc.Index.from_index(ix)
    lut, _ = gix.build_lut(torch.from_numpy(q))
    _same(_run(gix, lut, None, 200, 200, 32, lc.schedule(pool=1, table=1)),
          _run(gix, lut, None, 200, 200, 32, lc.schedule(pool=1, table=2)), "f32")
    gix.close()


@pytest.mark.parametrize("table", [1, 2])
def test_fp16_keys_follow_their_definition(torch, table):
    # every short-list key of an fp16 walk, recomputed on the host from the table lc_build_lut wrote: each
    # entry times its row's scale (exact), summed in float32 in sub-space order
    import paper_1804_09996_amd as lc
    w, ix, q = _index(56)
    gix = lc.Index.from_index(ix)
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    L = lut.cpu().numpy().view(np.float16).reshape(q.shape[0], w.m, 256).astype(np.float32)
    rs = sc.cpu().numpy().astype(np.float32)
    r = gix.search(lut, sc, ef=64, ef_max=64, S=16, sched=lc.schedule(pool=1, table=table))
    ids, adc, n = r.cand_ids.cpu().numpy(), r.cand_adc.cpu().numpy(), r.cand_n.cpu().numpy()
    codes = np.asarray(ix.codes)
    assert len(set(rs.ravel().tolist())) > 1, "rows with different scales"
    for i in range(q.shape[0]):
        for j in range(n[i]):
            c = codes[ids[i, j]]
            acc = np.float32(0.0)
            for s in range(w.m):
                acc = np.float32(acc + np.float32(L[i, s, c[s]] * rs[i, s]))
            assert acc.view(np.uint32) == np.float32(adc[i, j]).view(np.uint32), (i, j)
    gix.close()


def test_walk_plan_names_the_kernel(torch):
    # lc_walk_describe: the kernel the schedule rules pick, without launching it
    import paper_1804_09996_amd as lc
    w, ix, q = _index(56)
    gix = lc.Index.from_index(ix)
    f16, f32 = lc.LC_LUT_F16, lc.LC_LUT_F32
    p = gix.walk_plan(10_000, 256, 32, f16)
    assert p["kernel"] == "walk_rl_kernel<56, false>" and p["slots_per_cu"] == 8 and p["hash_bits"] == 12
    assert gix.walk_plan(10_000, 64, 32, f16)["kernel"] == "walk_rl_kernel<56, false>"
    assert gix.walk_plan(10_000, 64, 32, f16, lc.schedule(table=1))["kernel"] == "walk_reg_kernel<56, __half, 2, false>"
    assert gix.walk_plan(10_000, 256, 32, f16, lc.schedule(table=1))["kernel"] == "walk_kernel<56, __half, false>"
    assert gix.walk_plan(10_000, 64, 32, f32)["kernel"] == "walk_reg_kernel<56, float, 2, false>"
    assert gix.walk_plan(10_000, 256, 32, f32, lc.schedule(table=2))["kernel"] == "walk_kernel<56, float, false>"
    assert gix.walk_plan(10_000, 256, 32, f32, lc.schedule(visited=1))["kernel"] == "walk_cache_kernel<56, float, false>"
    assert gix.walk_plan(5, 256, 32, f16)["grid"] == 5  # never more slots than queries
    with pytest.raises(lc.LCError):
        gix.walk_plan(10, 64, 32, f16, lc.schedule(table=3))
    gix.close()
    # m = 32, pool 128: the register pool with the table in LDS keeps 8 slots per CU only with a 2^10-word
    # visited table; the table in registers keeps as many with 2^12 words and is taken
    w, ix, q = _index(32)
    gix = lc.Index.from_index(ix)
    p = gix.walk_plan(10_000, 128, 32, f16)
    assert p["kernel"] == "walk_rl_kernel<32, false>" and p["hash_bits"] == 12 and p["slots_per_cu"] == 8, p
    p = gix.walk_plan(10_000, 128, 32, f16, lc.schedule(table=1))
    assert p["kernel"] == "walk_reg_kernel<32, __half, 2, false>" and p["hash_bits"] == 10, p
    gix.close()
    # m = 16: the register pool with the table in LDS up to a pool of 128; beyond, the table in registers with
    # the visited table that keeps all 12 slots its registers allow (2^11 words)
    w, ix, q = _index(16)
    gix = lc.Index.from_index(ix)
    assert gix.walk_plan(10_000, 128, 32, f16)["kernel"] == "walk_reg_kernel<16, __half, 2, false>"
    p = gix.walk_plan(10_000, 256, 32, f16)
    assert p["kernel"] == "walk_rl_kernel<16, false>" and p["hash_bits"] == 11 and p["slots_per_cu"] == 12, p
    p = gix.walk_plan(10_000, 128, 32, f16, lc.schedule(table=2))
    assert p["hash_bits"] == 11 and p["slots_per_cu"] == 12, p
    gix.close()


def _oracle_view(ix):
    import oracle
    return oracle.Index(n=ix.n, d=ix.d, d_pad=ix.d_pad, m=ix.m, deg0=ix.deg0, deg_up=ix.deg_up, k_reg=ix.k_reg,
                        n_beta=ix.n_beta, entry=ix.entry, max_level=ix.max_level, proj=ix.proj, centroids=ix.centroids,
                        codes=ix.codes, adj0=ix.adj0, level=ix.level, up_base=ix.up_base, adj_up=ix.adj_up,
                        beta=ix.beta, beta_idx=ix.beta_idx, m_beta=ix.m_beta)


@pytest.mark.parametrize("m,table", [(16, 1), (16, 2), (32, 0), (56, 1), (56, 2), (56, 0)])
def test_fp16_walk_is_the_walk_on_its_table(torch, m, table):
    # the fp16 walk against the oracle's walk (Sec. 2: descent, best-first walk, short-list) on the same table
    # values (each fp16 entry times its row scale, exact in float64): short-lists, their lengths, E and D
    # identical on every query; keys within the float32 rounding of their m-term sums
    import paper_1804_09996_amd as lc
    w, ix, q = _index(m)
    gix = lc.Index.from_index(ix)
    lut, sc = gix.build_lut(torch.from_numpy(q), lc.LC_LUT_F16)
    tabs = (lut.cpu().numpy().view(np.float16).reshape(q.shape[0], m, 256).astype(np.float64)
            * sc.cpu().numpy().astype(np.float64)[:, :, None])
    oix = _oracle_view(ix)
    rng = np.random.default_rng(m + table)
    for ef, S in ((16, 16), (64, 16), (200, 32), (rng.integers(1, 257, q.shape[0]).astype(np.int32), 32)):
        ef_max = int(np.max(ef))
        o = oix.walk_tables(tabs, ef, S, nthreads=8)
        r = gix.search(lut, sc, ef=ef, ef_max=ef_max, S=S, sched=lc.schedule(table=table))
        ids, adc = r.cand_ids.cpu().numpy(), r.cand_adc.cpu().numpy().astype(np.float64)
        assert np.array_equal(ids, o["cand_ids"]), (ef_max, S)
        assert np.array_equal(r.cand_n.cpu().numpy(), o["cand_n"]) and np.array_equal(r.stats.cpu().numpy(), o["stats"])
        ok = ids >= 0
        bound = m * 2.0 ** -24 * np.abs(o["cand_adc"][ok]) + 1e-30
        assert np.all(np.abs(adc[ok] - o["cand_adc"][ok]) <= bound), (ef_max, S)
    gix.close()
