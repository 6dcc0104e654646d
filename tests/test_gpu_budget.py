"""Budget T on distance computations (Sec. 3.1) on the GPU against the oracle.

With max_evals = T a query's level-0 walk ends right after its T-th distance
evaluation: D = min(T, unbounded D), the links of that last expansion past
the budget are not evaluated, and the short-list is the best S of the pool at
that point.  The oracle's capped walk is pinned on the CPU
(tests/test_oracle.py); here every walk kernel (pool in registers, pool in
LDS, bitset visited set with an LDS cache, each in its dual-expansion or
single-expansion form) must give its short-list, E and D bit for bit.
"""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

# default (registers), pool in LDS, bitset + LDS cache, no prefetch with a small table
SCHEDULES = [None,
             dict(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, pool=1),
             dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=1, visited=1),
             dict(hash_bits=9, prefetch=0, waves_per_cu=0, queue=0, visited=0),
             dict(hash_bits=9, prefetch=1, waves_per_cu=0, queue=1, visited=0, codes=1)]
BUDGETS = [1, 2, 31, 32, 33, 100, 517, 4000]


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


@pytest.mark.parametrize("si", range(len(SCHEDULES)))
def test_budget_walk_matches_oracle(c1, torch, si):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    sc = None if SCHEDULES[si] is None else lc.schedule(**SCHEDULES[si])
    lut, _ = gix.build_lut(torch.from_numpy(q))
    free = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist, sched=sc)
    free_d = free.stats.cpu().numpy()[:, 1]
    for T in BUDGETS:
        o = ix.search(q, w.ef, w.shortlist, w.topk, max_evals=T)
        r = gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist, sched=sc, max_evals=T)
        ids, n, st = r.cand_ids.cpu().numpy(), r.cand_n.cpu().numpy(), r.stats.cpu().numpy()
        assert np.array_equal(st[:, 1], np.minimum(T, free_d)), T  # D = min(T, unbounded D)
        same = [np.array_equal(ids[i], o["cand_ids"][i]) and n[i] == o["cand_n"][i] and
                np.array_equal(st[i], o["stats"][i]) for i in range(w.nq)]
        print(f"schedule {si} T {T}: identical to the oracle on {sum(same)}/{w.nq}")
        assert np.mean(same) == 1.0, T
        ws = gix.workspace(q.shape[0], w.ef, w.shortlist, sc)
        assert int(ws.count_nonzero().item()) == 0, "workspace not left zeroed"


def test_budget_full_path_and_no_op(c1, torch):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    qt = torch.from_numpy(q)
    T = 150
    ids, d, _ = gix.query(qt, ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, max_evals=T)
    o = ix.search(q, w.ef, w.shortlist, w.topk, max_evals=T)
    s = parity.summarize(ix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    # a budget above every query's D is no budget at all
    a_ids, a_d, a_r = gix.query(qt, ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    big = int(a_r.stats[:, 1].max().item())
    b_ids, b_d, b_r = gix.query(qt, ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True, max_evals=big)
    assert np.array_equal(a_ids.cpu().numpy(), b_ids.cpu().numpy())
    assert np.array_equal(a_d.cpu().numpy().view(np.uint32), b_d.cpu().numpy().view(np.uint32))
    assert np.array_equal(a_r.stats.cpu().numpy(), b_r.stats.cpu().numpy())
    # fp16 tables under a budget: D is still min(T, unbounded D of the fp16 walk)
    lut16, sc16 = gix.build_lut(qt, lc.LC_LUT_F16)
    f16 = gix.search(lut16, sc16, ef=w.ef, ef_max=w.ef, S=w.shortlist)
    c16 = gix.search(lut16, sc16, ef=w.ef, ef_max=w.ef, S=w.shortlist, max_evals=40)
    assert np.array_equal(c16.stats.cpu().numpy()[:, 1], np.minimum(40, f16.stats.cpu().numpy()[:, 1]))


def test_negative_budget_is_rejected(c1, torch):
    import paper_1804_09996_amd as lc
    w, ix, gix, db, q = c1
    lut, _ = gix.build_lut(torch.from_numpy(q[:4]))
    with pytest.raises(lc.LCError) as e:
        gix.search(lut, ef=w.ef, ef_max=w.ef, S=w.shortlist, max_evals=-1)
    assert e.value.code == lc.LC_EINVAL
