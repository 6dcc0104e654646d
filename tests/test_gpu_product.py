"""Product regression codebook (Sec. 4.3, Eq. 9) on the GPU against the oracle.

The coordinates are cut into m_beta blocks of m / m_beta whole sub-spaces and
block jb of the refined vector takes its weights from codebook jb at the
vector's byte beta_idx[i][jb].  Indexes are built by the oracle; the product
codebooks are either drawn at random (every block and byte distinct, which
catches a wrong block or a transposed layout) or trained by the oracle.  Bars
as in test_gpu_parity: top-K EXACT on every query, every returned distance
within 1e-5 relative of the oracle's float64 refined distance.
"""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle
from tests import parity

pytestmark = pytest.mark.gpu

# (m, d) -> the specialised refine kernels (dsub 4, 6, 4, 2) and one shape
# that only the generic kernel covers (m 24, dsub 2)
SHAPES = {8: 32, 16: 96, 32: 128, 56: 112, 24: 48}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


_built = {}


def _base(m):
    if m not in _built:
        d = SHAPES[m]
        w = datagen.small(name=f"prod-{m}", n=1500, nq=24, d=d, m=m, n_train=1024, n_beta=8, n_beta_train=1500,
                          k_reg=6, ef=40, shortlist=48, topk=10)
        ix, db, q = oracle.build_workload(w, nthreads=4)
        _built[m] = (w, ix, db, q)
    return _built[m]


def _random_product(ix, mb, n_beta, seed):
    rs = np.random.default_rng(seed)
    B = (0.2 * rs.standard_normal((mb, n_beta, ix.k_reg + 1))).astype(np.float32)
    B[:, :, 0] += 0.9
    bidx = rs.integers(0, n_beta, (ix.n, mb)).astype(np.uint8)
    return dataclasses.replace(ix, beta=B, beta_idx=bidx, n_beta=n_beta, m_beta=mb)


def _oracle_topk(ixp, q, cand_ids, cand_n, K):
    """The oracle's refinement of a given short-list: float64 refined distance
    of every candidate (Eq. 5 / Eq. 9), then the K smallest (distance, id)."""
    ids = np.full((q.shape[0], K), -1, np.int32)
    d = np.full((q.shape[0], K), np.inf)
    for i in range(q.shape[0]):
        c = cand_ids[i, :max(int(cand_n[i]), 0)]
        dd = np.array([ixp.refined_distance(q[i], int(x)) for x in c])
        order = np.lexsort((c, dd))[:K]
        ids[i, :order.size] = c[order]
        d[i, :order.size] = dd[order]
    return {"ids": ids, "d": d}


def _check(ixp, q, w, torch, precisions=("f32", "f16")):
    import paper_1804_09996_amd as lc
    gix = lc.Index.from_index(ixp)
    o = ixp.search(q, w.ef, w.shortlist, w.topk)
    for prec in precisions:
        ids, d, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, precision=prec,
                              stats=True)
        cand, cn = r.cand_ids.cpu().numpy(), r.cand_n.cpu().numpy()
        same_walk = np.mean([np.array_equal(cand[i], o["cand_ids"][i]) for i in range(q.shape[0])])
        if prec == "f32":  # the walk does not read beta (the fp16 table walks its own way)
            assert same_walk == 1.0
        ref = _oracle_topk(ixp, q, cand, cn, w.topk)
        s = parity.summarize(ixp, q, ids.cpu().numpy(), d.cpu().numpy(), ref)
        print(f"m {ixp.m} m_beta {ixp.m_beta} {prec}: walk {same_walk:.2f} EXACT {s['exact_frac']:.3f} "
              f"max rel err {s['max_rel_err']:.1e}")
        assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()


@pytest.mark.parametrize("m", [8, 16, 32, 56])
@pytest.mark.parametrize("mb", [2, 4, 8])
def test_random_product_codebook_matches_oracle(torch, m, mb):
    w, ix, db, q = _base(m)
    _check(_random_product(ix, mb, 5, seed=100 * m + mb), q, w, torch)


def test_single_block_layouts_agree(torch):
    # m_beta = 1 given as [1, n_beta, k+1] / [n, 1] is the plain codebook
    import paper_1804_09996_amd as lc
    w, ix, db, q = _base(16)
    ix3 = dataclasses.replace(ix, beta=ix.beta[None], beta_idx=ix.beta_idx[:, None], m_beta=1)
    a = lc.Index.from_index(ix)
    b = lc.Index.from_index(ix3)
    ia, da, _ = a.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    ib, dbb, _ = b.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    assert np.array_equal(ia.cpu().numpy(), ib.cpu().numpy())
    assert np.array_equal(da.cpu().numpy().view(np.uint32), dbb.cpu().numpy().view(np.uint32))


def test_trained_product_codebook_matches_oracle(torch):
    w, ix, db, q = _base(16)
    ids = datagen.beta_train_ids(w)
    init = datagen.beta_init_ids(w, ids.size)
    B, _ = oracle.beta_train(db, ids, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, ix.k_reg, 8, init, 5, 3,
                             nthreads=4, m_beta=8)
    bidx = oracle.beta_assign(db, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, ix.k_reg, B, nthreads=4)
    _check(dataclasses.replace(ix, beta=B, beta_idx=bidx, n_beta=8, m_beta=8), q, w, torch)


@pytest.mark.parametrize("m,mb", [(24, 3), (16, 16)])
def test_generic_kernel_block_counts(torch, m, mb):
    # shapes or block counts without a specialised kernel take the generic
    # float32 kernel; the precision form needs a specialised one
    import paper_1804_09996_amd as lc
    w, ix, db, q = _base(m)
    ixp = _random_product(ix, mb, 4, seed=7 * m + mb)
    _check(ixp, q, w, torch, precisions=("f32",))
    gix = lc.Index.from_index(ixp)
    with pytest.raises(lc.LCError):
        gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, precision="f16+bf16")
    gix.close()


@pytest.mark.parametrize("m", [16, 24])
def test_out_of_range_block_byte_drops_the_candidate(torch, m):
    # a codebook byte >= n_beta in any block makes that vector no candidate
    import paper_1804_09996_amd as lc
    w, ix, db, q = _base(m)
    mb = 4 if m == 16 else 3
    ixp = _random_product(ix, mb, 5, seed=3)
    bad = np.arange(0, ix.n, 7)
    bidx = ixp.beta_idx.copy()
    bidx[bad, bad % mb] = 5
    gix = lc.Index.from_index(dataclasses.replace(ixp, beta_idx=bidx))
    ids, d, _ = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    ids = ids.cpu().numpy()
    assert not np.isin(ids, bad).any()
    # every other short-list entry is still refined exactly as the valid index does
    good = lc.Index.from_index(ixp)
    gi, gd, _ = good.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    d = d.cpu().numpy()
    for i in range(q.shape[0]):
        keep = [(a, b) for a, b in zip(gi[i], gd[i]) if a >= 0 and a not in set(bad.tolist())]
        got = [(a, b) for a, b in zip(ids[i], d[i]) if a >= 0]
        assert got[:len(keep)] == keep[:len(got)]
    gix.close()
    good.close()
