"""Regression-codebook assignment on the GPU (Sec. 4.3 Eq. 7; per block, Eq. 9)
against the oracle's assignment, through the C-ABI.

The arg-min is an integer decided by floating point; the kernel takes it in
float64 with the oracle's order of operations and no fused multiply-adds, so
the entries must be identical for every vector, not merely close.
"""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def test_assignment_matches_oracle_c1(c1_build, torch):
    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    gix = lc.Index.from_index(ix)
    got = gix.assign_beta(torch.from_numpy(db)).cpu().numpy()
    assert got.shape == (ix.n, 1)
    assert np.array_equal(got[:, 0], ix.beta_idx), int((got[:, 0] != ix.beta_idx).sum())
    # any sub-range, ragged, gives the same rows
    for n0, cnt in ((0, 1), (17, 63), (5000, 4999), (ix.n - 3, 3)):
        part = gix.assign_beta(torch.from_numpy(db[n0:n0 + cnt]), n0=n0).cpu().numpy()
        assert np.array_equal(part[:, 0], ix.beta_idx[n0:n0 + cnt])
    empty = gix.assign_beta(torch.zeros((0, w.d)), n0=ix.n)
    assert empty.shape == (0, 1)
    with pytest.raises(lc.LCError):
        gix.assign_beta(torch.from_numpy(db[:10]), n0=ix.n - 5)  # past the last vector
    gix.close()


def test_assignment_with_projection_and_product_codebook(torch):
    import paper_1804_09996_amd as lc
    # d 44 -> d_pad 48 through the orthonormal projection; product codebook of 4 blocks
    w = datagen.small(name="assign-proj", n=1800, nq=4, d=44, m=8, n_train=1024, n_beta=16, n_beta_train=1800,
                      k_reg=6, m_beta=4)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    assert ix.proj is not None and ix.beta.shape == (4, 16, 7) and ix.beta_idx.shape == (w.n, 4)
    gix = lc.Index.from_index(ix)
    got = gix.assign_beta(torch.from_numpy(db)).cpu().numpy()
    assert np.array_equal(got, ix.beta_idx), int((got != ix.beta_idx).sum())
    gix.close()
    # a single codebook on the same index: the oracle's assignment of it
    beta1, _ = oracle.beta_train(db, datagen.beta_train_ids(w), ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0,
                                 ix.k_reg, 16, datagen.beta_init_ids(w, w.n), 3, 2, nthreads=4)
    b1 = oracle.beta_assign(db, ix.proj, w.d_pad, ix.centroids, ix.codes, ix.adj0, ix.k_reg, beta1, nthreads=4)
    g1 = lc.Index.from_index(dataclasses.replace(ix, beta=beta1, beta_idx=b1, m_beta=1))
    got1 = g1.assign_beta(torch.from_numpy(db)).cpu().numpy()
    assert np.array_equal(got1[:, 0], b1)
    g1.close()
