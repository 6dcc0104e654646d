"""The host index builder of the package against the oracle's builder (CPU).

Both follow the same procedure from the paper (PQ k-means, levels, batched
graph build with the shrinking heuristic, regression codebook) but share no
code: the builder works in float32 with per-sub-space tables, the oracle in
float64 directly.  On these workloads every integer output is identical and
the float32 parameters agree bit for bit, which is what lets the larger
benchmark indexes come from the fast builder.
"""
import numpy as np
import pytest

import datagen
import oracle
from paper_1804_09996_amd import builder


def _compare(w, nthreads):
    bix, db, q = builder.build_workload(w, nthreads=nthreads)
    oix, _, _ = oracle.build_workload(w, nthreads=nthreads)
    assert np.array_equal(bix.codes, oix.codes)
    assert np.array_equal(bix.level, oix.level)
    assert (bix.entry, bix.max_level) == (oix.entry, oix.max_level)
    assert np.array_equal(bix.up_base, oix.up_base)
    assert np.array_equal(bix.adj_up, oix.adj_up)
    same_rows = np.all(bix.adj0 == oix.adj0, axis=1).mean()
    assert same_rows >= 0.999, same_rows
    np.testing.assert_allclose(bix.centroids, oix.centroids, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(bix.beta, oix.beta, rtol=1e-4, atol=1e-5)
    assert (bix.beta_idx == oix.beta_idx).mean() >= 0.999


def test_builder_matches_oracle_tiny(nthreads):
    _compare(datagen.small(), nthreads)


def test_builder_matches_oracle_c1(nthreads):
    _compare(datagen.C1, nthreads)


def test_builder_with_projection(nthreads):
    w = datagen.small(name="proj-b", n=1500, d=20, m=8, d_pad=24, n_train=1024, n_beta=8, n_beta_train=1500)
    _compare(w, nthreads)


def test_builder_product_codebook_matches_oracle(nthreads):
    # product regression codebook (Sec. 4.3, Eq. 9): 4 blocks of 2 sub-spaces
    w = datagen.small(name="prod-b", n=1500, d=32, m=8, n_beta=8, n_beta_train=1500, m_beta=4)
    bix, _, _ = builder.build_workload(w, nthreads=nthreads)
    oix, _, _ = oracle.build_workload(w, nthreads=nthreads)
    assert bix.beta.shape == oix.beta.shape == (4, 8, w.k_reg + 1)
    assert bix.beta_idx.shape == oix.beta_idx.shape == (w.n, 4)
    assert bix.m_beta == oix.m_beta == 4
    assert np.all(bix.adj0 == oix.adj0, axis=1).mean() >= 0.999
    np.testing.assert_allclose(bix.beta, oix.beta, rtol=1e-4, atol=1e-5)
    assert (bix.beta_idx == oix.beta_idx).mean() >= 0.999


def test_builder_is_thread_count_independent():
    w = datagen.small(name="threads", n=1200)
    a, _, _ = builder.build_workload(w, nthreads=1)
    b, _, _ = builder.build_workload(w, nthreads=7)
    for name in ("codes", "adj0", "adj_up", "beta", "beta_idx"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name


def test_index_cache_roundtrip(tmp_path):
    w = datagen.small(name="cache", n=700, n_beta=8, n_beta_train=700)
    a, _, _ = builder.build_workload(w, nthreads=2, cache_dir=str(tmp_path))
    b, _, _ = builder.build_workload(w, nthreads=2, cache_dir=str(tmp_path))
    for name in ("codes", "adj0", "up_base", "adj_up", "beta", "beta_idx", "centroids"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    assert (a.entry, a.max_level) == (b.entry, b.max_level)
