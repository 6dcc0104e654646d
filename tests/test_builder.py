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


# ---------------------------------------------------------------------------
# learned rotation ahead of PQ (OPQ; the codec of Sec. 4.1 / Sec. 5.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,D", [(12, 12), (12, 16), (40, 48)])
def test_procrustes_is_the_svd_closed_form(d, D):
    # argmax over P with orthonormal columns of tr(P S) = V U^T for S = U Sigma V^T
    rs = np.random.default_rng(d * 100 + D)
    S = rs.standard_normal((d, D))
    P = builder.procrustes(S)
    U, s, Vt = np.linalg.svd(S, full_matrices=False)
    np.testing.assert_allclose(P, Vt.T @ U.T, atol=1e-10)
    np.testing.assert_allclose(P.T @ P, np.eye(d), atol=1e-10)
    # and no rotation nearby does better
    for _ in range(5):
        Q, _ = np.linalg.qr(P + 1e-3 * rs.standard_normal(P.shape))
        assert np.trace(Q @ S) <= np.trace(P @ S) + 1e-9


def test_opq_lowers_distortion_and_is_thread_independent():
    w = datagen.small(name="opq-b", n=2000, d=32, m=8, n_train=4096)
    train = datagen.vectors(w, "train")
    init = datagen.pq_init_ids(w, train.shape[0])
    p1, h1 = builder.opq_train(train, w.d_pad, w.m, None, init, 5, 4, nthreads=1)
    p7, h7 = builder.opq_train(train, w.d_pad, w.m, None, init, 5, 4, nthreads=7)
    assert np.array_equal(p1, p7) and np.array_equal(h1, h7)
    assert np.all(np.diff(h1) <= 1e-6 * h1[0]), h1  # PQ steps and rotation steps never raise the distortion
    assert h1[-1] < 0.95 * h1[0]
    np.testing.assert_allclose(p1.T.astype(np.float64) @ p1, np.eye(32), atol=1e-5)
    # from a padded start (d 44 -> d_pad 48 through the seeded projection)
    wp = datagen.small(name="opq-p", n=2000, d=44, m=8, n_train=4096)
    tp = datagen.vectors(wp, "train")
    pp, hp = builder.opq_train(tp, wp.d_pad, wp.m, datagen.projection(wp), datagen.pq_init_ids(wp, tp.shape[0]), 4, 4)
    assert pp.shape == (48, 44) and np.all(np.diff(hp) <= 1e-6 * hp[0])
    np.testing.assert_allclose(pp.T.astype(np.float64) @ pp, np.eye(44), atol=1e-5)


def test_builder_with_learned_rotation_matches_oracle(nthreads):
    # the rotation is learned by the builder; given it, the rest of the build is the oracle's
    w = datagen.small(name="opq-build", n=1500, d=32, m=8, n_train=2048, n_beta=8, n_beta_train=1500, opq_iters=3)
    bix, db, q = builder.build_workload(w, nthreads=nthreads)
    assert bix.proj is not None and bix.proj.shape == (32, 32)
    oix = oracle.build_index(w, db, datagen.vectors(w, "train"), bix.proj, datagen.level_uniforms(w),
                             datagen.pq_init_ids(w, w.n_train), datagen.beta_train_ids(w),
                             datagen.beta_init_ids(w, min(w.n, w.n_beta_train)), nthreads)
    assert np.array_equal(bix.codes, oix.codes)
    assert np.all(bix.adj0 == oix.adj0, axis=1).mean() >= 0.999
    np.testing.assert_allclose(bix.centroids, oix.centroids, rtol=1e-6, atol=1e-7)
    assert (bix.beta_idx == oix.beta_idx).mean() >= 0.999


def test_builder_two_level_codec_matches_oracle(nthreads):
    # 2-level residual codec (Sec. 5.1): a first level of 2 x 32 centroids, PQ on the residual
    w = datagen.small(name="coarse-b", n=1500, d=32, m=8, n_beta=8, n_beta_train=1500, coarse_k=32)
    bix, _, _ = builder.build_workload(w, nthreads=nthreads)
    oix, _, _ = oracle.build_workload(w, nthreads=nthreads)
    assert bix.coarse_cent.shape == oix.coarse_cent.shape == (2, 32, 16)
    np.testing.assert_allclose(bix.coarse_cent, oix.coarse_cent, rtol=1e-6, atol=1e-7)
    assert np.array_equal(bix.coarse_codes, oix.coarse_codes)
    np.testing.assert_allclose(bix.centroids, oix.centroids, rtol=1e-5, atol=1e-6)
    assert (bix.codes == oix.codes).mean() >= 0.999
    np.testing.assert_allclose(bix.coarse_norm, oix.coarse_norm, rtol=1e-5, atol=1e-5)
    assert np.all(bix.adj0 == oix.adj0, axis=1).mean() >= 0.99
    np.testing.assert_allclose(bix.beta, oix.beta, rtol=1e-3, atol=1e-4)
    assert (bix.beta_idx == oix.beta_idx).mean() >= 0.99
