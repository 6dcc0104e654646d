"""Pins of the oracle's 2-level residual codec (Sec. 3.3 residual codecs; Sec. 5.1:
a first-level product quantizer over the two halves of the vector, whose
residual the PQ codes encode).  CPU only; every expected value is computed
here in plain numpy from the index arrays, or is a special case that reduces
to the one-level codec.
"""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle


@pytest.fixture(scope="module")
def coarse_build():
    w = datagen.small(name="coarse", coarse_k=16)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    return w, ix, db, q


def proj_np(ix, y):
    y = np.asarray(y, np.float64)
    return y if ix.proj is None else ix.proj.astype(np.float64) @ y


def first_level(ix) -> np.ndarray:
    h = ix.d_pad // 2
    c = np.empty((ix.n, ix.d_pad), np.float64)
    for half in range(2):
        c[:, half * h:(half + 1) * h] = ix.coarse_cent[half][ix.coarse_codes[:, half]]
    return c


def second_level(ix) -> np.ndarray:
    dsub = ix.d_pad // ix.m
    r = np.empty((ix.n, ix.d_pad), np.float64)
    for s in range(ix.m):
        r[:, s * dsub:(s + 1) * dsub] = ix.centroids[s][ix.codes[:, s]]
    return r


def test_coarse_encode_is_bruteforce_argmin():
    rs = np.random.default_rng(3)
    d, k = 10, 7
    x = rs.standard_normal((200, d)).astype(np.float32)
    proj = np.linalg.qr(rs.standard_normal((d, d)))[0].astype(np.float32)
    cent = rs.standard_normal((2, k, d // 2)).astype(np.float32)
    codes, resid = oracle.coarse_encode(x, proj, d, cent)
    xp = x.astype(np.float64) @ proj.astype(np.float64).T
    for half in range(2):
        part = xp[:, half * 5:(half + 1) * 5]
        dist = ((part[:, None, :] - cent[half][None].astype(np.float64)) ** 2).sum(-1)
        best = dist.argmin(1)
        assert np.array_equal(codes[:, half], best)
        np.testing.assert_allclose(resid[:, half * 5:(half + 1) * 5], part - cent[half][best], rtol=0, atol=1e-6)


def test_coarse_encode_ties_take_the_lower_index():
    x = np.zeros((3, 4), np.float32)
    cent = np.zeros((2, 5, 2), np.float32)  # all centroids equal: every entry ties
    codes, resid = oracle.coarse_encode(x, None, 4, cent)
    assert (codes == 0).all() and (resid == 0).all()


def test_two_level_walk_distance_is_the_reconstruction_distance(coarse_build):
    # the short-list's asymmetric distances are ||P y - (c + r)||^2 with both levels decoded here
    w, ix, db, q = coarse_build
    rec = first_level(ix) + second_level(ix)
    out = ix.search(q[:8], w.ef, w.shortlist, w.topk)
    for qi in range(8):
        yp = proj_np(ix, q[qi])
        for t in range(out["cand_n"][qi]):
            i = out["cand_ids"][qi, t]
            assert out["cand_adc"][qi, t] == pytest.approx(((yp - rec[i]) ** 2).sum(), rel=1e-12)


def test_coarse_norm_gives_the_decomposed_distance(coarse_build):
    # ||y - c - r||^2 = ||y^1 - c^1||^2 + ||y^2 - c^2||^2 - 2 sum_s <y^s, r^s> + norm
    w, ix, db, q = coarse_build
    c, r = first_level(ix), second_level(ix)
    h = ix.d_pad // 2
    for y in q[:4]:
        yp = proj_np(ix, y)
        direct = ((yp[None] - c - r) ** 2).sum(1)
        tables = ((yp[None, :h] - c[:, :h]) ** 2).sum(1) + ((yp[None, h:] - c[:, h:]) ** 2).sum(1)
        decomposed = tables - 2.0 * (r @ yp) + ix.coarse_norm.astype(np.float64)
        np.testing.assert_allclose(decomposed, direct, rtol=0, atol=1e-5 * direct.max())


def test_coarse_residual_codes_are_the_residual_pq(coarse_build):
    # the PQ codes are the nearest second-level centroids of P x - c
    w, ix, db, q = coarse_build
    c = first_level(ix)
    dsub = ix.d_pad // ix.m
    res = np.stack([proj_np(ix, x) for x in db[:300]]) - c[:300]
    for s in range(ix.m):
        part = res[:, s * dsub:(s + 1) * dsub]
        dist = ((part[:, None, :] - ix.centroids[s][None].astype(np.float64)) ** 2).sum(-1)
        assert np.mean(ix.codes[:300, s] == dist.argmin(1)) > 0.99  # the stored residual is rounded to f32


def test_zero_first_level_reduces_to_the_one_level_codec(tiny_build):
    # one first-level centroid at the origin: q(x) is the PQ reconstruction, so search is unchanged
    w, ix, db, q = tiny_build
    h = ix.d_pad // 2
    ixc = dataclasses.replace(ix, coarse_cent=np.zeros((2, 1, h), np.float32),
                              coarse_codes=np.zeros((ix.n, 2), np.uint16))
    a = ix.search(q, w.ef, w.shortlist, w.topk)
    b = ixc.search(q, w.ef, w.shortlist, w.topk)
    assert np.array_equal(a["cand_ids"], b["cand_ids"]) and np.array_equal(a["ids"], b["ids"])
    assert np.array_equal(a["stats"], b["stats"])
    np.testing.assert_allclose(b["d"], a["d"], rtol=1e-12)
    np.testing.assert_allclose(ixc.coarse_norms(), (second_level(ix) ** 2).sum(1), rtol=1e-6)


def test_two_level_refine_bruteforce(coarse_build):
    # x~ = sum_j beta_j (c(g_j) + r(g_j)), a -1 link a zero vector (Eq. 5 with the 2-level q)
    w, ix, db, q = coarse_build
    rec = first_level(ix) + second_level(ix)
    for y in q[:3]:
        yp = proj_np(ix, y)
        for i in range(0, ix.n, 97):
            G = np.stack([rec[i]] + [rec[g] if g >= 0 else np.zeros(ix.d_pad) for g in ix.adj0[i, :w.k_reg]], 1)
            xt = G @ ix.beta[ix.beta_idx[i]].astype(np.float64)
            assert ix.refined_distance(y, i) == pytest.approx(((yp - xt) ** 2).sum(), rel=1e-12)


def test_two_level_graph_lists_sorted_by_reconstruction_distance(coarse_build):
    # level-0 lists are ordered by ||x_i - q(x_j)||^2 with the 2-level q (Sec. 4.2)
    w, ix, db, q = coarse_build
    rec = first_level(ix) + second_level(ix)
    for i in range(0, ix.n, 53):
        row = ix.adj0[i][ix.adj0[i] >= 0]
        dd = ((proj_np(ix, db[i])[None] - rec[row]) ** 2).sum(1)
        assert np.all(np.diff(dd) >= -1e-9 * dd.max())


def test_two_level_beta_assignment_is_bruteforce_argmin(coarse_build):
    w, ix, db, q = coarse_build
    rec = first_level(ix) + second_level(ix)
    B = ix.beta.astype(np.float64)
    for i in range(0, ix.n, 61):
        G = np.stack([rec[i]] + [rec[g] if g >= 0 else np.zeros(ix.d_pad) for g in ix.adj0[i, :w.k_reg]], 1)
        loss = (((proj_np(ix, db[i])[:, None] - G @ B.T)) ** 2).sum(0)
        assert ix.beta_idx[i] == int(np.argmin(loss))


def test_two_level_codec_lowers_distortion(coarse_build, tiny_build):
    # same PQ size, a first level in front: the reconstruction error drops (Sec. 3.3, Table 1)
    w, ix, db, q = coarse_build
    w1, ix1, db1, _ = tiny_build
    assert w1.seed == w.seed and w1.d == w.d and w1.n == w.n
    xp = np.stack([proj_np(ix, x) for x in db])
    e2 = ((xp - first_level(ix) - second_level(ix)) ** 2).sum(1).mean()
    e1 = ((np.stack([proj_np(ix1, x) for x in db1]) - second_level(ix1)) ** 2).sum(1).mean()
    assert e2 < 0.9 * e1
