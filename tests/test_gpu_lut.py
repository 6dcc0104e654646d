"""The table kernel (lc_build_lut) on batches large enough that one block
takes several 16-query groups, with a ragged last group and a ragged last
block: each query's table — float32, and fp16 with its row scales — is bit for
bit the one it gets in a batch of 13 (one group per block), with the
projection done by the kernel or beforehand; and the float32 tables of a
sample of queries, the last ones included, lie within the expansion bound of
the oracle's float64 table (Sec. 4.1), the fp16 ones within half an fp16 ulp
of it as well."""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

F32_EPS = 2.0 ** -24
_BUILT = {}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _workload(m, nq):
    # d 96: projected to 112 at m = 56 (sub-space width 2), unprojected at m = 16 (width 6)
    if m not in _BUILT:
        w = datagen.small(name=f"lut-m{m}", n=1500, nq=nq, d=96, m=m, k_reg=4, n_beta=8, n_train=4096,
                          n_beta_train=1500, pq_iters=4, beta_kmeans_iters=2, em_iters=1)
        ix, db, q = oracle.build_workload(w, nthreads=8)
        _BUILT[m] = (w, ix, q)
    return _BUILT[m]


def _bound(ix, Q):
    """Float32 error of the table: the expansion ||y' - mu||^2 + ||c - mu||^2 - 2 <y' - mu, c - mu>, and, with a
    projection, that of y' = P y itself (each coordinate a float32 sum of d products: |e_t| <= (d + 2) eps
    sum_u |P_tu y_u|), which moves an entry by at most 2 sum_t |y'_t - c_t| e_t + sum_t e_t^2 over its sub-space."""
    dsub = ix.d_pad // ix.m
    C = ix.centroids.astype(np.float64)
    mu = C.mean(1)
    nc = ((C - mu[:, None, :]) ** 2).sum(-1)
    out = []
    for y in Q:
        yp = oracle.project(ix.proj, y, ix.d_pad)
        b = 16 * F32_EPS * (((yp.reshape(ix.m, dsub) - mu) ** 2).sum(-1)[:, None] + nc) + 1e-30
        if ix.proj is not None:
            d = y.shape[0]
            e = ((d + 2) * F32_EPS * (np.abs(np.asarray(ix.proj, np.float64)) @ np.abs(y.astype(np.float64))))
            e = e.reshape(ix.m, dsub)
            diff = np.abs(yp.reshape(ix.m, 1, dsub) - C)
            b = b + 2 * (diff * e[:, None, :]).sum(-1) + (e ** 2).sum(-1)[:, None]
        out.append(b)
    return np.stack(out)


# batch sizes that give 4 groups per block at m = 56 (5000 queries) and m = 16 (20000), a partial last group
@pytest.mark.parametrize("m,nq", [(56, 5000), (16, 20003)])
def test_tables_do_not_depend_on_the_batch(torch, m, nq):
    import paper_1804_09996_amd as lc
    w, ix, q = _workload(m, nq)
    gix = lc.Index.from_index(ix)
    qd = torch.from_numpy(q).to(gix.device)
    qp = gix.project(qd) if gix.has_projection else qd
    for dt in (lc.LC_LUT_F32, lc.LC_LUT_F16):
        for x, proj in ((qd, False), (qp, True)):
            if proj and not gix.has_projection:
                continue
            full, fsc = gix.build_lut(x, dt, projected=proj)
            full = full.cpu().numpy()
            fsc = None if fsc is None else fsc.cpu().numpy()
            idx = np.r_[0:260, nq - 300:nq]  # first and last blocks
            for c0 in range(0, len(idx), 13):
                rows = idx[c0:c0 + 13]
                part, psc = gix.build_lut(x[torch.from_numpy(rows).to(gix.device)], dt, projected=proj)
                assert np.array_equal(part.cpu().numpy().view(np.uint8), full[rows].view(np.uint8)), (dt, proj, c0)
                if psc is not None:
                    assert np.array_equal(psc.cpu().numpy(), fsc[rows]), (dt, proj, c0)
    gix.close()


@pytest.mark.parametrize("m,nq", [(56, 5000), (16, 20003)])
def test_tables_within_the_oracle_bound(torch, m, nq):
    import paper_1804_09996_amd as lc
    w, ix, q = _workload(m, nq)
    gix = lc.Index.from_index(ix)
    qd = torch.from_numpy(q).to(gix.device)
    rng = np.random.default_rng(m)
    idx = np.unique(np.r_[rng.integers(0, nq, 200), nq - 40:nq])
    ref = np.stack([ix.lut(q[i]) for i in idx])
    bound = _bound(ix, q[idx])
    lut, _ = gix.build_lut(qd)
    got = lut.cpu().numpy()[idx].astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))
    assert np.all(got >= 0) and not np.any(np.signbit(got))
    h, sc = gix.build_lut(qd, lc.LC_LUT_F16)
    h = h.cpu().numpy()[idx].astype(np.float64)
    sc = sc.cpu().numpy()[idx].astype(np.float64)
    mant, _ = np.frexp(sc)
    assert np.all(mant == 0.5), "scales are powers of two"
    assert np.all(h.max(-1) <= 32768.0)
    b16 = 2.0 ** -11 * np.abs(ref) + 2.0 ** -24 * sc[:, :, None] + bound
    assert np.all(np.abs(h * sc[:, :, None] - ref) <= b16)
    gix.close()


def test_unaligned_table_is_rejected(torch):
    # rows are written 8 or 16 bytes per lane: a table pointer off a 16-byte boundary is refused before launch
    import paper_1804_09996_amd as lc
    w, ix, q = _workload(16, 20003)
    gix = lc.Index.from_index(ix)
    qd = torch.from_numpy(q[:20]).to(gix.device)
    lut = torch.zeros(20 * 16 * 256 + 8, dtype=torch.float32, device=gix.device)
    sc = torch.zeros(20 * 16, dtype=torch.float32, device=gix.device)
    L = lc.lib()
    for off in (4, 8):
        assert L.lc_build_lut(gix.handle, qd.data_ptr(), 20, lc.LC_LUT_F32, lut.data_ptr() + off, None, None) \
            == lc.LC_EINVAL
        assert L.lc_build_lut(gix.handle, qd.data_ptr(), 20, lc.LC_LUT_F16, lut.data_ptr() + off, sc.data_ptr(),
                              None) == lc.LC_EINVAL
    assert L.lc_build_lut(gix.handle, qd.data_ptr(), 20, lc.LC_LUT_F32, lut.data_ptr(), None, None) == lc.LC_OK
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(lut[20 * 16 * 256:]).item()) == 0  # nothing past the table
    gix.close()
