"""Index build with its data-parallel steps on the GPU (gpu_build) against the
host builder, through the C-ABI: the projection, the PQ codes, the graph
(Sec. 5.1 batches, level-0 insertion on the GPU after the upper levels' nodes
on the host), the regression codebook and every vector's codebook entry are
the host builder's bit for bit."""
import dataclasses

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _inputs(w):
    db, train = datagen.vectors(w, "db"), datagen.vectors(w, "train")
    return (w, db, train, datagen.projection(w), datagen.level_uniforms(w), datagen.pq_init_ids(w, train.shape[0]),
            datagen.beta_train_ids(w), datagen.beta_init_ids(w, min(w.n, w.n_beta_train)))


def _compare(w, torch, log=print):
    from paper_1804_09996_amd import builder, gpu_build
    args = _inputs(w)
    h = builder.build_index(*args, nthreads=8)
    tm = {}
    g = gpu_build.build_index_gpu(*args, device="cuda", nthreads=8, timings=tm)
    log(f"{w.name}: n {w.n}, host part {tm['graph_host_nodes']} nodes, GPU batches {tm['graph_gpu_batches']}, "
        f"graph on the GPU {tm['graph_gpu_s']:.2f} s")
    assert tm["graph_gpu_batches"] > 0
    for k in ("codes", "adj0", "up_base", "adj_up", "level", "centroids", "beta", "beta_idx"):
        a, b = np.asarray(getattr(h, k)), np.asarray(getattr(g, k))
        assert a.shape == b.shape and np.array_equal(a, b), (k, int((a != b).sum()) if a.shape == b.shape else None)
    assert (h.entry, h.max_level) == (g.entry, g.max_level)
    if h.proj is not None:
        assert np.array_equal(h.proj, g.proj)
    return h, g


@pytest.mark.parametrize("kw", [dict(name="gb-small", n=3000, d=32, m=8),
                                dict(name="gb-pad", n=3000, d=28, m=8, d_pad=32),
                                dict(name="gb-m56", n=4000, d=96, m=56, d_pad=112, k_reg=32, n_beta=32),
                                dict(name="gb-m16", n=5000, d=96, m=16, k_reg=16, n_beta=64, ef_construction=64),
                                # sub-space width 8: the kernels with the width known only at run time
                                dict(name="gb-dsub8", n=3000, d=64, m=8)])
def test_gpu_build_equals_host_build(torch, kw):
    base = dict(nq=8, n_train=4096, n_beta_train=3000, pq_iters=6, beta_kmeans_iters=4, em_iters=3)
    base.update(kw)
    _compare(datagen.small(**base), torch)


def test_gpu_build_equals_host_build_10k(torch):
    # the 10k-vector workload's configuration (PQ 8x256, degree 32, efConstruction 64)
    _compare(datagen.C1, torch)


def test_gpu_build_equals_host_build_100k(torch):
    # 100k vectors, PQ 16x256, degree 32: thousands of reverse-link merges per batch, batches of up to 4096
    w = dataclasses.replace(datagen.C2, name="C2-100k", n=100_000, nq=100, n_train=16384, pq_iters=8,
                            n_beta_train=20_000, beta_kmeans_iters=5, em_iters=3)
    h, g = _compare(w, torch)
    # the search on the GPU-built index is the oracle's (same arrays)
    import oracle
    import paper_1804_09996_amd as lc
    from tests import parity
    q = datagen.vectors(w, "query")[:64]
    gix = lc.Index.from_index(g)
    ids, d, r = gix.query(torch.from_numpy(q), ef=w.ef, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    oix = oracle.Index(n=g.n, d=g.d, d_pad=g.d_pad, m=g.m, deg0=g.deg0, deg_up=g.deg_up, k_reg=g.k_reg,
                       n_beta=g.n_beta, entry=g.entry, max_level=g.max_level, proj=g.proj, centroids=g.centroids,
                       codes=g.codes, adj0=g.adj0, level=g.level, up_base=g.up_base, adj_up=g.adj_up, beta=g.beta,
                       beta_idx=g.beta_idx, m_beta=g.m_beta)
    o = oix.search(q, w.ef, w.shortlist, w.topk)
    s = parity.summarize(oix, q, ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
    gix.close()
