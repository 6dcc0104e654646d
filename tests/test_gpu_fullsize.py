"""Full-size parity: the 1M-vector workload in the launch configuration the
benchmark times (whole 10k-query batch, default schedule), checked against
the oracle on a seeded sample of queries.

The index comes from the package's host builder, whose output equals the
oracle builder's on the smaller workloads (tests/test_builder.py); both
search sides read the same arrays.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import torch

    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import builder
    w = datagen.C2
    ix, db, q = builder.build_workload(w, cache_dir="/tmp/lc_index_cache")
    oix = oracle.Index(n=ix.n, d=ix.d, d_pad=ix.d_pad, m=ix.m, deg0=ix.deg0, deg_up=ix.deg_up, k_reg=ix.k_reg,
                       n_beta=ix.n_beta, entry=ix.entry, max_level=ix.max_level, proj=ix.proj,
                       centroids=ix.centroids, codes=ix.codes, adj0=ix.adj0, level=ix.level, up_base=ix.up_base,
                       adj_up=ix.adj_up, beta=ix.beta, beta_idx=ix.beta_idx, m_beta=ix.m_beta)
    return w, oix, lc.Index.from_index(ix), torch.from_numpy(q).cuda(), q


def test_full_batch_against_oracle_sample(c2):
    w, oix, gix, qd, q = c2
    ids, d, r = gix.query(qd, ef=None, ef_max=w.ef, S=w.shortlist, K=w.topk, stats=True)
    sample = np.sort(datagen.sample_ids(w.seed, "MISC", q.shape[0], 600, sub=7))
    o = oix.search(q[sample], w.ef, w.shortlist, w.topk)
    ids, d = ids.cpu().numpy()[sample], d.cpu().numpy()[sample]
    st = r.stats.cpu().numpy()[sample]
    s = parity.summarize(oix, q[sample], ids, d, o)
    walk_same = np.mean([np.array_equal(st[i], o["stats"][i]) for i in range(len(sample))])
    print(f"1M: EXACT {s['exact_frac']:.4f}, (E,D) identical {walk_same:.4f}, max rel err {s['max_rel_err']:.2e}")
    assert s["exact_frac"] == 1.0 and walk_same == 1.0
    assert s["max_rel_err"] <= 1e-5


def test_largest_pool_on_a_sample(c2):
    # the biggest ef the walk accepts here, on a few queries: still the oracle's walk
    w, oix, gix, qd, q = c2
    ef = 1024
    ids, d, r = gix.query(qd[:24], ef=ef, ef_max=ef, S=w.shortlist, K=w.topk, stats=True)
    o = oix.search(q[:24], ef, w.shortlist, w.topk)
    same = np.mean([np.array_equal(r.stats.cpu().numpy()[i], o["stats"][i]) for i in range(24)])
    assert same == 1.0
    s = parity.summarize(oix, q[:24], ids.cpu().numpy(), d.cpu().numpy(), o)
    assert s["exact_frac"] == 1.0 and s["max_rel_err"] <= 1e-5
