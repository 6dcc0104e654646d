"""Serving loop on the GPU: every request's result is the same alone and in
the mix (bitwise), in both precision forms."""
import numpy as np
import pytest

from paper_1804_09996_amd import serve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,efs,split", [("f16", (16, 32, 64), True), ("f32", (16, 32, 64), True),
                                                 ("f16", (16, 64, 160, 256), True),
                                                 ("f16", (16, 64, 160, 256), False),
                                                 ("f16", (16, 64, 160, 256), None)])
def test_results_same_alone_and_in_the_mix(c1_build, precision, efs, split):
    # each launch is sized by its batch's largest ef (pools up to 128 in
    # registers, larger in LDS), or split into the two classes walked
    # concurrently; results never depend on it
    import torch

    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    gix = lc.Index.from_index(ix)
    S, K, ef_max = 32, 10, max(efs)
    reqs = serve.poisson_requests(w.d, q, rate_rps=4000.0, n_requests=40, seed=5, efs=efs, max_batch=48)
    eng = serve.GpuEngine(gix, n_slots=3, slot_queries=128, ef_max=ef_max, S=S, K=K, precision=precision,
                          split=split, record_walks=True)
    sch = serve.Scheduler(3, 128, mem_budget=200 * serve.query_bytes(w.m, S, K, w.d), bytes_per_query=
                          serve.query_bytes(w.m, S, K, w.d))
    stats = serve.serve(eng, sch, reqs)
    torch.cuda.synchronize()
    assert stats["requests"] == 40
    assert len({r.slot for r in reqs}) > 1
    for r in reqs:
        ids, d, _ = gix.query(torch.from_numpy(r.queries), ef=r.ef, ef_max=ef_max, S=S, K=K, precision=precision)
        assert np.array_equal(r.ids, ids.cpu().numpy()), r.rid
        assert np.array_equal(r.dist.view(np.uint32), d.cpu().numpy().view(np.uint32)), r.rid
    # the recorded walk launches cover every query once, with its (E, D)
    assert sum(x["n"] for x in eng.walk_log) == sum(r.size for r in reqs)
    assert all(x["stats"].shape == (x["n"], 2) and (x["stats"][:, 0] >= 1).all() for x in eng.walk_log)
    print(f"{precision}: {stats}")


def test_projected_index_same_alone_and_in_the_mix():
    # an index with a projection (d 28 -> d_pad 32): the serving loop projects each batch once, as
    # Index.query does, so a request's results do not depend on the batch it rides in
    import torch

    import datagen
    import oracle
    import paper_1804_09996_amd as lc
    w = datagen.small(name="serve-pad", n=1500, nq=200, d=28, m=8, n_train=2048, n_beta=8, n_beta_train=1500)
    ix, db, q = oracle.build_workload(w, nthreads=4)
    assert ix.proj is not None
    gix = lc.Index.from_index(ix)
    S, K, ef_max = 16, 5, 64
    reqs = serve.poisson_requests(w.d, q, rate_rps=4000.0, n_requests=30, seed=7, efs=(16, 64), max_batch=40)
    eng = serve.GpuEngine(gix, n_slots=3, slot_queries=128, ef_max=ef_max, S=S, K=K, precision="f16")
    bpq = serve.query_bytes(w.m, S, K, w.d, d_proj=w.d_pad)
    stats = serve.serve(eng, serve.Scheduler(3, 128, mem_budget=200 * bpq, bytes_per_query=bpq), reqs)
    torch.cuda.synchronize()
    assert stats["requests"] == 30
    for r in reqs:
        ids, d, _ = gix.query(torch.from_numpy(r.queries), ef=r.ef, ef_max=ef_max, S=S, K=K, precision="f16")
        assert np.array_equal(r.ids, ids.cpu().numpy()), r.rid
        assert np.array_equal(r.dist.view(np.uint32), d.cpu().numpy().view(np.uint32)), r.rid
