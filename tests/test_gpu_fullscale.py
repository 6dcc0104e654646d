"""Sampled parity at the large workloads' full sizes, in the launch
configurations the benchmark times, against the oracle searching the same
arrays (built by the GPU build steps, whose output equals the host
builder's: tests/test_gpu_build.py).

* 10M vectors, PQ 16, k = 16: the batched form (one step of 100k queries with
  per-query efSearch log-uniform 16..512, split into ef classes at pools 128
  and 256, longest ef first, replayed from a HIP graph), 600 sampled queries.
* 20M vectors, d 96 -> 112 through the projection, PQ 56, k = 32: the plain
  float32 path on a 10k-query batch (ef 128, short-list 32, top-10), 600
  sampled queries; the fp16 walk of the served form (table in registers) on
  the sample against the oracle's walk on the same fp16 table values; and the
  served fp16 form's requests against the path run alone.

Bars: top-K EXACT on every sampled query, every distance within 1e-5
relative of the oracle's float64 value, (E, D) identical on at least 99.5 %
of them: the walk's keys are float32 sums where the oracle's are float64, so
a near-tie between two keys at an admission or an expansion can resolve the
other way (a few queries in 10^3 at these sizes; the top-K stays EXACT).
"""
import dataclasses

import numpy as np
import pytest

import datagen
import oracle
from tests import parity

pytestmark = pytest.mark.gpu

WALK_BAR = 0.995  # (E, D) equality over the sample (float32 near-ties, see above)


def _oracle_view(ix):
    return oracle.Index(n=ix.n, d=ix.d, d_pad=ix.d_pad, m=ix.m, deg0=ix.deg0, deg_up=ix.deg_up, k_reg=ix.k_reg,
                        n_beta=ix.n_beta, entry=ix.entry, max_level=ix.max_level, proj=ix.proj, centroids=ix.centroids,
                        codes=ix.codes, adj0=ix.adj0, level=ix.level, up_base=ix.up_base, adj_up=ix.adj_up,
                        beta=ix.beta, beta_idx=ix.beta_idx, m_beta=ix.m_beta)


def test_batched_form_at_10M_against_oracle_sample():
    import torch

    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import gpu_build
    from paper_1804_09996_amd.batched import BatchedSearcher
    w = datagen.C4
    print("building the 10M index (GPU steps)", flush=True)
    ix, db, q = gpu_build.build_workload_gpu(w, device="cuda")
    del db
    gix = lc.Index.from_index(ix)
    ef = datagen.per_query_ef(w)
    K = S = w.topk
    bs = BatchedSearcher(gix, w.nq, ef_max=512, S=S, K=K, precision="f32")
    bs.set_inputs(q, ef)
    bs.set_classes([128, 256, 512])
    assert len(bs.ranges) == 3
    bs.capture()
    ids, d = bs.run()
    torch.cuda.synchronize()
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    # (E, D) of the same queries from the eager walk (the graph's statistics rows are permuted by class)
    st = np.empty((w.nq, 2), np.int32)
    inv = bs.inv.cpu().numpy()
    st[:] = bs.res.stats.cpu().numpy()[inv]
    samp = np.sort(datagen.sample_ids(w.seed, "MISC", w.nq, 600, sub=11))
    oix = _oracle_view(ix)
    o = oix.search(q[samp], ef[samp], S, K, nthreads=16)
    s = parity.summarize(oix, q[samp], ids[samp], d[samp], o)
    walk_same = np.mean([np.array_equal(st[samp][i], o["stats"][i]) for i in range(len(samp))])
    print(f"10M batched: EXACT {s['exact_frac']:.4f} (E,D) identical {walk_same:.4f} max rel err "
          f"{s['max_rel_err']:.2e}; ef of the sample {ef[samp].min()}..{ef[samp].max()}")
    assert s["exact_frac"] == 1.0 and walk_same >= WALK_BAR and s["max_rel_err"] <= 1e-5
    gix.close()


def test_serving_workload_at_20M_against_oracle_sample():
    import torch

    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import gpu_build, serve
    w = datagen.C5
    print("building the 20M index (GPU steps)", flush=True)
    ix, db, _ = gpu_build.build_workload_gpu(w, device="cuda")
    del db
    pool = datagen.vectors(dataclasses.replace(w, nq=10_000), "query")
    gix = lc.Index.from_index(ix)
    S, K, ef = 32, w.topk, 128
    ids, d, r = gix.query(torch.from_numpy(pool), ef=ef, ef_max=ef, S=S, K=K, stats=True)
    samp = np.sort(datagen.sample_ids(w.seed, "MISC", pool.shape[0], 600, sub=3))
    oix = _oracle_view(ix)
    o = oix.search(pool[samp], ef, S, K, nthreads=16)
    s = parity.summarize(oix, pool[samp], ids.cpu().numpy()[samp], d.cpu().numpy()[samp], o)
    st = r.stats.cpu().numpy()[samp]
    walk_same = np.mean([np.array_equal(st[i], o["stats"][i]) for i in range(len(samp))])
    print(f"20M plain fp32: EXACT {s['exact_frac']:.4f} (E,D) identical {walk_same:.4f} max rel err "
          f"{s['max_rel_err']:.2e}")
    assert s["exact_frac"] == 1.0 and walk_same >= WALK_BAR and s["max_rel_err"] <= 1e-5
    # the fp16 walk the served form runs (the default schedule: the table in registers) against the oracle's
    # walk on the same table values, on the sample with the serving ef mix (R34: near-ties of float32 sums)
    mix = np.asarray((32, 64, 128, 256))[np.random.default_rng(8).integers(0, 4, len(samp))].astype(np.int32)
    qp = gix.project(torch.from_numpy(pool[samp]).cuda())
    lut, sc = gix.build_lut(qp, lc.LC_LUT_F16, projected=True)
    r16 = gix.search(lut, sc, ef=mix, ef_max=256, S=S)
    tabs = (lut.cpu().numpy().view(np.float16).reshape(len(samp), w.m, 256).astype(np.float64)
            * sc.cpu().numpy().astype(np.float64)[:, :, None])
    o16 = oix.walk_tables(tabs, mix, S, nthreads=16)
    ids16 = r16.cand_ids.cpu().numpy()
    same16 = np.mean([np.array_equal(ids16[i], o16["cand_ids"][i]) and
                      np.array_equal(r16.stats.cpu().numpy()[i], o16["stats"][i]) for i in range(len(samp))])
    print(f"20M fp16 walk ({gix.walk_plan(len(samp), 256, S, lc.LC_LUT_F16)['kernel']}): short-list and (E,D) "
          f"identical to the oracle's walk on the same tables on {same16:.4f} of the sample")
    assert same16 >= WALK_BAR
    # the served fp16 form: every request as the path gives it alone, with small slots and with the
    # benchmark's (3 slots of 16384 queries, 150 requests at once so that batches fill them)
    bpq = serve.query_bytes(w.m, S, K, w.d, d_proj=w.d_pad)
    for n_slots, slot_q, n_req in ((4, 2048, 60), (3, 16384, 150)):
        reqs = serve.poisson_requests(w.d, pool, 1e9, n_req, 9, efs=(32, 64, 128, 256))
        for q_ in reqs:
            q_.arrival = 0.0
        eng = serve.GpuEngine(gix, n_slots=n_slots, slot_queries=slot_q, ef_max=256, S=S, K=K, precision="f16")
        serve.serve(eng, serve.Scheduler(n_slots, slot_q, int(0.75 * n_slots * slot_q) * bpq, bpq), reqs)
        torch.cuda.synchronize()
        for q_ in reqs[:: max(1, n_req // 20)]:
            i1, d1, _ = gix.query(torch.from_numpy(q_.queries), ef=q_.ef, ef_max=256, S=S, K=K, precision="f16")
            assert np.array_equal(q_.ids, i1.cpu().numpy()) and np.array_equal(q_.dist.view(np.uint32),
                                                                               d1.cpu().numpy().view(np.uint32))
        del eng
    gix.close()
