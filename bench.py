"""Benchmark of the Link & Code search path on one MI355X.

Default: the serving workload (20M vectors, PQ 56, k = 32): requests served by
continuous batching with fp16 tables against the plain float32 path at the
same 1-recall@1; one step = one backlog of requests, each request the whole
path (tables, walk + short-list, refinement + top-K) over its queries, already
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form serve|both|plain|batched|assign]
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("LCB_PROGRESS", "1")  # long index builds report progress on stderr

METRIC = "QPS at fixed 1-recall@1 (served FP16 vs plain FP32, 1 GPU); p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_bytes(w, E, D, S):
    """Algorithmic bytes of one walk launch: per query the LUT read
    (4 m 256), per expansion one adjacency row (4 deg0), per evaluated node
    its code (m), and the short-list written (8 S + 12)."""
    nq = E.shape[0]
    # 2-level codec: per evaluated node also its first-level codes (4), term (4) and two table entries (8)
    per_node = w.m + (16 if w.coarse_k else 0)
    return float(nq * (4 * w.m * 256 + 8 * S + 12) + 4 * w.deg0 * E.sum() + per_node * D.sum())


def walk_kernel_name(gix, nq, ef_max, S, precision, sched=None):
    """The walk kernel the library launches for this batch (lc_walk_describe),
    with its grid and LDS plan."""
    import paper_1804_09996_amd as lc
    dt = lc.LC_LUT_F32 if precision == "f32" else lc.LC_LUT_F16
    p = gix.walk_plan(nq, ef_max, S, dt, sched)
    return (f"{p['kernel']} ({p['grid']} slots, {p['slots_per_cu']} per CU, {p['lds_bytes']} B of LDS each, "
            f"visited table 2^{p['hash_bits']} words)")


def refine_bytes(w, cand_n, K):
    """Per candidate: its beta index (1 byte per codebook block), k links
    (4k), k+1 codes (m(k+1)); per query the output (8K)."""
    c = float(np.clip(cand_n, 0, None).sum())
    codes = w.m + (4 if w.coarse_k else 0)  # a 2-level code adds its two 16-bit first-level indices
    return c * (w.m_beta + 4 * w.k_reg + codes * (w.k_reg + 1)) + cand_n.shape[0] * 8 * K


def lut_bytes(w, nq):
    return float(nq) * (4 * w.d + 4 * (w.m * 256 + 2 * w.coarse_k))


def traffic_from_profiles(config):
    """HBM bytes per walk launch (FETCH_SIZE + WRITE_SIZE, each scaled by the
    calibration copy) from the committed counter summary
    profiles/walk_traffic.json, for the entry whose configuration equals
    `config`; valid only while the walk's source is the one the counters were
    taken on (its sha1), else None."""
    path = os.path.join(ROOT, "profiles", "walk_traffic.json")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha1(open(os.path.join(ROOT, "paper_1804_09996_amd", "csrc", "lc_walk.hip"), "rb").read()).hexdigest()
    for e in json.load(open(path)).get("entries", []):
        if e.get("kernel_sha1") == sha and e.get("config") == config:
            return e.get("bytes_per_launch")
    return None


def ground_truth(torch, db, q, dev, q_chunk=512, db_chunk=1 << 21):
    """Exact nearest neighbour (raw vectors, squared L2, lowest id on ties):
    the 8 best of every query by float32 products on the GPU (database in
    chunks), decided in float64 on the host."""
    dbt = torch.from_numpy(db).to(dev)
    nrm = (dbt * dbt).sum(1)
    gt = np.empty(q.shape[0], np.int64)
    for c0 in range(0, q.shape[0], q_chunk):
        qt = torch.from_numpy(q[c0:c0 + q_chunk]).to(dev)
        best_d = best_i = None
        for b0 in range(0, db.shape[0], db_chunk):
            d = nrm[None, b0:b0 + db_chunk] - 2.0 * qt @ dbt[b0:b0 + db_chunk].T
            v, i = torch.topk(d, min(8, d.shape[1]), dim=1, largest=False)
            i = i + b0
            if best_d is None:
                best_d, best_i = v, i
            else:
                v2, j = torch.topk(torch.cat([best_d, v], 1), min(8, best_d.shape[1] + v.shape[1]), dim=1,
                                   largest=False)
                best_d, best_i = v2, torch.gather(torch.cat([best_i, i], 1), 1, j)
        cand = best_i.cpu().numpy()
        for i in range(cand.shape[0]):
            cd = ((db[cand[i]].astype(np.float64) - q[c0 + i].astype(np.float64)) ** 2).sum(1)
            o = np.lexsort((cand[i], cd))
            gt[c0 + i] = cand[i][o[0]]
    del dbt, nrm
    return gt


def recall(ids, gt, r):
    return float(np.mean([gt[i] in ids[i, :r] for i in range(len(gt))]))


def cpu_baseline(ix, db, q, w, seconds=10.0):
    """The oracle, untuned, on a bounded sample of the query batch: a prefix
    of it, or the whole batch repeated until about `seconds` have passed."""
    import oracle
    oix = oracle.Index(n=ix.n, d=ix.d, d_pad=ix.d_pad, m=ix.m, deg0=ix.deg0, deg_up=ix.deg_up, k_reg=ix.k_reg,
                       n_beta=ix.n_beta, entry=ix.entry, max_level=ix.max_level, proj=ix.proj,
                       centroids=ix.centroids, codes=ix.codes, adj0=ix.adj0, level=ix.level, up_base=ix.up_base,
                       adj_up=ix.adj_up, beta=ix.beta, beta_idx=ix.beta_idx, m_beta=ix.m_beta)
    nt = oracle.default_threads()
    t0 = time.time()
    probe = oix.search(q[:nt], w.ef, w.shortlist, w.topk, nthreads=nt)
    per = (time.time() - t0) / nt * nt  # seconds per query per thread-round
    n = int(min(q.shape[0], max(nt, seconds / max(per, 1e-6) * nt)))
    n = max(nt, n // nt * nt)
    t0 = time.time()
    res = oix.search(q[:n], w.ef, w.shortlist, w.topk, nthreads=nt)
    passes = 1
    while time.time() - t0 < seconds and n == q.shape[0] and passes < 100:
        oix.search(q[:n], w.ef, w.shortlist, w.topk, nthreads=nt)
        passes += 1
    dt = time.time() - t0
    del probe
    what = f"first {n} of the {q.shape[0]} benchmark queries" if passes == 1 else \
        f"the {n} benchmark queries, {passes} passes"
    # and one thread on the first 1000 queries, in the paper's unit (ms per query)
    n1 = min(1000, q.shape[0])
    t1 = time.time()
    oix.search(q[:n1], w.ef, w.shortlist, w.topk, nthreads=1)
    ms1 = (time.time() - t1) / n1 * 1e3
    return {"value": n * passes / dt, "unit": "queries/s", "cores": nt, "kind": "oracle",
            "sample": f"{what}, float64 oracle search (LUT, walk, refine, top-{w.topk}), {nt} threads, "
                      f"{dt:.1f} s",
            "single_thread_ms_per_query": ms1, "single_thread_sample": f"first {n1} queries, 1 thread",
            "cpu_model": cpu_model()}, oix, res, n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def interp_at(points, r_target):
    """QPS at recall r_target, linear between the measured (recall, qps)
    points (None if r_target is outside their range)."""
    pts = sorted(points)
    for (r0, q0), (r1, q1) in zip(pts, pts[1:]):
        if r0 <= r_target <= r1:
            return q0 if r1 == r0 else q0 + (q1 - q0) * (r_target - r0) / (r1 - r0)
    if pts and abs(pts[-1][0] - r_target) < 1e-12:
        return pts[-1][1]
    return None


def ground_truth_sample(torch, db, q, dev, n_sample, seed):
    """Exact nearest neighbours of a seeded subsample of the queries."""
    import datagen
    idx = np.sort(datagen.sample_ids(seed, "MISC", q.shape[0], n_sample))
    return idx, ground_truth(torch, db, q[idx], dev)


def bench_batched(args):
    """Batched form: one batch, per-query ef log-uniform 16..512, longest ef
    first, autotuned walk schedule, the step replayed from a HIP graph."""
    import torch

    import datagen
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import gpu_build
    from paper_1804_09996_amd.batched import BatchedSearcher

    w = datagen.WORKLOADS[args.workload if args.workload not in ("C2-1M", "C5-20M") else "C4-10M"]
    dev = torch.device("cuda:0")
    t0 = time.time()
    ix, db, q = gpu_build.build_workload_gpu(w, device=dev, log=log, cache_dir=args.gpu_index_cache or None)
    log(f"index ready in {time.time() - t0:.1f}s (n={ix.n}, max_level={ix.max_level})")
    gix = lc.Index.from_index(ix, device=dev)
    nq, K = q.shape[0], w.topk
    ef = datagen.per_query_ef(w)
    S, ef_max = K, 512
    # --precision f16: fp16 tables in the walk (the refinement stays fp32 at this short-list: K = S leaves
    # nothing for a bf16 first pass to skip)
    prec = "f32" if args.precision == "f32" else "f16"
    bs = BatchedSearcher(gix, nq, ef_max=ef_max, S=S, K=K, precision=prec)
    bs.set_inputs(q, ef)
    if args.no_tune:  # the default schedule, one class: every step is one walk launch of one kernel
        import paper_1804_09996_amd as lc_
        sched = lc_.schedule()
        bs.sched, bs.table = sched, []
    else:
        sched = bs.tune(cache_path=None, log=log)
    bs.capture()
    for _ in range(args.warmup):
        bs.run()
    torch.cuda.synchronize()
    t_w = time.time()  # the device at its working clocks before the timed steps
    while time.time() - t_w < args.warm_seconds:
        bs.run()
        torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        ids, d = bs.run()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([a.elapsed_time(b) for a, b in evs])
    # per-kernel times of one eager step on the same buffers (the walk phase:
    # the concurrent launches of every ef class)
    lut_dt = bs.lut_dtype
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    qx, pj = bs._queries()
    lut, scale = gix.build_lut(qx, lut_dt, projected=pj)
    e[1].record()
    bs._walks(lut, scale)
    e[2].record()
    gix.refine(qx, bs.res.cand_ids, bs.res.cand_n, K, bs.refine_p, projected=pj)
    e[3].record()
    torch.cuda.synchronize()
    kms = [e[j].elapsed_time(e[j + 1]) for j in range(3)]
    st = bs.res.stats.cpu().numpy()
    # the walk alone (one launch over the whole batch, longest ef first) with other schedules and table types:
    # the codes fetched after the visited probe, fp16 tables in LDS and in registers (same walk results per
    # table type)
    variants = {}
    qx_all = torch.from_numpy(q).to(dev)
    ef_all = torch.from_numpy(ef).to(dev)
    order = torch.argsort(-ef_all, stable=True).to(torch.int32)
    l32, _ = gix.build_lut(qx_all, lc.LC_LUT_F32)
    l16, s16 = gix.build_lut(qx_all, lc.LC_LUT_F16)
    for name, lut_v, sc_v, sch in (("f32", l32, None, lc.schedule()), ("f32_codes_after_probe", l32, None,
                                                                        lc.schedule(codes=1)),
                                   ("f16_table_in_lds", l16, s16, lc.schedule(table=1)),
                                   ("f16_table_in_registers", l16, s16, lc.schedule(table=2))):
        wsv = gix.workspace(nq, ef_max, S, sch)
        ts = []
        for k in range(3):
            a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a_.record()
            gix.search(lut_v, sc_v, ef=ef_all, ef_max=ef_max, S=S, stats=False, sched=sch, ws=wsv, order=order)
            b_.record()
            b_.synchronize()
            ts.append(a_.elapsed_time(b_))
        plan = gix.walk_plan(nq, ef_max, S, lc.LC_LUT_F32 if sc_v is None else lc.LC_LUT_F16, sch)
        variants[name] = {"ms": float(np.median(ts[1:])), "kernel": plan["kernel"],
                          "slots_per_cu": plan["slots_per_cu"]}
        del wsv
    del l32, l16, s16
    E, D = st[:, 0].astype(np.int64), st[:, 1].astype(np.int64)
    wb = walk_bytes(w, E, D, S)
    if prec == "f16":
        wb += -nq * 2 * w.m * 256 + nq * 4 * w.m  # fp16 table + scales
    idx, gt = ground_truth_sample(torch, db, q, dev, 10_000, w.seed)
    ids_np = ids.cpu().numpy()[idx]
    rec = {f"R@{r_}": recall(ids_np, gt, r_) for r_ in (1, 10, 100) if r_ <= K}
    out = {"metric": "QPS, batched persistent form (per-query efSearch), 1 GPU", "value": nq * args.steps / wall,
           "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": prec, "data": "synthetic",
           "config": {"workload": f"{w.name}: N={w.n} d={w.d} Gaussian mixture ({w.n_comp} components), PQ {w.m}x256, "
                                  f"k={w.k_reg}, {nq} queries in one step, efSearch per query round(exp(U(ln16, "
                                  f"ln512))), pool max(ef, {S}), short-list {S}, top-{K}, longest ef first, "
                                  f"{'default' if args.no_tune else 'autotuned'} schedule {sched.as_dict()} and ef classes (pool limits "
                                  f"{bs.limits}: one concurrent walk launch per class), step replayed from a HIP "
                                  f"graph",
                      "ef_classes": [{"rows": r1 - r0, "ef_max": efm} for r0, r1, efm in bs.ranges]},
           "roofline": {"bound": "hbm", "achieved": wb / (kms[1] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": wb / (kms[1] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": traffic_from_profiles({"form": "batched", "workload": w.name, "table": prec,
                                                          "schedule": "default" if args.no_tune else "autotuned",
                                                          "S": S}) if args.no_tune else None,
                        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                        "kernel": "walk phase: " + "; ".join(walk_kernel_name(gix, r1 - r0, efm, S, prec, sched)
                                                             for r0, r1, efm in bs.ranges),
                        "algorithmic_bytes_per_launch": wb},
           "kernels_ms": dict(zip(("build_lut", "walk", "refine"), kms)),
           "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
           "recall_10k_sample": rec, "walk_mean_E": float(E.mean()), "walk_mean_D": float(D.mean()),
           "walk_variants_one_launch": variants,
           "autotune_table": bs.table}
    print(json.dumps(out), flush=True)


def bench_assign(args):
    """Index-build step on the GPU: the regression-codebook entry (Sec. 4.3
    Eq. 7; per block, Eq. 9) of every database vector, float64 arg-min, against
    the host builder's threaded assignment of a sample of the same vectors."""
    import ctypes as C

    import torch

    import datagen
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import builder

    w = datagen.WORKLOADS[args.workload]
    if args.m_beta != 1:
        w = dataclasses.replace(w, m_beta=args.m_beta)
    dev = torch.device("cuda:0")
    ix, db, q = builder.build_workload(w, cache_dir=args.cache, log=log)
    gix = lc.Index.from_index(ix, device=dev)
    x = torch.from_numpy(db).to(dev)
    out = gix.assign_beta(x)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(max(3, args.steps // 10)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = gix.assign_beta(x)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    got = out.cpu().numpy().reshape(ix.n, -1)
    agree = float((got == np.asarray(ix.beta_idx).reshape(ix.n, -1)).mean())
    # the host builder's assignment of a sample, its own threads
    L = builder.lib()
    ns = min(ix.n, 100_000)
    bidx = np.empty((ns, w.m_beta), np.uint8)
    p_ = lambda a_: None if a_ is None else a_.ctypes.data
    nt = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    rc = L.lcb_beta_assign(p_(np.ascontiguousarray(db[:ns])), ns, w.d, p_(ix.proj), w.d_pad, w.m, p_(ix.centroids),
                           p_(ix.codes), ix.codes.shape[1], p_(ix.adj0), w.deg0, w.k_reg, w.n_beta, w.m_beta,
                           p_(np.ascontiguousarray(ix.beta, np.float32)), nt, p_(bidx), None)
    cpu_s = time.perf_counter() - t0
    assert rc == 0
    print(json.dumps({"form": "beta assignment (index build)", "workload": w.name, "n": ix.n, "m_beta": w.m_beta,
                      "n_beta": w.n_beta, "k": w.k_reg, "gpu_ms": ms, "gpu_vectors_per_s": ix.n / (ms * 1e-3),
                      "agreement_with_host_builder": agree,
                      "host_builder": {"vectors": ns, "seconds": cpu_s, "vectors_per_s": ns / cpu_s, "threads": nt}}))


def host_cores():
    """Host cores this process may use: its CPU affinity, cut to the cgroup's
    CPU quota when one is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            n = min(n, max(1, int(float(quota) / float(period))))
    except (OSError, ValueError):
        pass
    return max(1, n)


SERVE_MIX = (32, 64, 128, 256)  # efSearch of the serving workload's requests


def serve_walk_bytes(m, S, E, D):
    """Algorithmic bytes of one fp16-table walk launch: per query the table
    (2 m 256) and its row scales (4 m), per expansion one adjacency row (128),
    per evaluated node its code (m), the short-list written (8 S + 12)."""
    nq = E.shape[0]
    return float(nq * (2 * m * 256 + 4 * m + 8 * S + 12) + 128 * E.sum() + m * D.sum())


def bench_serve(args):
    """The serving workload: a resident index, requests (a batch of queries,
    one efSearch each) served by continuous batching with fp16 tables, against
    the plain float32 path at the same 1-recall@1.

    Phases, in order: (1) the index build (GPU steps), (2) exact nearest
    neighbours of the query pool, (3) the walk alone on one stream (its kernel
    time and roofline), (4) the plain float32 path on fixed batches over an ef
    grid, (5) the served fp16 form at saturation over scaled ef mixes, (6) the
    timed steps: W + K backlogs of requests with the workload's ef mix, (7)
    Poisson loads at fractions of saturation (latency), (8) the oracle on the
    host cores (baseline and sampled parity)."""
    import torch

    import datagen
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import gpu_build, serve

    w = datagen.WORKLOADS[args.workload if args.workload != "C2-1M" else "C5-20M"]
    if args.n:
        w = dataclasses.replace(w, name=f"{w.name.split('-')[0]}-{args.n / 1e6:g}M", n=args.n)
    dev = torch.device("cuda:0")
    # (1) the index: data-parallel build steps on the GPU
    t0 = time.time()
    build_t = {}
    ix, db, _ = gpu_build.build_workload_gpu(w, device=dev, log=log, timings=build_t,
                                             cache_dir=args.gpu_index_cache or None)
    build_t["data_and_build_s"] = time.time() - t0
    pool = datagen.vectors(dataclasses.replace(w, nq=args.pool), "query")
    # (2) ground truth of every pool query
    t1 = time.time()
    gt = ground_truth(torch, db, pool, dev)
    log(f"ground truth of {pool.shape[0]} queries in {time.time() - t1:.1f}s")
    gix = lc.Index.from_index(ix, device=dev)
    del db
    S, K, ef_max = args.serve_shortlist, w.topk, 512
    m = w.m
    qd = torch.from_numpy(pool).to(dev)
    nq = pool.shape[0]
    mix_ef = np.asarray(SERVE_MIX)[datagen.rng(w.seed, "EF").integers(0, len(SERVE_MIX), nq)].astype(np.int32)

    # (3) the dominant kernel alone: fp16-table walk over the pool with the workload's ef mix, one stream.
    qp = gix.project(qd)
    lut16, sc16 = gix.build_lut(qp, lc.LC_LUT_F16, projected=True)
    ef_t = torch.from_numpy(mix_ef).to(dev)
    # slots take the queries longest ef first, as the serving engine lays out each launch
    ord_t = torch.argsort(ef_t, descending=True, stable=True).to(torch.int32)
    ws1 = gix.workspace(nq, int(mix_ef.max()), S)
    reps = max(5, args.steps // 2)

    def walk1():
        return gix.search(lut16, sc16, ef=ef_t, ef_max=int(mix_ef.max()), S=S, stats=True, ws=ws1, order=ord_t)

    # the device at its working clocks first: walks back to back for a second (a launch right after the
    # host-side build and ground truth has been measured up to 35 % slower than the same launch later)
    t_w, n_warm = time.time(), 0
    while time.time() - t_w < args.warm_seconds:
        walk1()
        torch.cuda.synchronize()
        n_warm += 1

    def back_to_back(fn, n):
        """Mean time per launch of n launches queued back to back on the current stream (events around the
        whole run, so host-side launch gaps are not counted while the queue is fed)."""
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            out = fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / n, out

    walk_ms, r1 = back_to_back(walk1, reps)
    st1 = r1.stats.cpu().numpy()
    E1, D1 = st1[:, 0].astype(np.int64), st1[:, 1].astype(np.int64)
    wb = serve_walk_bytes(m, S, E1, D1)
    kname = walk_kernel_name(gix, nq, int(mix_ef.max()), S, "f16")
    log(f"walk alone: {kname} {walk_ms:.3f} ms for {nq} queries, {wb / (walk_ms * 1e-3) / 1e9:.0f} GB/s algorithmic")

    # every kernel of the path on the same batch, one stream (mean of launches queued back to back)
    def timed(fn, reps_=10):
        return back_to_back(fn, reps_)[0]

    kern = {"project": timed(lambda: gix.project(qd)),
            "build_lut_f16": timed(lambda: gix.build_lut(qp, lc.LC_LUT_F16, projected=True)),
            "build_lut_f32": timed(lambda: gix.build_lut(qp, lc.LC_LUT_F32, projected=True)),
            "walk_f16": walk_ms}
    for hb in (10, 11, 12):  # the walk's visited-table sizes (same results; LDS per slot against capacity)
        sc_ = lc.schedule(hash_bits=hb)
        wsh = gix.workspace(nq, int(mix_ef.max()), S, sc_)
        kern[f"walk_f16_hash_bits_{hb}"] = timed(lambda: gix.search(lut16, sc16, ef=ef_t, ef_max=int(mix_ef.max()),
                                                                    S=S, stats=False, sched=sc_, ws=wsh, order=ord_t))
        del wsh
    for name, sc_ in (("walk_f16_codes_after_probe", lc.schedule(codes=1)),
                      ("walk_f16_table_in_lds", lc.schedule(table=1, pool=1))):
        wsh = gix.workspace(nq, int(mix_ef.max()), S, sc_)
        kern[name] = timed(lambda: gix.search(lut16, sc16, ef=ef_t, ef_max=int(mix_ef.max()), S=S, stats=False,
                                              sched=sc_, ws=wsh, order=ord_t))
        del wsh
    lut32, _ = gix.build_lut(qp, lc.LC_LUT_F32, projected=True)
    kern["walk_f32"] = timed(lambda: gix.search(lut32, None, ef=ef_t, ef_max=int(mix_ef.max()), S=S, stats=False,
                                                ws=ws1, order=ord_t))
    for name, prec in (("refine_f32", lc.LC_REFINE_F32), ("refine_bf16_rescore", lc.LC_REFINE_BF16_RESCORE)):
        kern[name] = timed(lambda: gix.refine(qp, r1.cand_ids, r1.cand_n, K, prec, projected=True))
    served_refine = args.serve_refine
    if served_refine == "auto":
        served_refine = "bf16" if kern["refine_bf16_rescore"] < kern["refine_f32"] else "f32"
    log("one-stream kernel times (ms, " + f"{nq} queries): " + ", ".join(f"{k} {v:.3f}" for k, v in kern.items())
        + f"; served refinement: {served_refine}")
    del ws1, lut16, sc16, qp, lut32

    # (4) the plain float32 path: tables, walk, refinement on fixed batches of the pool, three streams
    side = [torch.cuda.Stream(device=dev) for _ in range(3)]
    wsb = {}

    def plain_point(ef_, steps):
        """ef_: one efSearch for every query, or an array of per-query values."""
        per_q = not np.isscalar(ef_)
        ef_top = int(np.max(ef_)) if per_q else int(ef_)
        ef_dev = torch.from_numpy(np.asarray(ef_, np.int32)).to(dev) if per_q else None
        # per-query ef: slots take the queries longest ef first, as the served form's launches do
        ord_dev = torch.argsort(ef_dev, descending=True, stable=True).to(torch.int32) if per_q else None
        lanes = []
        for i, st_ in enumerate(side):
            nb = gix.workspace_bytes(nq, max(ef_top, S), S)
            if wsb.get(i) is None or wsb[i].numel() < nb:
                wsb[i] = torch.zeros(nb, dtype=torch.uint8, device=dev)
            lanes.append((st_, wsb[i]))
        torch.cuda.synchronize()

        def step(k):
            st_, ws_ = lanes[k % len(lanes)]
            with torch.cuda.stream(st_):
                qx = gix.project(qd)
                lut, _ = gix.build_lut(qx, lc.LC_LUT_F32, projected=True)
                r = gix.search(lut, None, ef=ef_dev, ef_max=ef_top, S=S, stats=False, ws=ws_, order=ord_dev)
                return gix.refine(qx, r.cand_ids, r.cand_n, K, lc.LC_REFINE_F32, projected=True)

        for k in range(len(lanes)):
            step(k)
        torch.cuda.synchronize()
        t_ = time.perf_counter()
        for k in range(steps):
            ids_, d_ = step(k)
        torch.cuda.synchronize()
        wall_ = time.perf_counter() - t_
        ids_np = ids_.cpu().numpy()
        return {"ef": (None if per_q else ef_), "S": S, "qps": nq * steps / wall_,
                "R@1": recall(ids_np, gt, 1), "R@10": recall(ids_np, gt, 10)}, ids_np, d_.cpu().numpy()

    # the same requests' queries with their own ef (the workload's mix, scaled for the curve) ...
    scales = (0.25, 0.5, 1.0, 2.0)
    plain_curve, plain_res = [], {}
    for sc_ in scales:
        efq = np.maximum(1, (mix_ef * sc_).astype(np.int32))
        pt, _, _ = plain_point(efq, max(3, args.steps // 4))
        pt.update({"ef_mix": [max(1, int(e * sc_)) for e in SERVE_MIX]})
        plain_curve.append(pt)
        log(f"plain fp32 ef mix x{sc_}: R@1 {pt['R@1']:.4f} R@10 {pt['R@10']:.4f} {pt['qps']:.0f} queries/s")
    # ... and one ef for every query (the cheapest way to a given recall on this pool)
    uniform_curve = []
    for ef_ in (32, 48, 64, 96, 128, 192, 256):
        pt, ids_np, d_np = plain_point(ef_, max(3, args.steps // 4))
        uniform_curve.append(pt)
        plain_res[ef_] = (ids_np, d_np)
        log(f"plain fp32 ef {ef_}: R@1 {pt['R@1']:.4f} R@10 {pt['R@10']:.4f} {pt['qps']:.0f} queries/s")
    del wsb

    # (5) + (6) the served fp16 form
    n_slots, slot_q = args.slots, args.slot_queries
    bpq = serve.query_bytes(m, S, K, w.d, d_proj=w.d_pad)
    budget = int(0.75 * n_slots * slot_q) * bpq  # below the slots' capacity: admission also waits on memory
    eng = serve.GpuEngine(gix, n_slots=n_slots, slot_queries=slot_q, ef_max=ef_max, S=S, K=K, precision="f16",
                          record_walks=True,
                          refine=lc.LC_REFINE_BF16_RESCORE if served_refine == "bf16" else lc.LC_REFINE_F32)

    def served_recall(reqs):
        hit1 = hit10 = tot = 0
        for r in reqs:
            g_ = gt[r.qidx]
            hit1 += int((r.ids[:, :1] == g_[:, None]).any(1).sum())
            hit10 += int((r.ids[:, :10] == g_[:, None]).any(1).sum())
            tot += r.size
        return hit1 / tot, hit10 / tot

    def backlog(efs, n_req, seed, timing=None):
        """n_req requests present at t = 0, served to completion; `timing`
        receives the wall time of the loop alone (requests drawn before it,
        recall taken after it)."""
        reqs = serve.poisson_requests(w.d, pool, 1e9, n_req, seed, efs=efs)
        for r in reqs:
            r.arrival = 0.0
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        res = serve.serve(eng, serve.Scheduler(n_slots, slot_q, budget, bpq), reqs)
        torch.cuda.synchronize()
        if timing is not None:
            timing.append(time.perf_counter() - t_b)
        res["R@1"], res["R@10"] = served_recall(reqs)
        return res, reqs

    served_curve = []
    for scale in scales:
        efs = tuple(max(1, int(e * scale)) for e in SERVE_MIX)
        res, _ = backlog(efs, args.step_requests * 4, w.seed + 11)
        served_curve.append({"efs": list(efs), "qps": res["qps"], "R@1": res["R@1"], "R@10": res["R@10"],
                             "p50_ms": res["latency_ms_p50"], "p99_ms": res["latency_ms_p99"]})
        log(f"served fp16 ef mix {efs}: R@1 {res['R@1']:.4f} R@10 {res['R@10']:.4f} {res['qps']:.0f} queries/s")

    # the timed steps: K steps of step_requests requests each (the workload's ef mix), all present at t = 0
    # and served back to back by the loop (as the plain path's batches follow each other on its streams)
    if args.warmup:
        backlog(SERVE_MIX, args.warmup * args.step_requests, w.seed + 100)
    eng.walk_log.clear()
    tw = []
    res_t, all_reqs = backlog(SERVE_MIX, args.steps * args.step_requests, w.seed + 200, timing=tw)
    wall = tw[0]
    served_q = res_t["queries"]
    value = served_q / wall
    r1_head, r10_head = res_t["R@1"], res_t["R@10"]
    timed_walks = list(eng.walk_log)
    log(f"served fp16 timed: {value:.0f} queries/s over {args.steps} steps, R@1 {r1_head:.4f}")

    # (7) latency at offered loads
    mean_batch = float(np.mean([r.size for r in all_reqs]))
    loads = []
    for frac in [float(x) for x in args.loads.split(",")]:
        rate = frac * value / mean_batch
        reqs = serve.poisson_requests(w.d, pool, rate, args.load_requests, w.seed + 2)
        res = serve.serve(eng, serve.Scheduler(n_slots, slot_q, budget, bpq), reqs)
        res["R@1"], res["R@10"] = served_recall(reqs)
        res.update({"offered_load_frac": frac, "offered_qps": rate * mean_batch, "request_rate": rate})
        loads.append(res)
        log(f"load {frac}: {res['qps']:.0f} queries/s p50 {res['latency_ms_p50']:.2f} ms p99 "
            f"{res['latency_ms_p99']:.2f} ms")

    # the plain path at the served form's recall (linear between its grid points)
    q_plain_r1 = interp_at([(c["R@1"], c["qps"]) for c in plain_curve], r1_head)
    q_plain_r10 = interp_at([(c["R@10"], c["qps"]) for c in plain_curve], r10_head)
    q_unif_r1 = interp_at([(c["R@1"], c["qps"]) for c in uniform_curve], r1_head)
    # served walks of the timed steps: their launch durations on the slot streams (overlapping launches)
    lw = [x for x in timed_walks if "stats" in x]
    served_walk = None
    if lw:
        sb = sum(serve_walk_bytes(m, S, x["stats"][:, 0].astype(np.int64), x["stats"][:, 1].astype(np.int64))
                 for x in lw)
        sd = sum(x["a"].elapsed_time(x["b"]) for x in lw)
        served_walk = {"launches": len(lw), "mean_launch_ms": sd / len(lw), "bytes": sb,
                       "GBps_per_launch_time": sb / (sd * 1e-3) / 1e9,
                       "note": "launches overlap over the slots' streams; each launch's time includes the others'"}

    out = {"metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
           "config": {"workload": f"{w.name}: N={w.n} d={w.d}->{w.d_pad} (seeded orthonormal projection), Gaussian "
                                  f"mixture ({w.n_comp} components, L2-normalised), PQ {w.m}x256, level-0 degree "
                                  f"{w.deg0}, k={w.k_reg}, beta codebook {w.n_beta}; resident index built by "
                                  f"gpu_build; requests of round(exp(U(0, ln1024))) queries, efSearch uniform over "
                                  f"{list(SERVE_MIX)}, short-list {S}, top-{K}; served by continuous batching "
                                  f"({n_slots} slots x {slot_q} queries, each on its own stream, memory budget "
                                  f"{budget} B = 75 % of the slots' capacity; each batch's walk "
                                  + ("split into its register-pool and LDS-pool classes on two streams" if eng.split
                                     else "one launch, queries longest ef first") +
                                  f") with fp16 tables and the "
                                  f"{served_refine} refinement; a step = {args.step_requests} requests; the K "
                                  f"timed steps' requests are present at t = 0 and served back to back",
                      "n": w.n, "queries_per_step": served_q / args.steps, "requests_per_step": args.step_requests,
                      "refinement": served_refine,
                      "query_pool": nq},
           "recall": {"R@1": r1_head, "R@10": r10_head},
           "plain_fp32": {"qps_at_same_R@1": q_plain_r1, "qps_at_same_R@10": q_plain_r10,
                          "form": "plain float32 path (tables, walk, refinement, fp32) on fixed batches of the "
                                  f"{nq}-query pool, each query with its request's ef (the workload's mix, scaled "
                                  f"x{list(scales)} for the curve; slots take them longest ef first), short-list {S}, "
                                  "consecutive batches over three streams",
                          "curve": plain_curve,
                          "one_ef_for_all": {"qps_at_same_R@1": q_unif_r1, "curve": uniform_curve,
                                             "note": "every query with the same ef: a different workload (no "
                                                     "request asks for its own ef), shown for context"}},
           "served_fp16_over_plain_fp32_at_same_R@1": None if not q_plain_r1 else value / q_plain_r1,
           "served_fp16_over_plain_fp32_at_same_R@10": None if not q_plain_r10 else value / q_plain_r10,
           "served_fp16_curve": served_curve,
           "latency_ms": {"p50": loads[-1]["latency_ms_p50"], "p99": loads[-1]["latency_ms_p99"],
                          "offered_load_frac": loads[-1]["offered_load_frac"]} if loads else None,
           "loads": loads,
           "roofline": {"bound": "hbm", "achieved": wb / (walk_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": wb / (walk_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": traffic_from_profiles({"form": "serve", "workload": w.name, "table": "f16",
                                                          "ef_mix": list(SERVE_MIX), "S": S, "queries": nq}),
                        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                        "kernel": kname, "algorithmic_bytes_per_launch": wb, "launch_ms": walk_ms,
                        "launches": reps, "queries_per_launch": nq,
                        # launches of this walk before the timed ones: the warm-up, then one untimed
                        "launches_before": n_warm + 1,
                        "measured": "one stream, the walk alone on the query pool with the workload's ef mix, "
                                    "slots taking queries longest ef first; launches queued back to back after "
                                    f"{args.warm_seconds:g} s of warm-up walks, mean per launch",
                        "walk_mean_E": float(E1.mean()), "walk_mean_D": float(D1.mean())},
           "served_walk_launches": served_walk,
           "one_stream_kernels_ms": kern,
           "index_build": build_t}
    if not args.no_cpu_baseline:
        import oracle
        from tests import parity
        oix = oracle.Index(n=ix.n, d=ix.d, d_pad=ix.d_pad, m=ix.m, deg0=ix.deg0, deg_up=ix.deg_up, k_reg=ix.k_reg,
                           n_beta=ix.n_beta, entry=ix.entry, max_level=ix.max_level, proj=ix.proj,
                           centroids=ix.centroids, codes=ix.codes, adj0=ix.adj0, level=ix.level,
                           up_base=ix.up_base, adj_up=ix.adj_up, beta=ix.beta, beta_idx=ix.beta_idx,
                           m_beta=ix.m_beta)
        nt = host_cores()
        # parity: the plain fp32 path at ef 128 against the oracle on a seeded sample of the pool
        ef_p = 128
        samp = np.sort(datagen.sample_ids(w.seed, "MISC", nq, args.parity_queries, sub=3))
        t2 = time.time()
        o = oix.search(pool[samp], ef_p, S, K, nthreads=nt)
        dt_par = time.time() - t2
        ids_p, d_p = plain_res[ef_p]
        sm = parity.summarize(oix, pool[samp], ids_p[samp], d_p[samp], o)
        out["parity_sample"] = {"form": f"plain fp32, ef {ef_p}, short-list {S}, top-{K}", "queries": len(samp),
                                "exact_frac": sm["exact_frac"], "strict_frac": sm["strict_frac"],
                                "max_rel_dist_err": sm["max_rel_err"]}
        # the oracle as a baseline: all host cores, the workload's ef mix, about cpu_seconds of work
        per_q = dt_par * nt / len(samp)
        n_b = int(min(nq, max(nt, args.cpu_seconds * nt / max(per_q, 1e-6))))
        t3 = time.time()
        passes = 0
        while True:  # the sample repeated until about cpu_seconds of work
            oix.search(pool[:n_b], mix_ef[:n_b], S, K, nthreads=nt)
            passes += 1
            if time.time() - t3 >= args.cpu_seconds or passes >= 50:
                break
        dt = time.time() - t3
        n1 = min(200, nq)
        t4 = time.time()
        oix.search(pool[:n1], mix_ef[:n1], S, K, nthreads=1)
        ms1 = (time.time() - t4) / n1 * 1e3
        out["cpu_baseline"] = {"value": n_b * passes / dt, "unit": "queries/s", "cores": nt, "kind": "oracle",
                               "sample": f"first {n_b} pool queries with the workload's ef mix ({passes} passes), "
                                         f"float64 oracle search (tables, walk, refinement, top-{K}) on the same "
                                         f"index, {nt} threads, {dt:.1f} s",
                               "single_thread_ms_per_query": ms1,
                               "single_thread_sample": f"first {n1} pool queries, 1 thread",
                               "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warm-seconds", type=float, default=1.0,
                    help="walks run back to back before the walk alone is timed (the device at working clocks)")
    ap.add_argument("--workload", default="C5-20M")
    ap.add_argument("--form", choices=("serve", "both", "plain", "batched", "assign"), default="serve")
    ap.add_argument("--n", type=int, default=0, help="override the database size (serving form; named in the line)")
    ap.add_argument("--loads", default="0.5,0.8", help="offered loads as fractions of saturation (serving form)")
    ap.add_argument("--load-requests", type=int, default=5000, help="requests per offered load (serving form)")
    ap.add_argument("--step-requests", type=int, default=250, help="requests per timed step (serving form)")
    ap.add_argument("--pool", type=int, default=10_000, help="query pool with exact neighbours (serving form)")
    ap.add_argument("--serve-shortlist", type=int, default=32, help="short-list size (serving form)")
    ap.add_argument("--slots", type=int, default=3, help="serving slots (each with its own streams; serving form)")
    ap.add_argument("--slot-queries", type=int, default=16384, help="queries per serving slot (serving form)")
    ap.add_argument("--serve-refine", choices=("auto", "f32", "bf16"), default="auto",
                    help="served refinement: fp32, bf16 with the fp32 re-score, or the faster of the two on the "
                         "one-stream measurement (serving form)")
    ap.add_argument("--parity-queries", type=int, default=600, help="oracle parity sample (serving form)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle baseline work (serving form)")
    ap.add_argument("--cache", default=os.environ.get("LC_INDEX_CACHE", os.path.join("/tmp", "lc_index_cache")))
    ap.add_argument("--gpu-index-cache", default="",
                    help="serving and batched forms: save the GPU-built index here, or load it if a build of the "
                         "same workload is there (the line then reports no build time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched form: the default walk schedule and one ef class (no autotuning)")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams that consecutive steps alternate on (1 = each step runs alone)")
    ap.add_argument("--precision", choices=("f32", "f16", "f16+bf16"), default=None,
                    help="form timed by --form plain (default: the plain fp32 path) and --form batched (default: "
                         "fp16 tables, the precision form)")
    ap.add_argument("--ef", type=int, default=0, help="efSearch for --form plain (default: the workload's)")
    ap.add_argument("--shortlist", type=int, default=0, help="short-list size for --form plain (default: the workload's)")
    ap.add_argument("--m-beta", type=int, default=1,
                    help="regression codebook blocks: 1 = one codebook, >1 = product codebook of that many blocks "
                         "(plain and both forms)")
    ap.add_argument("--n-beta", type=int, default=0,
                    help="regression codebook size (default: the workload's; 1 = one shared beta, the 0-byte form)")
    ap.add_argument("--opq-iters", type=int, default=0,
                    help="learn the rotation ahead of PQ (OPQ) with this many rotation steps (0 = the workload's)")
    ap.add_argument("--coarse-k", type=int, default=0,
                    help="2-level residual codec: first-level centroids per half (4096 = PQ2x12; plain form, f32 or f16)")
    ap.add_argument("--max-evals", type=int, default=0,
                    help="budget T on level-0 distance evaluations per query (0 = none; plain and both forms)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.precision is None:  # per form: fp16 tables for the batched form, the plain fp32 path otherwise
        args.precision = "f16" if args.form == "batched" else "f32"
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the search shards over GPUs by query "
                                   "slices or by database shards, each GPU running this path on its share",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import datagen
    import paper_1804_09996_amd as lc
    from paper_1804_09996_amd import builder

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read and written")
        del src, dst
    if args.form == "batched":
        return bench_batched(args)
    if args.form == "serve":
        return bench_serve(args)
    if args.form == "assign":
        return bench_assign(args)
    w = datagen.WORKLOADS[args.workload if args.workload != "C5-20M" else "C2-1M"]
    if args.m_beta != 1:
        w = dataclasses.replace(w, m_beta=args.m_beta)
    if args.n_beta:
        w = dataclasses.replace(w, n_beta=args.n_beta)
    if args.opq_iters:
        w = dataclasses.replace(w, opq_iters=args.opq_iters)
    if args.coarse_k:
        if args.form != "plain" or args.precision == "f16+bf16":
            raise SystemExit("--coarse-k takes --form plain with --precision f32 or f16 (the bf16 refinement covers "
                             "the one-level codec)")
        w = dataclasses.replace(w, coarse_k=args.coarse_k)
    dev = torch.device("cuda:0")
    t0 = time.time()
    if w.coarse_k:  # the 2-level codec is built on the host
        ix, db, q = builder.build_workload(w, cache_dir=args.cache, log=log)
    else:
        from paper_1804_09996_amd import gpu_build
        ix, db, q = gpu_build.build_workload_gpu(w, device=dev, log=log, cache_dir=args.gpu_index_cache or None)
    log(f"index ready in {time.time() - t0:.1f}s (n={ix.n}, max_level={ix.max_level})")
    gix = lc.Index.from_index(ix, device=dev)
    qd = torch.from_numpy(q).to(dev)
    nq = q.shape[0]
    K = w.topk
    gt = ground_truth(torch, db, q, dev)

    FORMS = {"f32": (lc.LC_LUT_F32, lc.LC_REFINE_F32), "f16": (lc.LC_LUT_F16, lc.LC_REFINE_F32),
             "f16+bf16": (lc.LC_LUT_F16, lc.LC_REFINE_BF16_RESCORE)}

    side_streams, ws_cache = [], {}

    def run(form, ef, S, steps, warmup, streams=None):
        """Time `steps` steps.  With several streams, step k runs on stream
        k mod streams with its own workspace and outputs, so consecutive
        batches overlap on the device (a batch's walk tail is filled by the
        next batch's walk, as in continuous batching); per-kernel times then
        come from a separate one-stream run, in which launches do not overlap."""
        streams = streams or args.streams
        lut_dt, ref_p = FORMS[form]
        if streams == 1:
            lanes = [(torch.cuda.current_stream(dev), gix.workspace(nq, max(ef, S), S))]
        else:
            # the same streams for every configuration of the run, each with its own workspace
            while len(side_streams) < streams:
                side_streams.append(torch.cuda.Stream(device=dev))
            nb = gix.workspace_bytes(nq, max(ef, S), S)
            if ws_cache.get("bytes", 0) < nb or len(ws_cache.get("ws", [])) < streams:
                ws_cache["ws"] = [torch.zeros(nb, dtype=torch.uint8, device=dev) for _ in range(streams)]
                ws_cache["bytes"] = nb
            lanes = list(zip(side_streams[:streams], ws_cache["ws"][:streams]))
        torch.cuda.synchronize()

        def step(k, ev=None):
            st_, ws = lanes[k % len(lanes)]
            with torch.cuda.stream(st_):
                if ev is not None:
                    ev[0].record()
                # an index with a projection projects the batch once (timed with the tables)
                qx = gix.project(qd) if gix.has_projection else qd
                lut, scale = gix.build_lut(qx, lut_dt, projected=gix.has_projection)
                if ev is not None:
                    ev[1].record()
                r = gix.search(lut, scale, ef=None, ef_max=ef, S=S, stats=True, ws=ws, max_evals=args.max_evals)
                if ev is not None:
                    ev[2].record()
                ids, d = gix.refine(qx, r.cand_ids, r.cand_n, K, ref_p, projected=gix.has_projection)
                if ev is not None:
                    ev[3].record()
            return ids, d, r

        for k in range(max(warmup, streams)):  # every stream's buffers exist before the timed steps
            step(k)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ids, d, r = step(k, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(3)] for k in range(steps)])
        step_ms = np.array([evs[k][0].elapsed_time(evs[k][3]) for k in range(steps)])
        ids_np = ids.cpu().numpy()
        st = r.stats.cpu().numpy()
        out = {"precision": form, "ef": ef, "S": S, "streams": streams, "qps": nq * steps / wall,
               "ms_per_step": wall / steps * 1e3,
               "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
               "recall": {f"R@{r_}": recall(ids_np, gt, r_) for r_ in (1, 10, 100) if r_ <= K},
               "ids": ids_np, "d": d.cpu().numpy(), "stats": st, "cand_n": r.cand_n.cpu().numpy()}
        if streams == 1:
            out["kernels_ms"] = dict(zip(("build_lut", "walk", "refine"), kern.mean(0).tolist()))
        else:
            one = run(form, ef, S, max(3, steps // 2), 1, streams=1)
            assert np.array_equal(one["ids"], ids_np) and np.array_equal(one["stats"], st)
            out["kernels_ms"] = one["kernels_ms"]
            out["one_stream"] = {k_: one[k_] for k_ in ("qps", "ms_per_step", "step_ms_p50", "step_ms_p99")}
        return out

    def end_to_end(form, ef, S, reps=7):
        """One batch from pinned host memory to results in pinned host memory
        (queries copied in, the whole path, ids and distances copied out), on
        one stream; the median over reps."""
        lut_dt, ref_p = FORMS[form]
        hq = torch.from_numpy(q).pin_memory()
        h_ids = torch.empty((nq, K), dtype=torch.int32).pin_memory()
        h_d = torch.empty((nq, K), dtype=torch.float32).pin_memory()
        qbuf = torch.empty_like(qd)
        ws = gix.workspace(nq, max(ef, S), S)
        times = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            qbuf.copy_(hq, non_blocking=True)
            qx = gix.project(qbuf) if gix.has_projection else qbuf
            lut, scale = gix.build_lut(qx, lut_dt, projected=gix.has_projection)
            r = gix.search(lut, scale, ef=None, ef_max=ef, S=S, stats=False, ws=ws, max_evals=args.max_evals)
            ids, d = gix.refine(qx, r.cand_ids, r.cand_n, K, ref_p, projected=gix.has_projection)
            h_ids.copy_(ids, non_blocking=True)
            h_d.copy_(d, non_blocking=True)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times[1:]))
        return {"ms_per_batch": ms, "qps": nq / (ms * 1e-3),
                "note": "one stream, queries from and results to pinned host memory (PCIe both ways)"}

    # the plain path at the workload's own operating point defines the target recall
    plain = run("f32", w.ef, w.shortlist, args.steps, args.warmup)
    r_target = plain["recall"]["R@1"]
    head = plain
    if args.form == "plain" and (args.precision, args.ef or w.ef, args.shortlist or w.shortlist) != \
            ("f32", w.ef, w.shortlist):
        head = run(args.precision, args.ef or w.ef, args.shortlist or w.shortlist, args.steps, args.warmup)
    curves = {}
    if args.form == "both":
        # the workload's operating point, smaller short-lists, and larger pools in steps fine enough near
        # it that a form just short of the recall target at one point meets it at the next
        grid = sorted({(w.ef, s_) for s_ in (K, (K + w.shortlist) // 2, w.shortlist) if s_ >= K} |
                      {(e_, w.shortlist) for e_ in (w.ef_eff + 16, w.ef_eff + 32, w.ef_eff + 64, w.ef_eff + 128)})
        for form in FORMS:
            curves[form] = []
            for ef_, s_ in grid:
                res = plain if (form == "f32" and (ef_, s_) == (w.ef, w.shortlist)) else \
                    run(form, ef_, s_, max(3, args.steps // 2), 1)
                curves[form].append(res)
                log(f"{form} ef={ef_} S={s_}: R@1 {res['recall']['R@1']:.4f} QPS {res['qps']:.0f}")

        def best_at_target(form):
            ok = [c for c in curves[form] if c["recall"]["R@1"] >= r_target]
            return max(ok, key=lambda c: c["qps"]) if ok else None

        best = {f: best_at_target(f) for f in FORMS}
        fp16 = [b for f, b in best.items() if f != "f32" and b is not None]
        if fp16:
            pick = max(fp16, key=lambda c: c["qps"])
            head = run(pick["precision"], pick["ef"], pick["S"], args.steps, args.warmup)  # the timed step
        log("at R@1 >= %.4f: " % r_target + ", ".join(
            f"{f}: {b['qps']:.0f} (ef {b['ef']}, S {b['S']})" for f, b in best.items() if b))

    E = head["stats"][:, 0].astype(np.int64)
    D = head["stats"][:, 1].astype(np.int64)
    S_h = head["S"]
    wm = head["kernels_ms"]["walk"]
    f16 = head["precision"] != "f32"
    wb = walk_bytes(w, E, D, S_h) if not f16 else \
        walk_bytes(w, E, D, S_h) - nq * 2 * w.m * 256 + nq * 4 * w.m  # fp16 table + scales
    rb = refine_bytes(w, head["cand_n"], K)
    lb = lut_bytes(w, nq) if not f16 else float(nq) * (4 * w.d + 2 * w.m * 256 + 4 * w.m)
    traffic = traffic_from_profiles({"form": "plain", "workload": w.name, "table": head["precision"].split("+")[0],
                                     "ef": head["ef"], "S": S_h})
    form = {"f32": "plain fp32 path",
            "f16": "fp16 tables in the walk, fp32 refinement",
            "f16+bf16": "precision form: fp16 tables, bf16 refinement, exact fp32 re-score of the best 2K"}[head["precision"]]
    if head is not plain and args.form == "plain":
        form += "; the configuration given on the command line"
    elif head is not plain:
        form += ("; the fastest measured (ef, shortlist) of the fp16 forms whose 1-recall@1 is at least the plain "
                 "path's at its own operating point (the same grid is swept for the plain path)")
    out = {
        "metric": METRIC, "value": head["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16" if f16 else "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.n} d={w.d} Gaussian mixture ({w.n_comp} components, "
                               f"L2-normalised), " + (f"learned rotation ({w.opq_iters} steps) + " if w.opq_iters else "") +
                               (f"2-level codec: first level 2x{w.coarse_k} centroids, residual " if w.coarse_k else "") +
                               f"PQ {w.m}x256, level-0 degree {w.deg0}, k={w.k_reg}, " +
                               (f"product beta codebook {w.m_beta} blocks x {w.n_beta}" if w.m_beta > 1
                                else f"beta codebook {w.n_beta}") +
                               (f", at most {args.max_evals} level-0 distance evaluations per query"
                                if args.max_evals else "") +
                               f", top-{K}, {nq} queries per step; {form}; "
                               f"efSearch {head['ef']}, shortlist {S_h}; " +
                               (f"consecutive steps alternate over {args.streams} streams (each with its own workspace "
                                f"and outputs), so one batch's walk tail overlaps the next batch" if args.streams > 1
                                else "each step runs alone"),
                   "queries_per_step": nq, "ef": head["ef"], "shortlist": S_h, "streams": args.streams,
                   "index": f"built from seed {w.seed} by " + ("liblc_build (host)" if w.coarse_k
                                                                  else "gpu_build (GPU steps, the host builder's arrays)")},
        "roofline": {"bound": "hbm", "achieved": wb / (wm * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": wb / (wm * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": walk_kernel_name(gix, nq, head["ef"], S_h, head["precision"]),
                     "algorithmic_bytes_per_launch": wb},
        "kernels_ms": head["kernels_ms"],
        "kernels_GBps_algorithmic": {"build_lut": lb / (head["kernels_ms"]["build_lut"] * 1e-3) / 1e9,
                                     "walk": wb / (wm * 1e-3) / 1e9,
                                     "refine": rb / (head["kernels_ms"]["refine"] * 1e-3) / 1e9},
        "recall": head["recall"], "batch_latency_ms": {"p50": head["step_ms_p50"], "p99": head["step_ms_p99"]},
        "one_stream": head.get("one_stream"),
        "end_to_end": end_to_end(head["precision"], head["ef"], S_h),
        "walk_mean_E": float(E.mean()), "walk_mean_D": float(D.mean()),
        "plain_fp32": {"qps": plain["qps"], "recall": plain["recall"], "ef": plain["ef"], "S": plain["S"],
                       "kernels_ms": plain["kernels_ms"], "one_stream": plain.get("one_stream")},
    }
    if curves:
        out["target_R@1"] = r_target
        out["curves"] = {f: [{"ef": c["ef"], "S": c["S"], "qps": c["qps"], "R@1": c["recall"]["R@1"],
                              "R@10": c["recall"].get("R@10"), "walk_ms": c["kernels_ms"]["walk"],
                              "refine_ms": c["kernels_ms"]["refine"],
                              "qps_one_stream": (c.get("one_stream") or {}).get("qps")} for c in cs]
                         for f, cs in curves.items()}
        out["qps_at_target_R@1"] = {f: (max((c["qps"] for c in cs if c["recall"]["R@1"] >= r_target), default=None))
                                    for f, cs in curves.items()}
    if not args.no_cpu_baseline:
        cb, oix, ores, n = cpu_baseline(ix, db, q, w)
        out["cpu_baseline"] = cb
        from tests import parity
        s = parity.summarize(oix, q[:n], plain["ids"][:n], plain["d"][:n], ores)
        walk_same = float(np.mean([np.array_equal(plain["stats"][i], ores["stats"][i]) for i in range(n)]))
        out["parity_sample"] = {"form": "plain fp32", "queries": n, "exact_frac": s["exact_frac"],
                                "strict_frac": s["strict_frac"], "max_rel_dist_err": s["max_rel_err"],
                                "walk_E_D_identical_frac": walk_same}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
