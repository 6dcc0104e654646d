"""Index build with its data-parallel steps on the GPU.

The same index as :func:`builder.build_index` (the host builder), with:

* the projection of the database and its PQ encoding on the GPU
  (``lc_project_exact``, ``lc_pq_encode``);
* the graph (Sec. 5.1: vectors added in batches, each searched against the
  graph as it stood when the batch began, then linked): the host builder
  inserts the nodes of the upper levels, which come first in the insertion
  order, then ``lc_graph_insert`` inserts every later batch (level-0 nodes
  only) on the GPU, with the same batch sizes;
* the regression-codebook assignment of every vector (``lc_assign_beta``).

The codebooks (PQ k-means on the training set, the regression codebook's
least squares on its training subset) stay on the host.  Every step takes its
floats in the order the host builder does, so the arrays are the host
builder's bit for bit (tests/test_gpu_build.py).  The 2-level codec is built
on the host only.
"""
from __future__ import annotations

import ctypes as C
import time
from typing import List, Optional, Tuple

import numpy as np

from . import LC_OK, Index, LCError, _check, _stream, lib
from . import builder as hb

BATCH_MAX = 4096


def batch_schedule(n: int, start: int) -> List[Tuple[int, int]]:
    """(position, size) of the insertion batches from position ``start`` of
    the insertion order: size clamp(position / 16, 1, 4096), the last one cut
    at n (the host builder's schedule)."""
    out, pos = [], max(1, int(start))
    while pos < n:
        bs = max(1, min(BATCH_MAX, pos // 16))
        bs = min(bs, n - pos)
        out.append((pos, bs))
        pos += bs
    return out


def build_index_gpu(w, db, train, proj, level_u, pq_init, beta_ids, beta_init, device="cuda",
                    nthreads: Optional[int] = None, log=None, timings: Optional[dict] = None) -> hb.BuiltIndex:
    import torch

    if getattr(w, "coarse_k", 0):
        raise ValueError("the 2-level codec is built by builder.build_index (host)")
    L, H = lib(), hb.lib()
    dev = torch.device(device)
    nt = nthreads or hb.threads()
    db, train, proj = hb._c(db, np.float32), hb._c(train, np.float32), hb._c(proj, np.float32)
    pq_init, level_u, beta_init = hb._c(pq_init, np.int64), hb._c(level_u, np.float64), hb._c(beta_init, np.int64)
    n, d = db.shape
    tm = {} if timings is None else timings
    t0 = time.time()
    if getattr(w, "opq_iters", 0) > 0:
        proj, _ = hb.opq_train(train, w.d_pad, w.m, proj, pq_init, w.opq_iters, max(2, w.pq_iters // 5), nt)
    cent = np.empty((w.m, 256, w.d_pad // w.m), np.float32)
    hb._ok(H.lcb_pq_train(hb._p(train), train.shape[0], d, hb._p(proj), w.d_pad, w.m, hb._p(pq_init), w.pq_iters,
                          nt, hb._p(cent)), "lcb_pq_train")
    tm["pq_train_s"] = time.time() - t0

    # projection and encoding of the database on the GPU
    t1 = time.time()
    cs = hb.code_stride_for(w.m)
    with torch.cuda.device(dev):
        st = _stream(torch, dev)
        x_g = torch.from_numpy(db).to(dev)
        xp_g = torch.empty((n, w.d_pad), dtype=torch.float32, device=dev)
        proj_g = None if proj is None else torch.from_numpy(proj).to(dev)
        _check(L.lc_project_exact(x_g.data_ptr(), n, d, None if proj_g is None else proj_g.data_ptr(), w.d_pad,
                                  xp_g.data_ptr(), st), "lc_project_exact")
        cent_g = torch.from_numpy(cent).to(dev)
        codes_g = torch.zeros((n, cs), dtype=torch.uint8, device=dev)
        _check(L.lc_pq_encode(xp_g.data_ptr(), n, w.d_pad, w.m, cent_g.data_ptr(), codes_g.data_ptr(), cs, st),
               "lc_pq_encode")
        codes = codes_g.cpu().numpy()
    tm["encode_s"] = time.time() - t1

    # the upper levels' nodes on the host
    t2 = time.time()
    level = np.empty(n, np.int8)
    rows = int(H.lcb_levels(hb._p(level_u), n, w.level_ratio, w.max_level_cap, hb._p(level)))
    adj0 = np.empty((n, w.deg0), np.int32)
    up_base = np.empty(n, np.int32)
    adj_up = np.empty((max(rows, 1), w.deg_up), np.int32)
    entry, maxl, next_pos = C.c_int32(), C.c_int32(), C.c_int64()
    hb._ok(H.lcb_graph_build_part(hb._p(db), n, d, hb._p(proj), w.d_pad, w.m, hb._p(cent), hb._p(codes), cs,
                                  hb._p(level), w.deg0, w.deg_up, w.ef_construction, nt, hb._p(adj0), hb._p(up_base),
                                  hb._p(adj_up), C.byref(entry), C.byref(maxl), None, 1, C.byref(next_pos)),
           "lcb_graph_build_part")
    adj_up = adj_up[:rows]
    tm["graph_host_s"] = time.time() - t2
    tm["graph_host_nodes"] = int(next_pos.value)

    # every later batch on the GPU
    t3 = time.time()
    order0 = np.flatnonzero(level == 0).astype(np.int32)  # the level-0 nodes, in insertion order
    n_up = n - order0.size
    sched = batch_schedule(n, int(next_pos.value))
    if sched:
        assert sched[0][0] >= n_up, "the host part stops at the first batch of level-0 nodes only"
        meta = {"d": d, "d_pad": w.d_pad, "m": w.m, "deg0": w.deg0, "deg_up": w.deg_up, "k_reg": w.k_reg,
                "entry": int(entry.value), "max_level": int(maxl.value)}
        arrays = {"proj": proj, "centroids": cent, "codes": codes, "adj0": adj0, "up_base": up_base,
                  "adj_up": adj_up, "beta": np.zeros((1, w.k_reg + 1), np.float32),
                  "beta_idx": np.zeros(n, np.uint8)}
        gix = Index(arrays, meta, device=dev)
        with torch.cuda.device(dev):
            st = _stream(torch, dev)
            nodes_g = torch.from_numpy(order0).to(dev)
            max_count = max(bs for _, bs in sched)
            nb = int(L.lc_graph_insert_workspace_bytes(gix.handle, max_count, w.ef_construction))
            if nb == 0:
                raise LCError(1, "lc_graph_insert_workspace_bytes")
            ws = torch.zeros(nb, dtype=torch.uint8, device=dev)
            adj0_g = gix.t["adj0"]
            base = nodes_g.data_ptr()
            last = time.time()
            for k, (pos, bs) in enumerate(sched):
                _check(L.lc_graph_insert(gix.handle, adj0_g.data_ptr(), xp_g.data_ptr(), base + 4 * (pos - n_up), bs,
                                         max_count, w.ef_construction, ws.data_ptr(), nb, st), "lc_graph_insert")
                if log and time.time() - last > 10.0 and k % 64 == 0:
                    torch.cuda.synchronize(dev)
                    last = time.time()
                    log(f"index build: GPU graph batch {k} / {len(sched)} (position {pos} of {n}, "
                        f"{last - t3:.0f} s)")
            adj0 = adj0_g.cpu().numpy()
            del ws, nodes_g
        gix.close()
        del gix
    tm["graph_gpu_s"] = time.time() - t3
    tm["graph_gpu_batches"] = len(sched)
    del xp_g

    # regression codebook on the host, the assignment of every vector on the GPU
    t4 = time.time()
    mb = w.m_beta
    beta = np.empty((w.n_beta, w.k_reg + 1) if mb == 1 else (mb, w.n_beta, w.k_reg + 1), np.float32)
    bids = hb._c(beta_ids, np.int64)
    hb._ok(H.lcb_beta_train(hb._p(db), hb._p(bids), bids.shape[0], d, hb._p(proj), w.d_pad, w.m, hb._p(cent),
                            hb._p(codes), cs, hb._p(adj0), w.deg0, w.k_reg, w.n_beta, mb, hb._p(beta_init),
                            w.beta_kmeans_iters, w.em_iters, nt, hb._p(beta), None, None), "lcb_beta_train")
    tm["beta_train_s"] = time.time() - t4
    t5 = time.time()
    ix = hb.BuiltIndex(n=n, d=d, d_pad=w.d_pad, m=w.m, deg0=w.deg0, deg_up=w.deg_up, k_reg=w.k_reg, n_beta=w.n_beta,
                       entry=int(entry.value), max_level=int(maxl.value), proj=proj, centroids=cent, codes=codes,
                       adj0=adj0, level=level, up_base=up_base, adj_up=adj_up, beta=beta,
                       beta_idx=np.zeros(n if mb == 1 else (n, mb), np.uint8), m_beta=mb)
    gix = Index.from_index(ix, device=dev)
    with torch.cuda.device(dev):
        bidx = gix.assign_beta(x_g).cpu().numpy()
    ix.beta_idx = bidx.reshape(n) if mb == 1 else bidx.reshape(n, mb)
    gix.close()
    del gix, x_g
    torch.cuda.empty_cache()
    tm["beta_assign_s"] = time.time() - t5
    tm["total_s"] = time.time() - t0
    if log:
        log("index build (GPU steps): " + ", ".join(f"{k} {v:.1f}" if isinstance(v, float) else f"{k} {v}"
                                                     for k, v in tm.items()))
    return ix


def build_workload_gpu(w, device="cuda", nthreads: Optional[int] = None, log=None, timings: Optional[dict] = None,
                       cache_dir: Optional[str] = None):
    """(index, db, queries) for a workload from its seed, built by build_index_gpu
    (or loaded from ``cache_dir``, where a build of the same workload fields was
    saved; ``timings`` then holds ``{"cached": 1}`` only)."""
    import os

    import datagen
    db = datagen.vectors(w, "db")
    q = datagen.vectors(w, "query")
    path = None
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        path = os.path.join(cache_dir, f"{w.name}-{w.key()}-gpu.npz")
        if os.path.exists(path):
            if timings is not None:
                timings["cached"] = 1
            if log:
                log(f"index loaded from {path}")
            return hb.BuiltIndex.load(path), db, q
    train = datagen.vectors(w, "train")
    ix = build_index_gpu(w, db, train, datagen.projection(w), datagen.level_uniforms(w),
                         datagen.pq_init_ids(w, train.shape[0]), datagen.beta_train_ids(w),
                         datagen.beta_init_ids(w, min(w.n, w.n_beta_train)), device, nthreads, log, timings)
    if path:
        ix.save(path + ".tmp.npz")
        os.replace(path + ".tmp.npz", path)
    return ix, db, q
