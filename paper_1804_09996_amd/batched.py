"""Batched form: one large batch of queries with per-query efSearch.

The whole path for the batch (tables, walk, refinement) runs on static device
buffers and is captured in a HIP graph; each step copies the queries and
their ef into the static inputs and replays the graph.  A batch whose ef
values change the class rows, a class's largest pool or a workspace is
recorded again before its first replay, so a captured launch never meets a
query beyond its pool or a freed workspace.  The walk is the
persistent kernel: resident slots take queries from an atomic counter, longest
ef first, so the long walks start early and the short ones fill the tail.

Queries are split into *ef classes* by the pool they need (max(ef, S),
rounded up to 64): each class is walked by its own launch whose slots are
sized for that class only (a pool of at most 128 entries lives in registers,
and smaller pools leave LDS for more resident slots), the launches of all
classes run concurrently inside the one graph (largest pools first), and the
refinement runs once over the whole batch.  On the host the batch is
permuted into (class, longest ef first) order so that every class is a
contiguous range of rows; the results are permuted back on the device.  The
class boundaries and the walk schedule come from the autotuner; neither
changes any result.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import LC_LUT_F16, LC_LUT_F32, SearchResult, _check, _stream, autotune, \
    lib


def class_limits_options(ef_max: int, S: int) -> List[List[int]]:
    """Candidate splits: pool limits (ascending, last = the batch's largest
    pool) at which the batch is cut into classes."""
    top = max(ef_max, S)
    top = (top + 63) // 64 * 64
    opts = [[top]]
    for cuts in ([128], [128, 256]):
        lim = [c for c in cuts if max(S, 1) <= c < top] + [top]
        if lim not in opts:
            opts.append(lim)
    return opts


def class_permutation(ef: np.ndarray, S: int, limits: Sequence[int]):
    """Order of the batch by (class, longest ef first) and the classes' row
    ranges (start, end, largest pool in the class).  A query's class is the
    first limit at or above its pool max(ef, S); pools above the last limit go
    to the last class."""
    ef = np.asarray(ef, dtype=np.int64).reshape(-1)
    limits = np.asarray(sorted(int(x) for x in limits))
    pool = np.maximum(ef, S)
    cls = np.minimum(np.searchsorted(limits, pool, side="left"), len(limits) - 1)
    perm = np.lexsort((-ef, cls)).astype(np.int64)  # class, then longest ef first (stable)
    ranges, start = [], 0
    for c, lim in enumerate(limits):
        n = int((cls == c).sum())
        if n:
            top = int(pool[perm[start:start + n]].max())  # the class's own largest pool sizes its launch
            ranges.append((start, start + n, top))
        start += n
    return perm, ranges


class BatchedSearcher:
    def __init__(self, gix, nq: int, ef_max: int, S: int, K: int, precision: str = "f32"):
        torch = gix.torch
        self.torch, self.gix = torch, gix
        self.nq, self.ef_max, self.S, self.K = nq, ef_max, S, K
        self.lut_dtype = LC_LUT_F16 if precision in ("f16", "f16+bf16") else LC_LUT_F32
        self.refine_p = gix.refine_mode(precision)
        dev = gix.device
        # the batch in (class, longest ef first) order, and the map back to query order
        self.q = torch.empty((nq, gix.d), dtype=torch.float32, device=dev)
        # an index with a projection: the batch projected once (static, so that a captured step reuses it)
        self.qp = torch.empty((nq, gix.d_pad), dtype=torch.float32, device=dev) if gix.has_projection else None
        self.ef = torch.empty(nq, dtype=torch.int32, device=dev)
        self.inv = torch.empty(nq, dtype=torch.int64, device=dev)
        self.res = SearchResult(torch.empty((nq, S), dtype=torch.int32, device=dev),
                                torch.empty((nq, S), dtype=torch.float32, device=dev),
                                torch.empty(nq, dtype=torch.int32, device=dev),
                                torch.empty((nq, 2), dtype=torch.int32, device=dev))
        self.sched = None
        self.limits = [max(ef_max, S)]
        self.ranges = [(0, nq, max(ef_max, S))]
        self.streams, self.ws = [], []
        self.graph = None
        self.table = None
        self._host_q = None
        self._host_ef = None

    # -- inputs -------------------------------------------------------------
    def set_inputs(self, q, ef):
        """Copy a batch in (query order); it is stored permuted by class and
        longest ef first."""
        self._host_q = np.ascontiguousarray(np.asarray(q, dtype=np.float32))
        self._host_ef = np.asarray(ef, dtype=np.int32).reshape(-1)
        self._apply()

    def _apply(self):
        torch = self.torch
        ef = self._host_ef
        perm, ranges = class_permutation(ef, self.S, self.limits)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        if self.graph is not None:
            # a replay still in flight reads the static inputs and workspaces
            torch.cuda.synchronize(self.gix.device)
        self.q.copy_(torch.from_numpy(self._host_q[perm]))
        self.ef.copy_(torch.from_numpy(ef[perm]))
        self.inv.copy_(torch.from_numpy(inv))
        old_ranges, old_ws = self.ranges, list(self.ws)
        self.ranges = ranges
        self._size_lanes()
        if self.graph is not None and (ranges != old_ranges or len(old_ws) != len(self.ws)
                                       or any(a is not b for a, b in zip(old_ws, self.ws))):
            # the captured launches hold the old class rows, pool limits and workspaces: record the step
            # again for the new ones (the old graph and workspaces are released only after that)
            retired = (self.graph, old_ws)
            self.graph = None
            self.capture()
            del retired

    def _size_lanes(self):
        torch, gix = self.torch, self.gix
        while len(self.streams) < len(self.ranges):
            self.streams.append(torch.cuda.Stream(device=gix.device))
        ws = []
        for i, (r0, r1, efm) in enumerate(self.ranges):
            nb = gix.workspace_bytes(r1 - r0, efm, self.S, self.sched)
            old = self.ws[i] if i < len(self.ws) else None
            ws.append(old if old is not None and old.numel() >= nb else
                      torch.zeros(max(nb, 1), dtype=torch.uint8, device=gix.device))
        self.ws = ws

    def set_classes(self, limits: Sequence[int]):
        """Pool limits of the ef classes (ascending); re-permutes the batch
        (and records the captured step again when its classes change)."""
        self.limits = sorted(int(x) for x in limits)
        if self._host_ef is not None:
            self._apply()

    # -- the step -----------------------------------------------------------
    def _walks(self, lut, scale, sched=None):
        """One walk launch per class, each on its own stream, joined back; the
        class of the largest pools first, so that the longest walks start
        first (a launch's resident slots take the device until its queue
        drains, and the next class fills the slots it frees)."""
        torch, gix = self.torch, self.gix
        main = torch.cuda.current_stream(gix.device)
        sched = sched if sched is not None else self.sched
        for i in reversed(range(len(self.ranges))):
            r0, r1, efm = self.ranges[i]
            st = self.streams[i]
            st.wait_stream(main)
            with torch.cuda.stream(st):
                out = SearchResult(self.res.cand_ids[r0:r1], self.res.cand_adc[r0:r1], self.res.cand_n[r0:r1],
                                   self.res.stats[r0:r1])
                gix.search(lut[r0:r1], None if scale is None else scale[r0:r1], ef=self.ef[r0:r1], ef_max=efm,
                           S=self.S, sched=sched, out=out, ws=self.ws[i])
        for i in range(len(self.ranges)):
            main.wait_stream(self.streams[i])

    def _queries(self):
        """The batch as the tables and the refinement take it (projected once
        when the index has a projection) and whether it is projected."""
        if self.qp is None:
            return self.q, False
        _check(lib().lc_project_queries(self.gix.handle, self.q.data_ptr(), self.nq, self.qp.data_ptr(),
                                        _stream(self.torch, self.gix.device)), "lc_project_queries")
        return self.qp, True

    def _step(self):
        gix = self.gix
        qx, pj = self._queries()
        lut, scale = gix.build_lut(qx, self.lut_dtype, projected=pj)
        self._walks(lut, scale)
        ids, d = gix.refine(qx, self.res.cand_ids, self.res.cand_n, self.K, self.refine_p, projected=pj)
        return ids.index_select(0, self.inv), d.index_select(0, self.inv)

    # -- tuning -------------------------------------------------------------
    def _time_walks(self, lut, scale, sched, reps: int) -> float:
        torch = self.torch
        self._walks(lut, scale, sched)  # warm up
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            self._walks(lut, scale, sched)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        return times[len(times) // 2]

    def tune(self, cands=None, reps: int = 3, cache_path: Optional[str] = autotune.DEFAULT_CACHE, log=None):
        """Pick the walk schedule for the whole batch (one class), then the
        class split, by timing the walk phase of this batch."""
        self.set_classes([max(self.ef_max, self.S)])
        qx, pj = self._queries()
        lut, scale = self.gix.build_lut(qx, self.lut_dtype, projected=pj)
        self.sched, self.table = autotune.tune(self.gix, lut, ef=self.ef, ef_max=self.ef_max, S=self.S,
                                               cands=cands, reps=reps, cache_path=cache_path, log=log, scale=scale)
        best = None
        for lim in class_limits_options(self.ef_max, self.S):
            self.set_classes(lim)
            qx, pj = self._queries()
            lut, scale = self.gix.build_lut(qx, self.lut_dtype, projected=pj)
            ms = self._time_walks(lut, scale, self.sched, reps)
            self.table.append({"classes": lim, "schedule": self.sched.as_dict(), "ms": ms})
            if log:
                log(f"autotune ef classes {lim}: {ms:.3f} ms")
            if best is None or ms < best[1]:
                best = (lim, ms)
        self.set_classes(best[0])
        return self.sched

    # -- graph ----------------------------------------------------------------
    def capture(self):
        """Record the step in a HIP graph (the workspaces are sized beforehand
        so that nothing is allocated or cleared by a memset inside the graph)."""
        torch = self.torch
        self._size_lanes()
        s = torch.cuda.Stream(device=self.gix.device)
        s.wait_stream(torch.cuda.current_stream(self.gix.device))
        with torch.cuda.stream(s):
            self._step()  # warm-up outside the graph (sets kernel attributes, pools)
        torch.cuda.current_stream(self.gix.device).wait_stream(s)
        torch.cuda.synchronize(self.gix.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.ids, self.d = self._step()
        return self.graph

    def run(self):
        """One step; returns (ids [nq, K], distances [nq, K]) in query order."""
        if self.graph is not None:
            self.graph.replay()
            return self.ids, self.d
        return self._step()
