"""Batched form: one large batch of queries with per-query efSearch.

The whole path for the batch (tables, walk, refinement) runs on static device
buffers and is captured once in a HIP graph; each step copies the queries and
their ef into the static inputs and replays the graph.  The walk is the
persistent kernel: resident slots take queries from an atomic counter, in an
order fixed on the host as longest ef first, so the long walks start early
and the short ones fill the tail.  The walk's schedule (visited-table size,
prefetch, queue) comes from the autotuner; every schedule gives the same
results.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import LC_LUT_F16, LC_LUT_F32, LC_REFINE_BF16_RESCORE, LC_REFINE_F32, SearchResult, autotune


class BatchedSearcher:
    def __init__(self, gix, nq: int, ef_max: int, S: int, K: int, precision: str = "f32"):
        torch = gix.torch
        self.torch, self.gix = torch, gix
        self.nq, self.ef_max, self.S, self.K = nq, ef_max, S, K
        self.lut_dtype = LC_LUT_F16 if precision == "f16" else LC_LUT_F32
        self.refine_p = LC_REFINE_BF16_RESCORE if precision == "f16" else LC_REFINE_F32
        dev = gix.device
        self.q = torch.empty((nq, gix.d), dtype=torch.float32, device=dev)
        self.ef = torch.empty(nq, dtype=torch.int32, device=dev)
        self.order = torch.empty(nq, dtype=torch.int32, device=dev)
        self.res = SearchResult(torch.empty((nq, S), dtype=torch.int32, device=dev),
                                torch.empty((nq, S), dtype=torch.float32, device=dev),
                                torch.empty(nq, dtype=torch.int32, device=dev),
                                torch.empty((nq, 2), dtype=torch.int32, device=dev))
        self.sched = None
        self.graph = None
        self.table = None

    def set_inputs(self, q, ef):
        """Copy a batch in; the processing order is longest ef first (stable)."""
        torch = self.torch
        ef = np.asarray(ef, dtype=np.int32).reshape(-1)
        order = np.argsort(-ef.astype(np.int64), kind="stable").astype(np.int32)
        self.q.copy_(torch.as_tensor(q, dtype=torch.float32))
        self.ef.copy_(torch.from_numpy(ef))
        self.order.copy_(torch.from_numpy(order))

    def _step(self):
        gix = self.gix
        lut, scale = gix.build_lut(self.q, self.lut_dtype)
        gix.search(lut, scale, ef=self.ef, ef_max=self.ef_max, S=self.S, sched=self.sched, order=self.order,
                   out=self.res)
        return gix.refine(self.q, self.res.cand_ids, self.res.cand_n, self.K, self.refine_p)

    def tune(self, cands=None, reps: int = 3, cache_path: Optional[str] = autotune.DEFAULT_CACHE, log=None):
        lut, scale = self.gix.build_lut(self.q, self.lut_dtype)
        self.sched, self.table = autotune.tune(self.gix, lut, ef=self.ef, ef_max=self.ef_max, S=self.S,
                                               cands=cands, reps=reps, cache_path=cache_path, log=log)
        return self.sched

    def capture(self):
        """Record the step in a HIP graph (the workspace is sized beforehand so
        that nothing is allocated or cleared by a memset inside the graph)."""
        torch = self.torch
        self.gix.workspace(self.nq, self.ef_max, self.S, self.sched)
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
