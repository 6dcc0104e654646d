"""Continuous-batching serving loop over a resident index.

Requests (a batch of queries and one efSearch each) arrive over time.  The
loop keeps a FIFO of arrived requests and a fixed set of *slots*; each slot
owns pre-allocated device buffers (queries, tables, pool output, results, its
own walk workspace) and its own stream.  Whenever a slot is free, the loop
admits arrived requests into it, in arrival order, while they fit the slot's
query capacity and the global memory budget (bytes of tables, pools and
short-lists of every query in flight), and launches the whole search path for
those queries on the slot's stream.  Slots run concurrently, so requests that
arrive while others are on the GPU start as soon as a slot and memory free
up, and their kernels overlap on the device with the ones already running.
A request is never split across slots; its latency runs from its (scheduled)
arrival to the moment its results are in host memory.

Results of a query do not depend on the batch it is launched with (every
kernel is per-query and the walk's schedule does not change results), which
the tests check as "same result alone and in the mix".

The scheduler is independent of the engine: :class:`GpuEngine` launches the
HIP kernels through the C-ABI; tests drive the scheduler with a fake engine on
a virtual clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    queries: np.ndarray  # [b, d] float32
    ef: int
    arrival: float       # seconds on the loop's clock
    start: float = -1.0  # launch time
    done: float = -1.0   # results on the host
    slot: int = -1
    ids: Optional[np.ndarray] = None
    dist: Optional[np.ndarray] = None
    qidx: Optional[np.ndarray] = None  # rows of the query pool the request carries

    @property
    def size(self) -> int:
        return int(self.queries.shape[0])

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def query_bytes(m: int, S: int, K: int, d: int, lut_bytes: int = 2, d_proj: int = 0, lut_entries: int = 0) -> int:
    """Device bytes one query holds while in flight: its table (+ scales),
    pool output (ids + distances), results, the query itself (and its
    projection, d_proj values, when the index has one) and its ef.
    ``lut_entries``: table entries per query when not m * 256 (the 2-level
    codec's row, Index.lut_stride)."""
    return (lut_entries or m * 256) * lut_bytes + 4 * m + 8 * S + 4 + 8 * K + 4 * d + 4 * d_proj + 4


class Scheduler:
    """Admission and slot bookkeeping (no device code)."""

    def __init__(self, n_slots: int, slot_queries: int, mem_budget: int, bytes_per_query: int):
        self.n_slots = n_slots
        self.slot_queries = slot_queries
        self.mem_budget = mem_budget
        self.bpq = bytes_per_query
        self.pending: collections.deque = collections.deque()
        self.free_slots: List[int] = list(range(n_slots))
        self.in_flight: Dict[int, List[Request]] = {}
        self.mem_used = 0
        self.max_mem_used = 0
        self.mem_waits = 0  # admissions cut short by the memory budget while the slot had room

    def arrive(self, req: Request):
        if req.size > self.slot_queries or req.size * self.bpq > self.mem_budget:
            raise ValueError(f"request {req.rid} of {req.size} queries can never be admitted")
        self.pending.append(req)

    def admit(self) -> Optional[tuple]:
        """Next (slot, requests) to launch, or None.  Takes requests from the
        head of the FIFO while they fit; never skips a request (FIFO fairness)."""
        if not self.free_slots or not self.pending:
            return None
        batch, nq = [], 0
        while self.pending:
            r = self.pending[0]
            need = r.size * self.bpq
            if nq + r.size > self.slot_queries:
                break
            if self.mem_used + need > self.mem_budget:
                self.mem_waits += 1
                break
            self.pending.popleft()
            batch.append(r)
            nq += r.size
            self.mem_used += need
        if not batch:
            return None
        self.max_mem_used = max(self.max_mem_used, self.mem_used)
        slot = self.free_slots.pop(0)
        for r in batch:
            r.slot = slot
        self.in_flight[slot] = batch
        return slot, batch

    def complete(self, slot: int) -> List[Request]:
        batch = self.in_flight.pop(slot)
        for r in batch:
            self.mem_used -= r.size * self.bpq
        self.free_slots.append(slot)
        return batch


class GpuEngine:
    """Launches the search path for one slot on its own stream."""

    def __init__(self, gix, n_slots: int, slot_queries: int, ef_max: int, S: int, K: int,
                 precision: str = "f16", sched=None, record_walks: bool = False, refine: Optional[int] = None,
                 split: Optional[bool] = None):
        import torch

        import paper_1804_09996_amd as lc
        self.torch, self.lc = torch, lc
        self.gix, self.ef_max, self.S, self.K = gix, ef_max, S, K
        self.sched = sched
        # record_walks: HIP events around every walk launch on its slot stream and the (E, D) counts of its
        # queries, for the walk's launch durations and algorithmic bytes (walk_log: one dict per launch)
        self.record_walks = record_walks
        self.walk_log: List[dict] = []
        self.lut_dtype = lc.LC_LUT_F16 if precision in ("f16", "f16+bf16") else lc.LC_LUT_F32
        # split: a batch's queries whose pool fits registers (<= 128 entries) are walked by their own launch,
        # concurrently with the larger pools' launch (each with its own workspace).  None: split when the two
        # classes take different walk kernels (the register pool beside the LDS pool); when both take the same
        # one (an fp16 table in registers keeps every pool in LDS) one launch per batch is faster (measured on
        # the 20M serving workload: 4.19M against 3.15M queries/s with 6 slots of 4096 queries)
        if split is None:
            k_small = gix.walk_plan(slot_queries, min(128, ef_max), S, self.lut_dtype, sched)["kernel"]
            k_big = gix.walk_plan(slot_queries, ef_max, S, self.lut_dtype, sched)["kernel"]
            split = ef_max > 128 and k_small != k_big
        self.split = split
        self.refine_p = gix.refine_mode(precision) if refine is None else int(refine)
        dev = gix.device
        Q, d, m = slot_queries, gix.d, gix.m
        # an index with a projection projects each batch once, for the tables and the refinement, as
        # Index.query does: the same rounding whatever the batch, so results never depend on it
        self.projected = gix.has_projection
        lut_t = torch.float16 if precision in ("f16", "f16+bf16") else torch.float32
        self.slots = []
        for _ in range(n_slots):
            # launches are sized by their batch's largest ef: smaller pools fit
            # more slots (more bitsets), larger ones longer id lists
            ws_bytes = max(lc.lib().lc_search_workspace_bytes_sched(gix.handle, Q, e, S,
                                                                    None if sched is None else lc.C.byref(sched))
                           for e in sorted(set(range(64, ef_max, 64)) | {1, ef_max}))
            ws2_bytes = max(lc.lib().lc_search_workspace_bytes_sched(gix.handle, Q, e, S,
                                                                     None if sched is None else lc.C.byref(sched))
                            for e in (1, 64, 128))
            self.slots.append({
                "stream": torch.cuda.Stream(device=dev),
                "q": torch.empty((Q, d), dtype=torch.float32, device=dev),
                "qp": torch.empty((Q, gix.d_pad) if self.projected else (1,), dtype=torch.float32, device=dev),
                "ef": torch.empty(Q, dtype=torch.int32, device=dev),
                "lut": torch.empty(((Q, gix.lut_stride_f16 if precision in ("f16", "f16+bf16") else gix.lut_stride) if gix.coarse_k
                                    else (Q, m, 256)), dtype=lut_t, device=dev),
                "scale": torch.empty((Q, m), dtype=torch.float32, device=dev),
                "cand_ids": torch.empty((Q, S), dtype=torch.int32, device=dev),
                "cand_adc": torch.empty((Q, S), dtype=torch.float32, device=dev),
                "cand_n": torch.empty(Q, dtype=torch.int32, device=dev),
                "ids": torch.empty((Q, K), dtype=torch.int32, device=dev),
                "d": torch.empty((Q, K), dtype=torch.float32, device=dev),
                "stats": torch.empty((Q, 2), dtype=torch.int32, device=dev),
                "h_stats": torch.empty((Q, 2), dtype=torch.int32).pin_memory(),
                "ws": torch.zeros(max(int(ws_bytes), 1), dtype=torch.uint8, device=dev),
                "ws2": torch.zeros(max(int(ws2_bytes), 1) if split else 1, dtype=torch.uint8, device=dev),
                "stream2": torch.cuda.Stream(device=dev),
                "h_q": torch.empty((Q, d), dtype=torch.float32).pin_memory(),
                "h_ef": torch.empty(Q, dtype=torch.int32).pin_memory(),
                "h_ids": torch.empty((Q, K), dtype=torch.int32).pin_memory(),
                "h_d": torch.empty((Q, K), dtype=torch.float32).pin_memory(),
                "event": None, "n": 0,
            })
        # the workspaces are zero-filled on the allocating stream; every slot stream must see that
        # before its first launch reads them
        torch.cuda.current_stream(dev).synchronize()

    def _walk(self, s, st, row0, rows, ef_launch, ws):
        """One walk launch over rows [row0, row0 + rows) of the slot's batch."""
        lc, C = self.lc, self.lc.C
        L, h = lc.lib(), self.gix.handle
        lut_row = s["lut"][0].numel() * s["lut"].element_size()
        rec = None
        if self.record_walks:
            rec = {"n": rows, "row0": row0, "ef_launch": ef_launch, "a": self.torch.cuda.Event(enable_timing=True),
                   "b": self.torch.cuda.Event(enable_timing=True)}
            rec["a"].record(st)
        scale = s["scale"].data_ptr() + 4 * self.gix.m * row0 if self.lut_dtype == lc.LC_LUT_F16 else None
        lc._check(L.lc_search_sched(h, s["lut"].data_ptr() + lut_row * row0, self.lut_dtype, scale, rows,
                                    s["ef"].data_ptr() + 4 * row0, ef_launch, self.S, None,
                                    s["cand_ids"].data_ptr() + 4 * self.S * row0,
                                    s["cand_adc"].data_ptr() + 4 * self.S * row0, s["cand_n"].data_ptr() + 4 * row0,
                                    s["stats"].data_ptr() + 8 * row0 if rec else None, ws.data_ptr(), ws.numel(),
                                    None if self.sched is None else C.byref(self.sched), C.c_void_p(st.cuda_stream)),
                  "lc_search")
        if rec is not None:
            rec["b"].record(st)
            s["recs"].append(rec)
            self.walk_log.append(rec)

    def launch(self, slot: int, batch: List[Request]):
        torch, lc, C = self.torch, self.lc, self.lc.C
        s = self.slots[slot]
        # requests longest ef first: the walk's slots take the long walks first, and the batch splits into
        # two contiguous classes (pools above 128 entries, then pools in registers)
        batch = sorted(batch, key=lambda r: -r.ef)
        s["batch"] = batch
        n = 0
        n_big = 0
        for r in batch:
            s["h_q"][n:n + r.size].copy_(torch.from_numpy(r.queries))
            s["h_ef"][n:n + r.size].fill_(int(r.ef))
            n += r.size
            if self._pool(r.ef) > 128:
                n_big = n
        s["n"] = n
        s["recs"] = []
        L, h = lc.lib(), self.gix.handle
        st = s["stream"]
        with torch.cuda.stream(st):
            s["q"][:n].copy_(s["h_q"][:n], non_blocking=True)
            s["ef"][:n].copy_(s["h_ef"][:n], non_blocking=True)
            sp = C.c_void_p(st.cuda_stream)
            scale = s["scale"].data_ptr() if self.lut_dtype == lc.LC_LUT_F16 else None
            proj = self.projected
            if proj:
                lc._check(L.lc_project_queries(h, s["q"].data_ptr(), n, s["qp"].data_ptr(), sp), "lc_project_queries")
                lc._check(L.lc_build_lut_projected(h, s["qp"].data_ptr(), n, self.lut_dtype, s["lut"].data_ptr(), scale,
                                                   sp), "lc_build_lut")
            else:
                lc._check(L.lc_build_lut(h, s["q"].data_ptr(), n, self.lut_dtype, s["lut"].data_ptr(), scale, sp),
                          "lc_build_lut")
            ef_top = int(batch[0].ef)
            if self.split and 0 < n_big < n:
                # the two classes concurrently: the large pools on the slot's second stream
                st2 = s["stream2"]
                st2.wait_stream(st)
                self._walk(s, st2, 0, n_big, ef_top, s["ws"])
                ef_small = max(int(r.ef) for r in batch if self._pool(r.ef) <= 128)
                self._walk(s, st, n_big, n - n_big, ef_small, s["ws2"])
                st.wait_stream(st2)
            else:
                self._walk(s, st, 0, n, ef_top, s["ws"])
            for rec in s["recs"]:
                s["h_stats"][rec["row0"]:rec["row0"] + rec["n"]].copy_(
                    s["stats"][rec["row0"]:rec["row0"] + rec["n"]], non_blocking=True)
            refine = L.lc_refine_projected if proj else L.lc_refine
            qin = s["qp"] if proj else s["q"]
            lc._check(refine(h, qin.data_ptr(), n, s["cand_ids"].data_ptr(), s["cand_n"].data_ptr(), self.S, self.K,
                             self.refine_p, s["ids"].data_ptr(), s["d"].data_ptr(), sp), "lc_refine")
            s["h_ids"][:n].copy_(s["ids"][:n], non_blocking=True)
            s["h_d"][:n].copy_(s["d"][:n], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
            s["event"] = ev

    def _pool(self, ef: int) -> int:
        """Pool entries of a query's walk: max(ef, S) rounded up to 64."""
        return (max(int(ef), self.S) + 63) // 64 * 64

    def ready(self, slot: int) -> bool:
        return self.slots[slot]["event"].query()

    def wait(self, slot: int):
        self.slots[slot]["event"].synchronize()

    def deliver(self, slot: int, batch: List[Request]):
        s = self.slots[slot]
        for rec in s.get("recs", []):
            rec["stats"] = s["h_stats"][rec["row0"]:rec["row0"] + rec["n"]].numpy().copy()
        n = 0
        for r in s["batch"]:  # the order the launch laid the requests out in
            r.ids = s["h_ids"][n:n + r.size].numpy().copy()
            r.dist = s["h_d"][n:n + r.size].numpy().copy()
            n += r.size


def serve(engine, sched: Scheduler, requests: List[Request], clock: Callable[[], float] = time.perf_counter,
          idle: Optional[Callable[[float], None]] = None) -> dict:
    """Run the loop until every request has its results.  ``requests`` carry
    arrival times relative to the start; a request is handed to the scheduler
    once the clock passes its arrival."""
    todo = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = clock()
    i = 0
    finished: List[Request] = []
    while len(finished) < len(todo):
        now = clock() - t0
        while i < len(todo) and todo[i].arrival <= now:
            sched.arrive(todo[i])
            i += 1
        progressed = False
        for slot in list(sched.in_flight):
            if engine.ready(slot):
                batch = sched.complete(slot)
                engine.deliver(slot, batch)
                t = clock() - t0
                for r in batch:
                    r.done = t
                finished.extend(batch)
                progressed = True
        while True:
            nxt = sched.admit()
            if nxt is None:
                break
            slot, batch = nxt
            t = clock() - t0
            for r in batch:
                r.start = t
            engine.launch(slot, batch)
            progressed = True
        if not progressed and idle is not None:
            nxt_arrival = todo[i].arrival if i < len(todo) else None
            idle(nxt_arrival if nxt_arrival is not None else now)
    wall = max(r.done for r in finished) - min(r.arrival for r in finished) if finished else 0.0
    lat = np.array([r.latency for r in finished]) * 1e3
    nqs = sum(r.size for r in finished)
    return {"requests": len(finished), "queries": nqs, "wall_s": wall, "qps": nqs / wall if wall > 0 else 0.0,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_mean": float(lat.mean()), "max_mem_used": sched.max_mem_used,
            "mem_waits": sched.mem_waits}


def poisson_requests(d: int, queries: np.ndarray, rate_rps: float, n_requests: int, seed: int,
                     efs=(32, 64, 128, 256), max_batch: int = 1024) -> List[Request]:
    """Seeded request stream: exponential inter-arrival times at `rate_rps`
    requests/s, batch sizes round(exp(U(0, ln max_batch))), ef uniform over
    `efs`; queries are taken from `queries` in order (wrapping)."""
    import datagen
    g = datagen.rng(seed, "ARRIVALS")
    gaps = g.exponential(1.0 / rate_rps, size=n_requests)
    sizes = np.rint(np.exp(g.random(n_requests) * np.log(max_batch))).astype(int).clip(1, max_batch)
    efv = np.asarray(efs)[g.integers(0, len(efs), n_requests)]
    t, pos, out = 0.0, 0, []
    for k in range(n_requests):
        t += float(gaps[k])
        idx = (pos + np.arange(sizes[k])) % queries.shape[0]
        pos = (pos + sizes[k]) % queries.shape[0]
        out.append(Request(rid=k, queries=np.ascontiguousarray(queries[idx]), ef=int(efv[k]), arrival=t, qidx=idx))
    return out
