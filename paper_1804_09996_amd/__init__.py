"""Link & Code search on AMD Instinct MI355X.

A thin ctypes binding of ``liblc.so`` (include/lc.h).  PyTorch supplies device
memory and the current stream; every step of the search runs in the library's
HIP kernels.  Importing the package does not need a GPU, but every call that
launches work raises if the native library is missing: there is no CPU
fallback.

Names follow the paper: ``build_lut`` (Sec. 4.1 asymmetric distances),
``search`` (Sec. 2 walk and the Sec. 4.1 short-list), ``refine`` (Sec. 4.2 /
4.3 regression refinement and top-K).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Union

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblc.so")

LC_OK, LC_EINVAL, LC_ENOSPC, LC_ENOTSUP, LC_EHIP = 0, 1, 2, 3, 4
LC_LUT_F32, LC_LUT_F16 = 0, 1
LC_REFINE_F32, LC_REFINE_BF16_RESCORE = 0, 1

_lib = None


class LCError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().lc_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class IndexView(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n", "d", "d_pad", "m", "ksub", "code_stride", "deg0", "deg_up", "k_reg",
                                          "n_beta", "entry", "max_level", "m_beta")] + \
               [("n_up_rows", C.c_int64)] + \
               [(n, C.c_void_p) for n in ("proj", "centroids", "codes", "adj0", "up_base", "adj_up", "beta",
                                          "beta_idx")] + \
               [("coarse_k", C.c_int32)] + \
               [(n, C.c_void_p) for n in ("coarse_cent", "coarse_codes", "coarse_norm")]


class Schedule(C.Structure):
    """Launch schedule of the walk (lc_schedule); every schedule gives the
    same results."""
    _fields_ = [("hash_bits", C.c_int32), ("prefetch", C.c_int32), ("waves_per_cu", C.c_int32),
                ("queue", C.c_int32), ("visited", C.c_int32), ("wide", C.c_int32), ("pool", C.c_int32),
                ("table", C.c_int32), ("codes", C.c_int32)]

    def __repr__(self):
        return (f"Schedule(hash_bits={self.hash_bits}, prefetch={self.prefetch}, "
                f"waves_per_cu={self.waves_per_cu}, queue={self.queue}, visited={self.visited}, wide={self.wide}, "
                f"pool={self.pool}, table={self.table}, codes={self.codes})")

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def schedule(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, wide=0, pool=0, table=0,
             codes=0) -> Schedule:
    return Schedule(hash_bits, prefetch, waves_per_cu, queue, visited, wide, pool, table, codes)


def lib():
    """The loaded ``liblc.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1804_09996_amd.build_ext`; "
                              "there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        L.lc_build_id.restype = C.c_char_p
        from .build_ext import source_id
        built, here = L.lc_build_id().decode(), source_id()
        if built != here:
            raise ImportError(f"{LIB_PATH} was built from other sources (build {built[:12]}, sources {here[:12]}): "
                              "rebuild it with `python -m paper_1804_09996_amd.build_ext`")
        p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.lc_strerror.argtypes = [C.c_int]
        L.lc_strerror.restype = C.c_char_p
        L.lc_index_bind.argtypes = [C.POINTER(IndexView), C.POINTER(p)]
        L.lc_index_release.argtypes = [p]
        L.lc_index_release.restype = None
        L.lc_build_lut.argtypes = [p, p, i64, C.c_int, p, p, p]
        L.lc_search_workspace_bytes.argtypes = [p, i64, i32, i32]
        L.lc_walk_describe.argtypes = [p, i64, i32, i32, C.c_int, p, C.c_char_p, sz]
        L.lc_search_workspace_bytes.restype = sz
        L.lc_search.argtypes = [p, p, C.c_int, p, i64, p, i32, i32, p, p, p, p, p, sz, p]
        L.lc_search_workspace_bytes_sched.argtypes = [p, i64, i32, i32, C.POINTER(Schedule)]
        L.lc_search_workspace_bytes_sched.restype = sz
        L.lc_search_sched.argtypes = [p, p, C.c_int, p, i64, p, i32, i32, p, p, p, p, p, p, sz, C.POINTER(Schedule), p]
        L.lc_search_budget.argtypes = [p, p, C.c_int, p, i64, p, i32, i32, i32, p, p, p, p, p, p, sz,
                                       C.POINTER(Schedule), p]
        L.lc_refine.argtypes = [p, p, i64, p, p, i32, i32, C.c_int, p, p, p]
        L.lc_assign_beta.argtypes = [p, p, i64, i64, p, p]
        L.lc_project_queries.argtypes = [p, p, i64, p, p]
        L.lc_build_lut_projected.argtypes = [p, p, i64, C.c_int, p, p, p]
        L.lc_refine_projected.argtypes = [p, p, i64, p, p, i32, i32, C.c_int, p, p, p]
        L.lc_lut_stride.argtypes = [p, C.c_int]
        L.lc_lut_stride.restype = i64
        L.lc_search_noalloc.argtypes = [p, p, C.c_int, p, i64, p, i32, i32, p, p, p, p, p]
        L.lc_project_exact.argtypes = [p, i64, C.c_int, p, C.c_int, p, p]
        L.lc_pq_encode.argtypes = [p, i64, C.c_int, C.c_int, p, p, C.c_int, p]
        L.lc_graph_insert_workspace_bytes.argtypes = [p, i32, i32]
        L.lc_graph_insert_workspace_bytes.restype = sz
        L.lc_graph_insert.argtypes = [p, p, p, p, i32, i32, i32, p, sz, p]
        _lib = L
    return _lib


def exported_symbols():
    return ["lc_build_id", "lc_strerror", "lc_index_bind", "lc_index_release", "lc_build_lut", "lc_search_workspace_bytes",
            "lc_search", "lc_refine", "lc_search_workspace_bytes_sched", "lc_search_sched", "lc_search_budget",
            "lc_assign_beta", "lc_project_queries", "lc_build_lut_projected", "lc_refine_projected", "lc_lut_stride",
            "lc_search_noalloc", "lc_project_exact", "lc_pq_encode", "lc_graph_insert_workspace_bytes",
            "lc_graph_insert", "lc_walk_describe"]


def _check(rc: int, where: str):
    if rc != LC_OK:
        raise LCError(rc, where)


def _stream(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class SearchResult:
    cand_ids: "object"
    cand_adc: "object"
    cand_n: "object"
    stats: "object"


class Index:
    """An index resident in device memory, bound to ``liblc``.

    ``arrays`` holds numpy arrays in the layout of include/lc.h (keys
    ``centroids, codes, adj0, up_base, adj_up, beta, beta_idx`` and optional
    ``proj``); ``meta`` the scalars ``d, d_pad, m, deg0, deg_up, k_reg,
    entry, max_level``.  ``beta`` is [n_beta, k+1] (one codebook) or
    [m_beta, n_beta, k+1] (product codebook), ``beta_idx`` [n] or [n, m_beta].
    A 2-level codec adds ``coarse_cent`` [2, k, d_pad/2], ``coarse_codes``
    [n, 2] (uint16) and ``coarse_norm`` [n].
    """

    def __init__(self, arrays: dict, meta: dict, device: Union[str, int] = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.meta = dict(meta)
        L = lib()

        def up(name, dtype):
            a = arrays.get(name)
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dtype)
            if a.size == 0:
                a = np.zeros(1, dtype=dtype)
            return torch.from_numpy(a).to(self.device)

        self.t = {
            "proj": up("proj", np.float32), "centroids": up("centroids", np.float32),
            "codes": up("codes", np.uint8), "adj0": up("adj0", np.int32), "up_base": up("up_base", np.int32),
            "adj_up": up("adj_up", np.int32), "beta": up("beta", np.float32), "beta_idx": up("beta_idx", np.uint8),
            "coarse_cent": up("coarse_cent", np.float32), "coarse_norm": up("coarse_norm", np.float32),
        }
        cc = arrays.get("coarse_codes")
        if cc is not None:
            # (c0, c1) pairs of uint16 travel as one 32-bit word per vector
            cc = np.ascontiguousarray(cc, np.uint16)
            if cc.ndim != 2 or cc.shape != (arrays["codes"].shape[0], 2):
                raise ValueError(f"coarse_codes has shape {cc.shape}, expected [n, 2]")
            self.t["coarse_codes"] = torch.from_numpy(cc.view(np.int32).reshape(-1).copy()).to(self.device)
        else:
            self.t["coarse_codes"] = None
        ccent = arrays.get("coarse_cent")
        if ccent is not None and (ccent.ndim != 3 or ccent.shape[0] != 2 or ccent.shape[2] * 2 != meta["d_pad"]
                                  or arrays.get("coarse_norm") is None or cc is None
                                  or np.asarray(arrays["coarse_norm"]).size != arrays["codes"].shape[0]):
            raise ValueError("coarse_cent [2, k, d_pad/2], coarse_codes [n, 2] and coarse_norm [n] go together")
        codes = arrays["codes"]
        beta, bidx = np.asarray(arrays["beta"]), np.asarray(arrays["beta_idx"])
        m_beta = beta.shape[0] if beta.ndim == 3 else 1
        n_beta = beta.shape[-2]
        # the kernels index beta and beta_idx by these sizes: check them before anything is bound
        if beta.ndim not in (2, 3) or beta.shape[-1] != meta["k_reg"] + 1:
            raise ValueError(f"beta has shape {beta.shape}, expected [(m_beta,) n_beta, {meta['k_reg'] + 1}]")
        if bidx.size != codes.shape[0] * m_beta:
            raise ValueError(f"beta_idx has {bidx.size} entries, expected n * m_beta = {codes.shape[0] * m_beta}")
        v = IndexView()
        v.n, v.d, v.d_pad, v.m = codes.shape[0], meta["d"], meta["d_pad"], meta["m"]
        v.ksub, v.code_stride = 256, codes.shape[1]
        v.deg0, v.deg_up, v.k_reg = meta["deg0"], meta["deg_up"], meta["k_reg"]
        v.n_beta, v.m_beta = n_beta, m_beta
        v.entry, v.max_level = meta["entry"], meta["max_level"]
        au = arrays.get("adj_up")
        v.n_up_rows = 0 if au is None else au.shape[0]
        for name in ("proj", "centroids", "codes", "adj0", "up_base", "adj_up", "beta", "beta_idx"):
            setattr(v, name, _ptr(self.t[name]))
        v.coarse_k = 0 if ccent is None else ccent.shape[1]
        for name in ("coarse_cent", "coarse_codes", "coarse_norm"):
            setattr(v, name, _ptr(self.t[name]))
        self.view = v
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.lc_index_bind(C.byref(v), C.byref(h)), "lc_index_bind")
        self.handle = h
        self.n, self.m, self.d, self.d_pad = v.n, v.m, v.d, v.d_pad
        self.k_reg = v.k_reg
        self.coarse_k = v.coarse_k
        self.lut_stride = int(L.lc_lut_stride(h, LC_LUT_F32))      # float32 table: floats per row
        self.lut_stride_f16 = int(L.lc_lut_stride(h, LC_LUT_F16))  # fp16 table: 16-bit elements per row
        self._ws = None

    @classmethod
    def from_index(cls, ix, device="cuda") -> "Index":
        """From any object with the index attributes (e.g. a built index)."""
        arrays = {k: getattr(ix, k) for k in ("proj", "centroids", "codes", "adj0", "up_base", "adj_up", "beta",
                                              "beta_idx")}
        for k in ("coarse_cent", "coarse_codes", "coarse_norm"):
            if getattr(ix, k, None) is not None:
                arrays[k] = getattr(ix, k)
        meta = {k: int(getattr(ix, k)) for k in ("d", "d_pad", "m", "deg0", "deg_up", "k_reg", "entry",
                                                 "max_level")}
        return cls(arrays, meta, device)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().lc_index_release(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refine_mode(self, precision: str) -> int:
        """Refinement for a precision name.  "f16" (fp16 tables) refines in
        float32: at the serving workload's shape the bf16 pass with its exact
        re-score takes 4.7x the float32 kernel's time (1.28 against 0.27 ms per
        10k queries), so the precision form keeps only the fp16 tables.
        "f16+bf16" selects the bf16 refinement with the exact fp32 re-score
        of the final candidates (one-level codec only)."""
        return LC_REFINE_BF16_RESCORE if precision == "f16+bf16" and not self.coarse_k else LC_REFINE_F32

    # -- the three calls of the path ---------------------------------------
    @property
    def has_projection(self) -> bool:
        return bool(self.view.proj)

    def project(self, q):
        """Projected queries P q [nq, d_pad] (a copy without a projection)."""
        torch = self.torch
        q = q.to(self.device, torch.float32).contiguous()
        out = torch.empty((q.shape[0], self.d_pad), dtype=torch.float32, device=self.device)
        _check(lib().lc_project_queries(self.handle, _ptr(q), q.shape[0], _ptr(out), _stream(torch, self.device)),
               "lc_project_queries")
        return out

    def build_lut(self, q, lut_dtype: int = LC_LUT_F32, projected: bool = False):
        """``projected``: q holds projected queries [nq, d_pad] (from project())."""
        torch = self.torch
        q = q.to(self.device, torch.float32).contiguous()
        nq = q.shape[0]
        if lut_dtype == LC_LUT_F32:
            shape = (nq, self.lut_stride) if self.coarse_k else (nq, self.m, 256)
            lut = torch.empty(shape, dtype=torch.float32, device=self.device)
            scale = None
        else:
            shape = (nq, self.lut_stride_f16) if self.coarse_k else (nq, self.m, 256)
            lut = torch.empty(shape, dtype=torch.float16, device=self.device)
            scale = torch.empty((nq, self.m), dtype=torch.float32, device=self.device)
        fn = lib().lc_build_lut_projected if projected else lib().lc_build_lut
        _check(fn(self.handle, _ptr(q), nq, lut_dtype, _ptr(lut), _ptr(scale), _stream(torch, self.device)),
               "lc_build_lut")
        return lut, scale

    def workspace_bytes(self, nq: int, ef_max: int, S: int, sched: Optional[Schedule] = None) -> int:
        return int(lib().lc_search_workspace_bytes_sched(self.handle, max(nq, 1), ef_max, S,
                                                         None if sched is None else C.byref(sched)))

    def walk_plan(self, nq: int, ef_max: int, S: int, lut_dtype: int = None, sched: Optional[Schedule] = None) -> dict:
        """The walk lc_search_sched would launch (lc_walk_describe): kernel
        name, grid, slots per CU, visited-table bits and LDS bytes per slot."""
        buf = C.create_string_buffer(256)
        dt = LC_LUT_F32 if lut_dtype is None else lut_dtype
        _check(lib().lc_walk_describe(self.handle, max(nq, 1), ef_max, S, dt,
                                      None if sched is None else C.byref(sched), buf, 256), "lc_walk_describe")
        kernel, _, rest = buf.value.decode().partition(">")
        out = {"kernel": kernel + ">"}
        for kv in rest.split():
            k, v = kv.split("=")
            out[k] = int(v)
        return out

    def workspace(self, nq: int, ef_max: int, S: int, sched: Optional[Schedule] = None):
        torch = self.torch
        need = self.workspace_bytes(nq, ef_max, S, sched)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.zeros(max(need, 1), dtype=torch.uint8, device=self.device)
        return self._ws

    def search(self, lut, scale=None, ef=None, ef_max: int = 64, S: int = 64, stats: bool = True,
               lut_dtype: Optional[int] = None, sched: Optional[Schedule] = None, order=None,
               out: Optional[SearchResult] = None, ws=None, max_evals: int = 0) -> SearchResult:
        """``ws``: a zero-filled uint8 device tensor of at least
        ``workspace_bytes(...)`` bytes, or None for the index's own (searches
        that may overlap on different streams need one each).  ``max_evals``
        > 0: the budget T on level-0 distance evaluations per query."""
        torch = self.torch
        nq = lut.shape[0]
        if lut_dtype is None:
            lut_dtype = LC_LUT_F16 if lut.dtype == torch.float16 else LC_LUT_F32
        ef_t = None
        if ef is not None:
            ef_t = torch.as_tensor(ef, dtype=torch.int32).to(self.device).contiguous()
            if ef_t.dim() == 0:
                ef_t = ef_t.expand(nq).contiguous()
        if out is not None:
            cand_ids, cand_adc, cand_n, st = out.cand_ids, out.cand_adc, out.cand_n, out.stats
        else:
            cand_ids = torch.empty((nq, S), dtype=torch.int32, device=self.device)
            cand_adc = torch.empty((nq, S), dtype=torch.float32, device=self.device)
            cand_n = torch.empty(nq, dtype=torch.int32, device=self.device)
            st = torch.empty((nq, 2), dtype=torch.int32, device=self.device) if stats else None
        if ws is None:
            ws = self.workspace(nq, ef_max, S, sched)
        elif ws.numel() < self.workspace_bytes(nq, ef_max, S, sched):
            raise LCError(LC_ENOSPC, "lc_search")
        if max_evals:
            rc = lib().lc_search_budget(self.handle, _ptr(lut), lut_dtype, _ptr(scale), nq, _ptr(ef_t), ef_max, S,
                                        int(max_evals), _ptr(order), _ptr(cand_ids), _ptr(cand_adc), _ptr(cand_n),
                                        _ptr(st), _ptr(ws), ws.numel(), None if sched is None else C.byref(sched),
                                        _stream(torch, self.device))
        elif sched is None and order is None:
            rc = lib().lc_search(self.handle, _ptr(lut), lut_dtype, _ptr(scale), nq, _ptr(ef_t), ef_max, S,
                                 _ptr(cand_ids), _ptr(cand_adc), _ptr(cand_n), _ptr(st), _ptr(ws), ws.numel(),
                                 _stream(torch, self.device))
        else:
            rc = lib().lc_search_sched(self.handle, _ptr(lut), lut_dtype, _ptr(scale), nq, _ptr(ef_t), ef_max, S,
                                       _ptr(order), _ptr(cand_ids), _ptr(cand_adc), _ptr(cand_n), _ptr(st), _ptr(ws),
                                       ws.numel(), None if sched is None else C.byref(sched),
                                       _stream(torch, self.device))
        _check(rc, "lc_search")
        return SearchResult(cand_ids, cand_adc, cand_n, st)

    def search_noalloc(self, lut, scale=None, ef=None, ef_max: int = 64, S: int = 64, out: SearchResult = None):
        """lc_search_noalloc: the walk with the library's fixed workspace array;
        ``out`` (a SearchResult with stats) holds the outputs, allocated here
        when None."""
        torch = self.torch
        nq = lut.shape[0]
        lut_dtype = LC_LUT_F16 if lut.dtype == torch.float16 else LC_LUT_F32
        ef_t = None if ef is None else torch.as_tensor(ef, dtype=torch.int32).to(self.device).contiguous()
        if out is None:
            out = SearchResult(torch.empty((nq, S), dtype=torch.int32, device=self.device),
                               torch.empty((nq, S), dtype=torch.float32, device=self.device),
                               torch.empty(nq, dtype=torch.int32, device=self.device),
                               torch.empty((nq, 2), dtype=torch.int32, device=self.device))
        _check(lib().lc_search_noalloc(self.handle, _ptr(lut), lut_dtype, _ptr(scale), nq, _ptr(ef_t), ef_max, S,
                                       _ptr(out.cand_ids), _ptr(out.cand_adc), _ptr(out.cand_n), _ptr(out.stats),
                                       _stream(torch, self.device)), "lc_search_noalloc")
        return out

    def refine(self, q, cand_ids, cand_n, K: int, precision: int = LC_REFINE_F32, projected: bool = False):
        torch = self.torch
        q = q.to(self.device, torch.float32).contiguous()
        nq, S = cand_ids.shape
        out_ids = torch.empty((nq, K), dtype=torch.int32, device=self.device)
        out_d = torch.empty((nq, K), dtype=torch.float32, device=self.device)
        fn = lib().lc_refine_projected if projected else lib().lc_refine
        _check(fn(self.handle, _ptr(q), nq, _ptr(cand_ids), _ptr(cand_n), S, K, precision, _ptr(out_ids),
                  _ptr(out_d), _stream(torch, self.device)), "lc_refine")
        return out_ids, out_d

    def assign_beta(self, x, n0: int = 0):
        """Codebook entries (Sec. 4.3 Eq. 7, per block Eq. 9) of the vectors
        n0 .. n0 + len(x) - 1 from their raw rows ``x`` [count, d]: a uint8
        device tensor [count, m_beta]."""
        torch = self.torch
        x = torch.as_tensor(x).to(self.device, torch.float32).contiguous()
        if x.dim() != 2 or x.shape[1] != self.d:
            raise ValueError(f"x must be [count, {self.d}]")
        out = torch.empty((x.shape[0], int(self.view.m_beta)), dtype=torch.uint8, device=self.device)
        _check(lib().lc_assign_beta(self.handle, _ptr(x), int(n0), x.shape[0], _ptr(out),
                                    _stream(torch, self.device)), "lc_assign_beta")
        return out

    def query(self, q, ef=None, ef_max: int = 64, S: int = 64, K: int = 10, stats: bool = False,
              sched: Optional[Schedule] = None, precision: str = "f32", max_evals: int = 0):
        """The whole path: tables, walk and short-list, refinement and top-K.
        ``precision="f16"`` selects the fp16 table (float32 refinement);
        ``"f16+bf16"`` the fp16 table and the bf16 refinement with exact fp32
        re-scoring of the final candidates (float32 on a 2-level index)."""
        lp = precision in ("f16", "f16+bf16")
        pj = self.has_projection  # project the batch once for the tables and the refinement
        if pj:
            q = self.project(q)
        lut, scale = self.build_lut(q, LC_LUT_F16 if lp else LC_LUT_F32, projected=pj)
        r = self.search(lut, scale, ef=ef, ef_max=ef_max, S=S, stats=stats, sched=sched, max_evals=max_evals)
        ids, d = self.refine(q, r.cand_ids, r.cand_n, K, self.refine_mode(precision), projected=pj)
        return ids, d, r
