"""Python binding of the Link & Code reference oracle (``liblc_oracle.so``).

TEST INFRASTRUCTURE ONLY: this package is loaded by the test-suite, by the
smoke check and by the CPU-baseline leg of the benchmark, never by the GPU
library.  It shares no code with ``paper_1804_09996_amd``.

Every function works in float64 (the index stores float32 parameters, which
are promoted) and follows the paper's definitions:

* PQ training/encoding: Sec. 3.3 and Sec. 4.1 ("Vector approximation").
* Node levels and the nested graph: Sec. 2 and Sec. 4.1 ("Graph-based
  structure": upper degree 32, level ratio 30), batched insertion (Sec. 5.1).
* 0-byte refinement: Sec. 4.2, Eq. (3)-(5); regression codebook: Sec. 4.3,
  Eq. (6)-(8).
* Search: greedy descent then best-first walk (Sec. 2), short-list and
  re-ranking (Sec. 4.1 "Refinement strategy").
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LC_ORACLE_LIB") or os.path.join(_HERE, "liblc_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_p = C.c_void_p
_i = C.c_int
_i64 = C.c_int64


class OrcCoarse(C.Structure):
    _fields_ = [("k", C.c_int32), ("cent", _p), ("codes", _p)]


class OrcIndex(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n", "d", "d_pad", "m", "ksub", "code_stride", "deg0", "deg_up",
                                          "k_reg", "n_beta", "entry", "max_level", "m_beta")] + \
               [(n, _p) for n in ("proj", "centroids", "codes", "adj0", "up_base", "adj_up", "beta", "beta_idx")] + \
               [("coarse", OrcCoarse)]


def _declare(L):
    L.orc_kmeans.argtypes = [_p, _i64, _i, _i, _p, _i, _i, _p, _p, _p]
    L.orc_pq_train.argtypes = [_p, _i64, _i, _p, _i, _i, _i, _p, _i, _i, _p, _p]
    L.orc_pq_encode.argtypes = [_p, _i64, _i, _p, _i, _i, _i, _p, _i, _p, _i]
    L.orc_levels.argtypes = [_p, _i64, _i, _i, _p]
    L.orc_levels.restype = _i64
    L.orc_hnsw_build.argtypes = [_p, _i64, _i, _p, _i, _i, _i, _p, _p, _i, _p, _i, _i, _i, _i, _p, _p, _p, _p, _p,
                                 C.POINTER(OrcCoarse)]
    L.orc_lsq_solve.argtypes = [_p, _p, _i, _p]
    L.orc_beta_train.argtypes = [_p, _p, _i64, _i, _p, _i, _i, _i, _p, _p, _i, _p, _i, _i, _i, _i, _p, _i, _i,
                                 _i, _p, _p, C.POINTER(OrcCoarse)]
    L.orc_beta_shared.argtypes = [_p, _p, _i64, _i, _p, _i, _i, _i, _p, _p, _i, _p, _i, _i, _p, C.POINTER(OrcCoarse)]
    L.orc_beta_assign.argtypes = [_p, _i64, _i, _p, _i, _i, _i, _p, _p, _i, _p, _i, _i, _i, _i, _p, _i, _p,
                                  C.POINTER(OrcCoarse)]
    L.orc_coarse_encode.argtypes = [_p, _i64, _i, _p, _i, _i, _p, _i, _p, _p]
    L.orc_coarse_norms.argtypes = [C.POINTER(OrcIndex), _p]
    L.orc_lut.argtypes = [C.POINTER(OrcIndex), _p, _p]
    L.orc_lut.restype = None
    L.orc_search.argtypes = [C.POINTER(OrcIndex), _p, _i64, _p, C.c_int32, C.c_int32, _i, _p, _p, _p, _p, _p, _p]
    L.orc_search_capped.argtypes = [C.POINTER(OrcIndex), _p, _i64, _p, C.c_int32, C.c_int32, C.c_int32, _i, _p, _p,
                                    _p, _p, _p, _p]
    L.orc_walk_tables.argtypes = [C.POINTER(OrcIndex), _p, _i64, _p, C.c_int32, _i, _p, _p, _p, _p]
    L.orc_refined_distance.argtypes = [C.POINTER(OrcIndex), _p, C.c_int32]
    L.orc_refined_distance.restype = C.c_double
    L.orc_walk_trace.argtypes = [C.POINTER(OrcIndex), _p, C.c_int32, _p, C.c_int32]
    L.orc_walk_trace.restype = C.c_int32
    L.orc_project.argtypes = [_p, _i, _i, _p, _p]
    L.orc_project.restype = None
    L.orc_build_trace.argtypes = [_p, _i64]
    L.orc_build_trace.restype = None
    L.orc_build_trace_used.argtypes = []
    L.orc_build_trace_used.restype = _i64


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def code_stride_for(m: int) -> int:
    """Row stride of the code array: the next power of two >= m."""
    s = 1
    while s < m:
        s *= 2
    return s


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------
def kmeans(x: np.ndarray, k: int, init: np.ndarray, iters: int, nthreads: int = 1):
    x = _c(x, np.float64)
    init = _c(init, np.int64)
    cent = np.empty((k, x.shape[1]), np.float64)
    assign = np.empty(x.shape[0], np.int32)
    hist = np.empty(iters + 1, np.float64)
    rc = _load().orc_kmeans(_ptr(x), x.shape[0], x.shape[1], k, _ptr(init), iters, nthreads, _ptr(cent),
                            _ptr(assign), _ptr(hist))
    if rc != 0:
        raise ValueError(f"orc_kmeans failed ({rc})")
    return cent, assign, hist


def project(proj: Optional[np.ndarray], y: np.ndarray, d_pad: int) -> np.ndarray:
    y = _c(y, np.float32)
    out = np.empty(d_pad, np.float64)
    proj = None if proj is None else _c(proj, np.float32)
    _load().orc_project(_ptr(proj), d_pad, y.shape[0], _ptr(y), _ptr(out))
    return out


def pq_train(train, proj, d_pad, m, init, iters, nthreads=1, ksub=256):
    train = _c(train, np.float32)
    proj = None if proj is None else _c(proj, np.float32)
    init = _c(init, np.int64)
    cent = np.empty((m, ksub, d_pad // m), np.float32)
    hist = np.empty((m, iters + 1), np.float64)
    rc = _load().orc_pq_train(_ptr(train), train.shape[0], train.shape[1], _ptr(proj), d_pad, m, ksub, _ptr(init),
                              iters, nthreads, _ptr(cent), _ptr(hist))
    if rc != 0:
        raise ValueError(f"orc_pq_train failed ({rc})")
    return cent, hist


def pq_encode(x, proj, d_pad, cent, nthreads=1, code_stride=None):
    x = _c(x, np.float32)
    proj = None if proj is None else _c(proj, np.float32)
    cent = _c(cent, np.float32)
    m, ksub = cent.shape[0], cent.shape[1]
    cs = code_stride or code_stride_for(m)
    codes = np.empty((x.shape[0], cs), np.uint8)
    rc = _load().orc_pq_encode(_ptr(x), x.shape[0], x.shape[1], _ptr(proj), d_pad, m, ksub, _ptr(cent), nthreads,
                               _ptr(codes), cs)
    if rc != 0:
        raise ValueError(f"orc_pq_encode failed ({rc})")
    return codes


def _coarse(coarse) -> Optional[OrcCoarse]:
    """(first-level centroids [2, k, d_pad/2] f32, codes [n, 2] u16) of a
    2-level codec as the C struct, or None for the one-level codec.  The
    arrays must stay alive while the struct is used."""
    if coarse is None:
        return None
    cent, codes = coarse
    if cent.dtype != np.float32 or codes.dtype != np.uint16 or not (cent.flags.c_contiguous and
                                                                       codes.flags.c_contiguous):
        raise ValueError("coarse codec arrays must be contiguous float32 / uint16")
    if cent.ndim != 3 or cent.shape[0] != 2 or codes.ndim != 2 or codes.shape[1] != 2:
        raise ValueError("coarse codec: centroids [2, k, d_pad/2], codes [n, 2]")
    return OrcCoarse(cent.shape[1], cent.ctypes.data, codes.ctypes.data)


def _cref(cs):
    return None if cs is None else C.byref(cs)


def coarse_encode(x, proj, d_pad, cent, nthreads=1):
    """First level of the 2-level codec: codes [n, 2] u16 and the residuals
    P x - c [n, d_pad] f32 that the second-level PQ encodes."""
    x = _c(x, np.float32)
    proj = None if proj is None else _c(proj, np.float32)
    cent = _c(cent, np.float32)
    codes = np.empty((x.shape[0], 2), np.uint16)
    resid = np.empty((x.shape[0], d_pad), np.float32)
    rc = _load().orc_coarse_encode(_ptr(x), x.shape[0], x.shape[1], _ptr(proj), d_pad, cent.shape[1], _ptr(cent),
                                   nthreads, _ptr(codes), _ptr(resid))
    if rc != 0:
        raise ValueError(f"orc_coarse_encode failed ({rc})")
    return codes, resid


def levels(u: np.ndarray, ratio: int = 30, cap: int = 16):
    u = _c(u, np.float64)
    lv = np.empty(u.shape[0], np.int8)
    rows = _load().orc_levels(_ptr(u), u.shape[0], ratio, cap, _ptr(lv))
    return lv, int(rows)


def hnsw_build(x, proj, d_pad, cent, codes, level, deg0, deg_up, efc, nthreads=1, coarse=None):
    x = _c(x, np.float32)
    proj = None if proj is None else _c(proj, np.float32)
    cent = _c(cent, np.float32)
    codes = _c(codes, np.uint8)
    level = _c(level, np.int8)
    n = x.shape[0]
    rows = int(level.astype(np.int64).sum())
    adj0 = np.empty((n, deg0), np.int32)
    up_base = np.empty(n, np.int32)
    adj_up = np.empty((max(rows, 1), deg_up), np.int32)
    entry = C.c_int32()
    maxl = C.c_int32()
    rc = _load().orc_hnsw_build(_ptr(x), n, x.shape[1], _ptr(proj), d_pad, cent.shape[0], cent.shape[1], _ptr(cent),
                                _ptr(codes), codes.shape[1], _ptr(level), deg0, deg_up, efc, nthreads, _ptr(adj0),
                                _ptr(up_base), _ptr(adj_up), C.byref(entry), C.byref(maxl), _cref(_coarse(coarse)))
    if rc != 0:
        raise ValueError(f"orc_hnsw_build failed ({rc})")
    if rows == 0:
        adj_up = adj_up[:0]
    return adj0, up_base, adj_up, int(entry.value), int(maxl.value)


def hnsw_build_traced(x, proj, d_pad, cent, codes, level, deg0, deg_up, efc, coarse=None, cap_words=1 << 24):
    """hnsw_build on one thread with the build trace on: (adj0, up_base,
    adj_up, entry, max_level, records), records a list of dicts
    {kind, level, owner, cand, out, by_test} in execution order (layout in
    lc_oracle.h)."""
    L = _load()
    buf = np.zeros(cap_words, np.int32)
    L.orc_build_trace(_ptr(buf), cap_words)
    try:
        out = hnsw_build(x, proj, d_pad, cent, codes, level, deg0, deg_up, efc, nthreads=1, coarse=coarse)
        used = int(L.orc_build_trace_used())
    finally:
        L.orc_build_trace(None, 0)
    if used < 0:
        raise ValueError("build trace overflowed its buffer")
    recs, i = [], 0
    while i < used:
        kind, lvl, owner, nc, nout = (int(v) for v in buf[i:i + 5])
        cand = buf[i + 5:i + 5 + nc].copy()
        o = buf[i + 5 + nc:i + 5 + nc + nout].copy()
        bt = buf[i + 5 + nc + nout:i + 5 + nc + 2 * nout].astype(bool)
        recs.append({"kind": kind, "level": lvl, "owner": owner, "cand": cand, "out": o, "by_test": bt})
        i += 5 + nc + 2 * nout
    return (*out, recs)


def lsq_solve(a: np.ndarray, c: np.ndarray):
    a = _c(a, np.float64)
    c = _c(c, np.float64)
    beta = np.empty(c.shape[0], np.float64)
    rc = _load().orc_lsq_solve(_ptr(a), _ptr(c), c.shape[0], _ptr(beta))
    return beta, int(rc)


def beta_train(x, ids, proj, d_pad, cent, codes, adj0, k_reg, n_beta, init, km_iters, em_iters, nthreads=1,
               m_beta=1, coarse=None):
    """Regression codebook(s): [n_beta, k+1] for one block, [m_beta, n_beta, k+1]
    for the product codebook (Eq. 9); the loss history likewise per block."""
    x = _c(x, np.float32)
    cent, codes, adj0 = _c(cent, np.float32), _c(codes, np.uint8), _c(adj0, np.int32)
    ids = _c(ids, np.int64)
    proj = None if proj is None else _c(proj, np.float32)
    init = _c(init, np.int64)
    beta = np.empty((m_beta, n_beta, k_reg + 1), np.float32)
    hist = np.empty((m_beta, em_iters + 1), np.float64)
    rc = _load().orc_beta_train(_ptr(x), _ptr(ids), ids.shape[0], x.shape[1], _ptr(proj), d_pad, cent.shape[0],
                                cent.shape[1], _ptr(cent), _ptr(codes), codes.shape[1],
                                _ptr(adj0), adj0.shape[1], k_reg, n_beta, m_beta, _ptr(init), km_iters,
                                em_iters, nthreads, _ptr(beta), _ptr(hist), _cref(_coarse(coarse)))
    if rc != 0:
        raise ValueError(f"orc_beta_train failed ({rc})")
    if m_beta == 1:
        return beta[0], hist[0]
    return beta, hist


def beta_shared(x, ids, proj, d_pad, cent, codes, adj0, k_reg, coarse=None):
    x = _c(x, np.float32)
    cent, codes, adj0 = _c(cent, np.float32), _c(codes, np.uint8), _c(adj0, np.int32)
    ids = _c(ids, np.int64)
    proj = None if proj is None else _c(proj, np.float32)
    beta = np.empty(k_reg + 1, np.float64)
    rc = _load().orc_beta_shared(_ptr(x), _ptr(ids), ids.shape[0], x.shape[1], _ptr(proj), d_pad, cent.shape[0],
                                 cent.shape[1], _ptr(cent), _ptr(codes), codes.shape[1],
                                 _ptr(adj0), adj0.shape[1], k_reg, _ptr(beta), _cref(_coarse(coarse)))
    if rc != 0:
        raise ValueError(f"orc_beta_shared failed ({rc})")
    return beta


def beta_assign(x, proj, d_pad, cent, codes, adj0, k_reg, beta, nthreads=1, coarse=None):
    """Entry per vector: [n] for a [n_beta, k+1] codebook, [n, m_beta] for a
    [m_beta, n_beta, k+1] product codebook."""
    x = _c(x, np.float32)
    cent, codes, adj0 = _c(cent, np.float32), _c(codes, np.uint8), _c(adj0, np.int32)
    proj = None if proj is None else _c(proj, np.float32)
    beta = _c(beta, np.float32)
    mb = 1 if beta.ndim == 2 else beta.shape[0]
    out = np.empty((x.shape[0], mb), np.uint8)
    rc = _load().orc_beta_assign(_ptr(x), x.shape[0], x.shape[1], _ptr(proj), d_pad, cent.shape[0], cent.shape[1],
                                 _ptr(cent), _ptr(codes), codes.shape[1],
                                 _ptr(adj0), adj0.shape[1], k_reg, beta.shape[-2], mb, _ptr(beta),
                                 nthreads, _ptr(out), _cref(_coarse(coarse)))
    if rc != 0:
        raise ValueError(f"orc_beta_assign failed ({rc})")
    return out[:, 0].copy() if beta.ndim == 2 else out


# ---------------------------------------------------------------------------
# index
# ---------------------------------------------------------------------------
@dataclass
class Index:
    """An index in the shared array layout (see ``lc_oracle.h``)."""
    n: int
    d: int
    d_pad: int
    m: int
    deg0: int
    deg_up: int
    k_reg: int
    n_beta: int
    entry: int
    max_level: int
    proj: Optional[np.ndarray]
    centroids: np.ndarray
    codes: np.ndarray
    adj0: np.ndarray
    level: np.ndarray
    up_base: np.ndarray
    adj_up: np.ndarray
    beta: np.ndarray
    beta_idx: np.ndarray
    ksub: int = 256
    m_beta: int = 1       # product codebook blocks (Eq. 9): beta [m_beta, n_beta, k+1], beta_idx [n, m_beta]
    # 2-level residual codec (Sec. 5.1): first-level centroids [2, k, d_pad/2] f32,
    # their codes [n, 2] u16 (the PQ codes then encode the residual), and the
    # per-node term ||c + r||^2 - ||c||^2 [n] f32 of the decomposed distance
    coarse_cent: Optional[np.ndarray] = None
    coarse_codes: Optional[np.ndarray] = None
    coarse_norm: Optional[np.ndarray] = None

    @property
    def coarse_k(self) -> int:
        return 0 if self.coarse_cent is None else int(self.coarse_cent.shape[1])

    def arrays(self) -> dict:
        names = ["proj", "centroids", "codes", "adj0", "level", "up_base", "adj_up", "beta", "beta_idx"]
        if self.coarse_cent is not None:
            names += ["coarse_cent", "coarse_codes", "coarse_norm"]
        return {k: getattr(self, k) for k in names}

    def _struct(self) -> OrcIndex:
        s = OrcIndex()
        s.n, s.d, s.d_pad, s.m, s.ksub = self.n, self.d, self.d_pad, self.m, self.ksub
        s.code_stride = self.codes.shape[1]
        s.deg0, s.deg_up, s.k_reg, s.n_beta = self.deg0, self.deg_up, self.k_reg, self.n_beta
        s.entry, s.max_level, s.m_beta = self.entry, self.max_level, self.m_beta
        if self.beta.size != self.m_beta * self.n_beta * (self.k_reg + 1) or self.beta_idx.size != self.n * self.m_beta:
            raise ValueError("beta / beta_idx do not match (m_beta, n_beta, k_reg, n)")
        for name in ("proj", "centroids", "codes", "adj0", "up_base", "adj_up", "beta", "beta_idx"):
            a = getattr(self, name)
            setattr(s, name, None if a is None or a.size == 0 else a.ctypes.data)
        if self.coarse_cent is not None:
            if (self.coarse_cent.shape != (2, self.coarse_k, self.d_pad // 2) or self.d_pad % 2
                    or self.coarse_codes.shape != (self.n, 2) or self.d_pad > self.m * self.ksub):
                raise ValueError("coarse codec arrays do not match (n, d_pad)")
            s.coarse = _coarse((self.coarse_cent, self.coarse_codes))
        return s

    def coarse_norms(self) -> np.ndarray:
        """Per-node term ||c + r||^2 - ||c||^2 of the 2-level asymmetric distance."""
        out = np.empty(self.n, np.float32)
        s = self._struct()
        if _load().orc_coarse_norms(C.byref(s), _ptr(out)) != 0:
            raise ValueError("orc_coarse_norms failed")
        return out

    def lut(self, y: np.ndarray) -> np.ndarray:
        out = np.empty((self.m, self.ksub), np.float64)
        s = self._struct()
        y = _c(y, np.float32)
        _load().orc_lut(C.byref(s), _ptr(y), _ptr(out))
        return out

    def refined_distance(self, y: np.ndarray, i: int) -> float:
        s = self._struct()
        y = _c(y, np.float32)
        return float(_load().orc_refined_distance(C.byref(s), _ptr(y), int(i)))

    def walk_trace(self, y: np.ndarray, ef_eff: int, cap: int = 1 << 20) -> np.ndarray:
        s = self._struct()
        out = np.empty(cap, np.int32)
        y = _c(y, np.float32)
        nt = _load().orc_walk_trace(C.byref(s), _ptr(y), int(ef_eff), _ptr(out), cap)
        return out[:nt].copy()

    def walk_tables(self, tables: np.ndarray, ef, S: int, nthreads: Optional[int] = None) -> dict:
        """The search's first stage (descent, level-0 walk, short-list) on the
        given ADC tables [nq][m][ksub] (float64) instead of the queries' own."""
        t = _c(tables, np.float64)
        nq = t.shape[0]
        assert t.shape[1:] == (self.m, 256)
        ef_arr = _c(np.broadcast_to(np.asarray(ef, dtype=np.int32), (nq,)), np.int32)
        out = {"cand_ids": np.empty((nq, S), np.int32), "cand_adc": np.empty((nq, S), np.float64),
               "cand_n": np.empty(nq, np.int32), "stats": np.empty((nq, 2), np.int32)}
        s = self._struct()
        rc = _load().orc_walk_tables(C.byref(s), _ptr(t), nq, _ptr(ef_arr), S, nthreads or default_threads(),
                                     _ptr(out["cand_ids"]), _ptr(out["cand_adc"]), _ptr(out["cand_n"]),
                                     _ptr(out["stats"]))
        if rc != 0:
            raise ValueError(f"orc_walk_tables failed ({rc})")
        return out

    def search(self, q: np.ndarray, ef, S: int, K: int, nthreads: Optional[int] = None, max_evals: int = 0) -> dict:
        """Full search; ``max_evals`` > 0 is the budget T on level-0 distance
        evaluations per query (Sec. 3.1), 0 none."""
        q = _c(q, np.float32)
        nq = q.shape[0]
        ef_arr = _c(np.broadcast_to(np.asarray(ef, dtype=np.int32), (nq,)), np.int32)
        out = {
            "ids": np.empty((nq, K), np.int32), "d": np.empty((nq, K), np.float64),
            "cand_ids": np.empty((nq, S), np.int32), "cand_adc": np.empty((nq, S), np.float64),
            "cand_n": np.empty(nq, np.int32), "stats": np.empty((nq, 2), np.int32),
        }
        s = self._struct()
        rc = _load().orc_search_capped(C.byref(s), _ptr(q), nq, _ptr(ef_arr), S, K, int(max_evals),
                                       nthreads or default_threads(), _ptr(out["ids"]), _ptr(out["d"]),
                                       _ptr(out["cand_ids"]), _ptr(out["cand_adc"]), _ptr(out["cand_n"]),
                                       _ptr(out["stats"]))
        if rc != 0:
            raise ValueError(f"orc_search failed ({rc})")
        return out


def build_index(w, db: np.ndarray, train: np.ndarray, proj: Optional[np.ndarray], level_u: np.ndarray,
                pq_init: np.ndarray, beta_ids: np.ndarray, beta_init: np.ndarray,
                nthreads: Optional[int] = None) -> Index:
    """Whole build from the seeded inputs: PQ (2-level when ``w.coarse_k``),
    levels, graph, regression codebook."""
    nt = nthreads or default_threads()
    coarse = None
    if getattr(w, "coarse_k", 0):
        import datagen
        ccent, _ = pq_train(train, proj, w.d_pad, 2, datagen.coarse_init_ids(w, train.shape[0]), w.pq_iters, nt,
                            ksub=w.coarse_k)
        _, rtrain = coarse_encode(train, proj, w.d_pad, ccent, nt)
        ccodes, rdb = coarse_encode(db, proj, w.d_pad, ccent, nt)
        cent, _ = pq_train(rtrain, None, w.d_pad, w.m, pq_init, w.pq_iters, nt)
        codes = pq_encode(rdb, None, w.d_pad, cent, nt)
        coarse = (ccent, ccodes)
    else:
        cent, _ = pq_train(train, proj, w.d_pad, w.m, pq_init, w.pq_iters, nt)
        codes = pq_encode(db, proj, w.d_pad, cent, nt)
    lv, _ = levels(level_u, w.level_ratio, w.max_level_cap)
    adj0, up_base, adj_up, entry, maxl = hnsw_build(db, proj, w.d_pad, cent, codes, lv, w.deg0, w.deg_up,
                                                    w.ef_construction, nt, coarse=coarse)
    beta, _ = beta_train(db, beta_ids, proj, w.d_pad, cent, codes, adj0, w.k_reg, w.n_beta, beta_init,
                         w.beta_kmeans_iters, w.em_iters, nt, m_beta=w.m_beta, coarse=coarse)
    bidx = beta_assign(db, proj, w.d_pad, cent, codes, adj0, w.k_reg, beta, nt, coarse=coarse)
    ix = Index(n=db.shape[0], d=db.shape[1], d_pad=w.d_pad, m=w.m, deg0=w.deg0, deg_up=w.deg_up, k_reg=w.k_reg,
               n_beta=w.n_beta, entry=entry, max_level=maxl, proj=proj, centroids=cent, codes=codes, adj0=adj0,
               level=lv, up_base=up_base, adj_up=adj_up, beta=beta, beta_idx=bidx, m_beta=w.m_beta)
    if coarse is not None:
        ix.coarse_cent, ix.coarse_codes = coarse
        ix.coarse_norm = ix.coarse_norms()
    return ix


def build_workload(w, nthreads: Optional[int] = None) -> tuple:
    """(index, db, queries) for a workload description, all from its seed."""
    import datagen
    db = datagen.vectors(w, "db")
    q = datagen.vectors(w, "query")
    train = datagen.vectors(w, "train")
    proj = datagen.projection(w)
    ix = build_index(w, db, train, proj, datagen.level_uniforms(w), datagen.pq_init_ids(w, train.shape[0]),
                     datagen.beta_train_ids(w), datagen.beta_init_ids(w, min(w.n, w.n_beta_train)), nthreads)
    return ix, db, q
