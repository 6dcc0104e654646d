"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the Link & Code method: it only draws
random numbers (database and query vectors, the uniforms from which node
levels are derived, random subsets used to initialise k-means and to pick the
regression training set, and a random orthonormal projection).  Everything the
method computes from those draws lives either in ``oracle/`` (the reference
implementation) or in the ``paper_1804_09996_amd`` package (the GPU path), and
the two never import each other.

Every array is a pure function of ``(seed, stream name, shape)``: the numpy
``Generator(PCG64(SeedSequence([seed, stream_id])))`` is deterministic across
platforms, so the oracle and the GPU path always see identical inputs.

Workload shapes follow the paper's data sets: 96-d L2-normalised CNN
descriptors (Deep1B, Sec. 3 and Sec. 5.2) are stood in for by an
L2-normalised Gaussian mixture, and 128-d SIFT descriptors (BIGANN, Sec. 5.2)
by non-negative integers with a heavy-tailed marginal.  None of those data
sets' own vectors are used or reproduced.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np

DEFAULT_SEED = 1804

# Named random streams.  The integer ids are arbitrary but frozen.
_STREAMS = {
    "DB": 1,
    "QUERY": 2,
    "TRAIN": 3,
    "MEANS": 4,
    "LEVELS": 5,
    "BETA": 6,
    "ARRIVALS": 7,
    "PQ_INIT": 8,
    "BETA_INIT": 9,
    "DIMS": 10,
    "PROJ": 11,
    "EF": 12,
    "MISC": 13,
    "COARSE_INIT": 14,
}


def rng(seed: int, stream: str, sub: int = 0) -> np.random.Generator:
    """Generator for one named stream (``sub`` splits a stream further)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), _STREAMS[stream], int(sub)])))


# ---------------------------------------------------------------------------
# Workload descriptions (sizes and knobs only).
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # database size
    nq: int                # number of queries
    d: int                 # input dimension
    dist: str              # "gmm" or "int128"
    n_comp: int            # mixture components (gmm)
    m: int                 # PQ sub-quantizers (8 bits each)
    d_pad: int             # dimension after the optional orthonormal projection
    deg0: int = 32         # level-0 degree
    deg_up: int = 32       # upper-level degree (Sec. 4.1)
    level_ratio: int = 30  # size ratio between two graph levels (Sec. 4.1)
    max_level_cap: int = 16
    k_reg: int = 16        # regression neighbours
    n_beta: int = 256      # beta codebook size (Sec. 4.3)
    ef: int = 128          # efSearch
    shortlist: int = 256   # S
    topk: int = 100        # K
    ef_construction: int = 64
    n_train: int = 65536   # PQ training vectors (a distinct draw)
    pq_iters: int = 25
    n_beta_train: int = 250_000   # regression-codebook training subset (Sec. 5.2)
    beta_kmeans_iters: int = 20
    em_iters: int = 10            # Sec. 5.2
    seed: int = DEFAULT_SEED
    m_beta: int = 1               # regression-codebook blocks (product codebook, Sec. 4.3 Eq. 9)
    opq_iters: int = 0            # learned rotation ahead of PQ (OPQ): rotation steps, 0 = none
    coarse_k: int = 0             # 2-level residual codec (Sec. 5.1): first-level centroids per half, 0 = none

    @property
    def dsub(self) -> int:
        return self.d_pad // self.m

    @property
    def ef_eff(self) -> int:
        return max(self.ef, self.shortlist)

    def key(self) -> str:
        """Stable hash of every field: names cached index files."""
        s = repr(dataclasses.astuple(self)).encode()
        return hashlib.sha1(s).hexdigest()[:16]


def _pad_for(d: int, m: int) -> int:
    return m * ((d + m - 1) // m)


C1 = Workload(name="C1-tiny", n=10_000, nq=100, d=96, dist="gmm", n_comp=64, m=8, d_pad=96,
              k_reg=8, ef=64, shortlist=64, topk=10, n_train=16384, pq_iters=20)
C2 = Workload(name="C2-1M", n=1_000_000, nq=10_000, d=96, dist="gmm", n_comp=1024, m=16, d_pad=96,
              k_reg=16, ef=128, shortlist=256, topk=100)
C3 = Workload(name="C3-int128", n=1_000_000, nq=10_000, d=128, dist="int128", n_comp=0, m=32, d_pad=128,
              k_reg=16, ef=128, shortlist=128, topk=10)
C4 = Workload(name="C4-10M", n=10_000_000, nq=100_000, d=96, dist="gmm", n_comp=1024, m=16, d_pad=96,
              k_reg=16, ef=128, shortlist=128, topk=100)
C5 = Workload(name="C5-20M", n=20_000_000, nq=1024, d=96, dist="gmm", n_comp=1024, m=56, d_pad=112,
              k_reg=32, ef=128, shortlist=128, topk=10)

WORKLOADS = {w.name: w for w in (C1, C2, C3, C4, C5)}


def small(name: str = "tiny", **kw) -> Workload:
    """A small workload for unit tests (defaults are C1's knobs)."""
    base = dict(name=name, n=2000, nq=32, d=24, dist="gmm", n_comp=8, m=4, d_pad=24, k_reg=4,
                ef=16, shortlist=16, topk=5, n_train=2048, pq_iters=8, n_beta=16,
                n_beta_train=2000, beta_kmeans_iters=5, em_iters=4, ef_construction=32)
    base.update(kw)
    if "d_pad" not in kw:
        base["d_pad"] = _pad_for(base["d"], base["m"])
    return Workload(**base)


# ---------------------------------------------------------------------------
# Vector generators.
# ---------------------------------------------------------------------------
def _gmm_params(w: Workload):
    """Component means and the fixed rotation of the mixture.

    The mixture is drawn in a latent basis where the spectrum decays like that
    of PCA-reduced CNN descriptors (mean spread ~ t^-1, within-component spread
    ~ t^-2 along latent axis t = 1..d, so the local intrinsic dimension is
    low), then turned by a seeded random rotation so that the variance is not
    aligned with any product-quantizer block."""
    t = np.arange(1, w.d + 1, dtype=np.float64)
    means = rng(w.seed, "MEANS").standard_normal((w.n_comp, w.d)) * np.sqrt(t ** -1.0)[None, :]
    a = rng(w.seed, "MEANS", 1).standard_normal((w.d, w.d))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    return means, np.sqrt(t ** -2.0), q


def _chunks(n: int, chunk: int, fill) -> None:
    """Run fill(c0, c1) over the chunks of range(n); chunks draw from their
    own sub-streams, so they run on a thread pool (numpy releases the GIL in
    its generators and matrix products) and the result does not depend on it."""
    starts = list(range(0, n, chunk))
    if len(starts) <= 1:
        for c0 in starts:
            fill(c0, min(n, c0 + chunk))
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1, len(starts)))) as ex:
        list(ex.map(lambda c0: fill(c0, min(n, c0 + chunk)), starts))


def gmm(w: Workload, n: int, stream: str, chunk: int = 1 << 18) -> np.ndarray:
    """``x = R (mu_c + eps)`` with c uniform over the components,
    ``mu_c ~ N(0, diag(t^-1))``, ``eps ~ N(0, diag(t^-2))`` and ``R`` a seeded
    rotation; drawn in float64, L2-normalised, rounded to float32."""
    means, noise_sd, rot = _gmm_params(w)
    out = np.empty((n, w.d), dtype=np.float32)

    def fill(c0, c1):
        g = rng(w.seed, stream, c0 // chunk)
        comp = g.integers(0, w.n_comp, size=c1 - c0)
        x = means[comp] + g.standard_normal((c1 - c0, w.d)) * noise_sd[None, :]
        x = x @ rot.T
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[c0:c1] = x

    _chunks(n, chunk, fill)
    return out


def int128(w: Workload, n: int, stream: str, chunk: int = 1 << 18) -> np.ndarray:
    """Non-negative integers 0..255 stored as float32: a seeded 70 % of the
    dimensions take ``min(floor(Exp(mean 20)), 255)``, the rest ``floor(256 U)``."""
    n_exp = int(round(0.7 * w.d))
    dims = np.sort(rng(w.seed, "DIMS").permutation(w.d)[:n_exp])
    is_exp = np.zeros(w.d, dtype=bool)
    is_exp[dims] = True
    out = np.empty((n, w.d), dtype=np.float32)

    def fill(c0, c1):
        g = rng(w.seed, stream, c0 // chunk)
        e = np.minimum(np.floor(g.exponential(20.0, size=(c1 - c0, w.d))), 255.0)
        u = np.floor(256.0 * g.random(size=(c1 - c0, w.d)))
        out[c0:c1] = np.where(is_exp[None, :], e, u).astype(np.float32)

    _chunks(n, chunk, fill)
    return out


def vectors(w: Workload, which: str) -> np.ndarray:
    """``which`` in {"db", "query", "train"}: the three disjoint draws."""
    n = {"db": w.n, "query": w.nq, "train": w.n_train}[which]
    stream = {"db": "DB", "query": "QUERY", "train": "TRAIN"}[which]
    if w.dist == "gmm":
        return gmm(w, n, stream)
    if w.dist == "int128":
        return int128(w, n, stream)
    raise ValueError(w.dist)


def projection(w: Workload) -> Optional[np.ndarray]:
    """Seeded orthonormal ``P`` of shape ``[d_pad, d]`` (``None`` when
    ``d_pad == d``): the first ``d`` columns of the Q factor of a Gaussian
    ``d_pad x d_pad`` matrix, column signs fixed so that diag(R) > 0."""
    if w.d_pad == w.d:
        return None
    a = rng(w.seed, "PROJ").standard_normal((w.d_pad, w.d_pad))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    return np.ascontiguousarray(q[:, : w.d]).astype(np.float32)


# ---------------------------------------------------------------------------
# Random draws that the method itself consumes.
# ---------------------------------------------------------------------------
def level_uniforms(w: Workload) -> np.ndarray:
    """``U_i`` in (0, 1], one per database vector (float64)."""
    return 1.0 - rng(w.seed, "LEVELS").random(w.n)


def sample_ids(seed: int, stream: str, n: int, k: int, sub: int = 0) -> np.ndarray:
    """``k`` distinct ids from ``range(n)`` (int64, in draw order)."""
    k = min(k, n)
    return rng(seed, stream, sub).permutation(n)[:k].astype(np.int64)


def pq_init_ids(w: Workload, n_train: int) -> np.ndarray:
    """Per-subspace k-means seeds: ``[m, 256]`` distinct training row ids."""
    return np.stack([sample_ids(w.seed, "PQ_INIT", n_train, 256, s) for s in range(w.m)])


def coarse_init_ids(w: Workload, n_train: int) -> np.ndarray:
    """k-means seeds of the 2-level codec's first level: ``[2, coarse_k]``
    distinct training row ids."""
    return np.stack([sample_ids(w.seed, "COARSE_INIT", n_train, w.coarse_k, h) for h in range(2)])


def beta_train_ids(w: Workload) -> np.ndarray:
    """Sorted regression training subset of ``min(n, n_beta_train)`` ids."""
    return np.sort(sample_ids(w.seed, "BETA", w.n, w.n_beta_train))


def beta_init_ids(w: Workload, n_sub: int) -> np.ndarray:
    """k-means seeds for the beta codebook: ids into the training subset."""
    return sample_ids(w.seed, "BETA_INIT", n_sub, w.n_beta)


def per_query_ef(w: Workload, lo: int = 16, hi: int = 512) -> np.ndarray:
    """efSearch per query, ``round(exp(U(ln lo, ln hi)))`` (int32)."""
    u = rng(w.seed, "EF").random(w.nq)
    return np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int32)
