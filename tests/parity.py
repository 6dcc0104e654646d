"""Comparison rules between the GPU path and the oracle (test infrastructure).

A query is EXACT when its ordered top-K ids equal the oracle's, except that at
a rank where they differ both ids must have oracle refined distances within
``rel`` of each other (float32 rounding may swap near-ties; which of two such
ids comes first is then not unique).  Independently, every returned distance
must be within ``rel`` of the oracle's float64 refined distance of that id.
"""
import numpy as np

REL = 1e-5


def query_exact(ix, y, gpu_ids, orc_ids, orc_d, rel=REL) -> bool:
    if len(gpu_ids) != len(orc_ids):
        return False
    valid = [int(g) for g in gpu_ids if g >= 0]
    if len(set(valid)) != len(valid):
        return False
    for r, (g, o) in enumerate(zip(gpu_ids, orc_ids)):
        if g == o:
            continue
        if g < 0 or o < 0:
            return False
        dg = ix.refined_distance(y, int(g))
        if abs(dg - orc_d[r]) > rel * max(abs(orc_d[r]), 1e-30):
            return False
    return True


def distance_errors(ix, q, ids, d):
    """Relative error of each returned distance against the oracle's float64
    refined distance of the same id (NaN for padding)."""
    err = np.full(ids.shape, np.nan)
    for i in range(ids.shape[0]):
        for r in range(ids.shape[1]):
            if ids[i, r] >= 0:
                ref = ix.refined_distance(q[i], int(ids[i, r]))
                err[i, r] = abs(float(d[i, r]) - ref) / max(abs(ref), 1e-30)
    return err


def summarize(ix, q, gpu_ids, gpu_d, orc):
    exact = np.array([query_exact(ix, q[i], gpu_ids[i], orc["ids"][i], orc["d"][i]) for i in range(q.shape[0])])
    strict = np.array([np.array_equal(gpu_ids[i], orc["ids"][i]) for i in range(q.shape[0])])
    err = distance_errors(ix, q, gpu_ids, gpu_d)
    return {"exact": exact, "exact_frac": float(exact.mean()) if exact.size else 1.0,
            "strict_frac": float(strict.mean()) if strict.size else 1.0,
            "max_rel_err": float(np.nanmax(err)) if np.isfinite(err).any() else 0.0}


def recall_at(ids, gt, r):
    return float(np.mean([gt[i] in ids[i, :r] for i in range(len(gt))]))
