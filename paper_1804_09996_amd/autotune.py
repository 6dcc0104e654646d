"""Schedule autotuner for the walk.

Every :class:`Schedule` returns identical results (the pool, the short-list
and the (E, D) counts do not depend on where the visited set lives, on the
prefetch, on occupancy or on the order in which slots pick queries), so the
tuner is free to pick the fastest.  It times each candidate on the caller's
batch with HIP events on the launch stream and caches the winner in a JSON
file keyed by device, index shape, ef, short-list size and batch size.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Iterable, Optional

from . import Schedule, schedule

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lc_autotune.json")


def candidates(ef_max: int, S: int, f16: bool = False) -> list:
    """Grid of schedules: where the visited set lives (LDS table, or workspace
    bitset behind an LDS cache), the LDS table size and id width, prefetch,
    the pool in registers or in LDS (pools up to 128 entries), the codes of
    every probed link or only of those the visited table does not hold, and
    (fp16 tables) the query's table in LDS or in registers; always the
    queue."""
    out = [schedule(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0)]  # the library's own choice
    if max(ef_max, S) <= 128:
        out.append(schedule(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, pool=1))
    for hb in (9, 10, 11, 12):
        out.append(schedule(hash_bits=hb, prefetch=1, waves_per_cu=0, queue=1, visited=0))
    out.append(schedule(hash_bits=11, prefetch=0, waves_per_cu=0, queue=1, visited=0))
    out.append(schedule(hash_bits=12, prefetch=1, waves_per_cu=0, queue=1, visited=0, wide=1))
    out.append(schedule(hash_bits=9, prefetch=0, waves_per_cu=0, queue=1, visited=1))
    out.append(schedule(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, codes=1))
    if f16:
        for t in (1, 2):
            out.append(schedule(hash_bits=0, prefetch=1, waves_per_cu=0, queue=1, visited=0, table=t))
    return out


def _key(gix, nq: int, ef_max: int, S: int, table: str = "f32") -> str:
    torch = gix.torch
    name = torch.cuda.get_device_properties(gix.device).name
    bucket = 1 << max(0, (int(nq) - 1).bit_length())
    return f"{name}|n={gix.n}|m={gix.m}|ef={ef_max}|S={S}|nq~{bucket}|table={table}|schedule-fields=9"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: dict):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_schedule(gix, lut, ef, ef_max: int, S: int, sc: Schedule, reps: int = 3, scale=None) -> float:
    """Median milliseconds of one walk launch with schedule ``sc`` (``scale``:
    the row scales of an fp16 table)."""
    torch = gix.torch
    gix.search(lut, scale, ef=ef, ef_max=ef_max, S=S, stats=False, sched=sc)  # warm up, size the workspace
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        gix.search(lut, scale, ef=ef, ef_max=ef_max, S=S, stats=False, sched=sc)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(gix, lut, ef=None, ef_max: int = 64, S: int = 64, cands: Optional[Iterable[Schedule]] = None,
         reps: int = 3, cache_path: Optional[str] = DEFAULT_CACHE, log=None, scale=None):
    """Best schedule for this index and batch, and the timing table (``scale``:
    the row scales when ``lut`` is an fp16 table)."""
    key = _key(gix, lut.shape[0], ef_max, S, "f16" if scale is not None else "f32")
    cache = load_cache(cache_path) if cache_path else {}
    if key in cache:
        return schedule(**cache[key]["schedule"]), cache[key]["table"]
    table = []
    for sc in (cands or candidates(ef_max, S, f16=scale is not None)):
        ms = time_schedule(gix, lut, ef, ef_max, S, sc, reps, scale=scale)
        table.append({"schedule": sc.as_dict(), "ms": ms})
        if log:
            log(f"autotune {sc}: {ms:.3f} ms")
    best = min(table, key=lambda r: r["ms"])
    if cache_path:
        cache[key] = {"schedule": best["schedule"], "table": table}
        save_cache(cache_path, cache)
    return schedule(**best["schedule"]), table
