"""Batched instances: subdomain layout per instance and the autotuner that picks it.

The batched driver (acch_batch_*) runs all instances' subdomain solves in one launch
per stage; the subdomain box size trades parallelism (more, smaller boxes: more
workgroups, shorter wavefront chains) against preconditioner quality (fewer GMRES
iterations with larger boxes).  The autotuner times whole batched steps for a few
box sizes on a copy of the batch and keeps the fastest, per tuning problem (the mix of
instance sizes, the precision, the overlap and the subdomain solver), optionally cached
in a JSON file.
"""
from __future__ import annotations

import json
import os
import tempfile
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from .binding import BatchSolver


def parts_for(n: int, box: int, overlap: int, periodic: bool) -> int:
    """Subdomains along an axis of n cells for a target owned width `box`; periodic
    axes need at least 2 parts and boxes (owned + 2 overlap) at most n - 2 wide."""
    k = max(1, int(round(n / box)))
    if periodic:
        k = max(2, k)
        while -(-n // k) + 2 * overlap > n - 2:
            k += 1
    return min(k, n)


def with_boxes(shapes: Sequence[Tuple[int, int]], params: List[Dict], box: int, overlap: int) -> List[Dict]:
    out = []
    for (ny, nx), p in zip(shapes, params):
        periodic = p.get("bc", "periodic") == "periodic"
        q = dict(p)
        q["sub"] = (parts_for(nx, box, overlap, periodic), parts_for(ny, box, overlap, periodic))
        out.append(q)
    return out


def tune_key(shapes: Sequence[Tuple[int, int]], precision: str, overlap: int, boxes: Sequence[int],
             solver: Tuple[str, int, float] = ("ilu0", 0, 0.0)) -> str:
    """Cache key of a tuning problem: the multiset of instance sizes, the precision, the
    overlap, the candidate box widths and the subdomain solver (name, fill level, diagonal
    shift), which decides both the iteration counts and the kernels that run."""
    counts: Dict[Tuple[int, int], int] = {}
    for s in shapes:
        counts[tuple(int(x) for x in s)] = counts.get(tuple(int(x) for x in s), 0) + 1
    return json.dumps({"shapes": sorted([list(k), v] for k, v in counts.items()), "precision": precision,
                       "overlap": int(overlap), "boxes": [int(b) for b in boxes],
                       "solver": [str(solver[0]), int(solver[1]), float(solver[2])]}, sort_keys=True)


def _load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _save_cache(path: str, data: Dict[str, dict]) -> None:
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)   # readers see the old or the new file, never a partial one


def time_box(fields, params, box: int, steps: int, **common) -> float:
    """Seconds per batched step with owned box width `box`, after one untimed step that
    also records the graphs."""
    import torch
    overlap = common.get("overlap", 1)
    shapes = [u.shape for u, _ in fields]
    with BatchSolver(fields, with_boxes(shapes, params, box, overlap), **common) as b:
        b.step(1)
        b.stream.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.stream.synchronize()
        t = (time.perf_counter() - t0) / steps
    torch.cuda.synchronize()
    return t


def autotune(fields, params, boxes: Sequence[int] = (24, 32, 48, 64), steps: int = 1, cache: Optional[str] = None,
             timer: Optional[Callable[..., float]] = None, **common):
    """Time `steps` batched steps for each candidate box size and return (best box,
    {box: seconds per step}).  With `cache` (a JSON file), a tuning problem already in
    the file (same instance sizes, precision, overlap, candidates and subdomain solver) is
    answered from it without timing, and a new result is added to it."""
    timer = timer or time_box
    solver = (common.get("subsolver", "ilu0"), common.get("fill_level", 0), common.get("ilu_shift", 0.0))
    key = tune_key([u.shape for u, _ in fields], common.get("precision", "fp64"), common.get("overlap", 1), boxes,
                   solver)
    if cache:
        hit = _load_cache(cache).get(key)
        if hit is not None:
            return int(hit["box"]), {int(k): float(v) for k, v in hit["seconds_per_step"].items()}
    timings = {int(box): timer(fields, params, box, steps, **common) for box in boxes}
    best = min(timings, key=timings.get)
    if cache:
        data = _load_cache(cache)
        data[key] = {"box": best, "seconds_per_step": {str(k): v for k, v in timings.items()}}
        _save_cache(cache, data)
    return best, timings
