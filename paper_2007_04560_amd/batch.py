"""Batched instances: subdomain layout per instance and the autotuner that picks it.

The batched driver (acch_batch_*) runs all instances' subdomain solves in one launch
per stage; the subdomain box size trades parallelism (more, smaller boxes: more
workgroups, shorter wavefront chains) against preconditioner quality (fewer GMRES
iterations with larger boxes).  The autotuner times whole batched steps for a few
box sizes on a copy of the batch and keeps the fastest.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence, Tuple

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


def autotune(fields, params, boxes: Sequence[int] = (24, 32, 48, 64), steps: int = 1, **common):
    """Time `steps` batched steps (after one untimed step that also records the
    graphs) for each candidate box size; returns (best box, {box: seconds per step})."""
    import torch
    overlap = common.get("overlap", 1)
    shapes = [u.shape for u, _ in fields]
    timings = {}
    for box in boxes:
        with BatchSolver(fields, with_boxes(shapes, params, box, overlap), **common) as b:
            b.step(1)
            b.stream.synchronize()
            t0 = time.perf_counter()
            b.step(steps)
            b.stream.synchronize()
            timings[box] = (time.perf_counter() - t0) / steps
        torch.cuda.synchronize()
    best = min(timings, key=timings.get)
    return best, timings
