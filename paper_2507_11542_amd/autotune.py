"""Tile-shape autotuner for batched solves.

For a batch composition it times a short run (a few RK steps from V0 through
hj_step_batch, on copies of the inputs) for each candidate launch shape
(nodes per tile, workgroups per round launch), with HIP events on the stream
the launches go to, keeps the fastest, and caches it in a JSON file keyed by
precision, ndim, dynamics, scheme and the batch's total node count (rounded to
a power of two).  Cache: $HJ_AUTOTUNE_CACHE, else ~/.cache/hj_mi355x/autotune.json.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

# (nodes per tile, workgroups per round launch); workgroups 0 = flat launches
# (one workgroup per 256-node tile)
CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (256, 0), (1024, 1024), (1024, 2048), (2048, 1024), (2048, 2048), (4096, 512), (4096, 1024),
    (4096, 2048), (8192, 1024), (8192, 2048), (16384, 1024),
)


def cache_path() -> str:
    p = os.environ.get("HJ_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "hj_mi355x", "autotune.json")


def cache_key(prec: str, problems) -> str:
    p0 = problems[0]
    total = sum(p.points for p in problems)
    bucket = 1 << max(0, int(math.ceil(math.log2(max(total, 1)))))
    return "%s/%dd/%s/%s/rk%d/%d" % (prec, p0.ndim, p0.dynamics, p0.scheme, p0.order, bucket)


def load() -> Dict[str, List[int]]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(key: str, value: Sequence[int]):
    data = load()
    data[key] = list(value)
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(problems, grids, v0s, prec: str, steps: int = 6, reps: int = 2,
         candidates: Sequence[Tuple[int, int]] = CANDIDATES, use_cache: bool = True,
         stream=None) -> Tuple[Tuple[int, int], Dict[str, float]]:
    """Returns the fastest (tile_nodes, workgroups) and the timings (ms per
    RK step of the whole batch) of every candidate."""
    import torch

    from . import hj

    key = cache_key(prec, problems)
    if use_cache:
        hit = load().get(key)
        if hit:
            return (int(hit[0]), int(hit[1])), {}
    stream = stream or torch.cuda.current_stream()
    work = [v.clone() for v in v0s]
    timings: Dict[str, float] = {}
    best: Optional[Tuple[float, Tuple[int, int]]] = None
    for tile, wg in candidates:
        b = hj.Batch(tile_nodes=tile, workgroups=wg, use_graph=True)
        try:
            for w, v in zip(work, v0s):
                w.copy_(v)
            ts = [p.t0 for p in problems]
            b.step(grids, v0s, work, [p.t0 for p in problems], ts, [p.tf for p in problems],
                   [p.mode for p in problems], 1, stream)  # capture, alpha
            b.wait(len(problems), stream)
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                ts = [p.t0 for p in problems]
                e0.record(stream)
                b.step(grids, v0s, work, [p.t0 for p in problems], ts,
                       [p.tf for p in problems], [p.mode for p in problems], steps, stream)
                e1.record(stream)
                b.wait(len(problems), stream)
                ms.append(e0.elapsed_time(e1) / steps)
            t = min(ms)
        finally:
            b.close()
        timings["%d/%d" % (tile, wg)] = t
        if best is None or t < best[0]:
            best = (t, (tile, wg))
    assert best is not None
    if use_cache:
        store(key, best[1])
    return best[1], timings
