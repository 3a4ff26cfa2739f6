"""Launch-configuration autotuner for batched replicas.

The tunables are the ones that change neither the arithmetic nor its order,
so every system's trajectory stays bit-identical whatever is chosen: the
number of steps replayed per run (the length of the captured graph, which
amortises the per-run kick and host round trip) and the workgroups per kernel
launch (tiles beyond the grid are taken in further passes of the same
workgroups).  Each candidate is timed on the batch's own admitted mix with
real runs -- the steps count toward the systems' targets -- and the fastest
per step is kept.
"""
from __future__ import annotations

import time
from typing import Dict, Iterable, List, Sequence, Tuple

DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (16, 2048), (32, 2048), (64, 2048), (64, 1024), (64, 4096), (64, 8192))


def autotune(batch, candidates: Iterable[Sequence[int]] = DEFAULT_CANDIDATES,
             runs: int = 2) -> Dict:
    """Time ``runs`` runs of ``batch`` per (steps_per_run, grid) candidate,
    after one untimed run that captures the candidate's graph; configure the
    batch with the fastest (seconds per step) and return the timings.
    ``batch.poll()`` synchronises, so each timing covers the device work."""
    trials: List[Dict] = []
    for spr, grid in candidates:
        batch.configure(int(spr), int(grid))
        batch.run()
        batch.poll()
        t0 = time.perf_counter()
        for _ in range(runs):
            batch.run()
        batch.poll()
        el = time.perf_counter() - t0
        trials.append({"steps_per_run": int(spr), "grid": int(grid),
                       "s_per_step": el / (runs * int(spr))})
    best = min(trials, key=lambda t: t["s_per_step"])
    batch.configure(best["steps_per_run"], best["grid"])
    return {"best": best, "trials": trials}
