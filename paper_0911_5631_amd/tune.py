"""Launch-configuration autotuner for batches and single systems.

The knobs are the ones that change neither the arithmetic nor its order, so
every system's trajectory stays bit-identical whatever is chosen:

  steps_per_run  length of the captured replay graph (amortises the per-run
                 kick and host round trip);
  grid           workgroups per step-kernel launch (tiles beyond the grid are
                 taken in further passes of the same workgroups);
  sort_grid      workgroups per sort launch;
  sort_split     workgroups sharing one 256-cell tile of the sort;
  tile_order     how the step kernel's workgroups walk the tiles across the 8
                 XCDs (passes of consecutive runs, or one slab of tiles per
                 XCD so that z-neighbour rows share an L2).

A batch is tuned on its own admitted mix with real runs (the steps count
toward the systems' targets).  A trial is scored by the atom-steps the batch
actually advanced per second, read from the device step counters before and
after it; a trial during which a system finished or was admitted (the work
per step changed) is discarded, and no trial is started that could finish a
system.  Results are kept in a JSON cache keyed by GPU architecture, kind
(batch or single system) and atom-count bucket.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, List, Mapping, Optional

KNOBS = ("steps_per_run", "grid", "sort_grid", "sort_split", "tile_order")

# tile_order: 1 passes, 2 XCD slabs (0 asks for the library's choice)
DEFAULT_CANDIDATES = (
    {"steps_per_run": 16, "grid": 2048, "sort_grid": 2048, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 32, "grid": 2048, "sort_grid": 2048, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 2048, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 2048, "sort_split": 1, "tile_order": 2},
    {"steps_per_run": 64, "grid": 1024, "sort_grid": 2048, "sort_split": 1, "tile_order": 2},
    {"steps_per_run": 64, "grid": 4096, "sort_grid": 2048, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 1024, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 4096, "sort_split": 1, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 2048, "sort_split": 2, "tile_order": 1},
)

SINGLE_CANDIDATES = (
    {"steps_per_run": 64, "grid": 0, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 0, "sort_grid": 0, "sort_split": 0, "tile_order": 1},
    {"steps_per_run": 64, "grid": 2048, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 0, "sort_grid": 256, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 0, "sort_grid": 1024, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 0, "sort_grid": 2048, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 0, "sort_grid": 4096, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 32, "grid": 0, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 4096, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 8192, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
    {"steps_per_run": 64, "grid": 16384, "sort_grid": 0, "sort_split": 0, "tile_order": 2},
)


def _cfg(c: Mapping) -> Dict[str, int]:
    return {k: int(c.get(k, 0)) for k in KNOBS}


def size_bucket(n_atoms: int) -> int:
    """Atom-count bucket: floor(log2 N) (systems within a factor of two share
    a tuned configuration)."""
    return int(math.floor(math.log2(max(int(n_atoms), 1))))


def cache_key(arch: str, kind: str, n_atoms: int) -> str:
    return f"{arch.split(':')[0]}/{kind}/{size_bucket(n_atoms)}"


def load_cache(path: Optional[str]) -> Dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(path: Optional[str], key: str, entry: Dict) -> None:
    if not path:
        return
    cache = load_cache(path)
    cache[key] = entry
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(batch, candidates: Iterable[Mapping] = DEFAULT_CANDIDATES, runs: int = 2,
             cache_path: Optional[str] = None, key: Optional[str] = None,
             clock=None, warm_runs: int = 0, trial_steps: int = 0) -> Dict:
    """Time ``runs`` runs of ``batch`` per candidate (after one untimed run
    that captures the candidate's graph), score each by atom-steps advanced
    per second, configure the batch with the best and return the trials.
    ``warm_runs`` untimed runs at the batch's configuration come first, so
    that no candidate is timed over the systems' first steps (from a lattice
    start they rebuild later than they will afterwards).  With
    ``trial_steps`` every candidate is timed over at least that many steps
    (more runs for shorter replays), so that candidates with short replays
    are not scored over a window that happens to hold fewer rebuilds.

    ``batch`` offers configure(**knobs), run(), poll() (synchronises) and
    progress() -> (atom-steps done, systems running, fewest steps left)."""
    clock = clock or time.perf_counter
    trials: List[Dict] = []
    _, running, left = batch.progress()
    for _ in range(warm_runs):
        if running == 0 or left <= 64:
            break
        batch.run()
        batch.poll()
        _, running, left = batch.progress()
    budget = left - 1          # steps every running system can still take safely
    for cand in candidates:
        c = _cfg(cand)
        spr = c["steps_per_run"] or 64
        n_runs = max(runs, -(-int(trial_steps) // spr))
        if running == 0 or (1 + n_runs) * spr > budget:
            trials.append({**c, "skipped": "a trial could finish a system"})
            continue
        batch.configure(**c)
        batch.run()            # captures this configuration's graph
        batch.poll()
        a0, k0, _ = batch.progress()
        t0 = clock()
        for _ in range(n_runs):
            batch.run()
        batch.poll()
        el = clock() - t0
        a1, k1, _ = batch.progress()
        budget -= (1 + n_runs) * spr
        if k1 != k0:
            trials.append({**c, "skipped": "the mix changed during the trial"})
            continue
        trials.append({**c, "atom_steps_per_s": (a1 - a0) / el if el > 0 else 0.0,
                       "seconds": el, "steps": n_runs * spr})
    scored = [t for t in trials if "atom_steps_per_s" in t]
    if not scored:
        return {"best": None, "trials": trials}
    best = max(scored, key=lambda t: t["atom_steps_per_s"])
    used = batch.configure(**{k: best[k] for k in KNOBS})
    if key:
        store(cache_path, key, {"config": {k: best[k] for k in KNOBS},
                                "atom_steps_per_s": best["atom_steps_per_s"]})
    return {"best": best, "in_use": used, "trials": trials}


def autotune_system(system, n_atoms: int, candidates: Iterable[Mapping] = SINGLE_CANDIDATES,
                    steps: int = 512, cache_path: Optional[str] = None,
                    key: Optional[str] = None, clock=None) -> Dict:
    """The same for one system: each candidate advances it ``steps`` real
    steps (after one untimed replay that warms the new graphs), timed to the
    synchronising props() call; the fastest is kept."""
    clock = clock or time.perf_counter
    trials: List[Dict] = []
    for cand in candidates:
        c = _cfg(cand)
        system.configure(**c)
        system.step(c["steps_per_run"] or 64)
        system.props()
        t0 = clock()
        system.step(steps)
        system.props()
        el = clock() - t0
        trials.append({**c, "atom_steps_per_s": n_atoms * steps / el if el > 0 else 0.0})
    best = max(trials, key=lambda t: t["atom_steps_per_s"])
    used = system.configure(**{k: best[k] for k in KNOBS})
    if key:
        store(cache_path, key, {"config": {k: best[k] for k in KNOBS},
                                "atom_steps_per_s": best["atom_steps_per_s"]})
    return {"best": best, "in_use": used, "trials": trials}


def apply_cached(target, path: Optional[str], key: str) -> Optional[Dict[str, int]]:
    """Configure ``target`` (a System or Batch) from the cache entry ``key``,
    if there is one; returns the configuration in use, else None."""
    entry = load_cache(path).get(key)
    if not entry:
        return None
    return target.configure(**entry["config"])
