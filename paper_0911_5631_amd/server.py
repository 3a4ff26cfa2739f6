"""Serving loop: requests arrive over time (a Poisson trace), are admitted into
one batch while their device memory fits the HBM budget and a slot is free,
advance together in graph replays (continuous batching: a finished system's
slot and memory go to the next queued request between replays), and leave
when their steps are done.

Reported per request: queueing delay (arrival -> admission) and latency
(arrival -> completion); for the run: p50 / p99 latency, offered load, and
aggregate atom-steps/s over the makespan.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .inputs import Request
from .md import Batch


@dataclasses.dataclass
class Served:
    name: str
    n: int
    steps: int
    arrival: float
    admitted: float
    done: float
    slot: int
    pos: Optional[np.ndarray] = None
    vel: Optional[np.ndarray] = None
    props: Optional[Dict[str, float]] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queueing(self) -> float:
        return self.admitted - self.arrival


def serve(requests: Sequence[Request], hbm_budget: int, *, max_slots: int = 64,
          steps_per_run: int = 64, time_scale: float = 1.0, keep_state: bool = False,
          dt: float = 0.005,
          clock: Callable[[], float] = time.perf_counter) -> Dict:
    """Serve ``requests`` (arrival times scaled by ``time_scale``) and return
    the per-request records and the run's statistics."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    batch = Batch(hbm_budget, max_slots, steps_per_run)
    queue: collections.deque = collections.deque()
    active: Dict[int, tuple] = {}
    served: List[Served] = []
    peak_bytes = 0
    t0 = clock()
    i = 0
    try:
        while i < len(reqs) or queue or active:
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival * time_scale <= now:
                queue.append(reqs[i])
                i += 1
            # admit in arrival order while the head of the queue fits
            while queue:
                r = queue[0]
                s = r.system()
                slot = batch.try_admit(s.pos, s.vel, s.box, r.steps, shell=s.shell, dt=dt,
                                       precision=s.precision)
                if slot is None:
                    break
                queue.popleft()
                active[slot] = (r, clock() - t0)
                peak_bytes = max(peak_bytes, batch.usage()[0])
            if not active:
                if queue:
                    raise RuntimeError(f"request {queue[0].name} does not fit an empty batch "
                                       f"(budget {hbm_budget} bytes)")
                if i < len(reqs):
                    time.sleep(max(0.0, reqs[i].arrival * time_scale - (clock() - t0)))
                continue
            batch.run()
            for slot in batch.poll():
                r, t_adm = active.pop(slot)
                t_done = clock() - t0
                rec = Served(r.name, r.n, r.steps, r.arrival * time_scale, t_adm, t_done, slot)
                rec.props = batch.props(slot)
                if keep_state:
                    rec.pos, rec.vel, _ = batch.get_state(slot)
                batch.release(slot)
                served.append(rec)
    finally:
        batch.close()
    makespan = max(r.done for r in served) if served else 0.0
    lat = np.array([r.latency for r in served])
    work = float(sum(r.n * r.steps for r in served))
    span = (reqs[-1].arrival - reqs[0].arrival) * time_scale if len(reqs) > 1 else 0.0
    return {
        "served": served,
        "n_requests": len(served),
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else 0.0,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else 0.0,
        "mean_queueing_s": float(np.mean([r.queueing for r in served])) if served else 0.0,
        "makespan_s": makespan,
        "atom_steps": work,
        "atom_steps_per_s": work / makespan if makespan > 0 else 0.0,
        "offered_atom_steps_per_s": work / span if span > 0 else float("inf"),
        "peak_bytes": peak_bytes,
    }
