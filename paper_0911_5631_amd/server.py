"""Serving loop: requests arrive over time (a Poisson trace), are admitted into
one batch while their device memory fits the HBM budget and a slot is free,
advance together in graph replays (continuous batching: a finished system's
slot and memory go to the next queued request between replays), and leave
when their steps are done.

Reported per request: queueing delay (arrival -> admission) and latency
(arrival -> completion); for the run: p50 / p99 latency, offered load,
aggregate atom-steps/s over the makespan, and the fraction of the makespan
the GPU spent on the batch's runs (``gpu_busy_fraction``).  The busy time is
measured with timing events recorded on the caller's stream before and after
every run: the library orders that stream after each call's device work, so
an event pair spans the run's device time (and no host idle time, since the
"before" event completes only when the stream reaches it).  The step-0
evaluations of admissions are not counted, so the fraction errs low.

While a run executes on the device, the host builds the start of the next
queued request (its lattice and velocities), so that this work does not
leave the device idle at the next admission.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .inputs import Request
from .md import Batch


class RunTimer:
    """Device time of the batch's runs: a pair of timing events on the
    caller's current stream around each run, summed at the end."""

    def __init__(self):
        import torch
        self._torch = torch
        self._stream = torch.cuda.current_stream()
        self._spans = []

    def before(self):
        ev = self._torch.cuda.Event(enable_timing=True)
        ev.record(self._stream)
        self._spans.append([ev, None])

    def after(self):
        ev = self._torch.cuda.Event(enable_timing=True)
        ev.record(self._stream)
        self._spans[-1][1] = ev

    def runs(self) -> int:
        return len(self._spans)

    def total_s(self) -> float:
        self._torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._spans) * 1e-3


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
    timer = RunTimer()
    queue: collections.deque = collections.deque()
    active: Dict[int, tuple] = {}
    served: List[Served] = []
    built: Dict[str, object] = {}       # starts built ahead, by request name
    peak_bytes = 0
    t0 = clock()
    i = 0

    def start_of(r):
        s = built.pop(r.name, None)
        return s if s is not None else r.system()

    try:
        while i < len(reqs) or queue or active:
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival * time_scale <= now:
                queue.append(reqs[i])
                i += 1
            # admit in arrival order while the head of the queue fits
            while queue:
                r = queue[0]
                s = start_of(r)
                slot = batch.try_admit(s.pos, s.vel, s.box, r.steps, shell=s.shell, dt=dt,
                                       precision=s.precision)
                if slot is None:
                    built[r.name] = s
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
            timer.before()
            batch.run()
            timer.after()
            # while the run executes: the start of the next request waiting
            nxt = queue[0] if queue else (reqs[i] if i < len(reqs) else None)
            if nxt is not None and nxt.name not in built:
                built[nxt.name] = nxt.system()
            for slot in batch.poll():
                r, t_adm = active.pop(slot)
                t_done = clock() - t0
                rec = Served(r.name, r.n, r.steps, r.arrival * time_scale, t_adm, t_done, slot)
                rec.props = batch.props(slot)
                if keep_state:
                    rec.pos, rec.vel, _ = batch.get_state(slot)
                batch.release(slot)
                served.append(rec)
            peak_bytes = max(peak_bytes, batch.usage()[0])
    finally:
        batch.close()
    busy = timer.total_s()
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
        "runs": timer.runs(),
        "gpu_busy_s": busy,
        "gpu_busy_fraction": busy / makespan if makespan > 0 else 0.0,
    }
