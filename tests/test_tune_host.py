"""Host logic of the launch-configuration autotuner (tune.py) on the CPU,
against a stand-in batch whose run time per step depends on the
configuration and a simulated clock: every candidate is timed after one
untimed run, the fastest per step is chosen, and the batch is left
configured with it.  The device path is covered by the GPU tests."""
import pytest

from paper_0911_5631_amd import tune


class Clock:
    t = 0.0

    def __call__(self):
        return self.t


class TimedBatch:
    def __init__(self, clock, cost):
        self.clock, self.cost = clock, cost      # cost(spr, grid) -> seconds per run
        self.config = None
        self.log = []

    def configure(self, spr, grid):
        self.config = (spr, grid)
        self.log.append(("configure", spr, grid))

    def run(self):
        self.clock.t += self.cost(*self.config)
        self.log.append(("run",) + self.config)

    def poll(self):
        return []


def test_fastest_per_step_is_kept(monkeypatch):
    clock = Clock()
    monkeypatch.setattr(tune.time, "perf_counter", clock)
    # per run: a fixed 40 us launch/host cost plus 1 us per step, and the
    # grid's own per-step cost (1024 the best)
    grid_cost = {2048: 0.20e-6, 1024: 0.05e-6, 4096: 0.30e-6, 8192: 0.50e-6}
    b = TimedBatch(clock, lambda spr, g: 40e-6 + spr * (1e-6 + grid_cost[g]))
    out = tune.autotune(b, runs=3)
    assert out["best"]["steps_per_run"] == 64 and out["best"]["grid"] == 1024
    assert b.config == (64, 1024)                      # left configured with the best
    assert len(out["trials"]) == len(tune.DEFAULT_CANDIDATES)
    for tr in out["trials"]:
        spr, g = tr["steps_per_run"], tr["grid"]
        assert tr["s_per_step"] == pytest.approx((40e-6 + spr * (1e-6 + grid_cost[g])) / spr)
    # each candidate: configure, one untimed run, then the timed runs
    for spr, g in tune.DEFAULT_CANDIDATES:
        k = b.log.index(("configure", spr, g))
        assert b.log[k + 1:k + 5] == [("run", spr, g)] * 4
