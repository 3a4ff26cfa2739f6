"""Host logic of the serving loop (paper_0911_5631_amd/server.py) on the CPU:
the scheduler runs against a stand-in batch with the same calls (admission
under a byte budget and a slot limit, runs of a fixed number of steps,
polling, release) and a simulated clock, so that admission order, budget,
slot reuse and the reported statistics can be checked exactly.  The device
path of the same loop is covered by the GPU tests."""
import numpy as np
import pytest

from paper_0911_5631_amd import inputs as I
from paper_0911_5631_amd import server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBatch:
    """Admits while the bytes fit and a slot is free; every run advances each
    admitted system by steps_per_run steps and takes run_s of the clock."""

    instances = []
    BYTES_PER_ATOM = 400

    def __init__(self, budget, max_slots, steps_per_run, clock=None, run_s=0.01):
        self.budget, self.max_slots, self.spr = budget, max_slots, steps_per_run
        self.clock, self.run_s = clock, run_s
        self.slots = {}
        self.peak = 0
        self.closed = False
        FakeBatch.instances.append(self)

    def usage(self):
        return sum(s["bytes"] for s in self.slots.values()), len(self.slots)

    def try_admit(self, pos, vel, box, n_steps, **params):
        need = len(pos) * self.BYTES_PER_ATOM
        if self.usage()[0] + need > self.budget or len(self.slots) >= self.max_slots:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = {"bytes": need, "left": int(n_steps), "n": len(pos), "done": 0}
        self.peak = max(self.peak, self.usage()[0])
        return slot

    def run(self):
        assert self.slots
        for s in self.slots.values():
            k = min(self.spr, s["left"])
            s["left"] -= k
            s["done"] += k
        self.clock.t += self.run_s

    def poll(self):
        return [k for k, s in self.slots.items() if s["left"] == 0]

    def props(self, slot):
        return {"step": self.slots[slot]["done"]}

    def get_state(self, slot):
        n = self.slots[slot]["n"]
        return np.zeros((n, 3)), np.zeros((n, 3)), self.slots[slot]["done"]

    def release(self, slot):
        del self.slots[slot]

    def close(self):
        self.closed = True


class FakeTimer:
    """Run spans read from the simulated clock."""

    clock = None

    def __init__(self):
        self.spans = []

    def before(self):
        self.spans.append([self.clock.t, None])

    def after(self):
        self.spans[-1][1] = self.clock.t

    def runs(self):
        return len(self.spans)

    def total_s(self):
        return sum(b - a for a, b in self.spans)


@pytest.fixture
def fake(monkeypatch):
    clock = FakeClock()
    FakeBatch.instances.clear()

    def make(budget, max_slots, spr):
        return FakeBatch(budget, max_slots, spr, clock=clock)

    monkeypatch.setattr(server, "Batch", make)
    FakeTimer.clock = clock
    monkeypatch.setattr(server, "RunTimer", FakeTimer)
    # the loop sleeps until the next arrival when nothing is active: advance
    # the simulated clock instead
    monkeypatch.setattr(server.time, "sleep", lambda s: setattr(clock, "t", clock.t + s))
    return clock


def _requests(spec):
    return [I.Request(arrival=a, name=f"r{k}", n_cells=c, rho=0.8, temperature=1.0,
                      steps=st, seed=k) for k, (a, c, st) in enumerate(spec)]


def test_every_request_served_once_in_budget(fake):
    reqs = _requests([(0.0, 3, 130), (0.0, 4, 64), (0.001, 3, 200), (0.05, 4, 64),
                      (0.05, 3, 10), (0.2, 4, 300)])
    budget = 4 * 4 ** 3 * 400 + 4 * 3 ** 3 * 400     # one 256-atom and one 108-atom system
    out = server.serve(reqs, budget, max_slots=8, steps_per_run=64, clock=fake)
    b = FakeBatch.instances[-1]
    assert b.closed and not b.slots
    assert out["n_requests"] == len(reqs)
    assert sorted(r.name for r in out["served"]) == sorted(r.name for r in reqs)
    assert b.peak <= budget and out["peak_bytes"] <= budget
    for r in out["served"]:
        req = next(q for q in reqs if q.name == r.name)
        assert r.props["step"] == req.steps                       # every step run
        assert r.arrival <= r.admitted <= r.done and r.latency >= r.queueing >= 0.0
    # arrival-order admission: no request is admitted before an earlier one
    adm = sorted(out["served"], key=lambda r: r.admitted)
    arr = [r.arrival for r in adm]
    assert arr == sorted(arr)
    work = sum(q.n * q.steps for q in reqs)
    assert out["atom_steps"] == work
    assert out["atom_steps_per_s"] == pytest.approx(work / out["makespan_s"])
    # every run takes run_s of the simulated clock: busy time is runs x run_s
    assert out["gpu_busy_s"] == pytest.approx(out["runs"] * b.run_s)
    assert out["gpu_busy_fraction"] == pytest.approx(out["gpu_busy_s"] / out["makespan_s"])
    assert 0.0 < out["gpu_busy_fraction"] <= 1.0 + 1e-12
    lat = np.array([r.latency for r in out["served"]])
    assert out["p50_latency_s"] == pytest.approx(np.percentile(lat, 50))
    assert out["p99_latency_s"] == pytest.approx(np.percentile(lat, 99))


def test_slot_limit_and_head_of_line_order(fake):
    # three slots, six equal requests at t = 0: admitted three at a time
    reqs = _requests([(0.0, 3, 64)] * 6)
    out = server.serve(reqs, 1 << 40, max_slots=3, steps_per_run=64, clock=fake)
    adm = sorted(r.admitted for r in out["served"])
    assert adm[:3] == [0.0, 0.0, 0.0] and min(adm[3:]) > 0.0
    assert {r.slot for r in out["served"]} == {0, 1, 2}      # freed slots reused


def test_idle_gap_waits_for_the_next_arrival(fake):
    reqs = _requests([(0.0, 3, 64), (5.0, 3, 64)])
    out = server.serve(reqs, 1 << 40, max_slots=4, steps_per_run=64, clock=fake)
    late = next(r for r in out["served"] if r.name == "r1")
    assert late.admitted >= 5.0 and late.queueing == pytest.approx(late.admitted - 5.0)


def test_request_larger_than_the_budget_is_an_error(fake):
    reqs = _requests([(0.0, 5, 64)])
    with pytest.raises(RuntimeError, match="does not fit an empty batch"):
        server.serve(reqs, 1000, max_slots=4, steps_per_run=64, clock=fake)
    assert FakeBatch.instances[-1].closed
