"""Host logic of the launch-configuration autotuner (tune.py) on the CPU,
against a stand-in batch with a simulated clock: systems of given sizes and
targets advance spr steps per run, each run costs a configuration-dependent
time per atom-step plus a fixed per-run cost.  Checked: the score is the
atom-steps actually advanced per second (a system that has finished no longer
counts); trials that would finish a system are not started; a trial during
which the mix changed is discarded; the batch is left configured with the
best; the cache is written and applied.  The device path is covered by the
GPU tests."""
import pytest

from paper_0911_5631_amd import tune


class Clock:
    t = 0.0

    def __call__(self):
        return self.t


class SimBatch:
    """n[i] atoms, target[i] steps; one run advances every running system
    by spr steps (capped at its target)."""

    def __init__(self, clock, sizes, targets, ns_per_atom_step, per_run=40e-6):
        self.clock, self.cost, self.per_run = clock, ns_per_atom_step, per_run
        self.n, self.target = list(sizes), list(targets)
        self.done = [0] * len(sizes)
        self.config = None
        self.log = []
        self.admit_at = None     # (run index, size, target): admit a system then

    def configure(self, steps_per_run=0, grid=0, sort_grid=0, sort_split=0, tile_order=0):
        self.config = (steps_per_run or 64, grid, sort_grid, sort_split, tile_order)
        self.log.append(("configure",) + self.config)
        return dict(zip(tune.KNOBS, self.config))

    def run(self):
        spr = self.config[0]
        work = 0
        for i, n in enumerate(self.n):
            k = min(spr, self.target[i] - self.done[i])
            self.done[i] += k
            work += n * k
        self.clock.t += self.per_run + work * self.cost(*self.config) * 1e-9
        self.log.append(("run",) + self.config)
        runs = sum(1 for e in self.log if e[0] == "run")
        if self.admit_at and runs == self.admit_at[0]:
            self.n.append(self.admit_at[1])
            self.target.append(self.admit_at[2])
            self.done.append(0)

    def poll(self):
        return [i for i in range(len(self.n)) if self.done[i] >= self.target[i]]

    def progress(self):
        running = [i for i in range(len(self.n)) if self.done[i] < self.target[i]]
        left = min((self.target[i] - self.done[i] for i in running), default=0)
        work = sum(n * d for n, d in zip(self.n, self.done))
        return work, len(running), left


def grid_cost(spr, grid, sort_grid, split, order=0):
    # ns per atom-step: grid 1024 and sort grid 4096 are the best
    return 0.12 + {1024: 0.0, 2048: 0.01, 4096: 0.03}[grid] + \
        {1024: 0.02, 2048: 0.01, 4096: 0.0}[sort_grid] + 0.005 * (split - 1)


def test_best_by_atom_steps_per_second(monkeypatch):
    clock = Clock()
    b = SimBatch(clock, [4000, 32000, 864], [100000] * 3, grid_cost)
    out = tune.autotune(b, runs=3, clock=clock)
    best = out["best"]
    assert (best["grid"], best["sort_grid"]) in {(1024, 2048), (2048, 4096)}
    assert b.config == tuple(best[k] for k in tune.KNOBS)
    for tr in out["trials"]:
        spr, g, sg, sp, order = (tr[k] for k in tune.KNOBS)
        per_run = 36864 * spr * grid_cost(spr, g, sg, sp, order) * 1e-9 + 40e-6
        assert tr["atom_steps_per_s"] == pytest.approx(36864 * spr / per_run, rel=1e-9)
    # each candidate: configure, one untimed run, then the timed runs
    for c in tune.DEFAULT_CANDIDATES:
        cfg = tuple(tune._cfg(c)[k] for k in tune.KNOBS)
        k = b.log.index(("configure",) + cfg)
        assert b.log[k + 1:k + 5] == [("run",) + cfg] * 4


def test_no_trial_may_finish_a_system():
    clock = Clock()
    # the smallest target (500 steps) allows trials of 3 x 16 .. 3 x 64 steps
    # only while the total stays below it
    b = SimBatch(clock, [4000, 8000], [500, 100000], grid_cost)
    out = tune.autotune(b, runs=2, clock=clock)
    assert all(d < t for d, t in zip(b.done, b.target))
    skipped = [t for t in out["trials"] if "skipped" in t]
    assert skipped and all("finish" in t["skipped"] for t in skipped)
    assert out["best"] is not None


def test_trial_during_which_the_mix_changed_is_discarded():
    clock = Clock()
    b = SimBatch(clock, [4000, 8000], [100000, 100000], grid_cost)
    b.admit_at = (3, 50000, 100000)    # admitted during the first candidate's timed runs
    out = tune.autotune(b, runs=2, clock=clock)
    assert "skipped" in out["trials"][0] and "changed" in out["trials"][0]["skipped"]
    assert all("atom_steps_per_s" in t for t in out["trials"][1:])


def test_cache_roundtrip(tmp_path):
    clock = Clock()
    path = str(tmp_path / "tune.json")
    b = SimBatch(clock, [4000, 32000], [100000] * 2, grid_cost)
    key = tune.cache_key("gfx950:sramecc+:xnack-", "batch", 36000)
    assert key == "gfx950/batch/15"
    out = tune.autotune(b, runs=2, clock=clock, cache_path=path, key=key)
    b2 = SimBatch(clock, [4000, 32000], [100000] * 2, grid_cost)
    used = tune.apply_cached(b2, path, key)
    assert used == {k: out["best"][k] for k in tune.KNOBS}
    assert tune.apply_cached(b2, path, "gfx950/batch/3") is None


def test_warm_runs_come_first_and_are_not_timed():
    clock = Clock()
    b = SimBatch(clock, [4000, 8000], [100000, 100000], grid_cost)
    b.configure(64, 2048, 2048, 1, 1)
    out = tune.autotune(b, runs=2, warm_runs=3, clock=clock)
    runs = [e for e in b.log if e[0] == "run"]
    assert runs[:3] == [("run", 64, 2048, 2048, 1, 1)] * 3     # at the batch's own config
    first = tune._cfg(tune.DEFAULT_CANDIDATES[0])
    assert b.log.index(("configure",) + tuple(first[k] for k in tune.KNOBS)) > 3
    assert all("atom_steps_per_s" in t for t in out["trials"])


def test_trial_steps_equalise_the_timed_window():
    clock = Clock()
    b = SimBatch(clock, [4000, 8000], [100000, 100000], grid_cost)
    out = tune.autotune(b, runs=2, trial_steps=192, clock=clock)
    for tr in out["trials"]:
        assert tr["steps"] == max(2 * tr["steps_per_run"], 192)
    # spr 16: one capture run and twelve timed runs
    first = tune._cfg(tune.DEFAULT_CANDIDATES[0])
    cfg = tuple(first[k] for k in tune.KNOBS)
    k = b.log.index(("configure",) + cfg)
    assert b.log[k + 1:k + 14] == [("run",) + cfg] * 13 and b.log[k + 14][0] == "configure"
