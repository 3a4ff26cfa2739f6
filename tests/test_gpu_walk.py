"""Tiles taken on demand by the step kernel.

A step launch with more tiles than workgroups hands out its tiles through
per-XCD claim counters instead of a fixed walk; which workgroup steps which
tile must change nothing.  Bar: bit-identical positions, velocities and
properties against the same system stepped with a grid at least as large as
its tile count (every workgroup at most one tile, the fixed walk), for both
tile orders, several grids, both precisions, over several calls (the
counters are reset by each launch for the next), and for a batch against
its systems run alone.
"""
import numpy as np
import pytest

from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

PASSES, SLABS = 1, 2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _fluid(nc, seed, rho=0.8):
    pos, L = I.fcc_lattice(nc, rho)
    pos = I.jitter(pos, L, 0.05, seed)
    vel = I.random_velocities(len(pos), 1.0, seed + 1)
    return pos, vel, L


def _run(pos, vel, L, precision, calls, shell=0.4, **cfg):
    from paper_0911_5631_amd.md import System
    s = System(pos, vel, L, shell=shell, precision=precision)
    used = s.configure(**cfg) if cfg else None
    for n in calls:
        s.step(n)
    p, v, _, step = s.get_state()
    pr = s.props()
    s.close()
    return p, v, step, pr, used


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_claimed_tiles_match_the_fixed_walk(precision):
    pos, vel, L = _fluid(13, 71)          # 8 788 atoms: 35 tiles
    nt = -(-len(pos) // 256)
    calls = (37, 64, 99)
    ref = _run(pos, vel, L, precision, calls, grid=64, tile_order=SLABS)
    assert ref[4]["grid"] >= nt          # the fixed walk
    for grid in (8, 12, 16, 24):         # 12: not a multiple of 8, a plain strided walk
        for order in (PASSES, SLABS):
            p, v, step, pr, used = _run(pos, vel, L, precision, calls, grid=grid,
                                        tile_order=order)
            assert used["grid"] == grid < nt
            assert step == ref[2] == sum(calls)
            assert np.array_equal(p, ref[0]) and np.array_equal(v, ref[1]), (grid, order)
            for key in ("ke", "pe", "virial", "n_rebuilds"):
                assert pr[key] == ref[3][key], (grid, order, key)


def test_claimed_tiles_in_a_batch_match_solo_runs():
    from paper_0911_5631_amd.md import Batch
    systems = I.replica_batch(n_replicas=5, k_lo=6, k_hi=11, steps=260, seed=77)
    for order in (PASSES, SLABS):
        b = Batch(1 << 31, 8, 32)
        slot_of = {b.admit(s.pos, s.vel, s.box, s.steps, shell=s.shell): k
                   for k, s in enumerate(systems)}
        b.configure(steps_per_run=32, grid=16, tile_order=order)
        out = {}
        for _ in range(40):
            if len(out) == len(systems):
                break
            b.run()
            for slot in b.poll():
                if slot_of[slot] not in out:
                    out[slot_of[slot]] = b.get_state(slot)
                    b.release(slot)
        b.close()
        assert len(out) == len(systems)
        for k, s in enumerate(systems):
            p, v, step, _, _ = _run(s.pos, s.vel, s.box, "fp32", (s.steps,), shell=s.shell)
            gp, gv, gstep = out[k]
            assert gstep == step == s.steps
            assert np.array_equal(gp, p) and np.array_equal(gv, v), (order, k)


def test_claimed_tiles_after_a_replay_cut_short():
    """A step whose rule fires without binned rows (a late binning) stops the
    rest of its replay: every workgroup skips those steps at once, which must
    still leave the claim counters reset for the launches after the host has
    binned the positions and resumed.  A lattice nearly at rest with one
    pair pushed to r = 0.9 and a shell of 0.004 (the maximum speed jumps
    from ~0.01 to ~0.7 in one step): same late binnings and bit-identical
    state as the fixed walk, for both tile orders."""
    pos, L = I.sc_lattice(16, 0.5)       # 4 096 atoms: 16 tiles
    rng = np.random.Generator(np.random.PCG64(61))
    vel = rng.uniform(-0.005, 0.005, pos.shape)
    vel -= vel.mean(0)
    d = pos[1] - pos[0]
    d -= L * np.round(d / L)
    pos[0] = pos[1] - d / np.linalg.norm(d) * 0.9
    nt = -(-len(pos) // 256)
    calls = (40, 24)
    ref = _run(pos, vel, L, "fp32", calls, shell=0.004, grid=64, tile_order=SLABS)
    assert ref[4]["grid"] >= nt and ref[3]["n_late_bins"] >= 1
    for order in (PASSES, SLABS):
        p, v, step, pr, used = _run(pos, vel, L, "fp32", calls, shell=0.004, grid=8,
                                    tile_order=order)
        assert used["grid"] == 8 < nt
        assert step == ref[2] == sum(calls)
        assert pr["n_late_bins"] == ref[3]["n_late_bins"]
        assert np.array_equal(p, ref[0]) and np.array_equal(v, ref[1]), order
