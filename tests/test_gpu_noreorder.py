"""MD_NO_REORDER (the ablation of Table 8) against the oracle.

Without reordering the atoms keep the caller's storage order for good: a
rebuild still bins them and finds the cell order (cell_start and a
permutation), wraps the positions in place and builds the neighbour list
through the permutation.  The method's results are unchanged, so the bars
are the usual ones: cells, cell order and pair sets bit for bit (the cell
order is the stable one, by storage index, which is the caller's order
here); forces, energies and trajectories at the tolerances of the
reordering method (FP64: summation order only).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

RC = 2.0 ** (1.0 / 6.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _system(*args, **kw):
    from paper_0911_5631_amd.md import System
    return System(*args, **kw)


def force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


def min_image(d, L):
    return d - L * np.round(d / L)


def _fluid(nc, seed, amp=0.12):
    pos, L = I.fcc_lattice(nc, 0.8)
    pos = I.jitter(pos, L, amp, seed)
    vel = I.random_velocities(len(pos), 1.0, seed + 1)
    pos, vel = I.shuffled(pos, vel, seed + 2)
    pos[::31, 1] += L                     # wrapped in place at creation
    return pos, vel, L


@pytest.mark.parametrize("nc,shell", [(13, 0.4), (9, 0.8)])
def test_no_reorder_bins_pairs_forces(nc, shell):
    pos, vel, L = _fluid(nc, 3 + nc)
    n = len(pos)
    rn = RC + shell
    s = _system(pos, vel, L, shell=shell, reorder=False)
    G = O.cells_per_edge(L, rn)
    wrapped = O.wrap(pos, L)
    p, _, f, _ = s.get_state()
    assert np.array_equal(p, wrapped)
    cells = O.cell_ids(wrapped, L, G)
    assert np.array_equal(s.cells(), cells)
    _, order, cs, _ = O.layers_reorder(cells, G)
    got_order, got_cs = s.bins()
    assert np.array_equal(got_cs, cs) and np.array_equal(got_order, order)
    rpi, rpj, rimg = O.pairs_cells(wrapped, L, G, rn)
    pi, pj = s.pairs()
    assert len(pi) == 2 * len(rpi)
    assert np.array_equal(O.pair_set(pi, pj), O.pair_set(rpi, rpj))
    ref = O.forces_pairs(wrapped, L, rpi, rpj, rimg)
    assert force_error(f, ref.force) <= 1e-5
    pr = s.props()
    assert abs(pr["pe"] - ref.pe) / n <= 1e-6 * max(abs(ref.pe) / n, 1.0)
    assert abs(pr["virial"] - ref.virial) / n <= 1e-6 * max(abs(ref.virial) / n, 1.0)
    s.close()


def test_no_reorder_sort_in_a_step_and_trajectory():
    """FP64 from an fcc start stored in a shuffled order: after the first
    rebuild inside md_step the cell order is the stable sort of the caller's
    order by the oracle's cells there; the trajectory follows the oracle's to
    summation order over 200 steps with several rebuilds."""
    pos, L = I.fcc_lattice(10, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 21)
    pos, vel = I.shuffled(pos, vel, 22)
    n = len(pos)
    G = O.cells_per_edge(L, RC + 0.4)
    sim = O.Sim(pos, vel, L, shell=0.4)
    k1 = 0
    while True:
        k1 += 1
        if sim.run(1)[0, 5]:
            break
        assert k1 < 200
    r1, _, _, _ = sim.state()
    s = _system(pos, vel, L, shell=0.4, precision="fp64", reorder=False)
    s.step(k1)
    assert s.props()["n_rebuilds"] == 1
    _, order, cs, _ = O.layers_reorder(O.cell_ids(r1, L, G), G)
    got_order, got_cs = s.bins()
    assert np.array_equal(got_cs, cs) and np.array_equal(got_order, order)
    s.step(200 - k1)
    tr = sim.run(200 - k1)
    p, v, f, step = s.get_state()
    rp, rv, rf, _ = sim.state()
    pr = s.props()
    sim.close()
    s.close()
    assert step == 200 and pr["n_rebuilds"] == 1 + int(tr[:, 5].sum()) >= 3
    assert np.abs(min_image(p - rp, L)).max() < 1e-9
    assert np.abs(v - rv).max() < 1e-8
    assert force_error(f, rf) < 1e-9
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10


def test_no_reorder_fp32_trajectory_and_batch():
    from paper_0911_5631_amd.md import Batch
    pos, vel, L = _fluid(9, 31, amp=0.05)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4, reorder=False)
    sim = O.Sim(pos, vel, L, shell=0.4)
    s.step(60)
    tr = sim.run(60)
    p, v, _, _ = s.get_state()
    rp, _, _, _ = sim.state()
    pr = s.props()
    sim.close()
    s.close()
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) >= 1
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-5
    # the same system as one replica of a batch beside a reordering one
    other = I.fcc_system("other", 6, 0.8, 1.0, seed=5)
    b = Batch(1 << 30, 2, 32)
    b.admit(other.pos, other.vel, other.box, 60, shell=0.4)
    slot = b.admit(pos, vel, L, 60, shell=0.4, reorder=False)
    for _ in range(10):
        b.run()
        if slot in b.poll():
            break
    bp, bv, bstep = b.get_state(slot)
    b.close()
    assert bstep == 60 and np.array_equal(bp, p) and np.array_equal(bv, v)


# ---------------------------------------------------------------------------
# the reorder interval N_R (Table 7): a rebuild reorders only when N_R steps
# have passed since the last reordering, and otherwise works like one under
# MD_NO_REORDER
# ---------------------------------------------------------------------------

def _first_rebuilds(pos, vel, L, shell, steps):
    sim = O.Sim(pos, vel, L, shell=shell)
    tr = sim.run(steps)
    sim.close()
    return [k + 1 for k in range(steps) if tr[k, 5]]


def test_reorder_interval_bins_at_a_rebuild_that_keeps_the_order():
    """N_R = 10^4: the creation sort reorders, the first rebuild in a step does
    not: its cell order is the stable sort by cell of the storage order left
    by the creation sort."""
    pos, L = I.fcc_lattice(10, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 41)
    pos, vel = I.shuffled(pos, vel, 42)
    G = O.cells_per_edge(L, RC + 0.4)
    k1 = _first_rebuilds(pos, vel, L, 0.4, 200)[0]
    s = _system(pos, vel, L, shell=0.4, precision="fp64", reorder_interval=10000)
    storage0, _ = s.bins()                 # original ids in storage order after creation
    s.step(k1)
    assert s.props()["n_rebuilds"] == 1
    sim = O.Sim(pos, vel, L, shell=0.4)
    sim.run(k1)
    r1, _, _, _ = sim.state()
    sim.close()
    cells1 = O.cell_ids(r1, L, G)
    expect = storage0[np.argsort(cells1[storage0], kind="stable")]
    _, _, cs, _ = O.layers_reorder(cells1, G)
    got_order, got_cs = s.bins()
    assert np.array_equal(got_cs, cs) and np.array_equal(got_order, expect)
    # the pair set of that rebuild is the oracle's
    rpi, rpj, _ = O.pairs_cells(r1, L, G, RC + 0.4)
    pi, pj = s.pairs()
    assert np.array_equal(O.pair_set(pi, pj), O.pair_set(rpi, rpj))
    s.close()


@pytest.mark.parametrize("nr", [30, 75])
def test_reorder_interval_fp64_trajectory(nr):
    """FP64 over 300 steps with rebuilds that reorder and rebuilds that do
    not: the oracle's trajectory to summation order, its rebuild count, and
    the reordering rebuilds where N_R says."""
    pos, L = I.fcc_lattice(10, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 51)
    n = len(pos)
    rb = _first_rebuilds(pos, vel, L, 0.4, 300)
    assert len(rb) >= 6
    s = _system(pos, vel, L, shell=0.4, precision="fp64", reorder_interval=nr)
    sim = O.Sim(pos, vel, L, shell=0.4)
    done = 0
    for k in rb:                      # calls that end at every rebuild step
        s.step(k - done)
        done = k
    s.step(300 - done)
    tr = sim.run(300)
    p, v, f, step = s.get_state()
    rp, rv, rf, _ = sim.state()
    pr = s.props()
    sim.close()
    s.close()
    assert step == 300 and pr["n_rebuilds"] == len(rb)
    assert np.abs(min_image(p - rp, L)).max() < 1e-9
    assert np.abs(v - rv).max() < 1e-8
    assert force_error(f, rf) < 1e-9
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10


def test_reorder_interval_fp32_batch_equals_solo_and_oracle():
    from paper_0911_5631_amd.md import Batch
    pos, vel, L = _fluid(9, 61, amp=0.05)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4, reorder_interval=40)
    s.step(150)
    p, v, _, _ = s.get_state()
    pr = s.props()
    s.close()
    sim = O.Sim(pos, vel, L, shell=0.4)
    tr = sim.run(150)
    rp, _, _, _ = sim.state()
    sim.close()
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) >= 3
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-5
    other = I.fcc_system("other", 6, 0.8, 1.0, seed=7)
    b = Batch(1 << 30, 2, 32)
    b.admit(other.pos, other.vel, other.box, 150, shell=0.4)
    slot = b.admit(pos, vel, L, 150, shell=0.4, reorder_interval=40)
    for _ in range(20):
        b.run()
        if slot in b.poll():
            break
    bp, bv, bstep = b.get_state(slot)
    b.close()
    assert bstep == 150 and np.array_equal(bp, p) and np.array_equal(bv, v)


def test_reorder_interval_refused_where_it_does_not_apply():
    from paper_0911_5631_amd._lib import MDError
    pos, vel, L = _fluid(7, 71)
    with pytest.raises(MDError) as e:
        _system(pos, vel, L, shell=0.4, reorder_interval=-1)
    assert e.value.code == -1
    s = _system(pos, vel, L, shell=0.4, reorder_interval=20)
    with pytest.raises(MDError) as e:
        s.newton3_ab()
    assert e.value.code == -8
    s.close()


# ---------------------------------------------------------------------------
# MD_NO_WINDOW: the LDS window switched off (the analogue of the paper's
# texture-cache experiment); the same candidates in the same order, so the
# same lists and sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nc,precision", [(12, "fp32"), (7, "fp32"), (10, "fp64")])
def test_no_window_is_bit_identical(nc, precision):
    pos, vel, L = _fluid(nc, 81 + nc)
    runs = []
    for window in (True, False):
        s = _system(pos, vel, L, shell=0.4, precision=precision, window=window)
        s.step(250)
        p, v, f, step = s.get_state()
        pi, pj = s.pairs()
        pr = s.props()
        s.close()
        runs.append((p, v, f, O.pair_set(pi, pj), pr))
    (p0, v0, f0, ps0, pr0), (p1, v1, f1, ps1, pr1) = runs
    assert pr0["n_rebuilds"] == pr1["n_rebuilds"] >= 3
    assert np.array_equal(p0, p1) and np.array_equal(v0, v1) and np.array_equal(f0, f1)
    assert np.array_equal(ps0, ps1)
    assert pr0["pe"] == pr1["pe"] and pr0["virial"] == pr1["virial"]
