"""Lennard-Jones with the longer cutoffs of the paper's LJ runs (r_c = 2.2,
2.5, 3.0; rho 0.38, T 1.2, delta 0.8: Sec. 5.1, Tables 1 and 3): the same
kernels without the soft-sphere shift, against the FP64 oracle.

Bars as for the soft spheres: pair sets bit-exact; FP32 forces
max_i |dF_i| / max(|F_i|, F_rms) <= 1e-5; PE and virial per atom 1e-6;
FP64 trajectories to 1e-9.  Then the equilibrated LJ fluid of Table 1's
size against the neighbour and layer counts the paper quotes for it.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-5
ENERGY_TOL = 1e-6
SHELL = 0.8


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


def lj_fluid(n_edge, seed, amp=0.2):
    pos, L = I.sc_lattice(n_edge, 0.38)
    pos = I.jitter(pos, L, amp, seed)
    vel = I.random_velocities(len(pos), 1.2, seed + 1000)
    return (*I.shuffled(pos, vel, seed + 2000), L)


def force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


def min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("rc,n_edge,seed", [(2.2, 14, 1), (2.5, 15, 2), (3.0, 17, 3)])
def test_lj_pairs_bit_exact(rc, n_edge, seed):
    pos, vel, L = lj_fluid(n_edge, seed)
    s = _system(pos, vel, L, r_cut=rc, shell=SHELL)
    pi, pj = s.pairs()      # raises if a list outgrew the default capacity
    wrapped = O.wrap(pos, L)
    rn = rc + SHELL
    ref = O.pair_set(*O.pairs_cells(wrapped, L, O.cells_per_edge(L, rn), rn)[:2])
    assert len(pi) == 2 * len(ref) and np.all(pi != pj)
    assert np.array_equal(O.pair_set(pi, pj), ref)
    pr = s.props()
    assert pr["n_pairs"] == len(ref)
    s.close()


@pytest.mark.parametrize("rc,n_edge,seed", [(3.0, 17, 11), (2.2, 20, 12)])
def test_lj_bins_bit_exact(rc, n_edge, seed):
    """Cells of 10-40 atoms: the sort ranks them cooperatively, and a cell
    tile is shared by several workgroups; the storage order must still be the
    stable counting sort (Sec. 3.4 layers read in cell order, Sec. 3.5)."""
    pos, vel, L = lj_fluid(n_edge, seed)
    s = _system(pos, vel, L, r_cut=rc, shell=SHELL)
    G = O.cells_per_edge(L, rc + SHELL)
    ref_cell = O.cell_ids(O.wrap(pos, L), L, G)
    assert np.array_equal(s.cells(), ref_cell)
    _, order, cs, _ = O.layers_reorder(ref_cell, G)
    got_order, got_cs = s.bins()
    assert np.array_equal(got_cs, cs) and np.array_equal(got_order, order)
    assert np.diff(cs).max() > 8                 # cells beyond the sorting network
    # after some steps (sorts inside the run), a stand-alone sort of the moved
    # atoms ranks each cell's members by their storage position, i.e. by the
    # order the last sort left
    s.step(40)
    before, _ = s.bins()
    s.bin_cells()
    after, cs2 = s.bins()
    p, _, _, _ = s.get_state()
    s.close()
    cell_now = O.cell_ids(O.wrap(p, L), L, G)
    want = before[np.argsort(cell_now[before], kind="stable")]
    assert np.array_equal(after, want)
    assert np.array_equal(cs2, np.concatenate([[0], np.cumsum(np.bincount(cell_now,
                                                                           minlength=G ** 3))]))


@pytest.mark.parametrize("rc,n_edge,seed", [(2.2, 14, 4), (2.5, 16, 5), (3.0, 18, 6)])
def test_lj_forces_fp32_within_tolerance(rc, n_edge, seed):
    pos, vel, L = lj_fluid(n_edge, seed)
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc, shell=SHELL, precision="fp32")
    _, _, f, _ = s.get_state()
    u, w = s.atom_energies()
    wrapped = O.wrap(pos, L)
    ref = O.forces_cells(wrapped, L, O.cells_per_edge(L, rc), rc=rc, ushift=0.0)
    assert force_error(f, ref.force) <= FORCE_TOL
    pr = s.props()
    assert abs(pr["pe"] - ref.pe) / n <= ENERGY_TOL * max(abs(ref.pe) / n, 1.0)
    assert abs(pr["virial"] - ref.virial) / n <= ENERGY_TOL * max(abs(ref.virial) / n, 1.0)
    assert np.abs(u - ref.u_atom).max() <= 1e-5 * max(np.abs(ref.u_atom).max(), 1.0)
    assert np.abs(w - ref.w_atom).max() <= 1e-5 * max(np.abs(ref.w_atom).max(), 1.0)
    s.close()


@pytest.mark.parametrize("rc", [2.2, 3.0])
def test_lj_fp64_trajectory_matches_oracle(rc):
    pos, vel, L = lj_fluid(15, 7, amp=0.1)
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc, shell=SHELL, precision="fp64")
    ref = O.Sim(pos, vel, L, shell=SHELL, rc=rc, ushift=0.0)
    s.step(150)
    tr = ref.run(150)
    p, v, _, step = s.get_state()
    rp, rv, _, _ = ref.state()
    assert step == 150
    assert np.abs(min_image(p - rp, L)).max() < 1e-9
    assert np.abs(v - rv).max() < 1e-8
    pr = s.props()
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10
    assert abs(pr["ke"] - tr[-1, 0]) / n < 1e-10
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) and pr["n_rebuilds"] > 2
    s.close()


def test_lj_fp32_trajectory_matches_oracle():
    pos, vel, L = lj_fluid(16, 8, amp=0.1)
    n = len(pos)
    s = _system(pos, vel, L, r_cut=2.5, shell=SHELL, precision="fp32")
    ref = O.Sim(pos, vel, L, shell=SHELL, rc=2.5, ushift=0.0)
    s.step(30)
    tr = ref.run(30)
    p, v, f, _ = s.get_state()
    rp, rv, rf, _ = ref.state()
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    assert force_error(f, rf) < 1e-4
    pr = s.props()
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-5
    assert abs(pr["ke"] - tr[-1, 0]) / n < 1e-5
    s.close()


def test_lj_table1_system_counts():
    """LJ r_c = 3.0 at Table 1's N_e = 48 (110 592 atoms): N_c = 4096 exactly;
    after the Sec. 5.1 equilibration the neighbour-list entries per atom,
    quoted as typically 89 for the LJ runs, are 87.6 in the FP64 oracle at
    N_e = 16 and 24 (the tolerance, 2.5 %, covers that and the rounding of
    the quote); the layer count N_l (largest cell occupancy at a sort) is
    quoted as 40-50; N_u as 14-15 steps for the largest systems (the oracle
    gives 16.7 at N_e = 24; the maximum speed, and with it the rebuild rate,
    grows with N), held to 13-17."""
    pos, L = I.sc_lattice(48, 0.38)
    vel = I.random_velocities(len(pos), 1.2, 81)
    s = _system(pos, vel, L, r_cut=3.0, shell=SHELL, even_cells=True)
    s.equilibrate_run(1000, 1.2)
    s.block_begin()
    s.step(2000)
    blk = s.block_end()
    pr = s.props()
    _, cs = s.bins()
    s.close()
    assert pr["cells_per_edge"] ** 3 == 4096
    assert abs(blk["nebr_per_atom"] - 89.0) <= 0.025 * 89.0, blk
    n_l = int(np.diff(cs).max())
    assert 38 <= n_l <= 52, n_l
    n_u = 3000 / pr["n_rebuilds"]
    assert 13.0 <= n_u <= 17.0, n_u
    assert abs(blk["ke_per_atom"] - 1.5 * 1.2) < 0.05


def test_lj_batch_equals_solo_bit_for_bit():
    """A batch sorts each cell tile with one workgroup, a single dense system
    shares it among several: the storage order (ranks by index) and so every
    trajectory are the same either way."""
    from paper_0911_5631_amd.md import Batch, System
    specs = [lj_fluid(13, 21, amp=0.1), lj_fluid(15, 22, amp=0.1)]
    b = Batch(1 << 31, 4, 16)
    slots = [b.admit(p, v, L, 120, r_cut=2.5, shell=SHELL) for p, v, L in specs]
    out = {}
    for _ in range(50):
        if len(out) == len(specs):
            break
        b.run()
        for slot in b.poll():
            out[slot] = b.get_state(slot)
            b.release(slot)
    b.close()
    for slot, (p, v, L) in zip(slots, specs):
        s = System(p, v, L, r_cut=2.5, shell=SHELL)
        s.step(120)
        sp, sv, _, step = s.get_state()
        s.close()
        gp, gv, gstep = out[slot]
        assert gstep == step == 120
        assert np.array_equal(gp, sp) and np.array_equal(gv, sv)
