"""Newton's-third-law A/B of the force phase (md_newton3_ab): the full list
(Sec. 3.3, no reaction forces) and the half list with atomic reactions (the
CPU form of Sec. 3.2) against the oracle and against each other.

Bar: list sizes exact (full = 2 x half = 2 x the oracle's pair count);
forces of both forms within the FP32 force bar of the other parity tests,
max_i |dF_i| / max(|F_i|, F_rms) <= 1e-5 (the half form's atomic sums come
in no fixed order, so it is held to the bar, not to bits); the full form
within 1e-6 of the step kernel's own forces at the same state.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

RC = 2.0 ** (1.0 / 6.0)
FORCE_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


@pytest.mark.parametrize("kind", ["sp", "lj"])
def test_full_and_half_forces_match_oracle(kind):
    from paper_0911_5631_amd.md import System
    if kind == "sp":
        pos, L = I.fcc_lattice(11, 0.8)           # 5 324 atoms: 20 tiles and a ragged tail
        pos = I.jitter(pos, L, 0.15, seed=91)
        vel = I.random_velocities(len(pos), 1.0, 92)
        rc, shell, ushift = RC, 0.4, 1.0
    else:
        pos, L = I.sc_lattice(17, 0.38)
        pos = I.jitter(pos, L, 0.2, seed=93)
        vel = I.random_velocities(len(pos), 1.2, 94)
        rc, shell, ushift = 2.5, 0.8, 0.0
    pos, vel = I.shuffled(pos, vel, 95)
    s = System(pos, vel, L, r_cut=rc, shell=shell)
    _, _, f_step, _ = s.get_state()
    full = s.newton3_ab(False, reps=2)
    half = s.newton3_ab(True, reps=2)
    n_pairs = s.props()["n_pairs"]
    s.close()
    wrapped = O.wrap(pos, L)
    ref = O.forces_cells(wrapped, L, O.cells_per_edge(L, rc), rc=rc, ushift=ushift)
    pi, _, _ = O.pairs_cells(wrapped, L, O.cells_per_edge(L, rc + shell), rc + shell)
    assert half["n_entries"] == len(pi) == n_pairs
    assert full["n_entries"] == 2 * len(pi)
    assert force_error(full["force"], ref.force) <= FORCE_TOL
    assert force_error(half["force"], ref.force) <= FORCE_TOL
    assert force_error(full["force"], f_step) <= 1e-6
    assert full["build_ms"] > 0 and full["force_ms"] > 0 and half["force_ms"] > 0


def test_ab_after_steps_and_state_kept():
    from paper_0911_5631_amd.md import System
    pos, L = I.fcc_lattice(8, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 96)
    s = System(pos, vel, L, shell=0.4)
    s.step(60)
    p0, v0, _, k0 = s.get_state()
    half = s.newton3_ab(True, reps=3)
    p1, v1, f1, k1 = s.get_state()
    # the A/B sorts the held state (as md_bin_cells) and changes nothing else
    assert k0 == k1 == 60
    assert np.array_equal(v0, v1)
    assert np.abs(p0 - p1 - L * np.round((p0 - p1) / L)).max() == 0.0
    assert force_error(half["force"], f1) <= FORCE_TOL
    s.step(10)
    assert s.props()["step"] == 70
    s.close()


@pytest.mark.parametrize("kind", ["sp", "lj3", "lj22"])
def test_cell_centric_build_matches_oracle_and_atom_centric(kind):
    """The cell-centric build (one workgroup per cell, one thread per
    occupant; Table 3's "old" organisation): its pair set bit for bit
    against the oracle's, its list equal to the atom-centric full list entry
    for entry (same order, so the forces are bit-identical), the half list's
    pairs the same set once each."""
    from paper_0911_5631_amd.md import System
    if kind == "sp":
        pos, L = I.fcc_lattice(12, 0.8)            # 6 912 atoms, ~3 per cell
        pos = I.jitter(pos, L, 0.15, seed=101)
        vel = I.random_velocities(len(pos), 1.0, 102)
        rc, shell = RC, 0.4
    else:
        rc = 3.0 if kind == "lj3" else 2.2        # up to ~45 occupants per cell
        pos, L = I.sc_lattice(18, 0.38)
        pos = I.jitter(pos, L, 0.2, seed=103)
        vel = I.random_velocities(len(pos), 1.2, 104)
        shell = 0.8
    pos, vel = I.shuffled(pos, vel, 105)
    s = System(pos, vel, L, r_cut=rc, shell=shell)
    wrapped = O.wrap(pos, L)
    rpi, rpj, _ = O.pairs_cells(wrapped, L, O.cells_per_edge(L, rc + shell), rc + shell)
    ref = O.pair_set(rpi, rpj)
    ci, cj = s.ab_pairs("cells")
    fi, fj = s.ab_pairs("full")
    hi, hj = s.ab_pairs("half")
    assert np.array_equal(ci, fi) and np.array_equal(cj, fj)
    assert len(ci) == 2 * len(ref) and np.array_equal(O.pair_set(ci, cj), ref)
    assert len(hi) == len(ref) and np.array_equal(O.pair_set(hi, hj), ref)
    cells = s.newton3_ab("cells", reps=2)
    full = s.newton3_ab("full", reps=2)
    s.close()
    assert cells["n_entries"] == full["n_entries"] == 2 * len(ref)
    assert np.array_equal(cells["force"], full["force"])
    assert cells["build_ms"] > 0
