"""Several species on the GPU (md_set_species) against the oracle's mixture
model (per species pair epsilon, sigma, cutoff, shift; Eq. (1) in the pair's
units).

Bars: a one-species table (sigma = epsilon = 1) reproduces the plain
kernels bit for bit; pair sets bit-exact; FP32 forces max_i |dF_i| /
max(|F_i|, F_rms) <= 1e-5, PE and virial per atom 1e-6; FP64 trajectories
1e-9; the checkerboard lattice sum in closed form.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

RC = 2.0 ** (1.0 / 6.0)
FORCE_TOL = 1e-5
ENERGY_TOL = 1e-6


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


def wca_binary(sig_aa=1.0, sig_bb=1.2, eps_aa=1.0, eps_bb=1.0, eps_ab=1.5):
    sig = np.array([[sig_aa, 0.5 * (sig_aa + sig_bb)], [0.5 * (sig_aa + sig_bb), sig_bb]])
    eps = np.array([[eps_aa, eps_ab], [eps_ab, eps_bb]])
    return eps, sig, RC * sig, eps.copy()


def force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


def min_image(d, L):
    return d - L * np.round(d / L)


def binary_fluid(n_edge, seed, rho=0.75, frac_b=0.4, amp=0.2):
    pos, L = I.sc_lattice(n_edge, rho)
    pos = I.jitter(pos, L, amp, seed)
    vel = I.random_velocities(len(pos), 1.0, seed + 1000)
    pos, vel = I.shuffled(pos, vel, seed + 2000)
    sp = (np.random.Generator(np.random.PCG64(seed + 3000)).random(len(pos)) < frac_b)
    return pos, vel, L, sp.astype(np.int32)


def test_one_species_table_is_bit_identical_to_the_plain_kernels():
    pos, vel, L, _ = binary_fluid(14, 1, rho=0.8)
    a = _system(pos, vel, L, shell=0.4)
    b = _system(pos, vel, L, shell=0.4)
    a.bin_cells()                         # the same re-sort and evaluation as set_species
    b.set_species(np.zeros(len(pos), np.int32), [[1.0]], [[1.0]], [[RC]], [[1.0]])
    for s in (a, b):
        s.step(150)
    pa, va, fa, _ = a.get_state()
    pb, vb, fb, _ = b.get_state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb) and np.array_equal(fa, fb)
    assert a.props()["pe"] == b.props()["pe"] and a.props()["n_rebuilds"] > 5
    a.close()
    b.close()


@pytest.mark.parametrize("n_edge,seed", [(12, 2), (17, 3)])
def test_binary_forces_and_pairs_match_oracle(n_edge, seed):
    pos, vel, L, sp = binary_fluid(n_edge, seed)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4)
    s.set_species(sp, eps, sig, rc, sh)
    _, _, f, _ = s.get_state()
    pr = s.props()
    pi, pj = s.pairs()
    s.close()
    wrapped = O.wrap(pos, L)
    mix = O.Mixture(sp, eps, sig, rc, sh)
    ref = O.forces_cells(wrapped, L, O.cells_per_edge(L, mix.max_cut), mix=mix)
    assert force_error(f, ref.force) <= FORCE_TOL
    assert abs(pr["pe"] - ref.pe) / n <= ENERGY_TOL * max(abs(ref.pe) / n, 1.0)
    assert abs(pr["virial"] - ref.virial) / n <= ENERGY_TOL * max(abs(ref.virial) / n, 1.0)
    rn = mix.max_cut + 0.4
    want = O.pair_set(*O.pairs_cells(wrapped, L, O.cells_per_edge(L, rn), rn)[:2])
    assert np.array_equal(O.pair_set(pi, pj), want)


def test_binary_fp64_trajectory_matches_oracle():
    pos, vel, L, sp = binary_fluid(13, 4, amp=0.08)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4, precision="fp64")
    s.set_species(sp, eps, sig, rc, sh)
    ref = O.Sim(pos, vel, L, shell=0.4, rc=rc.max(), ushift=0.0)
    ref.set_species(O.Mixture(sp, eps, sig, rc, sh))
    s.step(150)
    tr = ref.run(150)
    p, v, _, step = s.get_state()
    rp, rv, _, _ = ref.state()
    assert step == 150
    assert np.abs(min_image(p - rp, L)).max() < 1e-9
    assert np.abs(v - rv).max() < 1e-8
    pr = s.props()
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) and pr["n_rebuilds"] > 3
    s.close()
    ref.close()


@pytest.mark.parametrize("reorder_interval,reorder", [(40, True), (0, False)])
def test_binary_fp64_trajectory_without_reordering(reorder_interval, reorder):
    """The reorder interval and MD_NO_REORDER with a mixture: species stay
    with their atoms through rebuilds that keep the storage order (their
    candidates read through the cell-order permutation), and the trajectory
    is the oracle's to summation order."""
    pos, vel, L, sp = binary_fluid(13, 6, amp=0.08)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4, precision="fp64",
                reorder_interval=reorder_interval, reorder=reorder)
    s.set_species(sp, eps, sig, rc, sh)
    ref = O.Sim(pos, vel, L, shell=0.4, rc=rc.max(), ushift=0.0)
    ref.set_species(O.Mixture(sp, eps, sig, rc, sh))
    s.step(150)
    tr = ref.run(150)
    p, v, _, step = s.get_state()
    rp, rv, _, _ = ref.state()
    pr = s.props()
    s.close()
    ref.close()
    assert step == 150
    assert np.abs(min_image(p - rp, L)).max() < 1e-9
    assert np.abs(v - rv).max() < 1e-8
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) and pr["n_rebuilds"] > 3


def test_binary_fp32_trajectory_matches_oracle():
    pos, vel, L, sp = binary_fluid(15, 5, amp=0.08)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4)
    s.set_species(sp, eps, sig, rc, sh)
    ref = O.Sim(pos, vel, L, shell=0.4, rc=rc.max(), ushift=0.0)
    ref.set_species(O.Mixture(sp, eps, sig, rc, sh))
    s.step(30)
    tr = ref.run(30)
    p, _, f, _ = s.get_state()
    rp, _, rf, _ = ref.state()
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    assert force_error(f, rf) < 1e-4
    assert abs(s.props()["pe"] - tr[-1, 1]) / n < 1e-5
    s.close()
    ref.close()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("fp64", 1e-12)])
def test_checkerboard_closed_form_on_gpu(precision, tol):
    ne, a = 8, 1.1
    pos, L = I.sc_lattice(ne, 1.0 / a ** 3)
    g = np.arange(ne)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    sp = ((ix + iy + iz).ravel() % 2).astype(np.int32)
    eps, sig, rc, sh = wca_binary(sig_aa=1.0, sig_bb=1.2, eps_ab=1.5)
    s = _system(pos, np.zeros_like(pos), L, r_cut=rc.max(), shell=0.4, precision=precision)
    s.set_species(sp, eps, sig, rc, sh)
    pr = s.props()
    _, _, f, _ = s.get_state()
    s.close()
    print(f"checkerboard {precision}: PE/N error {abs(pr['pe_per_atom'] - 4.5):.3e}, "
          f"W/N error {abs(pr['virial_per_atom'] - 108.0):.3e}", flush=True)
    assert abs(pr["pe_per_atom"] - 4.5) < tol * 4.5
    assert abs(pr["virial_per_atom"] - 108.0) < tol * 108.0
    assert np.abs(f).max() < 1e3 * tol


def test_species_follow_atoms_through_sorts_and_set_state():
    # a gentle start (B atoms of sigma 1.2 sit closer than that on the lattice)
    pos, vel, L, sp = binary_fluid(12, 6, amp=0.08)
    eps, sig, rc, sh = wca_binary()
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4)
    s.set_species(sp, eps, sig, rc, sh)
    s.step(80)                                     # several rebuilds: species are re-sorted
    p, v, f, _ = s.get_state()
    wrapped = O.wrap(p, L)
    mix = O.Mixture(sp, eps, sig, rc, sh)
    ref = O.forces_cells(wrapped, L, O.cells_per_edge(L, mix.max_cut), mix=mix)
    assert force_error(f, ref.force) <= FORCE_TOL
    s.set_state(pos, vel)                           # back to the start, original indices
    _, _, f0, _ = s.get_state()
    ref0 = O.forces_cells(O.wrap(pos, L), L, O.cells_per_edge(L, mix.max_cut), mix=mix)
    assert force_error(f0, ref0.force) <= FORCE_TOL
    from paper_0911_5631_amd._lib import MDError
    with pytest.raises(MDError):
        s.set_species(sp, eps, sig, rc * 1.5, sh)  # beyond the system's cutoff
    s.close()


def test_mixture_block_means_match_oracle():
    """Block averages of a mixture (the accumulating mixture kernel) against
    the oracle's trace over the same steps, FP64."""
    pos, vel, L, sp = binary_fluid(11, 7, amp=0.08)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4, precision="fp64")
    s.set_species(sp, eps, sig, rc, sh)
    ref = O.Sim(pos, vel, L, shell=0.4, rc=rc.max(), ushift=0.0)
    ref.set_species(O.Mixture(sp, eps, sig, rc, sh))
    s.step(20)
    ref.run(20)
    s.block_begin()
    s.step(60)
    blk = s.block_end()
    want = O.block_means(ref.run(60), n, 1, 60)
    s.close()
    ref.close()
    assert blk["steps"] == 60
    for key in ("ke_per_atom", "pe_per_atom", "virial_per_atom"):
        assert abs(blk[key] - want[key]) <= 1e-10 * max(abs(want[key]), 1.0), key
    assert abs(blk["nebr_per_atom"] - want["nebr_per_atom"]) <= 1e-12 * want["nebr_per_atom"]


def test_mixture_energy_conservation_10k_steps():
    """The WCA mixture's pair energies are continuous at every cutoff (each
    shift is eps_ab), so the FP32-force trajectory conserves energy as the
    one-species one does: drift of the mean total energy per atom between
    the first and last 1 000 steps below 2e-4 over 10^4 steps."""
    pos, L = I.fcc_lattice(9, 0.75)
    vel = I.random_velocities(len(pos), 1.0, 13)
    sp = (np.random.Generator(np.random.PCG64(14)).random(len(pos)) < 0.5).astype(np.int32)
    eps, sig, rc, sh = wca_binary()
    n = len(pos)
    s = _system(pos, vel, L, r_cut=rc.max(), shell=0.4)
    s.set_species(sp, eps, sig, rc, sh)
    e = []
    for _ in range(100):
        s.step(100)
        pr = s.props()
        e.append((pr["ke"] + pr["pe"]) / n)
    e = np.array(e)
    assert abs(e[-10:].mean() - e[:10].mean()) / abs(e[:10].mean()) < 2e-4
    assert s.props()["step"] == 10000 and s.props()["n_rebuilds"] > 300
    s.close()
