"""Parity at the workloads' full sizes, in the launch configuration bench.py
times, and at the degenerate edges.

At N = 256 000 and 4 000 000 the oracle cannot evaluate the whole system in
seconds, so sampled atoms are checked one by one: the oracle's brute-force
per-atom force and neighbour set (every atom, minimum image, same expression
order) against the GPU's forces and neighbour-matrix rows.  Properties that
hold at any size (momentum, symmetry of the pair set) are checked for all
atoms.  Bars as in test_gpu_parity: forces max_i |dF_i| / max(|F_i|, F_rms)
<= 1e-5; neighbour sets bit-exact.
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


def _system(*args, **kw):
    from paper_0911_5631_amd.md import System
    return System(*args, **kw)


def _check_sampled_forces(pos, force, L, idx):
    f_ref, u_ref, _, _ = O.force_on_atoms(pos, L, idx)
    scale = np.maximum(np.linalg.norm(f_ref, axis=1), math.sqrt((f_ref ** 2).sum(1).mean()))
    err = float((np.linalg.norm(force[idx] - f_ref, axis=1) / scale).max())
    assert err <= FORCE_TOL, err
    return u_ref


def _check_sampled_neighbours(s, pos, L, rn, idx):
    pi, pj = s.pairs()
    order = np.argsort(pi, kind="stable")
    pi, pj = pi[order], pj[order]
    lo = np.searchsorted(pi, idx, side="left")
    hi = np.searchsorted(pi, idx, side="right")
    soa = O._soa(pos)
    for a, b, i in zip(lo, hi, idx):
        got = np.sort(pj[a:b])
        ref = np.sort(O.neighbors_of_atom(pos, L, rn, int(i), _soa_cache=soa))
        assert np.array_equal(got, ref), int(i)
    return pi, pj


@pytest.mark.parametrize("make,steps,n_sample", [(I.sp_256k, 25, 256), (I.sp_4m, 30, 48)],
                         ids=["sp_256k", "sp_4m"])
def test_full_size_sampled_parity(make, steps, n_sample):
    wl = make()
    n, L = wl.n, wl.box
    s = _system(wl.pos, wl.vel, L, shell=wl.shell, dt=wl.dt, precision=wl.precision)
    rng = np.random.Generator(np.random.PCG64(11))
    idx = np.sort(rng.choice(n, size=n_sample, replace=False)).astype(np.int64)
    # the fcc start: every separation exceeds r_c, so forces and PE vanish
    pos, vel, force, step = s.get_state()
    assert step == 0 and float(np.abs(force).max()) == 0.0 and s.props()["pe"] == 0.0
    # a few steps through graph replays and at least one rebuild
    s.step(steps)
    pr = s.props()
    assert pr["step"] == steps and pr["n_rebuilds"] >= 1
    pos, vel, force, step = s.get_state()
    assert np.isfinite(pos).all() and np.isfinite(force).all()
    u_ref = _check_sampled_forces(pos, force, L, idx)
    u_atom, _ = s.atom_energies()
    assert float(np.abs(u_atom[idx] - u_ref).max()) <= 1e-6 * max(1.0, float(np.abs(u_ref).max()))
    # total momentum stays at its start value (zero) up to FP32 force rounding
    p = vel.sum(0)
    assert float(np.abs(p).max()) <= 1e-6 * n ** 0.5 * steps
    # a list built at exactly these positions: sampled rows bit-exact, and the
    # pair set symmetric (each unordered pair once from each side)
    s.bin_cells()
    pos2, _, _, _ = s.get_state()
    assert np.array_equal(pos2, O.wrap(pos, L))
    pi, pj = _check_sampled_neighbours(s, pos2, L, RC + wl.shell, idx)
    key = pi.astype(np.int64) * n + pj
    rkey = pj.astype(np.int64) * n + pi
    assert np.array_equal(np.sort(key), np.sort(rkey))
    assert len(pi) == 2 * s.props()["n_pairs"]
    s.close()


def test_lj_full_size_sampled_parity():
    """Lennard-Jones at Table 1's largest size (N_e = 64, 262 144 atoms,
    r_c = 3.0, shell 0.8, rho 0.38): sampled forces and energies against the
    oracle's brute-force per-atom sums after steps with rebuilds, and sampled
    neighbour rows of a list built at those positions, bit-exact."""
    pos0, L = I.sc_lattice(64, 0.38)
    vel0 = I.random_velocities(len(pos0), 1.2, 17)
    n = len(pos0)
    s = _system(pos0, vel0, L, r_cut=3.0, shell=0.8, even_cells=True)
    s.step(40)
    assert s.props()["n_rebuilds"] >= 1
    pos, vel, force, _ = s.get_state()
    idx = np.sort(np.random.Generator(np.random.PCG64(18)).choice(n, 64, replace=False))
    f_ref, u_ref, _, _ = O.force_on_atoms(pos, L, idx.astype(np.int64), rc=3.0, ushift=0.0)
    scale = np.maximum(np.linalg.norm(f_ref, axis=1), math.sqrt((f_ref ** 2).sum(1).mean()))
    assert float((np.linalg.norm(force[idx] - f_ref, axis=1) / scale).max()) <= FORCE_TOL
    u_atom, _ = s.atom_energies()
    assert float(np.abs(u_atom[idx] - u_ref).max()) <= 1e-5 * max(1.0, float(np.abs(u_ref).max()))
    s.bin_cells()
    pos2, _, _, _ = s.get_state()
    _check_sampled_neighbours(s, pos2, L, 3.8, idx[:24])
    s.close()


def test_largest_system_the_index_width_allows():
    """The largest fcc system under the 25-bit storage index: n_c = 203,
    33 461 708 atoms (2^25 - 1 is the limit), 13.5 GB on the device.  After
    steps with a rebuild, sampled forces and energies against the oracle's
    brute-force sums, half of the sample stored at positions >= 2^24 (the
    top index bit set in their list entries); momentum as at 4 x 10^6."""
    from paper_0911_5631_amd.md import md_query_bytes, make_params
    from paper_0911_5631_amd._lib import MDError
    pos, L = I.fcc_lattice(203, 0.8)
    n = len(pos)
    assert n == 33_461_708 and n <= (1 << 25) - 1
    with pytest.raises(MDError):
        md_query_bytes(make_params(1 << 25, L, shell=0.4))
    vel = I.random_velocities(n, 1.0, 19)
    s = _system(pos, vel, L, shell=0.4, dt=0.005)
    del pos
    s.step(30)
    pr = s.props()
    assert pr["step"] == 30 and pr["n_rebuilds"] >= 1
    order, _ = s.bins()
    rng = np.random.Generator(np.random.PCG64(20))
    high = order[rng.choice(np.arange(1 << 24, n), 24, replace=False)]
    idx = np.unique(np.concatenate([high, rng.choice(n, 24, replace=False)])).astype(np.int64)
    pos, vel, force, _ = s.get_state()
    assert np.isfinite(pos).all() and np.isfinite(force).all()
    u_ref = _check_sampled_forces(pos, force, L, idx)
    u_atom, _ = s.atom_energies()
    s.close()
    assert float(np.abs(u_atom[idx] - u_ref).max()) <= 1e-6 * max(1.0, float(np.abs(u_ref).max()))
    assert float(np.abs(vel.sum(0)).max()) <= 1e-6 * n ** 0.5 * 30


def test_single_atom_and_pair():
    # one atom: no pairs, no force, nothing to do but drift
    L = 5.0
    s = _system(np.array([[0.1, -0.2, 0.3]]), np.array([[0.5, 0.0, -0.25]]), L, shell=0.4)
    s.step(10)
    p, v, f, step = s.get_state()
    assert step == 10 and float(np.abs(f).max()) == 0.0
    assert np.allclose(p, [[0.1 + 0.05 * 0.5 * 10 / 10, -0.2, 0.3 - 0.25 * 0.05]], atol=1e-12)
    assert s.props()["pe"] == 0.0
    s.close()
    # two atoms at separation r < r_c across the periodic boundary: the pair
    # force of Eq. (1), F = 48 r^-13 - 24 r^-7 along the separation
    r = 1.05
    pos = np.array([[L / 2 - r / 2 + 1e-3, 0.0, 0.0], [-L / 2 + r / 2 + 1e-3, 0.0, 0.0]])
    for prec, tol in (("fp32", 3e-6), ("fp64", 1e-13)):
        s = _system(pos, np.zeros((2, 3)), L, shell=0.4, precision=prec)
        _, _, f, _ = s.get_state()
        fmag = 48 * r ** -13 - 24 * r ** -7
        # atom 0 sits at +x, its image partner lies across the face at +L/2
        assert abs(f[0, 0] + fmag) <= tol * fmag and abs(f[1, 0] - fmag) <= tol * fmag
        u_ref = 4 * (r ** -12 - r ** -6) + 1
        assert abs(s.props()["pe"] - u_ref) <= tol * max(1.0, u_ref)
        s.close()


@pytest.mark.parametrize("n", [255, 256, 257, 343])
def test_minimal_box_and_ragged_tiles(n):
    # G = 3 (the smallest grid); tiles that end one atom short of, exactly
    # at, and one atom past a 256-atom boundary; against the oracle's brute
    # force over the 27 images.  Atoms: n sites of a jittered 7^3 simple
    # cubic lattice (spacing 0.857, so every pair force is finite).
    rng = np.random.Generator(np.random.PCG64(n))
    rn = RC + 0.4
    L = 6.0
    g = (np.arange(7) + 0.5) * (L / 7) - L / 2
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = sites[rng.permutation(len(sites))[:n]] + rng.uniform(-0.02, 0.02, size=(n, 3))
    vel = rng.normal(size=pos.shape) * 0.5
    s = _system(pos, vel, L, shell=0.4)
    assert s.props()["cells_per_edge"] == 3 and O.cells_per_edge(L, rn) == 3
    pi, pj = s.pairs()
    ref = O.pair_set(*O.pairs_brute(O.wrap(pos, L), L, rn)[:2])
    assert np.array_equal(O.pair_set(pi, pj), ref)
    _, _, f, _ = s.get_state()
    fr = O.forces_brute(O.wrap(pos, L), L)
    scale = np.maximum(np.linalg.norm(fr.force, axis=1), math.sqrt((fr.force ** 2).sum(1).mean()))
    assert float((np.linalg.norm(f - fr.force, axis=1) / scale).max()) <= FORCE_TOL
    # and a few steps on, against the oracle's own trajectory
    s.step(20)
    p, _, _, _ = s.get_state()
    sim = O.Sim(pos, vel, L, shell=0.4, dt=0.005)
    sim.run(20)
    pr, _, _, _ = sim.state()[:4]
    sim.close()
    d = p - pr
    d -= L * np.round(d / L)
    assert float(np.abs(d).max()) <= 1e-6
    s.close()
