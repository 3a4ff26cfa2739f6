"""Pins of the oracle's several-species pair model (the extension the paper
names in Sec. 3.5: per species pair epsilon, sigma, cutoff and
shift; Eq. (1) in the pair's units).  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

RC = 2.0 ** (1.0 / 6.0)


def wca_binary(species, sig_aa=1.0, sig_bb=1.2, eps_aa=1.0, eps_bb=1.0, eps_ab=1.5):
    """An additive soft-sphere (WCA) binary mixture: sigma_ab the mean, cutoff
    2^(1/6) sigma_ab, shift eps_ab so that u(r_c) = 0."""
    sig = np.array([[sig_aa, 0.5 * (sig_aa + sig_bb)], [0.5 * (sig_aa + sig_bb), sig_bb]])
    eps = np.array([[eps_aa, eps_ab], [eps_ab, eps_bb]])
    return O.Mixture(species, eps, sig, RC * sig, eps.copy())


def test_mixture_cells_and_lists_equal_brute_force():
    pos, L = I.sc_lattice(9, 0.75)
    pos = I.jitter(pos, L, 0.25, seed=41)
    sp = (np.random.Generator(np.random.PCG64(42)).random(len(pos)) < 0.4).astype(np.int32)
    mix = wca_binary(sp)
    ref = O.forces_brute(pos, L, mix=mix)
    scale = np.sqrt((ref.force ** 2).sum(1).mean())
    assert ref.n_inter > 0 and scale > 1.0
    rn = mix.max_cut + 0.4
    pi, pj, img = O.pairs_cells(pos, L, O.cells_per_edge(L, rn), rn)
    for f in (O.forces_cells(pos, L, O.cells_per_edge(L, mix.max_cut), mix=mix),
              O.forces_pairs(pos, L, pi, pj, img, mix=mix)):
        assert np.abs(f.force - ref.force).max() < 1e-12 * scale
        assert abs(f.pe - ref.pe) < 1e-12 * abs(ref.pe)
        assert abs(f.virial - ref.virial) < 1e-12 * abs(ref.virial)
        assert f.n_inter == ref.n_inter
    # Newton's third law holds pair by pair
    assert np.abs(ref.force.sum(0)).max() < 1e-11 * scale * len(pos)


def test_one_species_table_is_the_plain_potential():
    pos, L = I.fcc_lattice(5, 0.85)
    pos = I.jitter(pos, L, 0.2, seed=43)
    one = O.Mixture(np.zeros(len(pos), np.int32), [[1.0]], [[1.0]], [[RC]], [[1.0]])
    a = O.forces_cells(pos, L, O.cells_per_edge(L, RC), mix=one)
    b = O.forces_cells(pos, L, O.cells_per_edge(L, RC))
    scale = np.sqrt((b.force ** 2).sum(1).mean())
    # 1 / r^2 taken once (plain) or divided at the end (pair units): rounding only
    assert np.abs(a.force - b.force).max() < 1e-14 * scale
    assert abs(a.pe - b.pe) < 1e-14 * abs(b.pe) and a.n_inter == b.n_inter


def test_checkerboard_lattice_closed_form():
    # simple cubic of spacing a = sigma_ab = 1.1 with the two species on
    # alternate sites (the CsCl-like checkerboard): each atom has 6 unlike
    # neighbours at a, inside their cutoff 2^(1/6) 1.1 = 1.235, and its like
    # neighbours at sqrt(2) a = 1.556 lie beyond 2^(1/6) sigma_bb = 1.347.
    # At r = sigma the WCA energy is 4 eps (1 - 1) + eps = eps and f r^2 is
    # 48 eps (1 - 1/2) = 24 eps, so PE/N = 3 eps_ab, W/N = 72 eps_ab, F = 0.
    ne, a = 8, 1.1
    pos, L = I.sc_lattice(ne, 1.0 / a ** 3)
    assert abs(L / ne - a) < 1e-12
    g = np.arange(ne)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    sp = ((ix + iy + iz).ravel() % 2).astype(np.int32)
    mix = wca_binary(sp, sig_aa=1.0, sig_bb=1.2, eps_ab=1.5)
    n = len(pos)
    for f in (O.forces_brute(pos, L, mix=mix),
              O.forces_cells(pos, L, O.cells_per_edge(L, mix.max_cut), mix=mix)):
        assert abs(f.pe / n - 4.5) < 1e-12
        assert abs(f.virial / n - 108.0) < 1e-10
        assert np.abs(f.force).max() < 1e-11
        assert f.n_inter == 3 * n


def test_mixture_trajectory_conserves_energy_and_momentum():
    pos, L = I.sc_lattice(10, 0.7)
    pos = I.jitter(pos, L, 0.05, seed=44)
    vel = I.random_velocities(len(pos), 1.0, 45)
    sp = (np.arange(len(pos)) % 3 == 0).astype(np.int32)
    mix = wca_binary(sp)
    s = O.Sim(pos, vel, L, shell=0.4, rc=mix.max_cut, ushift=0.0)
    s.set_species(mix)
    tr = s.run(2000)
    e = (tr[:, 0] + tr[:, 1]) / len(pos)
    drift = abs(e[-200:].mean() - e[:200].mean()) / abs(e[:200].mean())
    assert drift < 2e-4
    v = s.state()[1]
    assert np.abs(v.sum(0)).max() < 1e-10
    s.close()


def test_set_species_rejects_a_cutoff_beyond_the_list():
    pos, L = I.fcc_lattice(4, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 46)
    s = O.Sim(pos, vel, L, shell=0.4)          # r_c = 2^(1/6)
    mix = wca_binary(np.zeros(len(pos), np.int32), sig_aa=1.1)
    with pytest.raises(ValueError):
        s.set_species(mix)
    s.close()
