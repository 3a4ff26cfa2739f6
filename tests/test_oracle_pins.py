"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics: printed cell counts, closed-form pair and lattice values, brute
force on tiny systems, library routines for the plain definitions, and
physical invariants of the leapfrog trajectory.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

RC = 2.0 ** (1.0 / 6.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Geometry: the paper's cell counts (Tables 1 and 5)
# ---------------------------------------------------------------------------

def _golden_cell_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_cell_counts.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            src, pot, ne, rho, rc, delta, nc = line.split()
            rc = RC if rc == "sp" else float(rc)
            rows.append((src, pot, int(ne), float(rho), rc, float(delta), int(nc)))
    return rows


@pytest.mark.parametrize("row", _golden_cell_rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}-{r[5]}")
def test_cell_counts_match_paper_tables(row):
    src, pot, ne, rho, rc, delta, nc = row
    L = ne / rho ** (1.0 / 3.0)           # Sec. 3.1: L = N_e / rho^(1/3)
    G = O.cells_per_edge(L, rc + delta, even=True)
    assert G ** 3 == nc


def test_cells_per_edge_text_rule():
    # floor(L / r_n) on values worked by hand
    assert O.cells_per_edge(10.0, 2.5) == 4
    assert O.cells_per_edge(10.0, 3.4) == 2
    assert O.cells_per_edge(68.39903786706787, RC + 0.4) == 44      # 68.399/1.5225 = 44.93
    assert O.cells_per_edge(68.39903786706787, RC + 0.4, even=True) == 44
    assert O.cells_per_edge(13.679807573413574, RC) == 12          # 13.68/1.1225 = 12.19
    assert O.cells_per_edge(170.99759466766967, RC + 0.4) == 112   # 171.0/1.5225 = 112.3
    assert O.cells_per_edge(10.5, 2.0, even=True) == 4


# ---------------------------------------------------------------------------
# Pair potential: special values of Eq. (1) with the soft-sphere shift
# ---------------------------------------------------------------------------

def test_pair_potential_special_values():
    u, fr = O.pair_potential(1.0)
    assert u == 1.0 and fr == 24.0                  # 4(1 - 1) + 1 ; 48 - 24
    r = 2.0 ** (-1.0 / 6.0)                         # r^-6 = 2
    u, fr = O.pair_potential(r)
    assert abs(u - 9.0) < 1e-12                     # 4(4 - 2) + 1
    assert abs(fr - 144.0 / r) < 1e-10              # (48*4 - 24*2) / r
    # Taylor expansion at r_c, derivatives worked by hand with r_c^-6 = 1/2:
    # u(r_c) = 0, u'(r_c) = 0, u''(r_c) = 72 r_c^-2, u'''(r_c) = -1512 r_c^-3,
    # u''''(r_c) = 26712 r_c^-4.
    u2 = 72.0 * 2.0 ** (-1.0 / 3.0)
    u3 = -1512.0 * 2.0 ** (-0.5)
    u4 = 26712.0 * 2.0 ** (-2.0 / 3.0)
    for eps in (1e-3, 1e-4, 1e-6):
        u, fr = O.pair_potential(RC - eps)
        expect_u = 0.5 * u2 * eps ** 2 - u3 * eps ** 3 / 6.0 + u4 * eps ** 4 / 24.0
        expect_fr = u2 * eps - 0.5 * u3 * eps ** 2 + u4 * eps ** 3 / 6.0
        assert abs(u - expect_u) < 0.1 * u4 * eps ** 4 + 1e-15
        assert abs(fr - expect_fr) < 0.1 * u4 * eps ** 3 + 1e-12
    assert O.pair_potential(RC) == (0.0, 0.0)
    assert O.pair_potential(1.5) == (0.0, 0.0)
    # plain truncated LJ (no shift): minimum -1 at 2^(1/6)
    u, fr = O.pair_potential(RC, rc=2.5, ushift=0.0)
    assert abs(u + 1.0) < 1e-12 and abs(fr) < 1e-12


def test_two_atom_force_direction_and_magnitude():
    L = 10.0
    for r in (0.95, 1.0, 1.05, 1.1):
        pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        f = O.forces_brute(pos, L)
        mag = 48.0 * r ** -13 - 24.0 * r ** -7
        # repulsive: atom 0 is pushed towards -x, atom 1 towards +x
        assert abs(f.force[0, 0] + mag) < 1e-10 * mag and abs(f.force[1, 0] - mag) < 1e-10 * mag
        assert np.all(f.force[:, 1:] == 0.0)
        assert abs(f.pe - (4 * (r ** -12 - r ** -6) + 1)) < 1e-12
        assert abs(f.virial - mag * r) < 1e-10 * mag * r
        # across the periodic boundary: same pair, split by the region edge
        pos2 = np.array([[L / 2 - 0.3, 0.0, 0.0], [-L / 2 + (r - 0.3), 0.0, 0.0]])
        g = O.forces_cells(pos2, L, O.cells_per_edge(L, RC))
        assert abs(g.force[0, 0] + mag) < 1e-9 * mag
        assert abs(g.pe - f.pe) < 1e-12


# ---------------------------------------------------------------------------
# Lattice sums (closed forms)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shell", [0.0, 0.4])
def test_sc_lattice_sums(shell):
    # sc at rho = 0.8: spacing a = rho^(-1/3) = 1.0772 < r_c < sqrt(2) a, so
    # each atom has 6 interacting neighbours at a, a^-6 = rho^2 = 0.64.
    # PE/N = 3 u(a) = 3 (4 (0.4096 - 0.64) + 1) = 0.2352
    # W/N  = 3 f(a) a^2 = 3 (48 * 0.4096 - 24 * 0.64) = 12.9024
    pos, L = I.sc_lattice(6, 0.8)
    n = len(pos)
    G = O.cells_per_edge(L, RC + shell)
    for f in (O.forces_cells(pos, L, O.cells_per_edge(L, RC)), O.forces_brute(pos, L),
              O.forces_pairs(pos, L, *O.pairs_cells(pos, L, G, RC + shell))):
        assert abs(f.pe / n - 0.2352) < 1e-12
        assert abs(f.virial / n - 12.9024) < 1e-11
        assert np.abs(f.force).max() < 1e-12
        assert f.n_inter == 3 * n


def test_fcc_lattice_sums():
    # fcc at rho = 1.2: nn = a / sqrt(2) = 1.0563 < r_c < a = 1.4938;
    # nn^-6 = rho^2 / 2 = 0.72.  PE/N = 6 u(nn) = 6 (4 (0.5184 - 0.72) + 1)
    # = 1.1616; W/N = 6 (48 * 0.5184 - 24 * 0.72) = 45.6192.
    pos, L = I.fcc_lattice(4, 1.2)
    n = len(pos)
    f = O.forces_cells(pos, L, O.cells_per_edge(L, RC))
    assert abs(f.pe / n - 1.1616) < 1e-12
    assert abs(f.virial / n - 45.6192) < 1e-10
    assert np.abs(f.force).max() < 1e-11
    # fcc at rho = 0.8 (every workload's start): nn = 1.209 > r_c, no forces;
    # with shell 0.4 (r_n = 1.5225 < a = 1.71) exactly the 12 nearest
    # neighbours are listed.
    pos, L = I.fcc_lattice(5, 0.8)
    n = len(pos)
    f = O.forces_brute(pos, L)
    assert f.pe == 0.0 and f.virial == 0.0 and np.all(f.force == 0.0)
    pi, pj, img = O.pairs_cells(pos, L, O.cells_per_edge(L, RC + 0.4), RC + 0.4)
    assert len(pi) == 6 * n
    assert np.all(np.bincount(np.concatenate([pi, pj]), minlength=n) == 12)


# ---------------------------------------------------------------------------
# Cells, wrap, layers
# ---------------------------------------------------------------------------

def test_wrap_half_open_and_exact():
    L = 7.5
    pos = np.array([[L / 2, -L / 2, 0.0], [-L / 2 - 0.25, L / 2 + 0.5, 3.7], [1.0, -3.0, L]])
    w = O.wrap(pos, L)
    assert np.array_equal(w[0], [-L / 2, -L / 2, 0.0])
    assert np.array_equal(w[1], [L / 2 - 0.25, -L / 2 + 0.5, 3.7])
    assert np.array_equal(w[2], [1.0, -3.0, 0.0])
    rng = np.random.default_rng(3)
    p = rng.uniform(-1.4 * L, 1.4 * L, (1000, 3))
    w = O.wrap(p, L)
    k = np.round((p - w) / L)
    assert np.all((w >= -L / 2) & (w < L / 2)) and np.array_equal(p - k * L, w)


def test_cell_ids_closed_form():
    # Sec. 3.1: c = ((c_z - 1) G + c_y - 1) G + c_x (1-based); 0-based here.
    L, G = 9.0, 6
    w = L / G
    pos = np.array([[-L / 2 + 0.5 * w, -L / 2 + 1.5 * w, -L / 2 + 2.5 * w],
                    [L / 2 - 0.1 * w, -L / 2, 0.0],
                    [0.0, 0.0, 0.0],
                    [np.nextafter(L / 2, 0), np.nextafter(L / 2, 0), -L / 2]])
    c = O.cell_ids(pos, L, G)
    assert c[0] == (2 * G + 1) * G + 0
    assert c[1] == (3 * G + 0) * G + 5
    assert c[2] == (3 * G + 3) * G + 3
    assert c[3] == (0 * G + 5) * G + 5          # clamped at the upper face
    # every atom lies inside its cell (up to rounding at the faces)
    rng = np.random.default_rng(5)
    p = rng.uniform(-L / 2, L / 2, (5000, 3))
    c = O.cell_ids(p, L, G)
    cc = np.stack([c % G, (c // G) % G, c // (G * G)], axis=1)
    lo = cc * w - L / 2
    assert np.all(p >= lo - 1e-12) and np.all(p < lo + w + 1e-12)


def test_layers_reorder_is_stable_counting_sort():
    rng = np.random.default_rng(11)
    G = 5
    cell = rng.integers(0, G ** 3, 3000).astype(np.int32)
    layer, order, cs, nl = O.layers_reorder(cell, G)
    assert np.array_equal(order, np.argsort(cell, kind="stable"))
    counts = np.bincount(cell, minlength=G ** 3)
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(counts)]))
    assert nl == counts.max()
    # layer = rank of the atom among earlier atoms of its cell
    for i in rng.integers(0, 3000, 50):
        assert layer[i] == np.count_nonzero(cell[:i] == cell[i])


# ---------------------------------------------------------------------------
# Pair sets and forces against brute force
# ---------------------------------------------------------------------------

def _fluid(nc, rho, amp, seed, shuffle=True):
    pos, L = I.fcc_lattice(nc, rho)
    pos = I.jitter(pos, L, amp, seed)
    vel = I.random_velocities(len(pos), 1.0, seed + 100)
    if shuffle:
        pos, vel = I.shuffled(pos, vel, seed + 200)
    return pos, vel, L


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("shell", [0.0, 0.3, 0.4, 0.8])
def test_pair_set_equals_brute_force(seed, shell):
    pos, _, L = _fluid(3, 0.8, 0.3, seed)
    rn = RC + shell
    ref = O.pair_set(*O.pairs_brute(pos, L, rn)[:2])
    G = O.cells_per_edge(L, rn)
    for g in {G, O.cells_per_edge(L, rn, even=True), max(G - 1, 3)}:
        if g < 3:
            continue
        pi, pj, img = O.pairs_cells(pos, L, g, rn)
        assert len(pi) == len(ref)                       # no pair twice
        assert np.array_equal(O.pair_set(pi, pj), ref)


def test_pair_images_match_brute_force():
    pos, _, L = _fluid(3, 0.8, 0.3, 9)
    rn = RC + 0.4
    bi, bj, bimg = O.pairs_brute(pos, L, rn)
    ci, cj, cimg = O.pairs_cells(pos, L, O.cells_per_edge(L, rn), rn)
    # the same unordered pair carries the opposite image when listed the other way
    key = {}
    for a, b, im in zip(bi, bj, bimg):
        key[(a, b)] = tuple(im)
    for a, b, im in zip(ci, cj, cimg):
        if (a, b) in key:
            assert key[(a, b)] == tuple(im)
        else:
            assert key[(b, a)] == tuple(-im)


@pytest.mark.parametrize("seed", [4, 5])
def test_forces_cell_methods_equal_brute_force(seed):
    pos, _, L = _fluid(3, 0.85, 0.25, seed)
    ref = O.forces_brute(pos, L)
    scale = np.sqrt((ref.force ** 2).sum(1).mean())
    assert ref.n_inter > 0 and scale > 1.0
    cel = O.forces_cells(pos, L, O.cells_per_edge(L, RC))
    lst = O.forces_pairs(pos, L, *O.pairs_cells(pos, L, O.cells_per_edge(L, RC + 0.4), RC + 0.4))
    for f in (cel, lst):
        assert np.abs(f.force - ref.force).max() < 1e-12 * scale
        assert abs(f.pe - ref.pe) < 1e-12 * abs(ref.pe)
        assert abs(f.virial - ref.virial) < 1e-12 * abs(ref.virial)
        assert f.n_inter == ref.n_inter
        assert np.allclose(f.u_atom, ref.u_atom, rtol=1e-12, atol=1e-12)
        assert abs(f.u_atom.sum() - 2 * f.pe) < 1e-10 * abs(f.pe)
    # Newton's third law: the total force vanishes to round-off
    assert np.abs(ref.force.sum(0)).max() < 1e-11 * scale * len(pos)


def test_force_on_atoms_and_neighbours_of_atom():
    pos, _, L = _fluid(3, 0.8, 0.3, 6)
    ref = O.forces_brute(pos, L)
    idx = np.array([0, 5, 17, 50, len(pos) - 1])
    F, u, w, cnt = O.force_on_atoms(pos, L, idx)
    scale = np.sqrt((ref.force ** 2).sum(1).mean())
    assert np.abs(F - ref.force[idx]).max() < 1e-12 * scale
    assert np.allclose(u, ref.u_atom[idx], rtol=1e-12, atol=1e-13)
    assert np.allclose(w, ref.w_atom[idx], rtol=1e-12, atol=1e-12)
    rn = RC + 0.4
    bi, bj, _ = O.pairs_brute(pos, L, rn)
    for i in idx:
        expect = np.sort(np.concatenate([bj[bi == i], bi[bj == i]]))
        assert np.array_equal(O.neighbors_of_atom(pos, L, rn, i), expect)


# ---------------------------------------------------------------------------
# The MD loop
# ---------------------------------------------------------------------------

def test_two_body_head_on_collision():
    # Two atoms approach along x with relative speed v.  Energy conservation
    # with reduced mass 1/2 puts the turning point where u(r_min) = v^2 / 4;
    # with y = r^-6: 4y^2 - 4y + 1 = v^2/4  =>  y = (1 + v/2) / 2.
    # After the collision the (equal-mass, elastic) velocities are exchanged.
    L = 12.0
    for v in (2.0, 4.0):
        pos = np.array([[-0.7, 0.0, 0.0], [0.7, 0.0, 0.0]])
        vel = np.array([[v / 2, 0.0, 0.0], [-v / 2, 0.0, 0.0]])
        dt = 0.0005
        sim = O.Sim(pos, vel, L, shell=0.4, dt=dt)
        rmin = 1e9
        for _ in range(3000):
            sim.run(1)
            p, vv, f, st = sim.state()
            rmin = min(rmin, p[1, 0] - p[0, 0])
        expect = ((1.0 + v / 2) / 2) ** (-1.0 / 6.0)
        assert abs(rmin - expect) < 2e-4
        assert np.allclose(vv, -vel, atol=1e-6)


def test_time_reversal():
    pos, vel, L = _fluid(3, 0.8, 0.1, 7)
    sim = O.Sim(pos, vel, L, shell=0.4)
    sim.run(150)
    p1, v1, f1, _ = sim.state()
    back = O.Sim(p1, -v1, L, shell=0.4)
    back.run(150)
    p2, v2, _, _ = back.state()
    d = p2 - O.wrap(pos, L)
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + vel).max() < 1e-9


def test_energy_momentum_conservation_10k_steps():
    pos, vel, L = _fluid(4, 0.8, 0.0, 8, shuffle=False)
    n = len(pos)
    sim = O.Sim(pos, vel, L, shell=0.4)
    tr = sim.run(10000)
    e = (tr[:, 0] + tr[:, 1]) / n
    drift = abs(e[-1000:].mean() - e[:1000].mean()) / abs(e[:1000].mean())
    assert drift < 2e-4                          # the paper's FP32 figure bounds FP64
    _, v, _, st = sim.state()
    assert np.abs(v.sum(0)).max() < 1e-10
    assert st.n_rebuilds > 100


@pytest.mark.parametrize("temp", [1.0, 3.0])
def test_rebuild_rule_misses_no_pair(temp):
    pos, L = I.fcc_lattice(4, 0.8)
    vel = I.random_velocities(len(pos), temp, 21)
    sim = O.Sim(pos, vel, L, shell=0.4, check_missed=True)
    tr = sim.run(400)
    _, _, _, st = sim.state()
    assert st.n_missed == 0 and st.n_rebuilds > 10
    # the recorded rebuilds follow "sum of vmax*dt exceeds delta/2"
    disp = math.sqrt(sim.start[3]) * 0.005
    for t in range(len(tr)):
        due = disp > 0.2
        assert bool(tr[t, 5]) == due
        disp = (0.0 if due else disp) + math.sqrt(tr[t, 3]) * 0.005


def test_cell_only_mode_matches_list_mode_trajectory():
    pos, vel, L = _fluid(3, 0.8, 0.05, 12)
    a = O.Sim(pos, vel, L, shell=0.0)
    b = O.Sim(pos, vel, L, shell=0.4)
    ta, tb = a.run(50), b.run(50)
    pa, va, _, _ = a.state()
    pb, vb, _, _ = b.state()
    d = pa - pb
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10 and np.abs(va - vb).max() < 1e-9
    assert np.allclose(ta[:, :3], tb[:, :3], rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------
# Lennard-Jones with the longer cutoffs of Sec. 5.1 (no shift)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rc", [2.2, 2.5, 3.0])
def test_lj_pair_set_and_forces_equal_brute_force(rc):
    # 729 atoms at rho 0.38: L = 12.43, three cells per edge at r_n = 3.8
    pos, L = I.sc_lattice(9, 0.38)
    pos = I.jitter(pos, L, 0.3, seed=int(rc * 10))
    rn = rc + 0.8
    G = O.cells_per_edge(L, rn)
    assert G >= 3
    ref = O.pair_set(*O.pairs_brute(pos, L, rn)[:2])
    pi, pj, _ = O.pairs_cells(pos, L, G, rn)
    assert len(pi) == len(ref) and np.array_equal(O.pair_set(pi, pj), ref)
    fb = O.forces_brute(pos, L, rc=rc, ushift=0.0)
    scale = np.sqrt((fb.force ** 2).sum(1).mean())
    for f in (O.forces_cells(pos, L, O.cells_per_edge(L, rc), rc=rc, ushift=0.0),
              O.forces_pairs(pos, L, pi, pj, _, rc=rc, ushift=0.0)):
        assert np.abs(f.force - fb.force).max() < 1e-12 * scale
        assert abs(f.pe - fb.pe) < 1e-12 * abs(fb.pe)
        assert f.n_inter == fb.n_inter


@pytest.mark.parametrize("rc", [2.2, 2.5, 3.0])
def test_lj_sc_lattice_sum_by_lattice_vectors(rc):
    # a simple cubic crystal: every atom sees the same shells, so PE/N is half
    # the sum of u(|n| a) over integer vectors n != 0 with |n| a < r_c (Eq. (1)
    # without shift), counted here by enumerating the vectors directly
    pos, L = I.sc_lattice(12, 0.38)
    a = L / 12
    k = int(rc / a) + 1
    g = np.arange(-k, k + 1)
    nx, ny, nz = np.meshgrid(g, g, g, indexing="ij")
    r2 = (nx ** 2 + ny ** 2 + nz ** 2).ravel() * a * a
    r2 = r2[(r2 > 0) & (r2 < rc * rc)]
    u = 4.0 * (r2 ** -6 - r2 ** -3)
    w = 48.0 * r2 ** -6 - 24.0 * r2 ** -3            # f(r) r^2
    f = O.forces_cells(pos, L, O.cells_per_edge(L, rc), rc=rc, ushift=0.0)
    n = len(pos)
    assert abs(f.pe / n - 0.5 * u.sum()) < 1e-12 * abs(u.sum())
    assert abs(f.virial / n - 0.5 * w.sum()) < 1e-11 * max(abs(w.sum()), 1.0)
    assert np.abs(f.force).max() < 1e-11
    assert f.n_inter == n * len(r2) // 2
