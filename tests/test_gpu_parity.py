"""Parity of the gfx950 path (through the C ABI) with the FP64 CPU oracle.

Bars (the stated tolerances of the GPU path, derived where none is stated):
  * cell assignment, storage order and neighbour-pair sets: bit-exact;
  * FP32 forces: max_i |dF_i| / max(|F_i|, F_rms) <= 1e-5 (a per-component
    relative error is undefined where F_i ~ 0, so the scale is the larger of
    the atom's own force and the rms force);
  * PE and virial per atom: |d(X/N)| <= 1e-6 * max(|X/N|, 1);
  * FP64 paths: the same quantities to ~1e-12 (summation order only).
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


def fluid(nc, rho=0.8, amp=0.15, seed=1, temp=1.0, shuffle=True):
    pos, L = I.fcc_lattice(nc, rho)
    pos = I.jitter(pos, L, amp, seed)
    vel = I.random_velocities(len(pos), temp, seed + 1000)
    if shuffle:
        pos, vel = I.shuffled(pos, vel, seed + 2000)
    return pos, vel, L


def force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


def min_image(d, L):
    return d - L * np.round(d / L)


# ---------------------------------------------------------------------------
# binning: bit-exact cells and stable cell order
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nc,shell,seed", [(10, 0.4, 1), (7, 0.0, 2), (13, 0.4, 3)])
def test_bin_cells_bit_exact(nc, shell, seed):
    pos, vel, L = fluid(nc, seed=seed)
    n = len(pos)
    s = _system(pos, vel, L, shell=shell)
    G = O.cells_per_edge(L, RC + shell)
    wrapped = O.wrap(pos, L)
    ref_cell = O.cell_ids(wrapped, L, G)
    assert np.array_equal(s.cells(), ref_cell)
    _, order, cs, _ = O.layers_reorder(ref_cell, G)
    got_order, got_cs = s.bins()
    assert np.array_equal(got_cs, cs)
    assert np.array_equal(got_order, order)
    # stand-alone re-binning of an already sorted system is the identity
    s.bin_cells()
    o2, cs2 = s.bins()
    assert np.array_equal(o2, order) and np.array_equal(cs2, cs)
    assert n % 256 != 0 or nc == 8
    s.close()


def test_bin_cells_even_rule_and_edges():
    # atoms exactly on the region faces and on cell faces
    pos, vel, L = fluid(9, amp=0.0, seed=4, shuffle=False)
    G = O.cells_per_edge(L, RC + 0.4, even=True)
    w = L / G
    pos[0] = [-L / 2, -L / 2, -L / 2]
    pos[1] = [np.nextafter(L / 2, 0), 0.0, 0.0]
    pos[2] = [-L / 2 + w, -L / 2 + 2 * w, 0.0]
    pos[3] = [L / 2, 0.0, -L / 2 - 0.1]        # outside: wrapped at creation
    s = _system(pos, vel, L, shell=0.4, even_cells=True)
    wrapped = O.wrap(pos, L)
    assert np.array_equal(s.cells(), O.cell_ids(wrapped, L, G))
    p, _, _, _ = s.get_state()
    assert np.array_equal(p, wrapped)
    s.close()


# ---------------------------------------------------------------------------
# neighbour matrix: bit-exact pair set
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nc,shell,seed", [(5, 0.4, 5), (10, 0.4, 6), (8, 0.8, 7)])
def test_neighbour_pairs_bit_exact(nc, shell, seed):
    pos, vel, L = fluid(nc, seed=seed, amp=0.25)
    s = _system(pos, vel, L, shell=shell)
    pi, pj = s.pairs()
    wrapped = O.wrap(pos, L)
    ref = O.pair_set(*O.pairs_cells(wrapped, L, O.cells_per_edge(L, RC + shell), RC + shell)[:2])
    if len(pos) <= 600:
        assert np.array_equal(ref, O.pair_set(*O.pairs_brute(wrapped, L, RC + shell)[:2]))
    # full list: every unordered pair twice, once from each side, never i == j
    assert len(pi) == 2 * len(ref)
    assert np.all(pi != pj)
    got = O.pair_set(pi, pj)
    assert np.array_equal(got, ref)
    fwd = set(zip(pi.tolist(), pj.tolist()))
    assert all((b, a) in fwd for a, b in list(fwd)[:2000])
    pr = s.props()
    assert pr["n_pairs"] == len(ref)
    s.close()


def test_fcc_start_has_twelve_neighbours_and_no_force():
    pos, L = I.fcc_lattice(10, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 3)
    s = _system(pos, vel, L, shell=0.4)
    pr = s.props()
    assert pr["n_pairs"] == 6 * len(pos) and pr["max_nebr"] == 12
    _, _, f, _ = s.get_state()
    assert np.all(f == 0.0) and pr["pe"] == 0.0 and pr["virial"] == 0.0
    s.close()


# ---------------------------------------------------------------------------
# forces and energies
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nc,amp,seed", [(6, 0.15, 8), (11, 0.2, 9)])
def test_forces_fp32_within_tolerance(nc, amp, seed):
    pos, vel, L = fluid(nc, amp=amp, seed=seed)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4, precision="fp32")
    _, _, f, _ = s.get_state()
    u, w = s.atom_energies()
    wrapped = O.wrap(pos, L)
    ref = O.forces_cells(wrapped, L, O.cells_per_edge(L, RC))
    assert force_error(f, ref.force) <= FORCE_TOL
    pr = s.props()
    assert abs(pr["pe"] - ref.pe) / n <= ENERGY_TOL * max(abs(ref.pe) / n, 1.0)
    assert abs(pr["virial"] - ref.virial) / n <= ENERGY_TOL * max(abs(ref.virial) / n, 1.0)
    assert abs(pr["ke"] - 0.5 * (vel ** 2).sum()) <= 1e-12 * pr["ke"]
    # per-atom diagnostics: FP32 sums of a few pair terms
    assert np.abs(u - ref.u_atom).max() <= 1e-5 * max(np.abs(ref.u_atom).max(), 1.0)
    assert np.abs(w - ref.w_atom).max() <= 1e-5 * max(np.abs(ref.w_atom).max(), 1.0)
    assert np.abs(f.sum(0)).max() <= 1e-4 * math.sqrt(n) * math.sqrt((ref.force ** 2).sum(1).mean())
    s.close()


@pytest.mark.parametrize("shell", [0.0, 0.4])
def test_forces_fp64(shell):
    pos, vel, L = fluid(7, amp=0.2, seed=10)
    n = len(pos)
    s = _system(pos, vel, L, shell=shell, precision="fp64")
    _, _, f, _ = s.get_state()
    ref = O.forces_cells(O.wrap(pos, L), L, O.cells_per_edge(L, RC))
    assert force_error(f, ref.force) <= 1e-12
    pr = s.props()
    assert abs(pr["pe"] - ref.pe) / n <= 1e-13 * max(abs(ref.pe) / n, 1.0)
    assert abs(pr["virial"] - ref.virial) / n <= 1e-13 * max(abs(ref.virial) / n, 1.0)
    s.close()


def test_sc_lattice_closed_form_on_gpu():
    # PE/N = 0.2352, W/N = 12.9024 for sc at rho = 0.8 (worked in the oracle
    # pins).  Every pair has the same separation, so FP32 rounding of the pair
    # terms is systematic here (it does not average out over pairs); held to
    # the stated bar 1e-6 max(|X/N|, 1) all the same.
    pos, L = I.sc_lattice(20, 0.8)
    vel = np.zeros_like(pos)
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-12)):
        s = _system(pos, vel, L, shell=0.4, precision=prec)
        pr = s.props()
        e_pe = abs(pr["pe_per_atom"] - 0.2352)
        e_w = abs(pr["virial_per_atom"] - 12.9024)
        print(f"sc lattice {prec}: PE/N error {e_pe:.3e}, W/N error {e_w:.3e}", flush=True)
        assert e_pe < tol * max(0.2352, 1.0) and e_w < tol * 12.9024
        s.close()


# ---------------------------------------------------------------------------
# trajectories
# ---------------------------------------------------------------------------

def test_cell_only_fp64_trajectory_matches_oracle():
    # the small workload's method: cell lists only, FP64 throughout
    pos, L = I.fcc_lattice(8, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 1)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.0, precision="fp64")
    ref = O.Sim(pos, vel, L, shell=0.0)
    for chunk in (1, 9, 90, 100):
        s.step(chunk)
        tr = ref.run(chunk)
        p, v, f, step = s.get_state()
        rp, rv, rf, _ = ref.state()
        assert np.abs(min_image(p - rp, L)).max() < 1e-9
        assert np.abs(v - rv).max() < 1e-8
        pr = s.props()
        assert abs(pr["ke"] - tr[-1, 0]) / n < 1e-10
        assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-10
    assert step == 200
    s.close()


def test_neighbour_list_fp32_trajectory_matches_oracle():
    pos, vel, L = fluid(10, amp=0.05, seed=11, temp=1.0)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4, precision="fp32")
    ref = O.Sim(pos, vel, L, shell=0.4)
    s.step(30)
    tr = ref.run(30)
    p, v, f, step = s.get_state()
    rp, rv, rf, _ = ref.state()
    assert step == 30
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    assert force_error(f, rf) < 1e-4
    pr = s.props()
    assert abs(pr["pe"] - tr[-1, 1]) / n < 1e-5
    assert abs(pr["ke"] - tr[-1, 0]) / n < 1e-5
    assert pr["n_rebuilds"] == int(tr[:, 5].sum())
    s.close()


def test_energy_and_momentum_conservation_10k_steps():
    pos, L = I.fcc_lattice(10, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 12)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4, precision="fp32")
    e = []
    for _ in range(100):
        s.step(100)
        pr = s.props()
        e.append((pr["ke"] + pr["pe"]) / n)
    e = np.array(e)
    drift = abs(e[-10:].mean() - e[:10].mean()) / abs(e[:10].mean())
    assert drift < 2e-4
    _, v, _, step = s.get_state()
    assert step == 10000
    # Pair forces are exactly antisymmetric (same FP32 arithmetic on -d), but
    # each atom sums its own pairs in FP32, so the total force per step is a
    # sum of N roundings: |sum F| ~ sqrt(N) 2^-24 F_rms, and the momentum
    # random-walks as sqrt(steps) dt of that.  Bound: 10x that with F_rms 50.
    bound = 10 * math.sqrt(10000) * 0.005 * math.sqrt(n) * 2.0 ** -24 * 50
    assert np.abs(v.sum(0)).max() < bound
    assert s.props()["n_rebuilds"] > 500
    s.close()


def test_resume_is_bit_identical():
    pos, vel, L = fluid(8, amp=0.1, seed=13)
    a = _system(pos, vel, L, shell=0.4)
    a.step(64)
    a.step(36)
    b = _system(pos, vel, L, shell=0.4)
    b.step(100)
    pa, va, fa, _ = a.get_state()
    pb, vb, fb, _ = b.get_state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb) and np.array_equal(fa, fb)
    a.close()
    b.close()


def test_cell_layer_overflow_is_bit_identical():
    # rows beyond the per-cell capacity go to an overflow list that is read in
    # the same ascending order, so a capacity of 2 changes nothing
    pos, vel, L = fluid(7, amp=0.1, seed=14)
    big = _system(pos, vel, L, shell=0.4)
    small = _system(pos, vel, L, shell=0.4, cell_cap=2)
    big.step(70)
    small.step(70)
    pa, va, _, _ = big.get_state()
    pb, vb, _, _ = small.get_state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    big.close()
    small.close()


def test_neighbour_overflow_stays_exact():
    # atoms whose list exceeds the capacity are evaluated from the cells every
    # step: the same pairs, summed in cell order (rounding differs only)
    pos, vel, L = fluid(7, amp=0.1, seed=15)
    big = _system(pos, vel, L, shell=0.4)
    small = _system(pos, vel, L, shell=0.4, nebr_cap=4)
    assert small.props()["max_nebr"] > 4
    _, _, fa, _ = big.get_state()
    _, _, fb, _ = small.get_state()
    assert force_error(fb, fa) < 1e-5
    big.step(50)
    small.step(50)
    pa, va, _, _ = big.get_state()
    pb, vb, _, _ = small.get_state()
    assert np.abs(min_image(pa - pb, L)).max() < 1e-6
    big.close()
    small.close()


def test_forces_call_reproduces_creation_forces():
    pos, vel, L = fluid(6, amp=0.2, seed=16)
    s = _system(pos, vel, L, shell=0.4)
    _, _, f0, _ = s.get_state()
    s.forces()
    _, _, f1, _ = s.get_state()
    assert np.array_equal(f0, f1)
    s.close()


def test_bin_cells_then_step_matches_oracle():
    pos, vel, L = fluid(8, amp=0.05, seed=17)
    n = len(pos)
    s = _system(pos, vel, L, shell=0.4)
    ref = O.Sim(pos, vel, L, shell=0.4)
    s.step(37)
    ref.run(37)
    s.bin_cells()                       # wrap, re-bin, reorder, rebuild at step 37
    order, cs = s.bins()
    p, _, _, _ = s.get_state()
    G = O.cells_per_edge(L, RC + 0.4)
    cells = O.cell_ids(p, L, G)
    assert np.all(np.diff(cells[order]) >= 0)          # storage is in cell order
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(np.bincount(cells, minlength=G ** 3))]))
    s.step(20)
    ref.run(20)
    p, v, _, step = s.get_state()
    rp, rv, _, _ = ref.state()
    assert step == 57
    assert np.abs(min_image(p - rp, L)).max() < 1e-6
    s.close()


def _run_batch(specs, steps_per_run=64, stagger=None):
    from paper_0911_5631_amd.md import Batch
    b = Batch(1 << 31, 8, steps_per_run)
    slots = {}
    pending = list(range(len(specs)))
    if stagger:
        first, later = pending[:stagger], pending[stagger:]
    else:
        first, later = pending, []
    def admit(k):
        pos, vel, L, n_steps = specs[k][:4]
        prm = specs[k][4] if len(specs[k]) > 4 else {"shell": 0.4}
        slots[b.admit(pos, vel, L, n_steps, **prm)] = k

    for k in first:
        admit(k)
    out = {}
    runs = 0
    while len(out) < len(specs):
        b.run()
        runs += 1
        if runs == 1:
            for k in later:
                admit(k)
        for slot in b.poll():
            if slot in slots and slots[slot] not in out:
                p, v, step = b.get_state(slot)
                out[slots[slot]] = (p, v, step, b.props(slot))
                b.release(slot)
        assert runs < 100
    b.close()
    return out


def test_batch_equals_solo_bit_for_bit():
    specs = []
    for k, (nc, rho, T, steps) in enumerate([(4, 0.8, 1.0, 150), (6, 0.7, 1.5, 100),
                                            (7, 0.9, 0.8, 200), (5, 0.85, 1.2, 64)]):
        pos, L = I.fcc_lattice(nc, rho)
        vel = I.random_velocities(len(pos), T, 40 + k)
        specs.append((pos, vel, L, steps))
    got = _run_batch(specs, stagger=2)
    for k, (pos, vel, L, steps) in enumerate(specs):
        s = _system(pos, vel, L, shell=0.4)
        s.step(steps)
        p, v, _, step = s.get_state()
        pr = s.props()
        gp, gv, gstep, gpr = got[k]
        assert gstep == step == steps
        assert np.array_equal(gp, p) and np.array_equal(gv, v), k
        assert gpr["n_rebuilds"] == pr["n_rebuilds"]
        assert gpr["pe"] == pr["pe"] and gpr["ke"] == pr["ke"]
        s.close()


def test_mixed_batch_equals_solo_bit_for_bit():
    """One batch holding FP32 and FP64 replicas of both potentials (the
    soft-sphere cutoff and LJ at r_c = 2.5 with a wider shell): each
    precision is its own step-kernel launch over the shared tables, each
    replica its own cutoff and list radius, and every trajectory equals the
    same system run alone."""
    specs = []
    for k, (prec, lj) in enumerate([("fp32", False), ("fp64", False), ("fp32", True),
                                    ("fp64", True), ("fp64", False)]):
        if lj:
            pos, L = I.sc_lattice(11 + k, 0.38)
            pos = I.jitter(pos, L, 0.1, 60 + k)
            vel = I.random_velocities(len(pos), 1.2, 70 + k)
            prm = {"r_cut": 2.5, "shell": 0.8, "precision": prec}
        else:
            pos, vel, L = fluid(4 + k, seed=80 + k)
            prm = {"shell": 0.4, "precision": prec}
        specs.append((pos, vel, L, 90 + 17 * k, prm))
    got = _run_batch(specs, steps_per_run=32, stagger=3)
    for k, (pos, vel, L, steps, prm) in enumerate(specs):
        s = _system(pos, vel, L, **prm)
        s.step(steps)
        p, v, _, step = s.get_state()
        pr = s.props()
        s.close()
        gp, gv, gstep, gpr = got[k]
        assert gstep == step == steps
        assert np.array_equal(gp, p) and np.array_equal(gv, v), (k, prm)
        assert gpr["n_rebuilds"] == pr["n_rebuilds"] and gpr["n_rebuilds"] > 0
        assert gpr["pe"] == pr["pe"] and gpr["ke"] == pr["ke"]


def test_one_slot_batch_reused_equals_solo():
    """A batch of one slot (its sort then takes the single-system path: idle
    workgroups stop after their first unit) run twice, the slot released and
    re-admitted in between, equals the systems run alone."""
    from paper_0911_5631_amd.md import Batch
    specs = [fluid(6, seed=71) + (170,), fluid(5, seed=72) + (90,)]
    b = Batch(1 << 31, 1, 32)
    got = []
    for pos, vel, L, steps in specs:
        slot = b.admit(pos, vel, L, steps, shell=0.4)
        assert slot == 0
        for _ in range(20):
            b.run()
            if b.poll():
                break
        got.append(b.get_state(slot) + (b.props(slot),))
        b.release(slot)
    b.close()
    for (pos, vel, L, steps), (gp, gv, gstep, gpr) in zip(specs, got):
        s = _system(pos, vel, L, shell=0.4)
        s.step(steps)
        p, v, _, step = s.get_state()
        pr = s.props()
        s.close()
        assert gstep == step == steps
        assert np.array_equal(gp, p) and np.array_equal(gv, v)
        assert gpr["n_rebuilds"] == pr["n_rebuilds"] > 0 and gpr["pe"] == pr["pe"]


def test_batch_admission_respects_budget():
    from paper_0911_5631_amd.md import Batch, md_query_bytes, make_params
    pos, L = I.fcc_lattice(6, 0.8)
    vel = I.random_velocities(len(pos), 1.0, 3)
    need = md_query_bytes(make_params(len(pos), L, shell=0.4))
    b = Batch(int(need * 1.5), 4, 64)
    assert b.try_admit(pos, vel, L, 10, shell=0.4) is not None
    assert b.try_admit(pos, vel, L, 10, shell=0.4) is None          # over budget: queue it
    used, k = b.usage()
    assert k == 1 and used == need
    b.close()


def test_errors_are_reported():
    from paper_0911_5631_amd._lib import MDError
    pos, vel, L = fluid(5, seed=15)
    bad = pos.copy()
    bad[7, 1] = np.nan
    with pytest.raises(MDError) as e:
        _system(bad, vel, L, shell=0.4)
    assert e.value.code == -7
    far = pos.copy()
    far[3, 0] = 2.0 * L
    with pytest.raises(MDError) as e:
        _system(far, vel, L, shell=0.4)
    assert e.value.code == -6
    with pytest.raises(MDError) as e:
        _system(pos[:10], vel[:10], 3.0, shell=0.4)
    assert e.value.code == -2


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-6)])
def test_rebuild_the_step_before_did_not_bin_for(precision, tol):
    """Positions are binned one step ahead only when the displacement rule
    could fire at the next step, judged from the previous maximum speed.  A
    lattice nearly at rest with one pair pushed to r = 0.9 and a shell of
    0.004: the pair's repulsion takes the maximum speed from 0.01 to ~0.7 in
    one step, so the rule fires at step 2 without rows; the library bins the
    held positions and resumes.  The trajectory and the rebuild steps equal
    the oracle's, in a single system and in a batch."""
    from paper_0911_5631_amd.md import Batch
    pos, L = I.sc_lattice(8, 0.5)
    rng = np.random.Generator(np.random.PCG64(61))
    vel = rng.uniform(-0.005, 0.005, pos.shape)
    vel -= vel.mean(0)
    d = pos[1] - pos[0]
    d -= L * np.round(d / L)
    pos[0] = pos[1] - d / np.linalg.norm(d) * 0.9
    n = len(pos)
    s = _system(pos, vel, L, shell=0.004, precision=precision)
    sim = O.Sim(pos, vel, L, shell=0.004)
    s.step(40)
    tr = sim.run(40)
    pr = s.props()
    p, v, _, step = s.get_state()
    rp, rv, _, _ = sim.state()
    sim.close()
    s.close()
    assert step == 40 and pr["n_late_bins"] >= 1
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) >= 2
    assert np.abs(min_image(p - rp, L)).max() < tol
    assert abs(pr["pe"] - tr[-1, 1]) / n < 10 * tol
    b = Batch(1 << 30, 2, 16)
    slot = b.admit(pos, vel, L, 40, shell=0.004, precision=precision)
    for _ in range(10):
        b.run()
        if b.poll():
            break
    bp, bv, bstep = b.get_state(slot)
    bpr = b.props(slot)
    b.close()
    assert bstep == 40 and bpr["n_late_bins"] == pr["n_late_bins"]
    assert np.array_equal(bp, p) and np.array_equal(bv, v)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_binning_ahead_covers_every_rebuild_of_a_fluid(precision):
    """Sec. 3.1's rule rebuilds when the accumulated max-speed displacement
    passes delta/2; positions are binned one step ahead when the same rule,
    with 1.5 times the last maximum speed, could fire at the next step (the
    sort kernel takes that decision for the step kernel).  In an ordinary
    fluid the maximum speed never grows 1.5-fold in one step, so every
    rebuild must find its rows binned ahead: no late binning, and the
    rebuild steps and the final state equal the oracle's."""
    pos, L = I.fcc_lattice(8, 0.8)                      # 2 048 atoms
    pos = I.jitter(pos, L, 0.05, 91)
    vel = I.random_velocities(len(pos), 1.0, 92)
    n, steps = len(pos), 300
    s = _system(pos, vel, L, shell=0.3, precision=precision)
    sim = O.Sim(pos, vel, L, shell=0.3)
    s.step(steps)
    tr = sim.run(steps)
    pr = s.props()
    p, _, _, step = s.get_state()
    rp, _, _, _ = sim.state()
    sim.close()
    s.close()
    assert step == steps and pr["n_late_bins"] == 0
    assert pr["n_rebuilds"] == int(tr[:, 5].sum()) >= 10
    tol = 1e-9 if precision == "fp64" else 1e-5
    assert np.abs(min_image(p - rp, L)).max() < tol
