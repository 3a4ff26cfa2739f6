"""Seeded input generators (shared by the oracle tests and the GPU path; they
hold none of the method's arithmetic): shapes, ranges, determinism."""
import math

import numpy as np

from paper_0911_5631_amd import inputs as I


def test_fcc_lattice_geometry():
    pos, L = I.fcc_lattice(5, 0.8)
    assert pos.shape == (500, 3) and abs(L - (500 / 0.8) ** (1 / 3)) < 1e-12
    assert (pos >= -L / 2).all() and (pos < L / 2).all()
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    a = L / 5
    assert abs(r.min() - a / math.sqrt(2)) < 1e-9          # fcc nearest neighbour
    assert (np.isclose(r, a / math.sqrt(2)).sum(1) == 12).all()


def test_random_velocities():
    v = I.random_velocities(4000, 1.3, 7)
    assert np.allclose(v.mean(0), 0.0, atol=1e-12)
    sp = np.linalg.norm(v + 0, axis=1)
    # speeds sqrt(3T) before the mean is removed: the mean is O(1/sqrt(N))
    assert abs(sp.mean() - math.sqrt(3 * 1.3)) < 0.02
    assert np.array_equal(v, I.random_velocities(4000, 1.3, 7))


def test_replica_batch_ranges():
    reps = I.replica_batch(n_replicas=40, k_lo=6, k_hi=20, steps=10, seed=4)
    for s in reps:
        k = round((s.n / 4) ** (1 / 3))
        assert 6 <= k <= 20 and s.n == 4 * k ** 3
        assert 0.7 <= s.rho <= 0.9 and 0.8 <= s.temperature <= 1.5
    again = I.replica_batch(n_replicas=40, k_lo=6, k_hi=20, steps=10, seed=4)
    assert all(np.array_equal(a.vel, b.vel) for a, b in zip(reps, again))


def test_served_stream_is_lazy_and_poisson():
    reqs = I.served_stream(n_requests=3000, rate=50.0, seed=5)
    t = np.array([r.arrival for r in reqs])
    assert (np.diff(t) > 0).all()
    assert abs(np.diff(t).mean() - 1 / 50.0) < 0.1 / 50.0     # mean gap 1/rate
    assert all(not hasattr(r, "pos") for r in reqs)          # parameters only
    r = reqs[0]
    s1, s2 = r.system(), r.system()
    assert s1.n == r.n == 4 * r.n_cells ** 3 and s1.steps == r.steps
    assert np.array_equal(s1.pos, s2.pos) and np.array_equal(s1.vel, s2.vel)
    assert 1000 <= min(q.steps for q in reqs) and max(q.steps for q in reqs) <= 20000
