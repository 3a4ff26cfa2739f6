"""Batched replicas and served requests against the FP64 CPU oracle.

A batch of 64 replicas drawn like the replica workload (N = 4 k^3 with k ~
U{6..20}, rho ~ U[0.7, 0.9], T ~ U[0.8, 1.5]), every other one FP64, with
uneven step counts of 50-80 (every replica rebuilds on the way), admitted
together and run to completion in one batch; then requests of a Poisson
trace served through the serving loop.  Each system's final positions,
velocities, kinetic and potential energy, virial and rebuild count are
compared with the oracle's own trajectory of the same start.

Bars (trajectories from an fcc start through rebuilds):
  FP64 replicas: positions 1e-9, velocities 1e-8, energies per atom 1e-10
    (summation order only);
  FP32 replicas: positions 1e-6, velocities 1e-4, energies per atom 1e-5
    (FP32 pair forces on an FP64 trajectory, the bars of the single-system
    trajectory tests);
  rebuild counts equal.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu

BARS = {"fp64": (1e-9, 1e-8, 1e-10), "fp32": (1e-6, 1e-4, 1e-5)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def min_image(d, L):
    return d - L * np.round(d / L)


def _compare(name, pos0, vel0, L, shell, steps, precision, got_p, got_v, got_props):
    sim = O.Sim(pos0, vel0, L, shell=shell, dt=0.005)
    tr = sim.run(steps)
    rp, rv, _, _ = sim.state()
    sim.close()
    n = len(pos0)
    tp, tv, te = BARS[precision]
    errs = {"pos": float(np.abs(min_image(got_p - rp, L)).max()),
            "vel": float(np.abs(got_v - rv).max()),
            "ke": abs(got_props["ke"] - tr[-1, 0]) / n,
            "pe": abs(got_props["pe"] - tr[-1, 1]) / n,
            "virial": abs(got_props["virial"] - tr[-1, 2]) / n}
    print(f"{name} {precision} n={n} steps={steps} " +
          " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert got_props["step"] == steps, name
    assert got_props["n_rebuilds"] == int(tr[:, 5].sum()) >= 1, name
    assert errs["pos"] < tp and errs["vel"] < tv, (name, errs)
    assert max(errs["ke"], errs["pe"], errs["virial"]) < te, (name, errs)
    return errs


def test_batch_of_64_uneven_replicas_matches_oracle():
    from paper_0911_5631_amd.md import Batch
    systems = I.replica_batch(n_replicas=64, k_lo=6, k_hi=20, steps=0, seed=81)
    steps = [50 + (7 * k) % 31 for k in range(64)]
    prec = ["fp64" if k % 2 else "fp32" for k in range(64)]
    b = Batch(16 << 30, 64, 32)
    slot_of = {}
    for k, s in enumerate(systems):
        slot_of[b.admit(s.pos, s.vel, s.box, steps[k], shell=s.shell, dt=s.dt,
                        precision=prec[k])] = k
    got = {}
    for _ in range(10):
        b.run()
        for slot in b.poll():
            k = slot_of[slot]
            if k not in got:
                p, v, step = b.get_state(slot)
                got[k] = (p, v, b.props(slot))
                assert step == steps[k]
                b.release(slot)
        if len(got) == len(systems):
            break
    b.close()
    assert len(got) == len(systems)
    worst = {}
    for k, s in enumerate(systems):
        p, v, pr = got[k]
        errs = _compare(s.name, s.pos, s.vel, s.box, s.shell, steps[k], prec[k], p, v, pr)
        w = worst.setdefault(prec[k], {})
        for key, e in errs.items():
            w[key] = max(w.get(key, 0.0), e)
    print("worst", worst, flush=True)


def test_served_requests_match_oracle():
    from paper_0911_5631_amd.md import make_params, md_query_bytes
    from paper_0911_5631_amd.server import serve
    reqs = I.served_stream(n_requests=12, rate=300.0, k_lo=6, k_hi=12, steps_lo=50,
                           steps_hi=120, seed=91)
    need = [md_query_bytes(make_params(r.n, r.system().box, shell=r.shell)) for r in reqs]
    res = serve(reqs, int(4.5 * max(need)), max_slots=8, steps_per_run=16, keep_state=True)
    assert res["n_requests"] == len(reqs)
    by_name = {r.name: r for r in reqs}
    for rec in res["served"]:
        s = by_name[rec.name].system()
        _compare(rec.name, s.pos, s.vel, s.box, s.shell, rec.steps, "fp32", rec.pos, rec.vel,
                 rec.props)
