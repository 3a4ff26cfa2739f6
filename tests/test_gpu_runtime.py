"""The runtime around the step on the GPU: where device memory comes from
(torch's caching allocator, or the library's own hipMalloc when no
allocator is given), which stream the work is ordered on (the caller's
current stream, or another one), and how the step kernel is launched
(graph replays, or one event-bracketed launch per step under md_profile).

Bar: every combination gives the same trajectory bit for bit, since none
of them changes the arithmetic or the order of any sum; the profiled run
counts exactly one step-kernel launch per step.
"""
import numpy as np
import pytest

from paper_0911_5631_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _start():
    pos, L = I.fcc_lattice(7, 0.8)                 # 1 372 atoms: 6 tiles, ragged tail
    pos = I.jitter(pos, L, 0.1, seed=31)
    vel = I.random_velocities(len(pos), 1.0, 32)
    pos, vel = I.shuffled(pos, vel, 33)
    return pos, vel, L


def _run(pos, vel, L, steps, **kw):
    from paper_0911_5631_amd.md import System
    s = System(pos, vel, L, shell=0.4, **kw)
    s.step(steps)
    out = s.get_state(), s.props()
    s.close()
    return out


def _same(a, b):
    (pa, va, fa, ka), pra = a
    (pb, vb, fb, kb), prb = b
    assert ka == kb
    assert np.array_equal(pa, pb) and np.array_equal(va, vb) and np.array_equal(fa, fb)
    for key in ("ke", "pe", "virial", "n_rebuilds"):
        assert pra[key] == prb[key], key


def test_allocator_and_stream_leave_the_trajectory_unchanged():
    import torch
    pos, vel, L = _start()
    ref = _run(pos, vel, L, 150)
    assert ref[1]["n_rebuilds"] > 3
    _same(_run(pos, vel, L, 150, allocator="hip"), ref)
    side = torch.cuda.Stream()
    _same(_run(pos, vel, L, 150, stream=side), ref)


def test_work_waits_for_the_callers_stream():
    """Device work of a call is ordered after what the caller's stream
    already holds: a copy into a torch tensor enqueued behind a long kernel
    on that stream, and the library's steps enqueued behind both, end in the
    same state as when nothing was pending."""
    import torch
    from paper_0911_5631_amd.md import System
    pos, vel, L = _start()
    ref = _run(pos, vel, L, 80)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = torch.randn(2048, 2048, device="cuda")
        s = System(pos, vel, L, shell=0.4, stream=side)
        for _ in range(8):
            a = a @ a / 64.0                           # pending work on the side stream
        s.step(80)
        b = a.clone()
    side.synchronize()
    assert torch.isfinite(b).all()
    got = s.get_state(), s.props()
    s.close()
    _same(got, ref)


def test_profiled_launches_equal_graph_replays():
    from paper_0911_5631_amd.md import System
    pos, vel, L = _start()
    ref = _run(pos, vel, L, 150)
    s = System(pos, vel, L, shell=0.4)
    s.step(50)
    s.profile(True)
    s.step(100)
    n, ms = s.kernel_time()
    s.profile(False)
    got = s.get_state(), s.props()
    s.close()
    assert n == 100 and ms > 0.0
    _same(got, ref)
