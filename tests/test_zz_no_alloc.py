"""md_newton3_ab_noalloc, the A/B entry point that allocates no device
memory (its buffers live in a static device array), against md_newton3_ab,
which allocates them: called through the C ABI on two systems in a row, the
second smaller than the first (what the first call left in the shared array
must not leak into the second).  Full list: forces bit for bit (same kernels,
same inputs, no atomics); half list: the reactions are added with atomics in
an unspecified order, so forces agree within the FP32 force bar; list
entries equal.  A system beyond the array's size is refused before any work.
"""
import math

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


def _force_error(f, ref):
    scale = np.maximum(np.linalg.norm(ref, axis=1), math.sqrt((ref ** 2).sum(1).mean()))
    return float((np.linalg.norm(f - ref, axis=1) / scale).max())


def test_noalloc_matches_allocating_entry_point_twice():
    from paper_0911_5631_amd.md import System
    for nc, steps, seed in ((14, 40, 3), (7, 25, 4)):          # 10 976 atoms, then 1 372
        pos, L = I.fcc_lattice(nc, 0.8)
        pos = I.jitter(pos, L, 0.1, seed)
        vel = I.random_velocities(len(pos), 1.0, seed + 10)
        s = System(pos, vel, L, shell=0.4)
        s.step(steps)
        for half in (False, True):
            ref = s.newton3_ab(half, reps=2)
            got = s.newton3_ab(half, reps=2, noalloc=True)
            assert got["n_entries"] == ref["n_entries"] > 0
            if half:
                assert _force_error(got["force"], ref["force"]) <= 1e-5
            else:
                assert np.array_equal(got["force"], ref["force"])
        s.close()


def test_noalloc_refuses_a_system_beyond_its_array():
    from paper_0911_5631_amd._lib import MDError
    from paper_0911_5631_amd.md import System
    pos, L = I.fcc_lattice(44, 0.8)                              # 340 736 atoms
    vel = I.random_velocities(len(pos), 1.0, 5)
    s = System(pos, vel, L, shell=0.4)
    with pytest.raises(MDError) as e:
        s.newton3_ab(False, noalloc=True)
    assert e.value.code == -3
    assert s.props()["step"] == 0                                # nothing ran
    s.close()
