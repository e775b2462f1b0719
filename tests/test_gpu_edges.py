"""Degenerate and boundary cases of the stepping path, through the C-ABI:
zero steps, a sample at zero steps, and the smallest lattices (one quad wide,
two rows high) against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def wrapped_diff(a, b):
    return np.abs(np.remainder(np.asarray(a) - np.asarray(b) + np.pi, 2 * np.pi) - np.pi)


SPEC = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.5)], seed=2, replica=1)


@pytest.mark.parametrize("dtype,fusion", [("f32", 2), ("f32", 1), ("f64", 1)])
def test_zero_steps_change_nothing(xyl, dtype, fusion):
    lat = xyl.Lattice(256, 16, dtype=dtype, **SPEC)
    lat.set_fusion(fusion)
    lat.init_random()
    lat.step(7)
    before = lat.get_state()
    lat.step(0)
    after = lat.get_state()
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    assert before[2] == after[2] == 7
    # a sampled run of zero steps: one sample, at the current step, equal to measure()
    s = lat.step_measured(0, 10)
    assert s.shape == (1, 6)
    np.testing.assert_array_equal(s[0], lat.measure())
    assert lat.step_index == 7
    lat.close()


@pytest.mark.parametrize("Lx,Ly", [(4, 2), (4, 9), (12, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_smallest_lattices_match_oracle(xyl, Lx, Ly, dtype):
    """One quad per row (Lx = 4: a lane is its own left and right neighbour
    across the periodic seam) and two rows (each row both y-neighbours of the
    other) against the oracle from the same start: FP64 over 300 steps to
    1e-12, FP32 over 100 steps to 1e-4."""
    say("smallest", Lx, Ly, dtype)
    lat = xyl.Lattice(Lx, Ly, dtype=dtype, **SPEC)
    o = oracle.Oracle(Lx, Ly, **SPEC)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    n = 300 if dtype == "f64" else 100
    s = lat.step_measured(n, 50)
    th, _, k = lat.get_state()
    tr, wr, so = o.run(th0, om0, 0, n, every=50)
    assert k == n
    d = wrapped_diff(th, tr).max()
    say("max|dtheta|", d)
    if dtype == "f64":
        assert d <= 1e-12
        np.testing.assert_allclose(s, so, rtol=1e-10, atol=1e-12)
    else:
        assert d <= 1e-4
        np.testing.assert_allclose(s, so, rtol=1e-4, atol=1e-5)
    lat.close()
