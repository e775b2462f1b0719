"""The oracle against itself: how far two FP64 runs drift apart when their
rounding differs.  These numbers fix the GPU parity bars that are looser than
the headline ones, so that the bars rest on a property of the dynamics that
anyone can recompute, not on a kernel's result.

Si(001) mapping (Sec. III.C: q = 2, field -h cos(p th) with p = 2.5, angles on
the half circle with a modulo after every step, Sec. III.D).  The field is not
pi-periodic, so its force jumps where an angle crosses +-pi/2: a site that one
run puts just above the boundary and the other just below takes a different
kick, and its neighbourhood follows.

* FP32 storage.  The oracle advanced one step at a time with its state rounded
  to binary32 after every step (what an FP32 kernel stores), against the plain
  FP64 oracle, 20 steps of the 4096^2 benchmark lattice at T_c: a handful of
  sites end beyond 1e-4 (at 9.4e-3 the worst), all but a 1e-5 fraction stay
  below it.  That is the bar tests/test_gpu_fullsize.py applies to the Si model
  (the XY model, whose field is 2 pi-periodic, keeps 1e-4 at every site: the
  same experiment at 2048^2 stays below 2e-6).
* FP32 arithmetic.  The same with one to four ulps of random relative error
  added to every angle and velocity after each step (the size of an FP32
  kernel's rounding), on the small lattices of tests/test_gpu_si.py, 100
  steps: some noise streams cross the cusp (at 64^2 the 1-ulp ones reproduce
  the GPU's 5.6e-3 at 6 sites), but none moves more than 1% of the sites
  beyond 1e-4 or the median beyond 1e-5 (it stays near 1e-6).  That is the
  FP32 bar of the small Si tests; a wrong force, draw or index moves most
  sites by far more.
* FP64 rounding.  Starts that differ by one ulp at every site (random
  direction) end 0.8-2e-10 apart after the 1000-step Si schedule of
  tests/test_gpu_si.py at 64^2 (3-5e-12 after 200 steps), while the XY model's
  spread stays below 1e-12.  The GPU's FP64 force (sine/cosine products) and
  the oracle's (sines of differences) differ by a few ulps per step, so the
  Si bars there are 1.2e-9 at 1000 steps and 6e-11 at 200, at least five times
  the spread measured here; the XY bar stays 1e-12.
"""
import numpy as np
import pytest

import oracle
from paper_2409_06412_amd import workloads


def wrapped(a, b, period):
    h = period / 2
    return np.abs(np.remainder(np.asarray(a) - np.asarray(b) + h, period) - h)


def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def run_f32_storage(o, th, om, nsteps, si):
    """The oracle's steps with the state rounded to binary32 after each one
    (and, for the half circle, mapped back if the rounding reached +pi_32/2)."""
    half = np.float64(np.float32(np.pi / 2))
    for k in range(nsteps):
        th, om = o.run(th, om, k, 1)
        th, om = to_f32(th), to_f32(om)
        if si:
            th = np.where(th >= half, th - np.float64(np.float32(np.pi)), th)
    return th, om


@pytest.mark.slow
def test_si_fp32_storage_sensitivity_at_full_size():
    L, nsteps = 4096, 20
    spec = workloads.si_lattice(L, L, seed=1)
    o = oracle.Oracle(**spec.oracle_kwargs())
    th0, om0 = o.init_random()
    th0 = to_f32(th0)
    a, _ = o.run(th0, om0, 0, nsteps)
    b, _ = run_f32_storage(o, th0, om0, nsteps, si=True)
    d = wrapped(a, b, np.pi)
    n_out = int(np.count_nonzero(d > 1e-4))
    # a bar of 1e-4 at every site is out of reach of FP32 storage itself ...
    assert n_out >= 1 and d.max() > 1e-3
    # ... while the bar the full-size GPU test uses holds for it
    assert n_out <= 1e-5 * L * L
    assert np.quantile(d, 1 - 1e-5) <= 1e-4


@pytest.mark.slow
def test_xy_fp32_storage_keeps_the_strict_bar():
    L, nsteps = 2048, 20
    spec = workloads.large_fp32(0, L)
    o = oracle.Oracle(**spec.oracle_kwargs())
    th0, om0 = o.init_random()
    th0 = to_f32(th0)
    a, _ = o.run(th0, om0, 0, nsteps)
    b, _ = run_f32_storage(o, th0, om0, nsteps, si=False)
    assert wrapped(a, b, 2 * np.pi).max() <= 1e-5


def run_with_arithmetic_noise(o, th, om, nsteps, ulps, rng):
    """The oracle's steps with the state perturbed by up to `ulps` binary32
    ulps (random relative error, uniform) and rounded to binary32 after each
    step, mapped back onto the half circle."""
    half, full = np.float64(np.float32(np.pi / 2)), np.float64(np.float32(np.pi))
    for k in range(nsteps):
        th, om = o.run(th, om, k, 1)
        th = to_f32(th * (1.0 + ulps * 2.0 ** -24 * rng.uniform(-1.0, 1.0, th.shape)))
        om = to_f32(om * (1.0 + ulps * 2.0 ** -24 * rng.uniform(-1.0, 1.0, om.shape)))
        th = np.where(th >= half, th - full, np.where(th < -half, th + full, th))
    return th, om


@pytest.mark.parametrize("Lx,Ly", [(64, 64), (300, 20)])
def test_si_fp32_arithmetic_noise_small_lattices(Lx, Ly):
    """The start of tests/test_gpu_si.py::test_fp32_parity, 100 steps."""
    spec = workloads.si_lattice(Lx, Ly, seed=3)
    o = oracle.Oracle(**spec.oracle_kwargs())
    th0, om0 = o.init_random()
    th0 = to_f32(th0)
    ref, _ = o.run(th0, om0, 0, 100)
    crossed = 0
    for ulps in (1, 4):
        for s in range(6):
            b, _ = run_with_arithmetic_noise(o, th0, om0, 100, ulps, np.random.default_rng(100 + s))
            d = wrapped(ref, b, np.pi)
            n_out = int(np.count_nonzero(d > 1e-4))
            crossed += n_out > 0
            assert n_out <= 0.01 * Lx * Ly
            assert np.median(d) <= 1e-5
    # a per-site 1e-4 bar over 100 steps is out of reach of FP32 rounding here
    assert crossed >= 2


def ulp_spread(o, th0, om0, nsteps, period, seeds=(0, 1, 2, 3)):
    """Largest final distance between the run from th0 and runs from th0
    moved by one ulp at every site in a random direction."""
    ref, _ = o.run(th0, om0, 0, nsteps)
    out = []
    for s in seeds:
        d = np.random.default_rng(s).choice([-1.0, 1.0], size=th0.shape)
        thp = np.nextafter(th0, th0 + d)
        if period == np.pi:      # stay on the half circle [-pi/2, pi/2)
            thp = np.where(thp >= np.pi / 2, th0, thp)
        tr, _ = o.run(thp, om0, 0, nsteps)
        out.append(wrapped(tr, ref, period).max())
    return max(out), min(out)


@pytest.mark.parametrize("Lx,Ly,nsteps,bar", [(64, 64, 1000, 1.2e-9), (260, 37, 200, 6e-11)])
def test_si_fp64_rounding_spread(Lx, Ly, nsteps, bar):
    """The schedule and start of tests/test_gpu_si.py::test_fp64_parity."""
    spec = workloads.si_lattice(Lx, Ly, seed=11, replica=2)
    kw = spec.oracle_kwargs()
    kw["schedule"] = [(0, 1.3 * workloads.SI_TC), (nsteps, 0.7 * workloads.SI_TC)]
    o = oracle.Oracle(**kw)
    th0, om0 = o.init_random()
    hi, lo = ulp_spread(o, th0, om0, nsteps, np.pi)
    # the strict FP64 bar (1e-12) is below what one ulp of rounding does here ...
    assert lo > 1e-12
    # ... and the bar used instead is at least five times the spread
    assert 5 * hi <= bar


def test_xy_fp64_rounding_spread_below_strict_bar():
    spec = workloads.small_fp64()
    o = oracle.Oracle(**spec.oracle_kwargs())
    th0, om0 = o.init_random()
    hi, _ = ulp_spread(o, th0, om0, 1000, 2 * np.pi, seeds=(0, 1))
    assert hi < 1e-12
