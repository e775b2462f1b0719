"""The two batched workloads at full size, in the configuration bench.py times
(App. B: many subsystems advanced together):

* the 288-replica finite-size-scaling ensemble (side lengths 32 to 512, 16
  temperatures, two seeds), autotuned and sampled every 100 steps: two-step
  classes on their streams, issued pass by pass, and the small replicas
  whole-in-LDS;
* the 60-replica 2048^2 quench batch (three ramp times, two dampings, two
  fields, five seeds), autotuned and stepped 100 steps without samples, one
  batched two-step pass per two steps;
* the 4096^2 lattice at its eight temperatures, batched as bench.py runs it
  (one class of 16-wave rows), sampled every 50 steps.

Chosen replicas (one per side length, the two extreme quench parameter sets,
the coldest and the hottest 4096^2 replica) are compared with the FP64 oracle
run from the replica's own start: the angles at every site after 100 steps
(XY: 1e-4, the single-lattice full-size bar) and, for the sampled runs, the
observables of the samples with the bars of the single-lattice full-size
test."""
import sys

import numpy as np
import pytest

import oracle
from paper_2409_06412_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def wrapped_diff(a, b, period=2 * np.pi):
    h = period / 2
    return np.abs(np.remainder(np.asarray(a) - np.asarray(b) + h, period) - h)


def check_replica(spec, start, end, nsteps, samples=None, every=0, tag=""):
    th0, om0, k0 = start
    th, om, k = end
    assert k0 == 0 and k == nsteps
    o = oracle.Oracle(**spec.oracle_kwargs())
    if every:
        tr, wr, so = o.run(th0, om0, 0, nsteps, every=every)
    else:
        tr, wr = o.run(th0, om0, 0, nsteps)
    d = wrapped_diff(th, tr)
    dom = np.abs(om - wr).max()
    say(tag, "%dx%d" % (spec.Lx, spec.Ly), "T0", spec.schedule[0][1], "max|dtheta|", d.max(), "max|domega|", dom)
    assert d.max() <= 1e-4
    assert dom <= 1e-3
    if samples is None:
        return
    N = spec.Lx * spec.Ly
    assert samples.shape == so.shape == (nsteps // every + 1, 6)
    np.testing.assert_allclose(samples[:, :3], so[:, :3], rtol=1e-4, atol=2e-6)
    # F(q) over N unit rotors: a per-term FP32 rotor error of two ulps of 1
    # moves F by up to 2 sqrt(F N) delta (see the single-lattice test)
    bound = 1e-4 * np.abs(so[:, 3:]) + 2.0 * np.sqrt(np.abs(so[:, 3:]) * N) * 2.0 ** -22
    assert np.all(np.abs(samples[:, 3:] - so[:, 3:]) <= bound)


def test_fss_ensemble_full_size_matches_oracle(xyl):
    specs = workloads.fss_ensemble(nsteps=10 ** 9)
    assert len(specs) == 288
    nsteps, every = 100, 100
    ens = xyl.Ensemble(specs, dtype="f32")
    try:
        launch = ens.autotune()
        say("FSS ensemble: launch", launch, "steps per pass", ens.fusion())
        # one replica per side length, at different temperatures
        sizes = sorted({s.Lx for s in specs})
        picks = [next(r for r, s in enumerate(specs) if s.Lx == L and s.replica % 32 == (3 * i) % 32)
                 for i, L in enumerate(sizes)]
        start = {r: ens.get_state(r) for r in picks}
        samples = ens.step(nsteps, every=every)
        end = {r: ens.get_state(r) for r in picks}
    finally:
        ens.close()
    for r in picks:
        check_replica(specs[r], start[r], end[r], nsteps, samples[r], every, "FSS replica %d" % r)


def test_quench_batch_full_size_matches_oracle(xyl):
    specs = workloads.kz_quench()
    assert len(specs) == 60 and all(s.Lx == s.Ly == 2048 for s in specs)
    nsteps = 100
    ens = xyl.Ensemble(specs, dtype="f32")
    try:
        launch = ens.autotune()
        say("quench batch: launch", launch, "steps per pass", ens.fusion())
        picks = [0, len(specs) - 1]
        start = {r: ens.get_state(r) for r in picks}
        ens.step(nsteps)
        end = {r: ens.get_state(r) for r in picks}
    finally:
        ens.close()
    for r in picks:
        check_replica(specs[r], start[r], end[r], nsteps, tag="quench replica %d" % r)


def test_eight_temperatures_full_size_matches_oracle(xyl):
    specs = [workloads.large_fp32(j) for j in range(8)]
    nsteps, every = 100, 50
    ens = xyl.Ensemble(specs, dtype="f32")
    try:
        launch = ens.autotune()
        say("4096^2 x 8 temperatures: launch", launch, "steps per pass", ens.fusion())
        picks = [0, len(specs) - 1]
        start = {r: ens.get_state(r) for r in picks}
        samples = ens.step(nsteps, every=every)
        end = {r: ens.get_state(r) for r in picks}
    finally:
        ens.close()
    for r in picks:
        check_replica(specs[r], start[r], end[r], nsteps, samples[r], every, "4096^2 replica %d" % r)
