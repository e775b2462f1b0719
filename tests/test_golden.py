"""Fixtures under tests/golden (CPU only).

* The oracle reproduces the runs `make_golden.py` stored from it: a change to
  the oracle's arithmetic, its random numbers or its initial state shows up
  here and has to be justified by the paper before the fixtures are rewritten.
* Values the paper prints: the z-collapse estimator resolves each published
  dynamic exponent to its raster step, and the Si(001) workloads sit at the
  paper's critical temperature.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import estimators

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden  # noqa: E402

# bars of the FP64 trajectory over the stored run lengths (the same as the GPU
# parity bars: the Si couplings make trajectories about a thousand times more
# sensitive to rounding than the XY ones)
BARS = {"xy_64x64_fp64": (1e-12, 1e-10), "si_36x20_fp64": (1e-10, 1e-9)}


def wrapped(d, period):
    return np.abs(np.remainder(d + period / 2, period) - period / 2)


def paper_values():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_values.txt")) as f:
        for ln in f:
            ln = ln.split("#")[0].split()
            if ln:
                vals[ln[0]] = [float(v) for v in ln[1:]]
    return vals


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_oracle_reproduces_stored_runs(name):
    g = make_golden.read(name)
    cfg, nsteps, every, _ = make_golden.CASES[name]
    assert g["config"] == cfg and (g["nsteps"], g["every"]) == (nsteps, every)
    o = oracle.Oracle(**cfg)
    th0, om0 = o.init_random()
    th, om, s = o.run(th0, om0, 0, nsteps, every=every)
    ang, rel = BARS[name]
    assert s.shape == (g["samples"].shape[0], 6)
    np.testing.assert_array_equal(g["samples"][:, 0], every * np.arange(len(s)))
    np.testing.assert_allclose(s, g["samples"][:, 1:], rtol=rel, atol=1e-12)
    period = np.pi if cfg["model"] == "si" else 2 * np.pi
    assert wrapped(th.ravel()[g["sites"]] - g["theta"], period).max() <= ang
    np.testing.assert_allclose(om.ravel()[g["sites"]], g["omega"], rtol=0, atol=100 * ang)


def test_stored_runs_are_physical():
    """Independent of the oracle's code: the stored samples start from omega = 0
    (no kinetic energy), and in the XY run at T = 0.5 the kinetic energy per
    site heads for equipartition, <omega^2>/2 = T/2 (App. A.1 with I = k_B = 1):
    within 20% once the first 500 steps have passed (the random start is still
    releasing potential energy then)."""
    for name in make_golden.CASES:
        g = make_golden.read(name)
        assert g["samples"][0, 2] == 0.0
    g = make_golden.read("xy_64x64_fp64")
    ekin = g["samples"][5:, 2]
    assert np.all(np.abs(ekin - 0.25) < 0.05)


def test_z_collapse_resolves_the_published_exponents():
    """The raster minimum of the Binder-relaxation collapse lands on each z the
    paper prints (its own and the Ising estimates it compares with) to the
    raster step, so that the paper's z = 2.13 and the Ising average 2.16 are
    told apart."""
    v = paper_values()
    f = lambda t: 1.2 + 1.8 * np.exp(-t / 40.0) + 0.1 * np.exp(-t / 7.0)
    t = np.linspace(0.0, 400.0, 200)
    zs = [v[k][0] for k in ("z", "z_ising_mc", "z_ising_rg_a", "z_ising_rg_b", "z_ising_ht", "z_ising_average")]
    got = []
    for z0 in zs:
        b = 144.0 / 112.0
        z, cost = estimators.z_collapse(t, f(b ** (-z0) * t), 144.0, t, f(t), 112.0, 1.5, 3.0, 0.01)
        assert z == pytest.approx(z0, abs=0.006)
        got.append(z)
    assert abs(got[0] - got[-1]) >= 0.025


def test_si_workloads_sit_at_the_published_critical_temperature():
    from paper_2409_06412_amd import workloads
    v = paper_values()
    assert workloads.SI_TC == pytest.approx(v["tc_over_jpar"][0] * abs(workloads.SI["Jx"]), rel=1e-15)
    temps = [s.schedule[0][1] for s in workloads.si_fss_ensemble()]
    assert min(temps) < workloads.SI_TC < max(temps)
