"""GPU parity of the Si(001) model variant (q = 2, p-fold field, half-circle
angles; Sec. III.C) against the FP64 oracle, through the C-ABI.

Bit-exact initial states, domain labels and ensemble states; observables of
an FP64 state within 1e-10; FP32 trajectories over 100 steps with at most 1%
of the sites beyond 1e-4 and a median within 1e-5 (sites that rounding puts
across the half-circle cusp; tests/test_oracle_sensitivity.py).  FP64
trajectories: within 1e-12 over 100 steps; over longer runs the bar follows the
trajectory's own sensitivity to rounding, which at the paper's couplings
(|Jx| = 10) is about a thousand times that of the XY model: two oracle runs
whose starts differ by one ulp per site (random direction) differ by up to
2e-10 within 1000 steps (4e-12 within 200), so the bars there are at least
five times that spread (tests/test_oracle_sensitivity.py recomputes it).  Angles are compared
modulo pi, the period of the half circle.  Besides the oracle, the GPU path is
pinned to the canonical distribution of rings of rotors (the paper's pair
benchmark, App. A.2, generalised to rings of four), computed by a transfer
matrix.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2409_06412_amd import workloads
from test_oracle_si import ring_distributions

pytestmark = pytest.mark.gpu


def half_circle_diff(a, b):
    return np.abs(np.remainder(np.asarray(a) - np.asarray(b) + np.pi / 2, np.pi) - np.pi / 2)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pair(xyl, Lx, Ly, dtype, T=workloads.SI_TC, **kw):
    spec = workloads.si_lattice(Lx, Ly, T, **kw)
    lat = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                      **spec.params())
    o = oracle.Oracle(**spec.oracle_kwargs())
    return lat, o


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_init_random_bit_exact(xyl, dtype):
    lat, o = make_pair(xyl, 260, 12, dtype, seed=9, replica=4)
    lat.init_random()
    th, om, k = lat.get_state()
    tr, _ = o.init_random()
    if dtype == "f32":
        tr = tr.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(th, tr)
    assert np.all(th >= -np.pi / 2) and np.all(th < np.float32(np.pi / 2))
    assert np.all(om == 0) and k == 0
    lat.close()


@pytest.mark.parametrize("Lx,Ly,nsteps,rows,wpb,tol", [
    (64, 64, 100, 16, 4, 1e-12),
    (64, 64, 1000, 16, 4, 1.2e-9),
    (260, 37, 200, 16, 4, 6e-11),
    (4, 2, 300, 1, 1, 1e-12),
])
def test_fp64_parity(xyl, Lx, Ly, nsteps, rows, wpb, tol):
    say("si fp64 parity", Lx, Ly, nsteps)
    lat, o = make_pair(xyl, Lx, Ly, "f64", seed=11, replica=2)
    lat.set_schedule([(0, 1.3 * workloads.SI_TC), (nsteps, 0.7 * workloads.SI_TC)])
    o = o.with_params(schedule=[(0, 1.3 * workloads.SI_TC), (nsteps, 0.7 * workloads.SI_TC)])
    lat.set_launch(rows, wpb)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    lat.step(nsteps)
    th, om, k = lat.get_state()
    tr, wr = o.run(th0, om0, 0, nsteps)
    assert k == nsteps
    dth = half_circle_diff(th, tr).max()
    dom = np.abs(om - wr).max()
    say("  max|dtheta|", dth, "max|domega|", dom)
    assert dth <= tol
    assert dom <= 10 * tol
    assert np.all(th >= -np.pi / 2) and np.all(th < np.pi / 2)
    lat.close()


@pytest.mark.parametrize("Lx,Ly", [(64, 64), (300, 20)])
def test_fp32_parity(xyl, Lx, Ly):
    """100 FP32 steps at T_c against the FP64 oracle from the same start.  A
    site that FP32 rounding puts on the other side of the half-circle cusp
    than FP64 takes a different kick, and the oracle itself does that under
    one ulp of rounding noise per step (tests/test_oracle_sensitivity.py): the
    bar is at most 1% of the sites beyond 1e-4 and a median within 1e-5."""
    lat, o = make_pair(xyl, Lx, Ly, "f32", seed=3)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    lat.step(100)
    th, om, _ = lat.get_state()
    tr, wr = o.run(th0, om0, 0, 100)
    d = half_circle_diff(th, tr)
    n_out = int(np.count_nonzero(d > 1e-4))
    say("si fp32 parity", Lx, Ly, "max|dtheta|", d.max(), "median", np.median(d), "sites beyond 1e-4", n_out)
    assert n_out <= 0.01 * Lx * Ly
    assert np.median(d) <= 1e-5
    lat.close()


def test_measured_relaxation_other_field_order(xyl):
    """Another corner of the parameter space (integer p = 2 with the opposite
    field sign, T = 0 relaxation, sampled observables) against the oracle."""
    lat, o = make_pair(xyl, 64, 64, "f64", T=0.0, Jx=-1.0, Jy=-0.1, h=0.5, p=2.0)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    s = lat.step_measured(500, 500)
    _, _, sr = o.run(th0, om0, 0, 500, every=500)
    np.testing.assert_allclose(s, sr, rtol=1e-9, atol=1e-12)
    lat.close()


def test_ordered_start_and_observables(xyl):
    for dtype in ("f64", "f32"):
        lat, o = make_pair(xyl, 64, 32, dtype)
        lat.init_ordered(-1)
        th, om, _ = lat.get_state()
        tr, _ = o.init_ordered(-1)
        want = tr if dtype == "f64" else tr.astype(np.float32).astype(np.float64)
        np.testing.assert_array_equal(th, want)
        obs = lat.measure()
        ref = o.observables(th, om)
        np.testing.assert_allclose(obs, ref, rtol=1e-6 if dtype == "f32" else 1e-12, atol=1e-12)
        assert obs[2] == pytest.approx(-math.sin(2 * math.pi / 2.5), rel=1e-6)
        lat.close()


def test_measured_samples_match_oracle(xyl):
    lat, o = make_pair(xyl, 64, 48, "f64", seed=5, replica=1)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    s = lat.step_measured(300, 50)
    _, _, sr = o.run(th0, om0, 0, 300, every=50)
    assert s.shape == sr.shape == (7, 6)
    np.testing.assert_allclose(s, sr, rtol=1e-10, atol=1e-12)
    lat.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_correlation_and_domains_match_oracle(xyl, dtype):
    lat, o = make_pair(xyl, 96, 40, dtype, Jx=10.0, seed=6)     # staggered along x
    th, om = workloads.half_circle_state(96, 40, seed=31)
    lat.set_state(th, om)
    th_dev, _, _ = lat.get_state()
    for axis, L in ((0, 96), (1, 40)):
        C = lat.correlation(axis, L // 2)
        np.testing.assert_allclose(C, o.correlation(th_dev, axis, L // 2), rtol=1e-10, atol=1e-12)
    lab, sizes, counts, nd, mx = lat.domains()
    want, nd_want = o.domains(th_dev)
    np.testing.assert_array_equal(lab, want)
    assert nd == nd_want
    assert int(np.sum(sizes * counts)) == 96 * 40
    lat.close()


def test_launch_shape_and_graph_invariance(xyl):
    states = []
    for rows, wpb, graphs in ((16, 4, 32), (1, 1, 0), (5, 2, 7)):
        lat, _ = make_pair(xyl, 520, 33, "f32", seed=8)
        lat.set_launch(rows, wpb)
        lat.set_graph_steps(graphs)
        lat.init_random()
        lat.step(77)
        states.append(lat.get_state())
        lat.close()
    for st in states[1:]:
        np.testing.assert_array_equal(st[0], states[0][0])
        np.testing.assert_array_equal(st[1], states[0][1])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ensemble_matches_single_lattices(xyl, dtype):
    """Whole-in-LDS replicas (FP32, L^2 <= 16384) and tile-path replicas of the
    SI model equal the same lattices run alone, bit for bit."""
    S = workloads.si_lattice
    specs = [S(32, 32, 2.0, seed=1, replica=0, nsteps=45),
             S(64, 48, 1.8, seed=2, replica=1, nsteps=60, Jx=10.0),
             S(144, 144, 2.1, seed=3, replica=2, nsteps=52),
             S(260, 40, 1.5, seed=4, replica=3, nsteps=65, p=3.0)]
    ens = xyl.Ensemble(specs, dtype=dtype)
    s1 = ens.step(25, every=10)
    s2 = ens.step(40, every=10)
    got = [ens.get_state(r) for r in range(len(specs))]
    ens.close()
    for r, sp in enumerate(specs):
        lat = xyl.Lattice(sp.Lx, sp.Ly, dtype=dtype, schedule=sp.schedule, seed=sp.seed, replica=sp.replica,
                          **sp.params())
        lat.init_random()
        n = min(sp.nsteps, 65)
        samples = lat.step_measured(n, 10)
        th, om, k = lat.get_state()
        eth, eom, ek = got[r]
        assert ek == k == n
        np.testing.assert_array_equal(eth, th)
        np.testing.assert_array_equal(eom, om)
        np.testing.assert_allclose(np.concatenate([s1[r], s2[r]]), samples, rtol=1e-12, atol=1e-14)
        lat.close()


def test_model_switch_and_errors(xyl):
    lat = xyl.Lattice(64, 8, dtype="f32", **workloads.SI)
    th, om = workloads.half_circle_state(64, 8, seed=2)
    bad = th.copy()
    bad[0, 0] = np.pi / 2                       # outside [-pi/2, pi/2)
    with pytest.raises(xyl.XylError) as e:
        lat.set_state(bad, om)
    assert e.value.code == -1
    lat.set_state(th, om)
    with pytest.raises(xyl.XylError) as e:
        lat.adjoint_forward(10, 5, 5)
    assert e.value.code == -5
    with pytest.raises(xyl.XylError):
        lat.set_model("xy", 2.5)                # the XY model has p = 2
    with pytest.raises(xyl.XylError):
        lat.set_model("si", 0.0)
    lat.set_model("xy", 2.0)
    with pytest.raises(xyl.XylError) as e:       # the state is undefined after a model change
        lat.step(1)
    assert e.value.code == -4
    lat.init_random()
    lat.step(3)
    lat.close()
    with pytest.raises(xyl.XylError):           # an ensemble needs one model
        xyl.Ensemble([workloads.si_lattice(32, 32), workloads.LatticeSpec(32, 32)])


def test_ring_canonical_distribution(xyl):
    """Rings of four rotors (a 4 x M lattice with Jy = 0) at the pair
    benchmark's field and temperature relax to the canonical distribution.
    BBK's stationary distribution deviates from it by O(dt^2) (about 0.4% of
    <cos p th> at dt = 0.005 for these stiff rings), which the statistics here
    resolve, so runs at dt and dt/2 are combined by Richardson extrapolation
    (4 m(dt/2) - m(dt)) / 3.  One-site and neighbour-pair moments must lie
    within 4 standard errors (spread over the independent rings) of the
    transfer-matrix values and clearly apart from those of a 10% different
    temperature."""
    M, T, P = 4096, 100.0, 2.5

    def run(dt, seed):
        lat = xyl.Lattice(4, M, dtype="f32", Jx=-20.0, Jy=0.0, h=-100.0, gamma=1.0, dt=dt, schedule=[(0, T)],
                          seed=seed, model="si", p=P)
        lat.init_random()
        lat.step(int(round(10.0 / dt)))
        every = int(round(0.2 / dt))
        acc = []
        for _ in range(300):
            lat.step(every)
            th, _, _ = lat.get_state()
            t1, t2 = th, np.roll(th, -1, axis=1)
            acc.append(np.stack([np.cos(P * th).mean(axis=1), (th * th).mean(axis=1),
                                 np.cos(2 * (t1 - t2)).mean(axis=1),
                                 (np.sin(2 * t1) * np.sin(2 * t2)).mean(axis=1)]))
        lat.close()
        per_ring = np.mean(acc, axis=0)             # [moment, ring]
        return per_ring.mean(axis=1), per_ring.std(axis=1, ddof=1) / math.sqrt(M)

    m1, s1 = run(0.005, 12)
    m2, s2 = run(0.0025, 13)
    sim = (4 * m2 - m1) / 3
    se = np.sqrt(16 * s2 ** 2 + s1 ** 2) / 3

    def canonical(TT):
        g, p1, p2 = ring_distributions(4, -20.0, -100.0, P, TT)
        d = g[1] - g[0]
        a, b = np.meshgrid(g, g, indexing="ij")
        return np.array([np.sum(np.cos(P * g) * p1) * d, np.sum(g * g * p1) * d,
                         np.sum(np.cos(2 * (a - b)) * p2) * d * d, np.sum(np.sin(2 * a) * np.sin(2 * b) * p2) * d * d])

    c = canonical(T)
    z = np.abs(sim - c) / se
    say("ring moments dt:", m1 - c, "dt/2:", m2 - c, "extrapolated z", z)
    assert np.all(z < 4), z
    assert np.max(np.abs(sim - canonical(1.1 * T)) / se) > 10
