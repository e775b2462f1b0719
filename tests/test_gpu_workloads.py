"""Small-scale versions of the configured workloads on the GPU, checked against
the oracle: a Kibble-Zurek quench ensemble (per-replica step counts, end-state
domains bit-exact), the finite-size-scaling analysis chain (samples -> Binder
cumulant and second-moment correlation length), long-axis correlation, and the
error paths of the C-ABI on a live device."""
import sys

import numpy as np
import pytest

import oracle
from oracle import estimators
from paper_2409_06412_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_quench_ensemble_domains(xyl):
    """Quench replicas (tau_Q x gamma x h) of 128^2 and 272x96 with a linear ramp
    1.5 -> 0 and a hold at T = 0; every replica's end state equals its solo run
    and its domain labels equal the oracle's flood fill bit for bit."""
    specs = workloads.kz_quench(L=128, taus=(100, 300), gammas=(0.1, 1.0), hs=(0.25, 0.5), seeds=range(1),
                                hold=50)
    specs.append(workloads.LatticeSpec(272, 96, h=0.5, gamma=1.0, schedule=((0, 1.5), (200, 0.0)), seed=3,
                                       replica=99, nsteps=250))
    ens = xyl.Ensemble(specs, dtype="f32")
    ens.step(400)
    for r, sp in enumerate(specs):
        th, om, k = ens.get_state(r)
        assert k == sp.nsteps
        lat = xyl.Lattice(sp.Lx, sp.Ly, dtype="f32", schedule=sp.schedule, seed=sp.seed, replica=sp.replica,
                          **sp.params())
        lat.init_random()
        lat.step(sp.nsteps)
        th1, om1, _ = lat.get_state()
        np.testing.assert_array_equal(th, th1)
        lat.close()
        labels, sizes, counts, nd, mx = ens.domains(r)
        o = oracle.Oracle(**sp.oracle_kwargs())
        lab_o, nd_o = o.domains(th, 32)
        np.testing.assert_array_equal(labels, lab_o)
        assert nd == nd_o and int(np.sum(sizes * counts)) == sp.Lx * sp.Ly
        say("replica", r, "tau", sp.schedule[-1][0], "gamma", sp.gamma, "h", sp.h, "domains", nd, "largest", mx)
    ens.close()


def test_fss_analysis_chain(xyl):
    """Three small replicas sampled every 100 steps: the host estimators of the
    library (Binder cumulant, second-moment correlation length, mean and
    error) agree with the oracle's on the same samples, and the sample series
    agree with single-lattice runs."""
    specs = workloads.fss_ensemble(sizes=(32, 64), ntemps=2, seeds=(0,), nsteps=3000)
    ens = xyl.Ensemble(specs, dtype="f32")
    samples = ens.step(3000, every=100)
    for r, sp in enumerate(specs):
        s = samples[r]
        assert s.shape == (31, 6)
        m = s[:, 2]
        U, U_se = xyl.binder(m, 6)
        assert U == pytest.approx(estimators.binder(m, 0.2), rel=1e-12)
        xi = estimators.xi_second_moment(s[6:, 3].mean(), s[6:, 4].mean(), sp.Lx)
        assert xyl.xi_second_moment(s, sp.Lx, 0, 6) == pytest.approx(xi, rel=1e-12)
        say("L", sp.Lx, "T", sp.schedule[0][1], "U", U, "+-", U_se, "xi_2nd", xi)
        assert 0.9 < U < 3.1
        mu, se, tau = xyl.mean_error(s[:, 0], 6)
        mo, seo, to = estimators.mean_and_error(s[:, 0], 0.2)
        assert mu == pytest.approx(mo, rel=1e-12) and se == pytest.approx(seo, rel=1e-9)
    ens.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_correlation_long_axis(xyl, dtype):
    Lx, Ly = 4096, 6
    lat = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=[(0, 0.4)], seed=8)
    lat.init_random()
    lat.step(50)
    th, _, _ = lat.get_state()
    C = lat.correlation(0, 2048)
    o = oracle.Oracle(Lx, Ly, schedule=[(0, 0.4)], seed=8)
    Cr = o.correlation(th, 0, 2048)
    np.testing.assert_allclose(C, Cr, atol=1e-6 if dtype == "f32" else 1e-12)
    C1 = lat.correlation(1, 3)
    np.testing.assert_allclose(C1, o.correlation(th, 1, 3), atol=1e-6 if dtype == "f32" else 1e-12)
    lat.close()


def test_error_paths_on_device(xyl):
    lat = xyl.Lattice(16, 8, dtype="f32")
    with pytest.raises(xyl.XylError) as e:
        lat.step(1)
    assert e.value.code == -4                                  # not initialised
    with pytest.raises(xyl.XylError) as e:
        lat.set_state(np.full((8, 16), np.nan), np.zeros((8, 16)))
    assert e.value.code == -1
    lat.init_random()
    with pytest.raises(xyl.XylError) as e:
        lat.adjoint_backward()
    assert e.value.code == -4                                  # no forward run
    with pytest.raises(xyl.XylError):
        lat.correlation(0, 9)                                  # rmax > L/2
    with pytest.raises(xyl.XylError):
        lat.set_params(1.0, -0.1, 0.5, 1.0, 0.0)               # dt <= 0
    with pytest.raises(xyl.XylError):
        lat.set_schedule([(10, 1.0), (5, 0.5)])                # knots not increasing
    with pytest.raises(xyl.XylError):
        lat.set_schedule([(0, -1.0)])                          # T < 0
    with pytest.raises(xyl.XylError):
        lat.set_launch(0, 3)                                   # waves per block not in {1, 2, 4, 8}
    lat.adjoint_forward(20, 5, 5)
    lat.step(1)
    with pytest.raises(xyl.XylError) as e:
        lat.adjoint_backward()                                 # stepped after the forward run
    assert e.value.code == -4
    lat.close()
    with pytest.raises(xyl.XylError) as e:
        xyl.Lattice(30, 8)
    assert e.value.code == -5


def test_graph_replays_across_state_resets(xyl):
    """Captured step graphs stay exact when the state is reset between replays."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.8)], seed=2, replica=0)
    lat = xyl.Lattice(64, 16, dtype="f64", **spec)
    o = oracle.Oracle(64, 16, **spec)
    lat.set_graph_steps(16)
    lat.init_random()
    lat.step(64)
    th0, om0 = workloads.random_state(64, 16, seed=5, omega_scale=0.3)
    lat.set_state(th0, om0, step=1000)
    lat.step(48)
    th, om, k = lat.get_state()
    tr, wr = o.run(th0, om0, 1000, 48)
    assert k == 1048
    assert np.abs(np.remainder(th - tr + np.pi, 2 * np.pi) - np.pi).max() < 1e-12
    lat.close()


def test_checkpoint_resume_is_bitwise(xyl, tmp_path):
    """The integrator's own state (get_raw_state/set_raw_state, and save/load,
    which use them) at step k, then continuing, equals the uninterrupted run
    bit for bit; a restart from the synchronized state (get_state/set_state: a
    fresh start at step k) agrees to rounding; a corrupted checkpoint is
    rejected."""
    for dtype in ("f32", "f64"):
        kw = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 1.0), (300, 0.2)], seed=9, replica=4)
        a = xyl.Lattice(96, 40, dtype=dtype, **kw)
        a.init_random()
        a.step(150)
        a.save(str(tmp_path / "ck.npz"))
        sync = a.get_state()
        raw = a.get_raw_state()
        assert raw[2] == 150 and not raw[3]
        a.step(100)
        ref = a.get_state()
        b = xyl.Lattice.load(str(tmp_path / "ck.npz"))
        b.step(100)
        got = b.get_state()
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        assert got[2] == ref[2] == 250
        b.set_raw_state(*raw)
        b.step(100)
        for x, y in zip(b.get_state(), ref):
            np.testing.assert_array_equal(x, y)
        b.set_state(sync[0], sync[1], sync[2])
        assert b.get_raw_state()[3]
        b.step(100)
        th = b.get_state()[0]
        d = np.abs(np.remainder(th - ref[0] + np.pi, 2 * np.pi) - np.pi).max()
        assert d <= (1e-4 if dtype == "f32" else 1e-12)
        a.close()
        b.close()
    z = dict(np.load(str(tmp_path / "ck.npz")))
    z["theta"][3, 7] += 1e-3
    np.savez(str(tmp_path / "bad.npz"), **z)
    with pytest.raises(xyl.XylError):
        xyl.Lattice.load(str(tmp_path / "bad.npz"))


def test_numeric_fault_is_reported(xyl):
    """A step size so large that the first drift overflows FP32 leaves
    non-finite values, which the synchronizing calls report as XYL_ENUMERIC."""
    lat = xyl.Lattice(32, 8, dtype="f32", dt=1e30, gamma=0.0, schedule=[(0, 0.0)])
    lat.init_random()
    lat.step(3)
    with pytest.raises(xyl.XylError) as e:
        lat.measure()
    assert e.value.code == -6
    with pytest.raises(xyl.XylError) as e:
        lat.get_state()
    assert e.value.code == -6
    lat.close()


def test_free_particle_equipartition_gpu(xyl):
    """Jx = Jy = h = 0: the stationary velocity variance of the BBK map with
    shared draws is exactly T/(1 + gamma dt/2) (0.8 T here); the FP32 GPU path
    must reproduce it within sampling error on 1M sites."""
    g, dt, T = 10.0, 0.05, 1.0
    lat = xyl.Lattice(1024, 1024, dtype="f32", Jx=0.0, Jy=0.0, h=0.0, gamma=g, dt=dt, schedule=[(0, T)], seed=4)
    lat.init_random()
    lat.step(80)
    _, om, _ = lat.get_state()
    v = np.mean(om ** 2)
    se = np.sqrt(2.0 / om.size) * v
    assert abs(v - T / (1 + 0.5 * g * dt)) < 5 * se
    lat.close()
