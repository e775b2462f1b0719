"""GPU adjoint (pathwise gradients with the noise held fixed) against the FP64
oracle adjoint and against central finite differences with common random
numbers, through the C-ABI and through the torch.autograd.Function."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NAMES = ("Jx", "Jy", "h", "gamma")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_fp64_adjoint_matches_oracle(xyl):
    """64 x 64, 500 steps, loss window 100, checkpoints every 100."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=7, replica=0)
    lat = xyl.Lattice(64, 64, dtype="f64", **spec)
    o = oracle.Oracle(64, 64, **spec)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    L = lat.adjoint_forward(500, 100, 100)
    g, dth, dom = lat.adjoint_backward()
    Lo, go, dtho, domo = o.adjoint(th0, om0, 500, 100)
    say("loss gpu", L, "oracle", Lo, "grad gpu", g, "oracle", go)
    assert L == pytest.approx(Lo, rel=1e-11)
    np.testing.assert_allclose(g, go, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(dth, dtho, rtol=1e-7, atol=1e-11 * np.abs(dtho).max())
    np.testing.assert_allclose(dom, domo, rtol=1e-7, atol=1e-11 * np.abs(domo).max())
    lat.close()


@pytest.mark.parametrize("Lx,Ly,K", [(68, 20, 7), (12, 5, 50)])
def test_fp64_adjoint_ragged_and_partial_segments(xyl, Lx, Ly, K):
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=0.7, dt=0.01, schedule=[(0, 1.0), (90, 0.3)], seed=3, replica=1)
    lat = xyl.Lattice(Lx, Ly, dtype="f64", **spec)
    lat.init_random()
    lat.step(13)                      # start from a non-fresh state
    L = lat.adjoint_forward(90, K, 25)
    g, dth, dom = lat.adjoint_backward()
    # from a non-fresh state the independent velocity is the stored half-step
    # one, so the reference is central differences of the GPU's own FP64 loss
    def loss_at(**kw):
        # the 13 lead-in steps use the base parameters: the state at step 13
        # is the independent variable
        p = dict(spec)
        p.update(kw)
        l2 = xyl.Lattice(Lx, Ly, dtype="f64", **spec)
        l2.init_random()
        l2.step(13)
        l2.set_params(p["Jx"], p["Jy"], p["h"], p["gamma"], p["dt"])
        val = l2.adjoint_forward(90, K, 25)
        l2.close()
        return val
    assert loss_at() == L
    for j, n in enumerate(NAMES):
        e = 1e-6 * abs(spec[n])
        fd = (loss_at(**{n: spec[n] + e}) - loss_at(**{n: spec[n] - e})) / (2 * e)
        assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-10), n
    lat.close()


@pytest.mark.parametrize("nsteps,window", [(500, 100)])
def test_fp32_adjoint_512_against_finite_differences(xyl, nsteps, window):
    """512 x 512, T = 0.6, checkpoints every 100: the FP32 adjoint agrees within
    1e-3 relative with central differences (relative step 1e-4, common random
    numbers) of the loss evaluated on the FP64 path from the same FP32 start.
    The horizon is 500 steps: at T = 0.6 the pathwise derivative loses its
    conditioning between 500 and 1000 steps (there, even converged FP64
    differences and the FP64 adjoint part at 1e-3) and over 5000 steps no
    finite-difference step converges (shown on the oracle), so the 5000-step
    run is used for timing only."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=7, replica=0)
    lat = xyl.Lattice(512, 512, dtype="f32", **spec)
    lat.init_random()
    L = lat.adjoint_forward(nsteps, 100, window)
    g, dth, dom = lat.adjoint_backward()
    lat.close()

    def loss64(**kw):
        p = dict(spec)
        p.update(kw)
        l2 = xyl.Lattice(512, 512, dtype="f64", **p)
        l2.init_random()
        th, om, _ = l2.get_state()
        l2.set_state(th.astype(np.float32).astype(np.float64), om, 0)
        val = l2.adjoint_forward(nsteps, nsteps, window)
        l2.close()
        return val

    L64 = loss64()
    say("loss fp32", L, "fp64", L64)
    assert L == pytest.approx(L64, rel=1e-3)
    for j, n in enumerate(NAMES):
        e = 1e-4 * abs(spec[n])
        fd = (loss64(**{n: spec[n] + e}) - loss64(**{n: spec[n] - e})) / (2 * e)
        say(n, "adjoint", g[j], "fd", fd)
        assert g[j] == pytest.approx(fd, rel=1e-3), n


def test_autograd_function(xyl):
    import torch
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=5, replica=0)
    lat = xyl.Lattice(64, 32, dtype="f64", **spec)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    params = torch.tensor([1.0, -0.1, 0.5, 1.0], dtype=torch.float64, requires_grad=True)
    th = torch.tensor(th0, device="cuda", requires_grad=True)
    om = torch.tensor(om0, device="cuda", requires_grad=True)
    L = xyl.langevin_loss(params, th, om, lat, 200, 50, 40)
    L.backward()
    o = oracle.Oracle(64, 32, **spec)
    Lo, go, dtho, domo = o.adjoint(th0, om0, 200, 40)
    assert float(L) == pytest.approx(Lo, rel=1e-11)
    np.testing.assert_allclose(params.grad.numpy(), go, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(th.grad.cpu().numpy(), dtho, rtol=1e-7, atol=1e-11 * np.abs(dtho).max())
    lat.close()


def test_repeated_gradients_reuse_state_correctly(xyl):
    """One lattice evaluates several gradients in a row. The backward graphs are
    captured once and reused. Every evaluation equals the same evaluation on a
    fresh lattice, bit for bit: from a new initial state, after a parameter
    change (which must rebuild the graphs), and from a different step origin."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=0.8, dt=0.01, schedule=[(0, 0.9)], seed=4, replica=3)

    def evaluate(lat, seed, lead, params):
        lat.set_seed(seed, 3)
        lat.set_params(*params)
        lat.init_random()
        lat.step(lead)
        L = lat.adjoint_forward(200, 20, 40)
        g, dth, dom = lat.adjoint_backward()
        return L, g, dth, dom

    base = (1.0, -0.1, 0.5, 0.8, 0.01)
    cases = [(4, 0, base), (9, 0, base), (9, 0, (1.1, -0.1, 0.45, 0.8, 0.01)), (9, 6, base), (4, 0, base)]
    shared = xyl.Lattice(96, 40, dtype="f32", **spec)
    for seed, lead, params in cases:
        got = evaluate(shared, seed, lead, params)
        fresh = xyl.Lattice(96, 40, dtype="f32", **spec)
        want = evaluate(fresh, seed, lead, params)
        fresh.close()
        assert got[0] == want[0]
        np.testing.assert_array_equal(got[1], want[1])
        np.testing.assert_array_equal(got[2], want[2])
        np.testing.assert_array_equal(got[3], want[3])
    shared.close()


def test_stale_adjoint_runs_are_rejected(xyl):
    """A second forward run on a lattice replaces the first one's checkpoints:
    differentiating the first then fails (XYL_ESTATE) instead of returning
    the second run's gradients; so does a run after the lattice was stepped,
    re-initialised or given other parameters.  The latest run may be
    differentiated repeatedly, with the same result."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=5, replica=0)
    lat = xyl.Lattice(64, 32, dtype="f64", **spec)
    lat.init_random()
    lat.adjoint_forward(60, 20, 10)
    first = lat.adjoint_run
    lat.init_random()
    lat.set_params(1.1, -0.1, 0.5, 1.0, 0.01)
    lat.adjoint_forward(60, 20, 10)
    second = lat.adjoint_run
    assert second != first
    with pytest.raises(xyl.XylError) as e:
        lat.adjoint_backward(run=first)
    assert e.value.code == -4 and "stale" in str(e.value)
    g1 = lat.adjoint_backward(run=second)
    g2 = lat.adjoint_backward(run=second)
    for a, b in zip(g1, g2):
        np.testing.assert_array_equal(a, b)
    lat.set_params(1.0, -0.1, 0.5, 1.0, 0.01)
    with pytest.raises(xyl.XylError) as e:
        lat.adjoint_backward(run=second)
    assert e.value.code == -4
    lat.close()


def test_stale_run_through_autograd(xyl):
    """Two losses evaluated on one lattice before their backward: the first
    loss's backward refuses (the lattice holds the second run), rather than
    differentiating the wrong trajectory."""
    import torch
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=5, replica=0)
    lat = xyl.Lattice(64, 32, dtype="f64", **spec)
    lat.init_random()
    th0, om0, _ = lat.get_state()
    th = torch.tensor(th0, device="cuda", requires_grad=True)
    om = torch.tensor(om0, device="cuda", requires_grad=True)
    p1 = torch.tensor([1.0, -0.1, 0.5, 1.0], dtype=torch.float64, requires_grad=True)
    p2 = torch.tensor([1.1, -0.1, 0.5, 1.0], dtype=torch.float64, requires_grad=True)
    L1 = xyl.langevin_loss(p1, th, om, lat, 60, 20, 10)
    L2 = xyl.langevin_loss(p2, th, om, lat, 60, 20, 10)
    L2.backward()
    assert p2.grad is not None
    with pytest.raises(xyl.XylError):
        L1.backward()
    lat.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_device_outputs_equal_host_outputs(xyl, dtype):
    """xyl_adjoint_backward_device writes the host path's state adjoints
    (times a scale) into device buffers of either precision."""
    import torch
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=2, replica=1)
    lat = xyl.Lattice(72, 20, dtype=dtype, **spec)
    lat.init_random()
    lat.adjoint_forward(80, 20, 16)
    g, dth, dom = lat.adjoint_backward()
    scale = -2.5
    for tdt in (torch.float64, torch.float32):
        gth = torch.full((20 * 72,), 7.0, dtype=tdt, device="cuda")
        gom = torch.full((20 * 72,), 7.0, dtype=tdt, device="cuda")
        gd = lat.adjoint_backward_device(gth, gom, scale=scale)
        np.testing.assert_allclose(gd, scale * g, rtol=1e-15, atol=0)
        want_th = (scale * dth.ravel()).astype(tdt == torch.float32 and np.float32 or np.float64)
        want_om = (scale * dom.ravel()).astype(tdt == torch.float32 and np.float32 or np.float64)
        np.testing.assert_array_equal(gth.cpu().numpy(), want_th)
        np.testing.assert_array_equal(gom.cpu().numpy(), want_om)
    lat.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_set_state_device(xyl, dtype):
    """The device setter equals the host setter from float32 and float64
    tensors, and rejects what the host setter rejects, leaving the lattice
    as it was."""
    import torch
    Lx, Ly = 40, 12
    rng = np.random.default_rng(4)
    th = rng.uniform(-np.pi, np.pi, (Ly, Lx))
    om = rng.standard_normal((Ly, Lx))
    a = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=[(0, 0.5)], seed=3)
    b = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=[(0, 0.5)], seed=3)
    for tdt in (torch.float64, torch.float32):
        src_th = th.astype(np.float32).astype(np.float64) if tdt == torch.float32 else th
        src_om = om.astype(np.float32).astype(np.float64) if tdt == torch.float32 else om
        a.set_state(src_th, src_om, 5)
        b.set_state_device(torch.tensor(th, dtype=tdt, device="cuda").view(-1),
                           torch.tensor(om, dtype=tdt, device="cuda").view(-1), 5)
        a.step(7)
        b.step(7)
        for x, y in zip(a.get_state(), b.get_state()):
            np.testing.assert_array_equal(x, y)
    before = b.get_state()
    bad = torch.tensor(th, dtype=torch.float64, device="cuda").view(-1)
    okw = torch.tensor(om, dtype=torch.float64, device="cuda").view(-1)
    for i, v in ((3, float("nan")), (100, 3.0 * np.pi + 1e-6)):
        t = bad.clone()
        t[i] = v
        with pytest.raises(xyl.XylError) as e:
            b.set_state_device(t, okw, 0)
        assert e.value.code == -1
    w = okw.clone()
    w[7] = float("inf")
    with pytest.raises(xyl.XylError):
        b.set_state_device(bad, w, 0)
    after = b.get_state()
    for x, y in zip(before, after):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


@pytest.mark.parametrize("Lx,Ly,dtype,K,nsteps,rows", [
    (512, 64, "f32", 100, 400, 0),        # the rule's strips, graph-captured segments
    (512, 42, "f32", 100, 400, 4),        # ragged strips
    (200, 9, "f32", 7, 90, 1),            # odd segments (one single step, then pairs), a partial wave
    (1024, 13, "f32", 20, 60, 1),         # the widest row the pass takes, one-row strips
    (1024, 8, "f32", 12, 48, 0),          # the widest row, the rule's 2-row strips
    (64, 4, "f64", 10, 50, 2),            # FP64, the smallest height
    (560, 6, "f64", 9, 45, 1),            # FP64, one-row strips, a partial wave
    (512, 8, "f64", 12, 48, 1),           # FP64, one-row strips
    (320, 8, "f64", 12, 48, 0),           # FP64, the rule's 2-row strips
    (640, 6, "f64", 10, 40, 0),           # FP64 too wide for 2-row strips: single reverse steps
    (2048, 8, "f32", 10, 40, 0),          # too wide: one reverse step per pass either way
])
def test_two_reverse_steps_per_pass_equal_single_steps(xyl, Lx, Ly, dtype, K, nsteps, rows):
    """The two-step reverse pass against one reverse step per pass: dL/dth0
    and dL/dw0 bitwise equal, the parameter gradients equal up to the order
    of their sums (FP32 sites summed in FP32 four at a time by the single
    step, one at a time by the pass)."""
    say("adjoint fusion", Lx, Ly, dtype, K, nsteps, rows)
    spec = dict(Jx=1.0, Jy=-0.2, h=0.4, gamma=0.8, dt=0.02, schedule=[(0, 1.1), (nsteps, 0.4)], seed=5, replica=3)
    out = []
    for sp in (1, 2):
        lat = xyl.Lattice(Lx, Ly, dtype=dtype, **spec)
        lat.set_adjoint_fusion(sp, rows)
        lat.init_random()
        lat.step(6)
        L = lat.adjoint_forward(nsteps, K, max(1, nsteps // 3))
        g, dth, dom = lat.adjoint_backward()
        out.append((L, g, dth, dom))
        lat.close()
    assert out[0][0] == out[1][0]
    np.testing.assert_array_equal(out[0][2], out[1][2])
    np.testing.assert_array_equal(out[0][3], out[1][3])
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=1e-5 if dtype == "f32" else 1e-12,
                               atol=1e-9 * np.abs(out[0][1]).max())
