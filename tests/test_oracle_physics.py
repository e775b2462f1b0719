"""Pins of the oracle's physics (CPU only).

Each test checks the oracle against something other than itself: a closed form,
a mathematical invariant, a library routine (numpy FFT, scipy labelling, scipy
Lyapunov solver) or brute-force finite differences.  Together they are chosen
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import estimators
from paper_2409_06412_amd import workloads


def wrapped(d):
    return np.remainder(d + np.pi, 2 * np.pi) - np.pi


# ----------------------------------------------------------------- energy
@pytest.mark.parametrize("Jx,Jy,h", [(1.0, -0.1, 0.5), (-1.0, 0.1, 0.25), (0.7, 0.3, 0.0)])
def test_ground_state_energy_closed_form(Jx, Jy, h):
    """Staggered ordered state: every bond and the field at their minimum,
    E/N = -(|Jx| + |Jy| + h) (h >= 0)."""
    o = oracle.Oracle(8, 6, Jx=Jx, Jy=Jy, h=h)
    for sign in (1, -1):
        th, om = o.init_ordered(sign)
        assert o.energy_pot(th) / o.N == pytest.approx(-(abs(Jx) + abs(Jy) + h), abs=1e-14)
        obs = o.observables(th, om)
        assert obs[2] == pytest.approx(float(sign), abs=1e-15)   # staggered order parameter


def test_uniform_state_energy_closed_form():
    o = oracle.Oracle(6, 4, Jx=1.0, Jy=-0.1, h=0.5)
    phi = 0.3
    th = np.full((4, 6), phi)
    assert o.energy_pot(th) / o.N == pytest.approx(1.0 - 0.1 - 0.5 * math.cos(2 * phi), abs=1e-14)


@pytest.mark.parametrize("Lx,Ly", [(4, 4), (2, 3), (5, 4)])
def test_force_is_minus_energy_gradient(Lx, Ly):
    """Brute-force central differences of E_pot on small lattices (incl. Lx = 2,
    where the two x bonds of a pair are both counted)."""
    o = oracle.Oracle(Lx, Ly, Jx=1.0, Jy=-0.1, h=0.5)
    th, _ = workloads.random_state(Lx, Ly, seed=11)
    F = o.force(th).ravel()
    eps = 1e-6
    for i in range(o.N):
        tp = th.ravel().copy(); tp[i] += eps
        tm = th.ravel().copy(); tm[i] -= eps
        fd = -(o.energy_pot(tp) - o.energy_pot(tm)) / (2 * eps)
        assert F[i] == pytest.approx(fd, abs=1e-8)


# ------------------------------------------------------------- dynamics
def test_zero_temperature_relaxation_to_ground_state():
    o = oracle.Oracle(16, 16, gamma=1.0, dt=0.01, schedule=[(0, 0.0)])
    th, om = workloads.perturbed_ground_state(16, 16, o.stagger(), 0.3, seed=2)
    th, om, s = o.run(th, om, 0, 4000, every=4000)
    assert s[-1, 0] == pytest.approx(-1.6, abs=1e-9)
    assert s[-1, 1] < 1e-12
    assert abs(s[-1, 2]) == pytest.approx(1.0, abs=1e-5)


def test_energy_conservation_is_second_order():
    """gamma = T = 0 reduces BBK to velocity Verlet: the total-energy error is
    bounded, quarters when dt halves, and does not drift."""
    dev = {}
    for dt, n in ((0.02, 1000), (0.01, 2000)):
        o = oracle.Oracle(16, 16, gamma=0.0, dt=dt, schedule=[(0, 0.0)])
        th, om = workloads.perturbed_ground_state(16, 16, o.stagger(), 0.6, seed=3)
        _, _, s = o.run(th, om, 0, n, every=1)
        E = s[:, 0] + s[:, 1]
        d = E - E[0]
        dev[dt] = np.max(np.abs(d))
        q = len(d) // 4
        assert abs(d[-q:].mean() - d[:q].mean()) < 0.5 * dev[dt]
    ratio = dev[0.02] / dev[0.01]
    assert 3.3 < ratio < 4.7


@pytest.mark.parametrize("m,n", [(1, 0), (0, 1), (2, 3), (8, 0), (0, 8), (5, 8)])
def test_linear_dispersion(m, n):
    """Small oscillations about the ordered state: Omega^2 = 4h + 2|Jx|(1 - cos kx)
    + 2|Jy|(1 - cos ky); velocity Verlet gives r2 + r0 = (2 - Omega^2 dt^2) r1 for
    the projections r_j of the mode after j steps."""
    Lx = Ly = 16
    Jx, Jy, h, dt, A = 1.0, -0.1, 0.5, 0.1, 1e-5
    o = oracle.Oracle(Lx, Ly, Jx=Jx, Jy=Jy, h=h, gamma=0.0, dt=dt, schedule=[(0, 0.0)])
    th0, om = o.init_ordered(1)
    y, x = np.mgrid[0:Ly, 0:Lx]
    kx, ky = 2 * np.pi * m / Lx, 2 * np.pi * n / Ly
    mode = np.cos(kx * x + ky * y)
    th = wrapped(th0 + A * mode)
    r = []
    for j in range(3):
        t, _ = o.run(th, om, 0, j)
        r.append(np.sum(wrapped(t - th0) * mode))
    Om2 = 4 * h + 2 * abs(Jx) * (1 - math.cos(kx)) + 2 * abs(Jy) * (1 - math.cos(ky))
    assert (r[2] + r[0]) / r[1] == pytest.approx(2 - Om2 * dt * dt, abs=1e-8)


def msd_harmonic(t, eta, w2, T):
    """Second moment <x^2>(t) of a thermal harmonic oscillator from rest
    (App. A.2, Eq. MSD-HO, m = kB = 1), evaluated in complex arithmetic."""
    root = np.sqrt(complex(eta * eta - 4 * w2))
    lp, lm = 0.5 * (eta + root), 0.5 * (eta - root)
    s = lp + lm
    val = eta * T / (lp - lm) ** 2 * (s / (lp * lm) + 4 / s * (np.exp(-s * t) - 1)
                                      - np.exp(-2 * lp * t) / lp - np.exp(-2 * lm * t) / lm)
    return val.real


def bbk_linear_maps(w2, g, dt, T):
    """Linear BBK map of one oscillator on the state (x_k, w_k, n_k):
    wh = a w - hdt w2 x + hs n ; x' = x + dt wh ; w' = c (wh - hdt w2 x' + hs n')
    with n' a fresh draw; returns (M, B) with s' = M s + B n'."""
    a, c, hdt = 1 - 0.5 * g * dt, 1 / (1 + 0.5 * g * dt), 0.5 * dt
    hs = 0.5 * math.sqrt(2 * g * T * dt)
    Awh = np.array([-hdt * w2, a, hs])
    Ax = np.array([1.0, 0, 0]) + dt * Awh
    Aw = c * (Awh - hdt * w2 * Ax)
    M = np.vstack([Ax, Aw, [0, 0, 0]])
    B = np.array([0, c * hs, 1.0])
    return M, B


@pytest.mark.parametrize("eta", [1.0, 10.0])
def test_harmonic_oscillator_benchmark(eta):
    """The paper's first benchmark (App. A.2): Jx = Jy = 0 and a small-amplitude
    field well -h cos(2 th) ~ 2 h th^2 give independent oscillators with
    omega^2 = 4 h = 20 (the paper's value), 131072 paths from rest, dt = 0.01.
    The sample <th^2>(t) must match the exact second moment of the discrete
    linear BBK map (covariance propagation) at every time, and, from t = 1 on,
    the paper's continuous closed form Eq. MSD-HO within 1 %."""
    Lx, Ly, h, T, dt = 512, 256, 5.0, 0.005, 0.01
    o = oracle.Oracle(Lx, Ly, Jx=0.0, Jy=0.0, h=h, gamma=eta, dt=dt, schedule=[(0, T)], seed=9)
    M, B = bbk_linear_maps(4 * h, eta, dt, T)
    S = np.diag([0.0, 0.0, 1.0])
    th = np.zeros((Ly, Lx)); om = np.zeros((Ly, Lx))
    k = 0
    for t in (0.1, 0.3, 1.0, 3.0):
        steps = int(round(t / dt)) - k
        th, om = o.run(th, om, k, steps)
        for _ in range(steps):
            S = M @ S @ M.T + np.outer(B, B)
        k += steps
        x2 = np.mean(th ** 2)
        se = math.sqrt(np.var(th ** 2) / th.size)
        assert abs(x2 - S[0, 0]) < 5 * se + 2e-3 * x2
        if t >= 1.0:
            assert S[0, 0] == pytest.approx(msd_harmonic(t, eta, 4 * h, T), rel=0.01)


def test_free_particle_equipartition():
    """Jx = Jy = h = 0: with one Gaussian draw shared by the two half-kicks around
    each time, the stationary velocity variance of BBK is exactly T/(1 + gamma dt/2);
    independent draws per half-kick would give T/2.  gamma dt = 0.5 makes the
    factor 0.8 so the reading is resolved."""
    g, dt, T = 10.0, 0.05, 1.0
    o = oracle.Oracle(256, 256, Jx=0.0, Jy=0.0, h=0.0, gamma=g, dt=dt, schedule=[(0, T)], seed=4)
    th = np.zeros((256, 256)); om = np.zeros((256, 256))
    th, om = o.run(th, om, 0, 80)
    v = np.mean(om ** 2)
    se = math.sqrt(2.0 / om.size) * v
    assert abs(v - T / (1 + 0.5 * g * dt)) < 5 * se


def test_harmonic_stationary_covariance_discrete_lyapunov():
    """For the linearised map (oscillator, omega^2 = 4h) the stationary covariance
    of the stored BBK state solves a discrete Lyapunov equation; the oracle's
    late-time <th^2> and <omega^2> must match it within sampling error."""
    h, T, g, dt = 5.0, 0.005, 2.0, 0.05
    M, Bn = bbk_linear_maps(4 * h, g, dt, T)
    S = scipy.linalg.solve_discrete_lyapunov(M, np.outer(Bn, Bn))
    o = oracle.Oracle(256, 256, Jx=0.0, Jy=0.0, h=h, gamma=g, dt=dt, schedule=[(0, T)], seed=12)
    th = np.zeros((256, 256)); om = np.zeros((256, 256))
    th, om = o.run(th, om, 0, 400)
    for got, want, arr in ((np.mean(th ** 2), S[0, 0], th), (np.mean(om ** 2), S[1, 1], om)):
        se = math.sqrt(np.var(arr ** 2) / arr.size)
        assert abs(got - want) < 5 * se + 2e-3 * want


# ------------------------------------------------------------ observables
def test_observables_match_fft():
    Lx, Ly = 12, 8
    o = oracle.Oracle(Lx, Ly)
    th, om = workloads.random_state(Lx, Ly, seed=21)
    eps = o.stagger()
    s0, s1 = eps * np.cos(th), eps * np.sin(th)
    X0, X1 = np.fft.fft2(s0), np.fft.fft2(s1)
    N = Lx * Ly
    F = lambda l, k: (abs(X0[l, k]) ** 2 + abs(X1[l, k]) ** 2) / N
    obs = o.observables(th, om)
    assert obs[1] == pytest.approx(np.mean(0.5 * om ** 2), rel=1e-13)
    assert obs[2] == pytest.approx(X0[0, 0].real / N, rel=1e-12)
    assert obs[3] == pytest.approx(F(0, 0), rel=1e-12)
    assert obs[4] == pytest.approx(F(0, 1), rel=1e-12)
    assert obs[5] == pytest.approx(F(1, 0), rel=1e-12)


@pytest.mark.parametrize("axis", [0, 1])
def test_correlation_fourier_identity(axis):
    """App. C: the Fourier transform of C_delta(r) equals the summed squared lattice
    Fourier transform of the two rotor components (numpy FFT)."""
    Lx, Ly = 10, 6
    o = oracle.Oracle(Lx, Ly)
    th, _ = workloads.random_state(Lx, Ly, seed=22)
    eps = o.stagger()
    s = [eps * np.cos(th), eps * np.sin(th)]
    L = Lx if axis == 0 else Ly
    C = o.correlation(th, axis, L - 1)
    S = np.fft.fft(C)
    N = Lx * Ly
    ax = 1 if axis == 0 else 0
    want = sum(np.sum(np.abs(np.fft.fft(sk, axis=ax)) ** 2, axis=1 - ax) for sk in s) / N
    np.testing.assert_allclose(S.real, want, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(S.imag, 0, atol=1e-11)
    # the paper's form: S(k) = (1/(N L_other)) sum_l sum_kappa |FFT2(s^kappa)_{k,l}|^2
    other = Ly if axis == 0 else Lx
    X = [np.fft.fft2(sk) for sk in s]
    want2 = sum(np.sum(np.abs(Xk) ** 2, axis=0 if axis == 0 else 1) for Xk in X) / (N * other)
    np.testing.assert_allclose(S.real, want2, rtol=1e-11, atol=1e-12)
    assert C[0] == pytest.approx(1.0, abs=1e-14)


def test_second_moment_xi_on_planted_field():
    """A field with C(r) = exp(-|r|/xi) (periodic, summed images) has
    F(0)/F(k1) = S(0)/S(k1) computable by FFT; the estimator returns xi exactly
    for the Lorentzian case and tends to xi for the exponential."""
    L, xi = 64, 3.0
    r = np.arange(L)
    C = np.exp(-np.minimum(r, L - r) / xi)
    S = np.fft.fft(C).real
    est = estimators.xi_second_moment(S[0], S[1], L)
    assert est == pytest.approx(xi, rel=0.03)
    # exact Lorentzian in k: S(k) = 1/(1 + 4 xi^2 sin^2(pi k / L))
    S0, S1 = 1.0, 1.0 / (1 + 4 * xi * xi * math.sin(math.pi / L) ** 2)
    assert estimators.xi_second_moment(S0, S1, L) == pytest.approx(xi, rel=1e-12)


# --------------------------------------------------------------- Binder
def test_binder_limits():
    assert estimators.binder(np.full(100, 0.37), 0.0) == pytest.approx(1.0, abs=1e-15)
    o = oracle.Oracle(2, 2)
    rng = np.random.default_rng(5)
    ms = []
    for _ in range(40000):
        th = rng.uniform(-np.pi, np.pi, size=(2, 2))
        ms.append(o.observables(th, np.zeros((2, 2)))[2])
    ms = np.array(ms)
    U = estimators.binder(ms, 0.0)
    # iid uniform angles: E m^4 / (E m^2)^2 = 3 - 3/(2N)
    boot = [estimators.binder(rng.choice(ms, ms.size), 0.0) for _ in range(50)]
    assert abs(U - (3 - 3 / 8)) < 5 * np.std(boot)
    assert abs(U - 3.0) > 10 * np.std(boot)


def test_tau_int_ar1():
    rng = np.random.default_rng(6)
    phi = 0.8
    x = np.empty(200000)
    x[0] = 0
    e = rng.standard_normal(x.size)
    for t in range(1, x.size):
        x[t] = phi * x[t - 1] + e[t]
    want = 0.5 * (1 + phi) / (1 - phi)
    assert estimators.tau_int(x[:20000]) == pytest.approx(want, rel=0.15)


# ---------------------------------------------------------------- domains
def periodic_labels(spin):
    """Independent route: scipy's open-boundary labelling plus a union-find over the
    periodic seams; each cluster is named by its smallest linear index."""
    from scipy import ndimage
    Ly, Lx = spin.shape
    lab = np.zeros(spin.shape, dtype=np.int64)
    nxt = 0
    for v in (1, -1):
        l, n = ndimage.label(spin == v)
        lab = np.where(l > 0, l + nxt, lab)
        nxt += n
    parent = list(range(nxt + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for y in range(Ly):
        if spin[y, 0] == spin[y, Lx - 1]:
            parent[find(lab[y, 0])] = find(lab[y, Lx - 1])
    for x in range(Lx):
        if spin[0, x] == spin[Ly - 1, x]:
            parent[find(lab[0, x])] = find(lab[Ly - 1, x])
    roots = np.vectorize(find)(lab).ravel()
    first = {}
    for i, r in enumerate(roots):
        first.setdefault(r, i)
    return np.array([first[r] for r in roots]).reshape(spin.shape)


def theta_for_spins(spin, eps):
    """An angle with the requested staggered spin: 0.2 if eps*spin = +1, else 2.9."""
    return np.where(spin * eps > 0, 0.2, 2.9)


@pytest.mark.parametrize("Lx,Ly,p,seed", [(16, 16, 0.5, 1), (17, 9, 0.4, 2), (32, 8, 0.6, 3), (2, 2, 0.5, 4)])
def test_domains_match_independent_labelling(Lx, Ly, p, seed):
    o = oracle.Oracle(Lx, Ly)
    eps = o.stagger()
    spin = np.where(np.random.default_rng(seed).random((Ly, Lx)) < p, 1, -1)
    lab, nd = o.domains(theta_for_spins(spin, eps))
    want = periodic_labels(spin)
    np.testing.assert_array_equal(lab, want)
    assert nd == len(np.unique(want))


def test_domain_invariants():
    o = oracle.Oracle(12, 10)
    eps = o.stagger()
    # stripes along x that wrap: each row of spins constant, alternating in pairs of rows
    spin = np.repeat(np.array([1, 1, -1, -1, 1, 1, -1, -1, 1, 1])[:, None], 12, axis=1)
    lab, nd = o.domains(theta_for_spins(spin, eps))
    # rows 8,9 (+1) join rows 0,1 across the y seam
    assert nd == 4
    assert np.all(lab[8:10] == 0)
    # a pattern that alternates in both directions gives N singletons
    chk = np.where((np.add.outer(np.arange(10), np.arange(12)) % 2) == 0, 1, -1)
    lab, nd = o.domains(theta_for_spins(chk, eps))
    assert nd == 120
    np.testing.assert_array_equal(lab.ravel(), np.arange(120))
    # ordered state: one domain of size N
    th, _ = o.init_ordered(1)
    lab, nd = o.domains(th)
    assert nd == 1 and np.all(lab == 0)


def test_domain_spin_threshold():
    """|th| <= pi_p/2 counts as +1 (before staggering), just above counts as -1."""
    o = oracle.Oracle(2, 1, Jx=1.0)
    for bits, pi_p in ((64, math.pi), (32, float(np.float32(math.pi)))):
        half = pi_p / 2
        th = np.array([[half, 0.0]])       # eps = (+1, -1): spins (+1, -1) -> 2 domains
        _, nd = o.domains(th, bits)
        assert nd == 2
        th = np.array([[np.nextafter(half, 4.0), 0.0]])   # spins (-1, -1) -> 1 domain
        _, nd = o.domains(th, bits)
        assert nd == 1


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_central_differences():
    spec = dict(Lx=8, Ly=6, Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=7)
    o = oracle.Oracle(**spec)
    th0, om0 = o.init_random()
    om0 = om0 + 0.1 * np.random.default_rng(1).standard_normal(om0.shape)
    nsteps, window = 80, 30
    L, g, dth, dom = o.adjoint(th0, om0, nsteps, window)
    assert L == pytest.approx(o.loss(th0, om0, nsteps, window), rel=1e-14)
    for j, name in enumerate(("Jx", "Jy", "h", "gamma")):
        p = spec[name]
        e = 1e-5 * abs(p)
        lp = o.with_params(**{name: p + e}).loss(th0, om0, nsteps, window)
        lm = o.with_params(**{name: p - e}).loss(th0, om0, nsteps, window)
        fd = (lp - lm) / (2 * e)
        assert g[j] == pytest.approx(fd, rel=2e-6, abs=1e-12), name
    for i in (0, 7, 23, 47):
        for arr, grad in ((th0, dth), (om0, dom)):
            e = 1e-6
            a = arr.ravel().copy(); a[i] += e
            b = arr.ravel().copy(); b[i] -= e
            if arr is th0:
                fd = (o.loss(a.reshape(arr.shape), om0, nsteps, window) - o.loss(b.reshape(arr.shape), om0, nsteps, window)) / (2 * e)
            else:
                fd = (o.loss(th0, a.reshape(arr.shape), nsteps, window) - o.loss(th0, b.reshape(arr.shape), nsteps, window)) / (2 * e)
            assert grad.ravel()[i] == pytest.approx(fd, rel=1e-5, abs=1e-11)


@pytest.mark.slow
def test_pathwise_gradient_conditioning_horizon():
    """At T = 0.6 (64 x 64) the pathwise derivative of the windowed m_s^2 loss is
    well conditioned over 1000 steps (finite differences converge to the adjoint)
    but not over 5000 steps, where chaotic growth makes finite differences at
    relative steps 1e-3 .. 1e-6 disagree wildly with each other."""
    spec = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.6)], seed=7)
    o = oracle.Oracle(64, 64, **spec)
    th, om = o.init_random()

    def fd(N, rel):
        W = N // 5
        return (o.with_params(Jx=1 + rel).loss(th, om, N, W) - o.with_params(Jx=1 - rel).loss(th, om, N, W)) / (2 * rel)

    _, g, _, _ = o.adjoint(th, om, 1000, 200)
    for rel in (1e-4, 1e-5, 1e-6):
        assert fd(1000, rel) == pytest.approx(g[0], rel=1e-3)
    long = [fd(5000, rel) for rel in (1e-3, 1e-4, 1e-5, 1e-6)]
    assert max(long) - min(long) > 10 * max(abs(v) for v in long[:1])


# ------------------------------------------------- structure factor (App. C)
def test_structure_factor_definition_matches_lattice_fft():
    """Eq. FT-Corr-delta (transform of C) equals Eq. S-as-lattice-FT (summed
    squared lattice transforms of the rotor components), for both axes, both
    models."""
    for model, Lx, Ly, q in (("xy", 12, 8, 1.0), ("si", 10, 6, 2.0)):
        o = oracle.Oracle(Lx, Ly, model=model, p=2.5 if model == "si" else 2.0)
        rng = np.random.default_rng(41)
        W = np.pi if model == "xy" else np.pi / 2
        th = rng.uniform(-W, W, size=(Ly, Lx))
        eps = o.stagger()
        X = [np.fft.fft2(eps * np.cos(q * th)), np.fft.fft2(eps * np.sin(q * th))]
        N = Lx * Ly
        for axis, L in ((0, Lx), (1, Ly)):
            S = estimators.structure_factor(o.correlation(th, axis, L - 1))
            other = Ly if axis == 0 else Lx
            want = sum(np.sum(np.abs(Xk) ** 2, axis=0 if axis == 0 else 1) for Xk in X) / (N * other)
            np.testing.assert_allclose(S, want, rtol=1e-11, atol=1e-12)
            assert np.sum(S) == pytest.approx(L, rel=1e-12)          # sum rule: L C(0) = L


def test_lorentzian_fit_recovers_xi():
    N = 512
    k = np.arange(N)
    for xi in (3.0, 12.5, 40.0):
        S = estimators.lorentzian(np.minimum(k, N - k), xi, 0.7, N)
        got, A = estimators.lorentzian_xi(S, N, 0, 20)
        assert got == pytest.approx(xi, rel=1e-7)
        assert A == pytest.approx(0.7, rel=1e-7)
    # exponential correlations C(r) = exp(-|r|/xi) (periodic images): the
    # Lorentzian is their transform's small-k form, good to O(1/xi)
    for xi in (10.0, 30.0):
        r = np.arange(N)
        S = estimators.structure_factor(np.exp(-np.minimum(r, N - r) / xi))
        got, _ = estimators.lorentzian_xi(S, N, 0, int(N / (2 * np.pi * xi)) + 2)
        assert got == pytest.approx(xi, rel=0.05)


# ------------------------------------- time-resolved Binder cumulant, z
def test_binder_relaxation_pins():
    # hand-computed: two replicas, four samples, bins of two
    m = np.array([[1.0, 2.0, 0.5, 0.5], [1.0, 0.0, 1.5, 0.5]])
    U = estimators.binder_relaxation(m, 2)
    x = np.array([1.0, 2.0, 1.0, 0.0])
    assert U[0] == pytest.approx(np.mean(x ** 4) / np.mean(x ** 2) ** 2, rel=1e-15)
    assert U[0] == pytest.approx((1 + 16 + 1) / 4 / ((1 + 4 + 1) / 4) ** 2, rel=1e-15)
    # constant magnitude: U = 1; Gaussian magnetisation: U = 3
    assert np.all(estimators.binder_relaxation(np.full((5, 6), -0.3), 3) == pytest.approx(1.0, abs=1e-15))
    g = np.random.default_rng(2).standard_normal((4000, 20))
    Ug = estimators.binder_relaxation(g, 10)
    assert np.all(np.abs(Ug - 3.0) < 0.15)


def test_z_collapse_recovers_planted_exponent():
    """U(t, L1) = f(b^-z t) with f the relaxation of U(t, L2): the raster
    minimum lies at the planted z (to its step), for either size order."""
    f = lambda t: 1.2 + 1.8 * np.exp(-t / 40.0) + 0.1 * np.exp(-t / 7.0)
    t = np.linspace(0.0, 400.0, 200)
    for z0, L1, L2 in ((2.13, 144.0, 112.0), (2.17, 80.0, 112.0)):
        b = L1 / L2
        U1 = f(b ** (-z0) * t)
        z, cost = estimators.z_collapse(t, U1, L1, t, f(t), L2, 1.5, 3.0, 0.01)
        assert z == pytest.approx(z0, abs=0.006)
        assert cost < 1e-5


# ------------------------------------------------ quench schedules (Sec. II.B, V)
def test_schedule_shapes():
    """Piecewise schedules: linear segments (Eq. Linear-Quench), power-law
    segments w = f^g (eps ~ t^g, Sec. V) and their mirror 1 - (1 - f)^g,
    checked against the closed forms; held outside the knots."""
    sched = [(100, 2.0, 3), (200, 1.0, -2), (300, 1.0), (400, 0.5, 1)]
    o = oracle.Oracle(4, 4, schedule=sched)
    for k in range(0, 500, 7):
        if k <= 100:
            want = 2.0
        elif k < 200:
            f = (k - 100) / 100
            want = 2.0 - 1.0 * f ** 3
        elif k < 300:
            f = (k - 200) / 100
            want = 1.0 + 0.0 * (1 - (1 - f) ** 2)
        elif k < 400:
            want = 1.0 - 0.5 * (k - 300) / 100
        else:
            want = 0.5
        assert o.temperature(k) == pytest.approx(want, rel=1e-14, abs=1e-15), k
    # a symmetric protocol through T_c: decelerating into the critical point,
    # accelerating out of it, eps(t) = -sign(t) |t / tau|^2 about the crossing
    Tc, tau = 1.0, 1000
    o = oracle.Oracle(4, 4, schedule=[(0, 1.25, -2), (tau, Tc, 2), (2 * tau, 0.75)])
    for t in (-900, -400, -37, 0, 52, 300, 999):
        eps = -np.sign(t) * (abs(t) / tau) ** 2 * 0.25
        assert o.temperature(tau + t) == pytest.approx(Tc * (1 + eps), rel=1e-13), t


def test_adaptive_sampling_rule():
    """The rule ds' = clamp(floor(ds tau / 10 + 1/2)) on series of known
    autocorrelation: white noise (tau = 1/2) drives ds to ds_min, a slow AR(1)
    series (tau = 0.5 (1 + phi) / (1 - phi) = 19.5 samples) to ds_max within a
    few blocks, and every spacing stays inside the clamp; the plan ends at
    k0 + nsteps."""
    rng = np.random.default_rng(3)
    white = rng.standard_normal(10000)
    st = estimators.adaptive_steps(white, 7, 20000, 40, 10, 400, 64)
    d = np.diff(st)
    assert st[0] == 7 and st[-1] == 20007
    assert np.all(d[:-1] >= 10) and np.all(d <= 400)
    assert np.all(d[64:-1] == 10)
    phi = 0.95                                   # tau = 19.5 samples: ds roughly doubles per block
    x = np.empty(12000)
    x[0] = 0.0
    for t in range(1, x.size):
        x[t] = phi * x[t - 1] + rng.standard_normal()
    st = estimators.adaptive_steps(x, 0, 1000000, 20, 10, 400, 1024)
    d = np.diff(st)
    assert d[0] == 20 and np.max(d) == 400 and np.all(d[:-1] >= 10)
    # every decision follows the rule on its block
    blocks = [x[i * 1024:(i + 1) * 1024] for i in range(3)]
    ds = 20
    for b in blocks:
        ds = int(min(max(np.floor(ds * estimators.tau_int(b) / 10 + 0.5), 10), 400))
    assert d[3 * 1024 - 1] == ds
