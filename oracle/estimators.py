"""Host-side estimators of the oracle (TEST INFRASTRUCTURE ONLY).

Written from their definitions, in numpy, for a reader to check by eye:
  * Binder cumulant U = <M^4> / <M^2>^2 (Sec. IV.A, Eq. Def-Binder-Cum), the
    averages being plain means over the retained samples (App. B, Eq.
    ensemble-average-calculation with the time integral as a sample mean).
  * Integrated autocorrelation time and error of a time-series mean (App. B,
    Eqs. Autocorrelation-Function, Autocorrelation-Time, Time-Series-Var):
    tau = 1/2 + sum_{t>=1} rho(t) in units of the sampling interval and
    var(mean) = 2 tau sigma^2 / n.  The sum is cut by the automatic window of
    Madras and Sokal (the reference the paper cites for this), the smallest M
    with M >= c tau(M), c = 6.
  * Second-moment correlation length from the structure factor at k = 0 and
    at the smallest nonzero wave number (the Lorentzian of App. C, Eq.
    Lorentzian-Peak, evaluated at those two points).
  * Directional structure factor S(k) = sum_r C(r) exp(-2 pi i k r / N), the
    Fourier transform of the correlation function (App. C, Eq. FT-Corr-delta),
    written as that sum; and the correlation length as the parameter of a
    least-squares fit of the Lorentzian A 2 xi / (1 + 4 pi^2 xi^2 (k/N)^2)
    around k = 0 (App. C, Eq. Lorentzian-Peak, with k read as k / N), by
    scipy's curve_fit.
  * Adaptive sampling (App. B: ds ~ tau_C / 10, adapted during the run): the
    plan of sample steps that the rule ds' = clamp(floor(ds tau / 10 + 1/2))
    produces from the samples' values, tau of each block of samples in
    samples.
  * Time-resolved Binder cumulant U(t) (Sec. IV.B; App. B: the ensemble
    average over replicas restricted to a time bin) and the dynamic exponent
    z from the collapse U(t, L1) = U(b^-z t, L2), b = L1 / L2, by a raster of
    z in steps of 0.01 minimising the squared deviation of the curves, the
    second linearly interpolated (numpy.interp).
"""
from __future__ import annotations

import numpy as np


def discard_count(n: int, discard_fraction: float) -> int:
    return int(np.floor(discard_fraction * n))


def binder(m, discard_fraction: float = 0.2) -> float:
    m = np.asarray(m, dtype=np.float64)
    m = m[discard_count(len(m), discard_fraction):]
    m2 = np.mean(m ** 2)
    m4 = np.mean(m ** 4)
    return m4 / (m2 * m2)


def autocorrelation(f) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    n = len(f)
    d = f - f.mean()
    c0 = np.dot(d, d) / n
    rho = np.empty(n)
    for t in range(n):
        rho[t] = np.dot(d[: n - t], d[t:]) / n / c0 if c0 > 0 else 0.0
    return rho


def tau_int(f, c: float = 6.0) -> float:
    rho = autocorrelation(f)
    n = len(rho)
    tau = 0.5
    for M in range(1, n):
        tau += rho[M]
        if M >= c * tau:
            return max(tau, 0.5)
    return max(tau, 0.5)


def mean_and_error(f, discard_fraction: float = 0.0):
    f = np.asarray(f, dtype=np.float64)
    f = f[discard_count(len(f), discard_fraction):]
    n = len(f)
    tau = tau_int(f)
    var = np.var(f)
    return float(f.mean()), float(np.sqrt(2.0 * tau * var / n)), float(tau)


def xi_second_moment(F0_mean: float, Fk_mean: float, L: int) -> float:
    r = F0_mean / Fk_mean - 1.0
    if r <= 0:
        return 0.0
    return float(np.sqrt(r) / (2.0 * np.sin(np.pi / L)))


def structure_factor(C) -> np.ndarray:
    """S(k) for k = 0..N-1 from C(r), r = 0..N-1 (the full periodic range)."""
    C = np.asarray(C, dtype=np.float64)
    N = len(C)
    r = np.arange(N)
    S = np.empty(N)
    for k in range(N):
        ph = 2.0 * np.pi * k * r / N
        re = np.sum(C * np.cos(ph))
        im = -np.sum(C * np.sin(ph))
        assert abs(im) <= 1e-9 * max(1.0, abs(re)), "C(r) is not symmetric"
        S[k] = re
    return S


def lorentzian(k, xi, amplitude, N):
    return amplitude * 2.0 * xi / (1.0 + 4.0 * np.pi ** 2 * xi ** 2 * (np.asarray(k, dtype=np.float64) / N) ** 2)


def lorentzian_xi(S, N: int, k_first: int, k_last: int):
    """Least-squares fit of S(k), k_first <= k <= k_last, to the Lorentzian;
    returns (xi, amplitude).  Start values from the straight line 1/S against
    (k/N)^2."""
    from scipy.optimize import curve_fit
    k = np.arange(k_first, k_last + 1)
    y = np.asarray(S, dtype=np.float64)[k_first:k_last + 1]
    u = (k / N) ** 2
    b, a = np.polyfit(u, 1.0 / y, 1)
    xi0 = np.sqrt(max(b / a, 1e-12)) / (2 * np.pi)
    A0 = 1.0 / (2.0 * a * xi0)
    (xi, A), _ = curve_fit(lambda kk, xi, A: lorentzian(kk, xi, A, N), k, y, p0=(xi0, A0), maxfev=10000)
    return float(abs(xi)), float(A)


def binder_relaxation(m, bin: int):
    """m: (nrep, nt) series; U per bin of `bin` consecutive samples, averages
    over all replicas and the bin's samples."""
    m = np.asarray(m, dtype=np.float64)
    nrep, nt = m.shape
    out = []
    for b in range(nt // bin):
        x = m[:, b * bin:(b + 1) * bin]
        out.append(np.mean(x ** 4) / np.mean(x ** 2) ** 2)
    return np.array(out)


def z_collapse(t1, U1, L1, t2, U2, L2, z_lo=1.0, z_hi=3.5, z_step=0.01):
    b = L1 / L2
    best = (np.inf, np.nan)
    t1, U1, t2, U2 = (np.asarray(v, dtype=np.float64) for v in (t1, U1, t2, U2))
    nz = int(np.floor((z_hi - z_lo) / z_step + 1e-9)) + 1
    for j in range(nz):
        z = z_lo + j * z_step
        t = b ** (-z) * t1
        inside = (t >= t2[0]) & (t <= t2[-1])
        if inside.sum() < 3:
            continue
        cost = np.mean((U1[inside] - np.interp(t[inside], t2, U2)) ** 2)
        if cost < best[0]:
            best = (cost, z)
    return best[1], best[0]


def adaptive_steps(values, k0: int, nsteps: int, ds0: int, ds_min: int, ds_max: int, block: int):
    """Sample steps of the adaptive rule, replayed from the sequence of the
    chosen observable's sample values (one per sample, in order)."""
    steps = [k0]
    ds = ds0
    blk = [values[0]]
    i = 0
    while steps[-1] < k0 + nsteps:
        if len(blk) == block:
            tau = tau_int(np.array(blk))
            ds = int(min(max(np.floor(ds * tau / 10.0 + 0.5), ds_min), ds_max))
            blk = []
        steps.append(steps[-1] + min(ds, k0 + nsteps - steps[-1]))
        i += 1
        blk.append(values[i])
    return steps

