"""GPU parity of the directional structure factor S_delta(k) and the
Lorentzian correlation length (App. C) through the C-ABI.

S(k) is compared with the oracle's definition, the Fourier sum of the oracle's
correlation function over the full periodic range (Eq. FT-Corr-delta), to
1e-9 relative.  Power-of-two axes go through the per-line FFT, other lengths
through the direct sum; both are covered.  At the benchmark's 4096^2 the
check is by properties: the sum rule sum_k S(k) = L C(0) = L, positivity,
and agreement with the transform of the GPU correlation function.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import estimators
from paper_2409_06412_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def full_spectrum(S_half, L):
    """S(0..L-1) from S(0..L/2) by S(L - k) = S(k)."""
    S = np.empty(L)
    S[: L // 2 + 1] = S_half
    S[L // 2 + 1:] = S_half[1: L - L // 2][::-1]
    return S


@pytest.mark.parametrize("model,dtype,Lx,Ly", [
    ("xy", "f64", 64, 32),      # FFT along both axes
    ("xy", "f32", 96, 40),      # direct sums along both axes
    ("xy", "f64", 260, 16),     # direct along x, FFT along y
    ("si", "f64", 64, 48),      # q = 2 rotors; FFT along x, direct along y
    ("si", "f32", 128, 128),
    ("xy", "f64", 8, 2048),     # one radix-8 pass along x; radix 16, 16, 8 along y
    ("xy", "f64", 512, 4),      # radix 16, 16, 2 along x; one radix-4 pass along y
    ("si", "f64", 256, 2),      # two radix-16 passes along x; a single radix-2 pass along y
])
def test_structure_factor_matches_oracle(xyl, model, dtype, Lx, Ly):
    say("structure factor", model, dtype, Lx, Ly)
    if model == "si":
        spec = workloads.si_lattice(Lx, Ly, Jx=10.0, seed=4)
        th, om = workloads.half_circle_state(Lx, Ly, seed=17)
    else:
        spec = workloads.LatticeSpec(Lx, Ly, seed=4)
        th, om = workloads.random_state(Lx, Ly, seed=17)
    lat = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=spec.schedule, seed=spec.seed, **spec.params())
    lat.set_state(th, om)
    lat.step(20)                                     # correlated, non-trivial state
    th_dev, _, _ = lat.get_state()
    o = oracle.Oracle(**spec.oracle_kwargs())
    for axis, L in ((0, Lx), (1, Ly)):
        S = lat.structure_factor(axis, L // 2)
        want = estimators.structure_factor(o.correlation(th_dev, axis, L - 1))[: L // 2 + 1]
        np.testing.assert_allclose(S, want, rtol=1e-9, atol=1e-9 * L)
        assert np.sum(full_spectrum(S, L)) == pytest.approx(L, rel=1e-10)
    lat.close()


def test_structure_factor_full_size_properties(xyl):
    """4096^2 FP32 (the benchmark's lattice) after 300 steps at T = 0.3: sum
    rule and positivity of S(k) along both axes, and the correlation function
    (computed on the GPU from the same transform, App. C) against the oracle's
    direct pair sums for r <= 8 on the same state."""
    spec = workloads.large_fp32(0, 4096)
    lat = xyl.Lattice(4096, 4096, dtype="f32", schedule=spec.schedule, seed=spec.seed, **spec.params())
    lat.init_random()
    lat.step(300)
    for axis in (0, 1):
        S = lat.structure_factor(axis, 2048)
        assert np.all(S > 0)
        assert np.sum(full_spectrum(S, 4096)) == pytest.approx(4096.0, rel=1e-10)
    th, _, _ = lat.get_state()
    o = oracle.Oracle(**spec.oracle_kwargs())
    for axis in (0, 1):
        np.testing.assert_allclose(lat.correlation(axis, 8), o.correlation(th, axis, 8), rtol=0, atol=1e-10)
    S = lat.structure_factor(0, 2048)
    # the peak of an ordering lattice: a Lorentzian fit over it gives a finite xi
    xi, A = xyl.lorentzian_xi(S, 4096, 1, 40)
    say("4096^2 xi_x", xi)
    assert 0.5 < xi < 4096
    lat.close()


def test_lorentzian_fit_of_gpu_spectrum_matches_oracle_fit(xyl):
    """Above T_c the peak is a Lorentzian; the library fit of the GPU's S(k)
    equals scipy's fit of the oracle's S(k) of the same state."""
    L = 256
    spec = workloads.LatticeSpec(L, L, schedule=((0, 1.2),), seed=6)
    lat = xyl.Lattice(L, L, dtype="f64", schedule=spec.schedule, seed=spec.seed, **spec.params())
    lat.init_random()
    lat.step(2000)
    th, _, _ = lat.get_state()
    o = oracle.Oracle(**spec.oracle_kwargs())
    for axis in (0, 1):
        S = lat.structure_factor(axis, L // 2)
        So = estimators.structure_factor(o.correlation(th, axis, L - 1))
        xi, A = xyl.lorentzian_xi(S, L, 0, 24)
        xo, Ao = estimators.lorentzian_xi(So, L, 0, 24)
        say("axis", axis, "xi", xi, "oracle fit", xo)
        assert xi == pytest.approx(xo, rel=1e-6)
    lat.close()


def test_ensemble_structure_factor_equals_single(xyl):
    specs = [workloads.LatticeSpec(64, 64, seed=1, replica=0, nsteps=30),
             workloads.LatticeSpec(300, 24, seed=2, replica=1, nsteps=30)]
    ens = xyl.Ensemble(specs, dtype="f32")
    ens.step(30)
    for r, sp in enumerate(specs):
        lat = xyl.Lattice(sp.Lx, sp.Ly, dtype="f32", schedule=sp.schedule, seed=sp.seed, replica=sp.replica,
                          **sp.params())
        lat.init_random()
        lat.step(30)
        for axis, L in ((0, sp.Lx), (1, sp.Ly)):
            np.testing.assert_array_equal(ens.structure_factor(r, axis, L // 2), lat.structure_factor(axis, L // 2))
        lat.close()
    ens.close()


def test_structure_factor_errors(xyl):
    lat = xyl.Lattice(64, 16, dtype="f32")
    with pytest.raises(xyl.XylError):
        lat.structure_factor(0, 4)                   # no state yet
    lat.init_random()
    with pytest.raises(xyl.XylError):
        lat.structure_factor(2, 4)
    with pytest.raises(xyl.XylError):
        lat.structure_factor(1, 9)                   # kmax > Ly/2
    lat.close()
