"""The cumulant-relaxation pipeline of Sec. IV.B on the GPU: batched replicas
of the Si(001) model at T_c from disordered starts, their order-parameter
series, the time-resolved Binder cumulant U(t) (App. B bins) and the dynamic
exponent from the curve collapse.

Parity: the FP64 ensemble's series against the oracle's runs of the same
replicas, then every later stage on the two sets of series.  At production
shape (FP32, whole-in-LDS replicas) the pipeline's invariants: U(0) of a
disordered start, relaxation below it, a finite z inside the raster.
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


def relaxation_specs(sizes, nrep, nsteps, r0=0):
    out = []
    r = r0
    for L in sizes:
        for i in range(nrep):
            out.append(workloads.si_lattice(L, L, workloads.SI_TC, seed=3, replica=r, nsteps=nsteps))
            r += 1
    return out


def test_relaxation_pipeline_matches_oracle(xyl):
    sizes, nrep, nsteps, every = (8, 12), 6, 400, 10
    specs = relaxation_specs(sizes, nrep, nsteps)
    ens = xyl.Ensemble(specs, dtype="f64")
    samples = ens.step(nsteps, every=every)
    ens.close()
    t = np.arange(nsteps // every + 1) * every * workloads.SI["dt"]
    curves = {}
    for iL, L in enumerate(sizes):
        m_gpu, m_ora = [], []
        for i in range(nrep):
            sp = specs[iL * nrep + i]
            o = oracle.Oracle(**sp.oracle_kwargs())
            th, om = o.init_random()
            _, _, so = o.run(th, om, 0, nsteps, every=every)
            m_gpu.append(samples[iL * nrep + i][:, 2])
            m_ora.append(so[:, 2])
        m_gpu, m_ora = np.array(m_gpu), np.array(m_ora)
        d = np.abs(m_gpu - m_ora).max()
        say("L", L, "max |m_gpu - m_oracle|", d)
        assert d <= 1e-8
        U, se = xyl.binder_relaxation(m_gpu, 2)
        np.testing.assert_allclose(U, estimators.binder_relaxation(m_ora, 2), rtol=1e-6)
        curves[L] = (t[: 2 * U.size].reshape(-1, 2).mean(axis=1), U, estimators.binder_relaxation(m_ora, 2))
    (ta, Ua, Uao), (tb, Ub, Ubo) = curves[12], curves[8]
    z, _ = xyl.z_collapse(ta, Ua, 12, tb, Ub, 8, 0.5, 4.0, 0.01)
    zo, _ = estimators.z_collapse(ta, Uao, 12, tb, Ubo, 8, 0.5, 4.0, 0.01)
    say("z (gpu series, library)", z, "z (oracle series, oracle estimator)", zo)
    assert abs(z - zo) <= 0.011


def test_relaxation_at_production_shape(xyl):
    """512 replicas each of 16^2 and 24^2, FP32, whole-in-LDS, started ordered
    (th = pi/p everywhere, U = 1 exactly, the paper's Binder start) and run at
    1.5 T_c: U rises from 1 towards the disordered value, and the collapse
    returns an exponent inside its raster.  (From disordered starts at these
    sizes U hardly moves: rows order but stay independent, J_perp = J_par/100.)"""
    sizes, nrep, nsteps, every = (16, 24), 512, 2000, 20
    specs = []
    r = 0
    for L in sizes:
        for i in range(nrep):
            specs.append(workloads.si_lattice(L, L, 1.5 * workloads.SI_TC, seed=5, replica=r, nsteps=nsteps))
            r += 1
    ens = xyl.Ensemble(specs, dtype="f32")
    for r, sp in enumerate(specs):
        ens.set_state(r, np.full((sp.Ly, sp.Lx), np.pi / sp.p), np.zeros((sp.Ly, sp.Lx)))
    samples = ens.step(nsteps, every=every)
    ens.close()
    t = np.arange(nsteps // every + 1) * every * workloads.SI["dt"]
    curves = {}
    for iL, L in enumerate(sizes):
        m = np.array([samples[iL * nrep + i][:, 2] for i in range(nrep)])
        assert np.all(m[:, 0] == m[0, 0])
        U, se = xyl.binder_relaxation(m, 1)
        late = U[len(U) // 2:].mean()
        say("L", L, "U(0)", U[0], "U(late)", late, "se(late)", se[-1])
        assert U[0] == pytest.approx(1.0, abs=1e-12)
        assert late > 1.8
        curves[L] = (t, U)
    z, cost = xyl.z_collapse(*curves[24], 24, *curves[16], 16, 0.5, 4.0, 0.01)
    say("z", z, "cost", cost)
    assert 0.5 <= z <= 4.0 and np.isfinite(cost)
