"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: only the parameter sets of the
lattices that are simulated and numpy-seeded arbitrary states for tests that
need a state other than the method's own initial conditions.  Both the HIP
path and the oracle receive what this module produces as plain inputs.

Parameter sets (all with J_x = +1 along the dimer rows, J_y = -0.1 across
them, the two-fold field h and damping gamma, dt = 0.01):
  * ``small_fp64``  64 x 64, FP64, T = 0.5, seed 0, 10,000 steps, sampled
    every 100 steps (the size the oracle finishes in seconds).
  * ``large_fp32``  4096 x 4096, FP32 state, eight temperatures evenly spaced
    in [0.3, 1.2], seed 1, sampled every 500 steps.
  * ``fss_ensemble`` 288 replicas: L in {32, ..., 512} x 16 temperatures in
    [0.3, 1.2] x 2 seeds, 50,000 steps.
  * ``kz_quench``   60 replicas of 2048 x 2048: tau_Q in {1e3, 1e4, 1e5}
    steps x gamma in {0.1, 1} x h in {0.25, 0.5} x 5 seeds; T ramps linearly
    from 1.5 to 0 over tau_Q steps, then holds at 0 for 1000 steps.
  * ``adjoint_512`` 512 x 512, FP32, T = 0.6, seed 7, 5000 steps, loss window
    1000, checkpoints every 100 steps.
Si(001) model variant (the paper's own mapping, Sec. III.C and IV): q = 2,
p = 2.5, angles in [-pi/2, pi/2), I J_par = 10, I J_perp = 0.1, I h = 1, eta = 1
(Sec. IV), i.e. Jx = -10, Jy = -0.1, h = -1 in this project's sign convention;
the Binder crossing of the paper puts T_c at 0.1969 J_par:
  * ``si_lattice``   one lattice at a given temperature.
  * ``si_fss_ensemble`` L in {32, 48, 64, 80, 96, 112, 128, 144} x 8
    temperatures in [0.94, 1.06] T_c x 2 seeds (the paper starts its Binder runs
    ordered, Fig. 4; an ensemble starts from the init stream, and ordered
    states can be set per replica).
  * ``si_quench``    symmetric linear quench T_c (1 + e) -> T_c (1 - e) at rate
    1/tau_Q in reduced temperature (Sec. II.B, Eq. Linear-Quench), stopped at the
    end of the ramp (Sec. V).
The paper runs on synthetic lattices only (no dataset), so nothing here stands
in for external data.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

JX, JY, H, GAMMA, DT = 1.0, -0.1, 0.5, 1.0, 0.01


@dataclass
class LatticeSpec:
    Lx: int
    Ly: int
    Jx: float = JX
    Jy: float = JY
    h: float = H
    gamma: float = GAMMA
    dt: float = DT
    schedule: Sequence[Tuple[int, float]] = ((0, 0.5),)
    seed: int = 0
    replica: int = 0
    nsteps: int = 0
    model: str = "xy"
    p: float = 2.0

    def params(self):
        return dict(Jx=self.Jx, Jy=self.Jy, h=self.h, gamma=self.gamma, dt=self.dt, model=self.model, p=self.p)

    def oracle_kwargs(self):
        return dict(Lx=self.Lx, Ly=self.Ly, Jx=self.Jx, Jy=self.Jy, h=self.h, gamma=self.gamma,
                    dt=self.dt, schedule=list(self.schedule), seed=self.seed, replica=self.replica,
                    model=self.model, p=self.p)


def small_fp64() -> LatticeSpec:
    return LatticeSpec(64, 64, schedule=((0, 0.5),), seed=0, replica=0, nsteps=10_000)


def large_temperatures() -> List[float]:
    return [0.3 + 0.9 * j / 7 for j in range(8)]


def large_fp32(j: int = 0, L: int = 4096) -> LatticeSpec:
    return LatticeSpec(L, L, schedule=((0, large_temperatures()[j]),), seed=1, replica=j,
                       nsteps=100_000)


FSS_SIZES = (32, 48, 64, 96, 128, 192, 256, 384, 512)


def fss_ensemble(sizes: Sequence[int] = FSS_SIZES, ntemps: int = 16, seeds=(0, 1),
                 nsteps: int = 50_000) -> List[LatticeSpec]:
    out = []
    temps = [0.3 + 0.06 * t for t in range(ntemps)]
    for iL, L in enumerate(sizes):
        for iT, T in enumerate(temps):
            for iS, s in enumerate(seeds):
                r = (iL * ntemps + iT) * len(seeds) + iS
                out.append(LatticeSpec(L, L, schedule=((0, T),), seed=s, replica=r, nsteps=nsteps))
    return out


def kz_quench(L: int = 2048, taus=(1_000, 10_000, 100_000), gammas=(0.1, 1.0), hs=(0.25, 0.5),
              seeds=range(5), hold: int = 1000) -> List[LatticeSpec]:
    out = []
    r = 0
    for tq in taus:
        for g in gammas:
            for hh in hs:
                for s in seeds:
                    out.append(LatticeSpec(L, L, h=hh, gamma=g, schedule=((0, 1.5), (tq, 0.0)),
                                           seed=s, replica=r, nsteps=tq + hold))
                    r += 1
    return out


def adjoint_512(L: int = 512) -> LatticeSpec:
    return LatticeSpec(L, L, schedule=((0, 0.6),), seed=7, replica=0, nsteps=5000)


SI = dict(Jx=-10.0, Jy=-0.1, h=-1.0, gamma=1.0, dt=0.01, model="si", p=2.5)
SI_TC = 0.1969 * 10.0


def si_lattice(Lx: int, Ly: int, T: float = SI_TC, seed: int = 0, replica: int = 0, nsteps: int = 0,
               **overrides) -> LatticeSpec:
    args = dict(SI)
    args.update(overrides)
    return LatticeSpec(Lx, Ly, schedule=((0, T),), seed=seed, replica=replica, nsteps=nsteps, **args)


def si_fss_ensemble(sizes: Sequence[int] = (32, 48, 64, 80, 96, 112, 128, 144), ntemps: int = 8,
                    seeds=(0, 1), nsteps: int = 100_000) -> List[LatticeSpec]:
    temps = [SI_TC * (0.94 + 0.12 * t / (ntemps - 1)) for t in range(ntemps)]
    out = []
    for iL, L in enumerate(sizes):
        for iT, T in enumerate(temps):
            for iS, sd in enumerate(seeds):
                r = (iL * ntemps + iT) * len(seeds) + iS
                out.append(si_lattice(L, L, T, seed=sd, replica=r, nsteps=nsteps))
    return out


def si_quench(L: int = 1024, taus=(100.0, 1000.0), eps: float = 0.25, seeds=range(2)) -> List[LatticeSpec]:
    """tau_Q in time units; the ramp from eps to -eps lasts 2 eps tau_Q time units."""
    out = []
    r = 0
    for tq in taus:
        n = int(round(2 * eps * tq / SI["dt"]))
        for sd in seeds:
            out.append(LatticeSpec(L, L, schedule=((0, SI_TC * (1 + eps)), (n, SI_TC * (1 - eps))), seed=sd,
                                   replica=r, nsteps=n, **SI))
            r += 1
    return out


def half_circle_state(Lx: int, Ly: int, seed: int, omega_scale: float = 1.0):
    """Arbitrary (theta, omega) of the SI model: theta uniform in [-pi/2, pi/2)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi / 2, np.pi / 2, size=(Ly, Lx))
    # keep the FP32 rounding inside the half circle too
    th = np.where(th.astype(np.float32) >= np.float32(np.pi / 2), -np.pi / 2, th)
    om = omega_scale * rng.standard_normal((Ly, Lx))
    return th, om


def random_state(Lx: int, Ly: int, seed: int, omega_scale: float = 1.0, dtype=np.float64):
    """Arbitrary (theta, omega): theta uniform in [-pi, pi), omega ~ N(0, omega_scale^2)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=(Ly, Lx)).astype(dtype)
    om = (omega_scale * rng.standard_normal((Ly, Lx))).astype(dtype)
    return th.astype(np.float64), om.astype(np.float64)


def perturbed_ground_state(Lx: int, Ly: int, stagger: np.ndarray, amplitude: float, seed: int):
    """Staggered ground state (theta = 0 where the stagger sign is +1, -pi where it
    is -1) plus uniform noise of the given amplitude, omega = 0."""
    rng = np.random.default_rng(seed)
    th = np.where(stagger > 0, 0.0, -np.pi) + rng.uniform(-amplitude, amplitude, size=(Ly, Lx))
    th = np.where(th < -np.pi, th + 2 * np.pi, th)
    return th, np.zeros((Ly, Lx))
