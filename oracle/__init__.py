"""Plain FP64 CPU oracle for the Langevin-XY hot path (arXiv:2409.06412).

TEST INFRASTRUCTURE ONLY: this package checks the HIP product path.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with ``paper_2409_06412_amd`` and never imports it.

The arithmetic lives in ``xyo.c`` (plain C, IEEE binary64, no contraction);
this module only marshals numpy arrays into it.  ``estimators`` holds the
host-side statistics (Binder cumulant, autocorrelation time, correlation
length) written from their definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xyo.c")
_LIB = os.path.join(_HERE, "libxyo.so")
MAX_KNOTS = 16
NOBS = 6


def build(force: bool = False) -> str:
    """Compile ``xyo.c`` into ``libxyo.so`` with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Model(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("Jx", ctypes.c_double), ("Jy", ctypes.c_double), ("h", ctypes.c_double),
        ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
        ("nknots", ctypes.c_int32),
        ("knot_step", ctypes.c_uint64 * MAX_KNOTS),
        ("knot_T", ctypes.c_double * MAX_KNOTS),
        ("model", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("knot_gamma", ctypes.c_int32 * MAX_KNOTS),
    ]


MODELS = {"xy": 0, "si": 1}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, u32, u64, i32, i64 = (ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_int32, ctypes.c_int64)
        P = ctypes.POINTER
        pm = P(Model)
        pd = P(d)
        sig = {
            "xyo_philox4x32_10": (None, [P(u32), P(u32), P(u32)]),
            "xyo_uniform": (d, [u32]),
            "xyo_normal": (d, [pm, u64, i64]),
            "xyo_normals": (None, [pm, u64, pd]),
            "xyo_temperature": (d, [pm, u64]),
            "xyo_init_random": (None, [pm, pd, pd]),
            "xyo_init_ordered": (None, [pm, i32, pd, pd]),
            "xyo_stagger": (i32, [pm, i64]),
            "xyo_energy_pot": (d, [pm, pd]),
            "xyo_force": (None, [pm, pd, pd]),
            "xyo_run": (i32, [pm, pd, pd, u64, u64]),
            "xyo_run_measured": (i64, [pm, pd, pd, u64, u64, u64, pd]),
            "xyo_observables": (None, [pm, pd, pd, pd]),
            "xyo_correlation": (None, [pm, pd, i32, i32, pd]),
            "xyo_domains": (i64, [pm, pd, i32, P(i32)]),
            "xyo_adjoint": (d, [pm, pd, pd, u64, u64, pd, pd, pd]),
            "xyo_loss": (d, [pm, pd, pd, u64, u64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's loops use (its OpenMP runtime's
    omp_set_num_threads)."""
    lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(n))


def max_threads() -> int:
    lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    return int(gomp.omp_get_max_threads())


def _pd(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One lattice model: couplings, damping, step size, schedule and noise key.

    model "xy": q = 1, p = 2, angles in [-pi, pi); model "si": the Si(001)
    mapping, q = 2 with field order p, angles in [-pi/2, pi/2)."""

    def __init__(self, Lx, Ly, Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01,
                 schedule=((0, 0.5),), seed=0, replica=0, model="xy", p=2.0):
        m = Model()
        m.model = MODELS[model]
        m.p = float(p)
        self.model = model
        m.Lx, m.Ly = int(Lx), int(Ly)
        m.Jx, m.Jy, m.h, m.gamma, m.dt = float(Jx), float(Jy), float(h), float(gamma), float(dt)
        m.seed, m.replica = int(seed), int(replica)
        sched = list(schedule)
        if not 1 <= len(sched) <= MAX_KNOTS:
            raise ValueError("schedule needs 1..16 knots")
        m.nknots = len(sched)
        for j, kt in enumerate(sched):
            m.knot_step[j] = int(kt[0])
            m.knot_T[j] = float(kt[1])
            m.knot_gamma[j] = int(kt[2]) if len(kt) > 2 else 1
        self.m = m
        self.N = m.Lx * m.Ly
        self._p = ctypes.byref(m)

    @property
    def shape(self):
        return (self.m.Ly, self.m.Lx)

    # -- noise and schedule -------------------------------------------------
    def temperature(self, k: int) -> float:
        return lib().xyo_temperature(self._p, int(k))

    def normals(self, k: int) -> np.ndarray:
        n = np.empty(self.N)
        lib().xyo_normals(self._p, int(k), _pd(n))
        return n.reshape(self.shape)

    # -- states ---------------------------------------------------------------
    def init_random(self):
        th, om = np.empty(self.N), np.empty(self.N)
        lib().xyo_init_random(self._p, _pd(th), _pd(om))
        return th.reshape(self.shape), om.reshape(self.shape)

    def init_ordered(self, sign=1):
        th, om = np.empty(self.N), np.empty(self.N)
        lib().xyo_init_ordered(self._p, int(sign), _pd(th), _pd(om))
        return th.reshape(self.shape), om.reshape(self.shape)

    def stagger(self) -> np.ndarray:
        return np.array([lib().xyo_stagger(self._p, i) for i in range(self.N)],
                        dtype=np.int32).reshape(self.shape)

    # -- physics ------------------------------------------------------------
    def energy_pot(self, theta) -> float:
        th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        return lib().xyo_energy_pot(self._p, _pd(th))

    def force(self, theta) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        F = np.empty(self.N)
        lib().xyo_force(self._p, _pd(th), _pd(F))
        return F.reshape(self.shape)

    def run(self, theta, omega, k0: int, nsteps: int, every: int = 0):
        """Advance copies of (theta, omega) by nsteps from step k0.

        Returns (theta, omega) or, with every > 0, (theta, omega, samples) where
        samples[j] = observables at step k0 + j*every."""
        th = np.array(theta, dtype=np.float64).ravel()
        om = np.array(omega, dtype=np.float64).ravel()
        if every:
            ns = nsteps // every + 1
            out = np.empty((ns, NOBS))
            rc = lib().xyo_run_measured(self._p, _pd(th), _pd(om), int(k0), int(nsteps), int(every), _pd(out))
            if rc < 0:
                raise FloatingPointError("oracle: numeric fault")
            return th.reshape(self.shape), om.reshape(self.shape), out[:rc]
        rc = lib().xyo_run(self._p, _pd(th), _pd(om), int(k0), int(nsteps))
        if rc < 0:
            raise FloatingPointError("oracle: numeric fault")
        return th.reshape(self.shape), om.reshape(self.shape)

    def observables(self, theta, omega) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        om = np.ascontiguousarray(omega, dtype=np.float64).ravel()
        out = np.empty(NOBS)
        lib().xyo_observables(self._p, _pd(th), _pd(om), _pd(out))
        return out

    def correlation(self, theta, axis: int, rmax: int) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        C = np.empty(rmax + 1)
        lib().xyo_correlation(self._p, _pd(th), int(axis), int(rmax), _pd(C))
        return C

    def domains(self, theta, precision_bits: int = 64):
        th = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        lab = np.empty(self.N, dtype=np.int32)
        nd = lib().xyo_domains(self._p, _pd(th), int(precision_bits),
                               lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if nd < 0:
            raise MemoryError("oracle: domains")
        return lab.reshape(self.shape), int(nd)

    def adjoint(self, theta0, omega0, nsteps: int, window: int):
        th = np.ascontiguousarray(theta0, dtype=np.float64).ravel()
        om = np.ascontiguousarray(omega0, dtype=np.float64).ravel()
        g = np.zeros(4)
        dth = np.empty(self.N)
        dom = np.empty(self.N)
        L = lib().xyo_adjoint(self._p, _pd(th), _pd(om), int(nsteps), int(window), _pd(g), _pd(dth), _pd(dom))
        if not np.isfinite(L):
            raise FloatingPointError("oracle: adjoint failed")
        return L, g, dth.reshape(self.shape), dom.reshape(self.shape)

    def loss(self, theta0, omega0, nsteps: int, window: int) -> float:
        th = np.ascontiguousarray(theta0, dtype=np.float64).ravel()
        om = np.ascontiguousarray(omega0, dtype=np.float64).ravel()
        return lib().xyo_loss(self._p, _pd(th), _pd(om), int(nsteps), int(window))

    def with_params(self, **kw) -> "Oracle":
        m = self.m
        args = dict(Lx=m.Lx, Ly=m.Ly, Jx=m.Jx, Jy=m.Jy, h=m.h, gamma=m.gamma, dt=m.dt,
                    schedule=[(m.knot_step[j], m.knot_T[j], m.knot_gamma[j]) for j in range(m.nknots)],
                    seed=m.seed, replica=m.replica, model=self.model, p=m.p)
        args.update(kw)
        return Oracle(**args)


def philox(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().xyo_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def uniform(r: int) -> float:
    return lib().xyo_uniform(int(r) & 0xFFFFFFFF)
