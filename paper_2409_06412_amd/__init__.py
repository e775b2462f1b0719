"""Python binding of ``libxyl.so``, the MI355X (gfx950) Langevin-XY library.

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C-ABI declared in ``include/xyl.h``.  PyTorch provides the
device memory of the state (three tensors per lattice) and the stream.  There
is no CPU fallback: if the library or a gfx950 device is missing, every call
raises.

    import paper_2409_06412_amd as xyl
    lat = xyl.Lattice(4096, 4096, dtype="f32", schedule=[(0, 0.5)], seed=1)
    lat.init_random()
    lat.step(1000)
    samples = lat.step_measured(10_000, every=500)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxyl.so")

F32, F64 = 0, 1
MAX_KNOTS = 16
OBS_FIELDS = ("e_pot", "e_kin", "m_s", "f0", "fkx", "fky")

_ERRORS = {-1: "XYL_EINVAL", -2: "XYL_ENOMEM", -3: "XYL_EDEVICE", -4: "XYL_ESTATE",
           -5: "XYL_EUNSUPPORTED", -6: "XYL_ENUMERIC"}


class XylError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_ERRORS.get(code, str(code)), msg))
        self.code = code


class ReplicaDesc(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("Jx", ctypes.c_double), ("Jy", ctypes.c_double), ("h", ctypes.c_double),
        ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
        ("nknots", ctypes.c_int32),
        ("knot_step", ctypes.c_uint64 * MAX_KNOTS),
        ("knot_T", ctypes.c_double * MAX_KNOTS),
        ("nsteps", ctypes.c_uint64),
        ("model", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("knot_gamma", ctypes.c_int32 * MAX_KNOTS),
    ]


# XYL_MODEL_*: the XY lattice with a two-fold field, and the paper's Si(001)
# dimer mapping (q = 2, p-fold field, half-circle angles)
MODELS = {"xy": 0, "si": 1}


def _model_code(model) -> int:
    return MODELS[model] if isinstance(model, str) else int(model)


_lib = None
P = ctypes.POINTER
_d, _u64, _u32, _i32, _vp = ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p

_SIGS = {
    "xyl_abi_version": (_i32, []),
    "xyl_last_error": (ctypes.c_char_p, []),
    "xyl_device_count": (_i32, []),
    "xyl_create": (_i32, [P(_vp), _i32, _i32, _i32, _i32]),
    "xyl_create_wrapped": (_i32, [P(_vp), _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "xyl_destroy": (_i32, [_vp]),
    "xyl_set_stream": (_i32, [_vp, _vp]),
    "xyl_set_params": (_i32, [_vp, _d, _d, _d, _d, _d]),
    "xyl_set_model": (_i32, [_vp, _i32, _d]),
    "xyl_set_fusion": (_i32, [_vp, _i32]),
    "xyl_get_fusion": (_i32, [_vp, P(_i32), P(_i32)]),
    "xyl_set_step2_shape": (_i32, [_vp, _i32, _i32]),
    "xyl_get_step2_shape": (_i32, [_vp, P(_i32), P(_i32), P(_i32)]),
    "xyl_ensemble_set_fusion": (_i32, [_vp, _i32]),
    "xyl_ensemble_set_graphs": (_i32, [_vp, _i32]),
    "xyl_ensemble_get_fusion": (_i32, [_vp, P(_i32)]),
    "xyl_stream_ceiling": (_i32, [_i32, _u64, _i32, P(_d)]),
    "xyl_set_schedule_shaped": (_i32, [_vp, P(_u64), P(_d), P(_i32), _i32]),
    "xyl_step_adaptive": (_i32, [_vp, _u64, _u64, _u64, _u64, _i32, _u64, P(_d), P(_u64), _u64, P(_u64)]),
    "xyl_structure_factor": (_i32, [_vp, _i32, _i32, P(_d)]),
    "xyl_ensemble_structure_factor": (_i32, [_vp, _i32, _i32, _i32, P(_d)]),
    "xyl_lorentzian_xi": (_i32, [P(_d), _i32, _i32, _i32, P(_d), P(_d)]),
    "xyl_binder_relaxation": (_i32, [P(_d), _u64, _u64, _u64, P(_d), P(_d)]),
    "xyl_z_collapse": (_i32, [P(_d), P(_d), _u64, _d, P(_d), P(_d), _u64, _d, _d, _d, _d, P(_d), P(_d)]),
    "xyl_set_schedule": (_i32, [_vp, P(_u64), P(_d), _i32]),
    "xyl_set_seed": (_i32, [_vp, _u64, _u32]),
    "xyl_init_random": (_i32, [_vp]),
    "xyl_init_ordered": (_i32, [_vp, _i32]),
    "xyl_set_state": (_i32, [_vp, P(_d), P(_d), _u64]),
    "xyl_get_state": (_i32, [_vp, P(_d), P(_d), P(_u64)]),
    "xyl_state_buffers": (_i32, [_vp, P(_vp), P(_vp), P(_i32)]),
    "xyl_step": (_i32, [_vp, _u64]),
    "xyl_step_measured": (_i32, [_vp, _u64, _u64, P(_d), _u64, P(_u64)]),
    "xyl_measure": (_i32, [_vp, P(_d)]),
    "xyl_correlation": (_i32, [_vp, _i32, _i32, P(_d)]),
    "xyl_domains": (_i32, [_vp, P(_i32), P(_u64), P(_u64), _u64, P(_u64), P(_u64), P(_u64)]),
    "xyl_sync": (_i32, [_vp]),
    "xyl_set_launch": (_i32, [_vp, _i32, _i32]),
    "xyl_get_launch": (_i32, [_vp, P(_i32), P(_i32)]),
    "xyl_autotune": (_i32, [_vp]),
    "xyl_set_graph_steps": (_i32, [_vp, _i32]),
    "xyl_philox_blocks": (_i32, [_i32, _u64, P(_u32), P(_u32), _u64]),
    "xyl_noise": (_i32, [_vp, _u64, P(_d)]),
    "xyl_binder": (_i32, [P(_d), _u64, _u64, P(_d), P(_d)]),
    "xyl_mean_error": (_i32, [P(_d), _u64, _u64, P(_d), P(_d), P(_d)]),
    "xyl_xi_second_moment": (_i32, [P(_d), _u64, _u64, _i32, _i32, P(_d)]),
    "xyl_ensemble_create": (_i32, [P(_vp), P(ReplicaDesc), _i32, _i32, _i32]),
    "xyl_ensemble_destroy": (_i32, [_vp]),
    "xyl_ensemble_set_stream": (_i32, [_vp, _vp]),
    "xyl_ensemble_step": (_i32, [_vp, _u64, _u64, P(_d), _u64, P(_u64)]),
    "xyl_ensemble_set_mode": (_i32, [_vp, _i32]),
    "xyl_ensemble_autotune": (_i32, [_vp]),
    "xyl_ensemble_get_launch": (_i32, [_vp, P(_i32), P(_i32)]),
    "xyl_ensemble_get_state": (_i32, [_vp, _i32, P(_d), P(_d), P(_u64)]),
    "xyl_ensemble_set_state": (_i32, [_vp, _i32, P(_d), P(_d), _u64]),
    "xyl_ensemble_domains": (_i32, [_vp, _i32, P(_i32), P(_u64), P(_u64), _u64, P(_u64), P(_u64), P(_u64)]),
    "xyl_ensemble_sync": (_i32, [_vp]),
    "xyl_adjoint_forward": (_i32, [_vp, _u64, _u64, _u64, P(_d), P(_u64)]),
    "xyl_adjoint_backward": (_i32, [_vp, _u64, P(_d), P(_d), P(_d)]),
    "xyl_adjoint_backward_device": (_i32, [_vp, _u64, _d, P(_d), _vp, _vp, _i32]),
    "xyl_set_adjoint_fusion": (_i32, [_vp, _i32, _i32]),
    "xyl_set_state_device": (_i32, [_vp, _vp, _vp, _i32, _u64]),
    "xyl_domains_noalloc": (_i32, [_vp, P(_i32), P(_u64), P(_u64), _u64, P(_u64), P(_u64), P(_u64)]),
    "xyl_get_raw_state": (_i32, [_vp, P(_d), P(_d), P(_u64), P(_i32)]),
    "xyl_set_raw_state": (_i32, [_vp, P(_d), P(_d), _u64, _i32]),
}


def load():
    """Loads ``libxyl.so`` (built in-tree by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libxyl.so is not built: run `python -m paper_2409_06412_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise XylError(rc, load().xyl_last_error().decode())


def _pd(a: np.ndarray):
    return a.ctypes.data_as(P(_d))


def _f64(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _sched_arrays(schedule):
    """Knots (k, T) or (k, T, g): g is the shape of the segment that starts
    at the knot (1 linear, g > 1 power law, g < 0 mirrored power law)."""
    sched = list(schedule)
    ks = (_u64 * len(sched))(*[int(kt[0]) for kt in sched])
    Ts = (_d * len(sched))(*[float(kt[1]) for kt in sched])
    gs = (_i32 * len(sched))(*[int(kt[2]) if len(kt) > 2 else 1 for kt in sched])
    return ks, Ts, gs, len(sched)


def _dtype_code(dtype) -> int:
    if dtype in ("f32", "float32", F32):
        return F32
    if dtype in ("f64", "float64", F64):
        return F64
    raise ValueError("dtype must be 'f32' or 'f64'")


def device_count() -> int:
    return load().xyl_device_count()


class Lattice:
    """One periodic Lx x Ly lattice whose state lives in three torch tensors on
    ``cuda:device`` (two angle buffers and the velocity buffer)."""

    def __init__(self, Lx: int, Ly: int, dtype="f32", device: int = 0, *, Jx=1.0, Jy=-0.1, h=0.5,
                 gamma=1.0, dt=0.01, schedule: Sequence[Tuple[int, float]] = ((0, 0.0),), seed=0,
                 replica=0, stream=None, torch_buffers: bool = True, model="xy", p=2.0):
        import torch
        lib = load()
        self.Lx, self.Ly, self.N = int(Lx), int(Ly), int(Lx) * int(Ly)
        self.dtype = _dtype_code(dtype)
        self.device = int(device)
        self._h = _vp()
        self._bufs = None
        self.adjoint_run = 0
        if torch_buffers:
            tdt = torch.float32 if self.dtype == F32 else torch.float64
            dev = torch.device("cuda", self.device)
            self._bufs = [torch.zeros(self.N, dtype=tdt, device=dev) for _ in range(3)]
            _check(lib.xyl_create_wrapped(ctypes.byref(self._h), self.Lx, self.Ly, self.dtype, self.device,
                                          *[_vp(b.data_ptr()) for b in self._bufs]))
        else:
            _check(lib.xyl_create(ctypes.byref(self._h), self.Lx, self.Ly, self.dtype, self.device))
        if stream is not None:
            _check(lib.xyl_set_stream(self._h, _vp(int(stream))))
        self.set_params(Jx, Jy, h, gamma, dt)
        self.set_model(model, p)
        self.set_schedule(schedule)
        self.set_seed(seed, replica)

    # -- lifetime --------------------------------------------------------------
    def close(self):
        if self._h:
            _check(load().xyl_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- configuration -----------------------------------------------------------
    def set_params(self, Jx, Jy, h, gamma, dt):
        self.params = dict(Jx=float(Jx), Jy=float(Jy), h=float(h), gamma=float(gamma), dt=float(dt))
        _check(load().xyl_set_params(self._h, float(Jx), float(Jy), float(h), float(gamma), float(dt)))

    def set_model(self, model="xy", p=2.0):
        """"xy" (q = 1, p = 2) or "si" (the Si(001) mapping: q = 2, field order p,
        angles in [-pi/2, pi/2)).  The state must be initialised again afterwards."""
        code = _model_code(model)
        _check(load().xyl_set_model(self._h, code, float(p)))
        self.model, self.p = code, float(p)

    def set_schedule(self, schedule):
        ks, Ts, gs, n = _sched_arrays(schedule)
        _check(load().xyl_set_schedule_shaped(self._h, ks, Ts, gs, n))
        self._schedule = [(int(kt[0]), float(kt[1]), int(kt[2]) if len(kt) > 2 else 1) for kt in schedule]

    def set_seed(self, seed, replica=0):
        _check(load().xyl_set_seed(self._h, int(seed), int(replica)))
        self._seed, self._replica = int(seed), int(replica)

    def set_stream(self, stream):
        _check(load().xyl_set_stream(self._h, _vp(int(stream) if stream is not None else 0)))

    def set_fusion(self, steps_per_pass: int):
        """1: one step per pass over the state; 2: two (FP32, width up to 4096
        using at least 3/4 of the lanes of its waves of 256 sites and two of
        the last); results are identical."""
        _check(load().xyl_set_fusion(self._h, int(steps_per_pass)))

    def fusion(self):
        """(steps per pass, rows per strip of the two-step pass or 0 where it
        does not apply)."""
        sp, rows = _i32(), _i32()
        _check(load().xyl_get_fusion(self._h, ctypes.byref(sp), ctypes.byref(rows)))
        return sp.value, rows.value

    def set_step2_shape(self, rows=0, tile_waves=0):
        """Rows per strip of the two-step pass and, for widths above 4096, the
        most waves per column tile (0 keeps the current value)."""
        _check(load().xyl_set_step2_shape(self._h, int(rows), int(tile_waves)))

    def step2_shape(self):
        """(rows per strip, most waves per tile, number of column tiles) of
        the two-step pass; zeros where it does not apply."""
        r, w, t = _i32(), _i32(), _i32()
        _check(load().xyl_get_step2_shape(self._h, ctypes.byref(r), ctypes.byref(w), ctypes.byref(t)))
        return r.value, w.value, t.value

    def set_launch(self, rows_per_strip=0, waves_per_block=0):
        _check(load().xyl_set_launch(self._h, int(rows_per_strip), int(waves_per_block)))

    def launch(self):
        r, w = _i32(), _i32()
        _check(load().xyl_get_launch(self._h, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    def autotune(self):
        _check(load().xyl_autotune(self._h))
        return self.launch()

    def set_graph_steps(self, steps: int):
        _check(load().xyl_set_graph_steps(self._h, int(steps)))

    # -- state -------------------------------------------------------------------
    def init_random(self):
        _check(load().xyl_init_random(self._h))

    def init_ordered(self, sign=1):
        _check(load().xyl_init_ordered(self._h, int(sign)))

    def set_state(self, theta, omega, step: int = 0):
        th = _f64(theta, (self.Ly, self.Lx))
        om = _f64(omega, (self.Ly, self.Lx))
        _check(load().xyl_set_state(self._h, _pd(th), _pd(om), int(step)))

    def set_state_device(self, theta, omega, step: int = 0):
        """The state from two CUDA tensors of Lx*Ly float32 or float64 elements
        (same dtype, on the lattice's device): checked and converted on the
        device; nothing per site crosses to the host."""
        th, om = _device_arrays(theta, omega, self.N, self.device)
        _check(load().xyl_set_state_device(self._h, _vp(th.data_ptr()), _vp(om.data_ptr()),
                                           _dtype_code_torch(th.dtype), int(step)))

    def get_state(self):
        th = np.empty((self.Ly, self.Lx))
        om = np.empty((self.Ly, self.Lx))
        k = _u64()
        _check(load().xyl_get_state(self._h, _pd(th), _pd(om), ctypes.byref(k)))
        return th, om, k.value

    def get_raw_state(self):
        """(theta, u, step, fresh): the integrator's own state, u being the
        half-step velocity (or w^k when fresh); set_raw_state continues from it
        bit for bit."""
        th = np.empty((self.Ly, self.Lx))
        u = np.empty((self.Ly, self.Lx))
        k, f = _u64(), _i32()
        _check(load().xyl_get_raw_state(self._h, _pd(th), _pd(u), ctypes.byref(k), ctypes.byref(f)))
        return th, u, k.value, bool(f.value)

    def set_raw_state(self, theta, u, step: int, fresh: bool):
        th = _f64(theta, (self.Ly, self.Lx))
        uu = _f64(u, (self.Ly, self.Lx))
        _check(load().xyl_set_raw_state(self._h, _pd(th), _pd(uu), int(step), 1 if fresh else 0))

    @property
    def step_index(self) -> int:
        k = _u64()
        _check(load().xyl_get_state(self._h, None, None, ctypes.byref(k)))
        return k.value

    def state_buffers(self):
        """(theta_ptr, vel_ptr, fresh): device pointers of the current angles and
        of the velocity buffer (w^k if fresh, else w^{k-1/2})."""
        t, v, f = _vp(), _vp(), _i32()
        _check(load().xyl_state_buffers(self._h, ctypes.byref(t), ctypes.byref(v), ctypes.byref(f)))
        return t.value, v.value, bool(f.value)

    def theta_tensor(self):
        """The current angles as a (Ly, Lx) torch view (torch-backed lattices only)."""
        if self._bufs is None:
            raise RuntimeError("lattice was created without torch buffers")
        ptr = self.state_buffers()[0]
        for b in self._bufs[:2]:
            if b.data_ptr() == ptr:
                return b.view(self.Ly, self.Lx)
        raise RuntimeError("current angle buffer not found")

    # -- stepping and measurement ------------------------------------------------------
    def step(self, nsteps: int):
        _check(load().xyl_step(self._h, int(nsteps)))

    def step_measured(self, nsteps: int, every: int) -> np.ndarray:
        ns = int(nsteps) // int(every) + 1
        out = np.empty((ns, 6))
        nout = _u64()
        _check(load().xyl_step_measured(self._h, int(nsteps), int(every), _pd(out), ns, ctypes.byref(nout)))
        return out[: nout.value]

    def step_adaptive(self, nsteps: int, ds0: int, ds_min: int, ds_max: int, which: int = 2, block: int = 32):
        """Samples whose spacing follows tau_C / 10 of observable `which`;
        returns (steps, samples)."""
        cap = int(nsteps) // int(ds_min) + 2
        out = np.empty((cap, 6))
        steps = np.empty(cap, dtype=np.uint64)
        n = _u64()
        _check(load().xyl_step_adaptive(self._h, int(nsteps), int(ds0), int(ds_min), int(ds_max), int(which),
                                        int(block), _pd(out), steps.ctypes.data_as(P(_u64)), cap, ctypes.byref(n)))
        return steps[: n.value].astype(np.int64), out[: n.value]

    def measure(self) -> np.ndarray:
        out = np.empty(6)
        _check(load().xyl_measure(self._h, _pd(out)))
        return out

    def correlation(self, axis: int, rmax: int) -> np.ndarray:
        C = np.empty(int(rmax) + 1)
        _check(load().xyl_correlation(self._h, int(axis), int(rmax), _pd(C)))
        return C

    def structure_factor(self, axis: int, kmax: int) -> np.ndarray:
        """S(k), k = 0..kmax, along axis 0 (x) or 1 (y)."""
        S = np.empty(int(kmax) + 1)
        _check(load().xyl_structure_factor(self._h, int(axis), int(kmax), _pd(S)))
        return S

    def domains(self, want_labels: bool = True):
        """Returns (labels or None, sizes, counts, n_domains, max_size)."""
        return _domains(lambda *a: load().xyl_domains(self._h, *a), self.N, (self.Ly, self.Lx), want_labels)

    def domains_noalloc(self, want_labels: bool = True):
        """``domains`` through the library's allocation-free entry point (lattices
        of at most 2^22 sites)."""
        return _domains(lambda *a: load().xyl_domains_noalloc(self._h, *a), self.N, (self.Ly, self.Lx), want_labels)

    def noise(self, k: int) -> np.ndarray:
        out = np.empty((self.Ly, self.Lx))
        _check(load().xyl_noise(self._h, int(k), _pd(out)))
        return out

    def sync(self):
        _check(load().xyl_sync(self._h))

    # -- checkpoint --------------------------------------------------------------------
    def save(self, path: str):
        """Writes the integrator's state (angles, stored velocities and whether
        they are synchronized), the synchronized velocities for reference, the
        step index, parameters, schedule and noise key to an .npz file with a
        checksum; resuming from it continues bit for bit."""
        th, u, k, fresh = self.get_raw_state()
        _, om, _ = self.get_state()
        payload = dict(theta=th, u=u, fresh=np.int32(fresh), omega=om, step=np.uint64(k), Lx=self.Lx, Ly=self.Ly,
                       dtype=self.dtype,
                       params=np.array([self.params[n] for n in ("Jx", "Jy", "h", "gamma", "dt")]),
                       model=np.int32(self.model), p=np.float64(self.p),
                       schedule=np.array(self._schedule, dtype=np.float64),
                       key=np.array([self._seed, self._replica], dtype=np.uint64))
        payload["checksum"] = np.frombuffer(_checksum(payload), dtype=np.uint8)
        np.savez(path, **payload)

    @classmethod
    def load(cls, path: str, device: int = 0, stream=None) -> "Lattice":
        with np.load(path, allow_pickle=False) as z:
            d = {k: z[k] for k in z.files}
        if bytes(d.pop("checksum")) != _checksum(d):
            raise XylError(-1, "checkpoint %s is corrupt (checksum mismatch)" % path)
        p = d["params"]
        sched = [(int(row[0]), float(row[1])) + ((int(row[2]),) if len(row) > 2 else ()) for row in d["schedule"]]
        seed, rep = (int(v) for v in d["key"])
        lat = cls(int(d["Lx"]), int(d["Ly"]), dtype=int(d["dtype"]), device=device, Jx=p[0], Jy=p[1], h=p[2],
                  gamma=p[3], dt=p[4], schedule=sched, seed=seed, replica=rep, stream=stream,
                  model=int(d["model"]), p=float(d["p"]))
        lat.set_raw_state(d["theta"], d["u"], int(d["step"]), bool(d["fresh"]))
        return lat

    # -- gradients ---------------------------------------------------------------------
    def adjoint_forward(self, nsteps: int, ckpt_every: int, window: int) -> float:
        """Runs the forward pass and returns the loss; the run's identifier is
        kept as ``adjoint_run`` (what ``adjoint_backward`` differentiates)."""
        L, run = _d(), _u64()
        _check(load().xyl_adjoint_forward(self._h, int(nsteps), int(ckpt_every), int(window), ctypes.byref(L),
                                          ctypes.byref(run)))
        self.adjoint_run = run.value
        return L.value

    def set_adjoint_fusion(self, steps_per_pass: int, rows: int = 0):
        """Reverse steps per pass of the backward sweep (2 where a row fits a
        workgroup, else 1) and rows per strip of the two-step pass (0 keeps
        it); dL/dtheta0 and dL/domega0 are identical either way."""
        _check(load().xyl_set_adjoint_fusion(self._h, int(steps_per_pass), int(rows)))

    def adjoint_backward(self, run: Optional[int] = None):
        """(dL/d[Jx, Jy, h, gamma], dL/dtheta0, dL/domega0) as host arrays, of
        the forward run `run` (default: the latest)."""
        g = np.empty(4)
        dth = np.empty((self.Ly, self.Lx))
        dom = np.empty((self.Ly, self.Lx))
        run = self.adjoint_run if run is None else int(run)
        _check(load().xyl_adjoint_backward(self._h, run, _pd(g), _pd(dth), _pd(dom)))
        return g, dth, dom

    def adjoint_backward_device(self, dtheta0, domega0, run: Optional[int] = None, scale: float = 1.0):
        """dL/d[Jx, Jy, h, gamma] times `scale` (host array); writes scale *
        dL/dtheta0 and scale * dL/domega0 into two CUDA tensors of Lx*Ly float32
        or float64 elements (either may be None)."""
        g = np.empty(4)
        run = self.adjoint_run if run is None else int(run)
        ptrs, code = [], F64
        for t in (dtheta0, domega0):
            if t is None:
                ptrs.append(None)
                continue
            _device_arrays(t, t, self.N, self.device)
            code = _dtype_code_torch(t.dtype)
            ptrs.append(_vp(t.data_ptr()))
        if dtheta0 is not None and domega0 is not None and dtheta0.dtype != domega0.dtype:
            raise ValueError("dtheta0 and domega0 must have the same dtype")
        _check(load().xyl_adjoint_backward_device(self._h, run, float(scale), _pd(g), ptrs[0], ptrs[1], code))
        return g


def _dtype_code_torch(dt) -> int:
    import torch
    if dt == torch.float32:
        return F32
    if dt == torch.float64:
        return F64
    raise ValueError("device arrays must be float32 or float64")


def _device_arrays(a, b, n, device):
    """Checks that a and b are contiguous CUDA tensors of n elements of one
    floating dtype on `device` (no copies are made)."""
    for t in (a, b):
        if not getattr(t, "is_cuda", False) or t.device.index != device:
            raise ValueError("expected CUDA tensors on device %d" % device)
        if t.numel() != n or not t.is_contiguous():
            raise ValueError("expected contiguous tensors of %d elements" % n)
    if a.dtype != b.dtype:
        raise ValueError("theta and omega must have the same dtype")
    _dtype_code_torch(a.dtype)
    return a, b


def _checksum(d) -> bytes:
    import hashlib
    h = hashlib.sha256()
    for k in sorted(d):
        a = np.ascontiguousarray(d[k])
        h.update(k.encode())
        h.update(str(a.dtype).encode())
        h.update(a.tobytes())
    return h.digest()


def _domains(call, N, shape, want_labels):
    labels = np.empty(shape, dtype=np.int32) if want_labels else None
    ns, nd, mx = _u64(), _u64(), _u64()
    lab_p = labels.ctypes.data_as(P(_i32)) if want_labels else None
    # distinct cluster sizes s_1 < s_2 < ... sum to at most N, so there are
    # fewer than sqrt(2 N) + 1 of them
    cap = int(np.sqrt(2.0 * N)) + 2
    sizes = np.empty(cap, dtype=np.uint64)
    counts = np.empty(cap, dtype=np.uint64)
    _check(call(lab_p, sizes.ctypes.data_as(P(_u64)), counts.ctypes.data_as(P(_u64)), cap,
                ctypes.byref(ns), ctypes.byref(nd), ctypes.byref(mx)))
    return labels, sizes[: ns.value], counts[: ns.value], nd.value, mx.value


class Ensemble:
    """Replicas of possibly different size, parameters, schedule, seed and step
    count, stepped together in batched launches."""

    def __init__(self, specs, dtype="f32", device: int = 0, stream=None):
        self.specs = list(specs)
        n = len(self.specs)
        arr = (ReplicaDesc * n)()
        for d, s in zip(arr, self.specs):
            d.Lx, d.Ly = s.Lx, s.Ly
            d.Jx, d.Jy, d.h, d.gamma, d.dt = s.Jx, s.Jy, s.h, s.gamma, s.dt
            d.seed, d.replica = s.seed, s.replica
            sched = list(s.schedule)
            d.nknots = len(sched)
            for j, kt in enumerate(sched):
                d.knot_step[j] = int(kt[0])
                d.knot_T[j] = float(kt[1])
                d.knot_gamma[j] = int(kt[2]) if len(kt) > 2 else 1
            d.nsteps = int(s.nsteps)
            d.model = _model_code(getattr(s, "model", "xy"))
            d.p = float(getattr(s, "p", 2.0))
        self.dtype = _dtype_code(dtype)
        self._h = _vp()
        _check(load().xyl_ensemble_create(ctypes.byref(self._h), arr, n, self.dtype, int(device)))
        if stream is not None:
            _check(load().xyl_ensemble_set_stream(self._h, _vp(int(stream))))
        self.n = n

    def close(self):
        if self._h:
            _check(load().xyl_ensemble_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, mode: int):
        _check(load().xyl_ensemble_set_mode(self._h, int(mode)))

    def set_fusion(self, steps_per_pass: int):
        """2 (default): FP32 replicas on the tile path whose width the two-step
        pass takes advance two steps per pass between samples, batched by
        waves per row; 1: every step is one batched launch.  Results are
        identical."""
        _check(load().xyl_ensemble_set_fusion(self._h, int(steps_per_pass)))

    def fusion(self) -> int:
        """Steps per pass in effect for the batched mode."""
        sp = _i32()
        _check(load().xyl_ensemble_get_fusion(self._h, ctypes.byref(sp)))
        return sp.value

    def set_graphs(self, enable):
        """Capture repeated chunks of batched stepping as graphs: 0 (or False)
        never, 1 (or True, the default) for chunks with at most one class of
        two-step passes, 2 for every repeated chunk; results are identical."""
        _check(load().xyl_ensemble_set_graphs(self._h, int(enable)))

    def autotune(self):
        _check(load().xyl_ensemble_autotune(self._h))
        return self.launch()

    def launch(self):
        r, w = _i32(), _i32()
        _check(load().xyl_ensemble_get_launch(self._h, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    def step(self, nsteps: int, every: int = 0, cap: int = 0):
        """Advances; with every > 0 returns a list of (n_r, 6) sample arrays."""
        if not every:
            _check(load().xyl_ensemble_step(self._h, int(nsteps), 0, None, 0, None))
            return None
        cap = cap or int(nsteps) // int(every) + 2
        out = np.empty((self.n, cap, 6))
        nout = np.zeros(self.n, dtype=np.uint64)
        _check(load().xyl_ensemble_step(self._h, int(nsteps), int(every), _pd(out), cap,
                                        nout.ctypes.data_as(P(_u64))))
        counts = nout.tolist()
        return [out[r, : counts[r]] for r in range(self.n)]

    def get_state(self, r: int):
        s = self.specs[r]
        th = np.empty((s.Ly, s.Lx))
        om = np.empty((s.Ly, s.Lx))
        k = _u64()
        _check(load().xyl_ensemble_get_state(self._h, int(r), _pd(th), _pd(om), ctypes.byref(k)))
        return th, om, k.value

    def set_state(self, r: int, theta, omega, step: int = 0):
        s = self.specs[r]
        th = _f64(theta, (s.Ly, s.Lx))
        om = _f64(omega, (s.Ly, s.Lx))
        _check(load().xyl_ensemble_set_state(self._h, int(r), _pd(th), _pd(om), int(step)))

    def domains(self, r: int, want_labels: bool = True):
        s = self.specs[r]
        return _domains(lambda *a: load().xyl_ensemble_domains(self._h, int(r), *a), s.Lx * s.Ly,
                        (s.Ly, s.Lx), want_labels)

    def structure_factor(self, r: int, axis: int, kmax: int) -> np.ndarray:
        S = np.empty(int(kmax) + 1)
        _check(load().xyl_ensemble_structure_factor(self._h, int(r), int(axis), int(kmax), _pd(S)))
        return S

    def sync(self):
        _check(load().xyl_ensemble_sync(self._h))


def stream_ceiling(n: int, reps: int = 100, device: int = 0) -> float:
    """GB/s of a plain read-two/write-two float stream over n elements per array."""
    g = _d()
    _check(load().xyl_stream_ceiling(int(device), int(n), int(reps), ctypes.byref(g)))
    return g.value


def philox_blocks(counters: np.ndarray, seed: int, device: int = 0) -> np.ndarray:
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    _check(load().xyl_philox_blocks(int(device), int(seed), c.ctypes.data_as(P(_u32)),
                                    out.ctypes.data_as(P(_u32)), c.shape[0]))
    return out


def binder(m, discard: int = 0):
    m = np.ascontiguousarray(m, dtype=np.float64)
    U, se = _d(), _d()
    _check(load().xyl_binder(_pd(m), m.size, int(discard), ctypes.byref(U), ctypes.byref(se)))
    return U.value, se.value


def binder_relaxation(m, bin: int = 1):
    """U(t) per bin of `bin` samples from an (nrep, nt) array of order-parameter
    series; returns (U, U_se)."""
    m = np.ascontiguousarray(m, dtype=np.float64)
    if m.ndim != 2:
        raise ValueError("m must be (nrep, nt)")
    nrep, nt = m.shape
    nb = nt // int(bin) if bin >= 1 else 0
    U, se = np.empty(max(nb, 1)), np.empty(max(nb, 1))
    _check(load().xyl_binder_relaxation(_pd(m), nrep, nt, int(bin), _pd(U), _pd(se)))
    return U[:nb], se[:nb]


def z_collapse(t1, U1, L1, t2, U2, L2, z_lo=1.0, z_hi=3.5, z_step=0.01):
    """(z, cost) collapsing U(t, L1) onto U(b^-z t, L2), b = L1 / L2."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (t1, U1, t2, U2)]
    if a[0].size != a[1].size or a[2].size != a[3].size:
        raise ValueError("t and U arrays differ in length")
    z, c = _d(), _d()
    _check(load().xyl_z_collapse(_pd(a[0]), _pd(a[1]), a[0].size, float(L1), _pd(a[2]), _pd(a[3]), a[2].size,
                                 float(L2), float(z_lo), float(z_hi), float(z_step), ctypes.byref(z), ctypes.byref(c)))
    return z.value, c.value


def lorentzian_xi(S, L: int, k_first: int, k_last: int):
    """(xi, amplitude) of the Lorentzian fitted to S[k_first..k_last]."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    if S.size <= k_last:
        raise ValueError("S needs k_last + 1 entries")
    xi, A = _d(), _d()
    _check(load().xyl_lorentzian_xi(_pd(S), int(L), int(k_first), int(k_last), ctypes.byref(xi), ctypes.byref(A)))
    return xi.value, A.value


def xi_second_moment(samples, L: int, axis: int = 0, discard: int = 0) -> float:
    """Second-moment correlation length along axis 0 (x) or 1 (y) from an
    (n, 6) array of samples as the measuring calls return them."""
    s = np.ascontiguousarray(samples, dtype=np.float64)
    if s.ndim != 2 or s.shape[1] != 6:
        raise ValueError("samples must be (n, 6)")
    xi = _d()
    _check(load().xyl_xi_second_moment(_pd(s), s.shape[0], int(discard), int(axis),
                                       int(L), ctypes.byref(xi)))
    return xi.value


def mean_error(f, discard: int = 0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    mu, se, tau = _d(), _d(), _d()
    _check(load().xyl_mean_error(_pd(f), f.size, int(discard), ctypes.byref(mu), ctypes.byref(se),
                                 ctypes.byref(tau)))
    return mu.value, se.value, tau.value


def _langevin_loss_class():
    import torch

    class LangevinLoss(torch.autograd.Function):
        """Pathwise loss L = (1/W) sum over the last W steps of m_s^2 after
        `nsteps` BBK steps from (theta0, omega0), with the lattice's noise held
        fixed; differentiable in params = [Jx, Jy, h, gamma] (float64 tensor)
        and in the initial state.  The backward pass is the library's adjoint
        (checkpoints every `ckpt_every` steps, segments recomputed on the GPU)."""

        @staticmethod
        def forward(ctx, params, theta0, omega0, lattice, nsteps, ckpt_every, window):
            # the four parameters are host scalars; the initial state stays on
            # the device (the library checks and converts it there)
            p = [float(v) for v in params.detach().cpu().double().tolist()]
            lattice.set_params(p[0], p[1], p[2], p[3], lattice.params["dt"])
            th = theta0.detach().contiguous()
            om = omega0.detach().contiguous()
            if th.is_cuda:
                # the library works on the lattice's stream: torch's pending
                # writes of the inputs must be done first
                torch.cuda.current_stream(th.device).synchronize()
                lattice.set_state_device(th.view(-1), om.view(-1), 0)
            else:
                lattice.set_state(th.double().numpy(), om.double().numpy(), 0)
            L = lattice.adjoint_forward(int(nsteps), int(ckpt_every), int(window))
            ctx.lattice = lattice
            ctx.run = lattice.adjoint_run
            ctx.meta = (params.dtype, params.device, theta0.dtype, theta0.device, theta0.shape)
            return torch.tensor(L, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gL):
            pdt, pdev, tdt, tdev, shape = ctx.meta
            # outputs are allocated by torch and filled by the library's
            # kernels, scaled by the upstream derivative; a later forward on
            # the same lattice makes ctx.run stale (the library then raises)
            if tdev.type == "cuda":
                gth = torch.empty(shape, dtype=tdt, device=tdev)
                gom = torch.empty(shape, dtype=tdt, device=tdev)
                g = ctx.lattice.adjoint_backward_device(gth.view(-1), gom.view(-1), run=ctx.run, scale=float(gL))
            else:
                g, dth, dom = ctx.lattice.adjoint_backward(run=ctx.run)
                g = g * float(gL)
                gth = torch.from_numpy(dth * float(gL)).to(tdt).reshape(shape)
                gom = torch.from_numpy(dom * float(gL)).to(tdt).reshape(shape)
            gp = torch.tensor(g, dtype=pdt, device=pdev)
            return gp, gth, gom, None, None, None, None

    return LangevinLoss


_LL = None


def langevin_loss(params, theta0, omega0, lattice: "Lattice", nsteps: int, ckpt_every: int, window: int):
    """Functional form of ``LangevinLoss.apply``."""
    global _LL
    if _LL is None:
        _LL = _langevin_loss_class()
    return _LL.apply(params, theta0, omega0, lattice, nsteps, ckpt_every, window)
