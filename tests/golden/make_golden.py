"""Writes the oracle-generated fixtures of this folder.

Only the FP64 oracle (``oracle/``) and numpy are used: no value here comes from
the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py

Each fixture holds a short run of one configuration from the oracle's own
random start (the init stream, omega = 0): the observables every `every` steps
and the final angle and velocity of a fixed sample of sites.  The tests read
them back to check that the oracle still reproduces them (a change to its
arithmetic shows up here) and that the FP64 HIP path meets them.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

OBS = ("e_pot", "e_kin", "m_s", "f0", "fkx", "fky")

# name -> (oracle configuration, steps, sample spacing, description)
CASES = {
    # the small FP64 configuration (Sec. III, Eq. Hamiltonian; BBK, App. A.1)
    "xy_64x64_fp64": (dict(Lx=64, Ly=64, Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01, schedule=[(0, 0.5)],
                           seed=0, replica=0, model="xy", p=2.0), 1000, 100,
                      "XY model, 64 x 64, Jx = 1, Jy = -0.1, h = 0.5, gamma = 1, dt = 0.01, T = 0.5, seed 0, "
                      "replica 0"),
    # the Si(001) mapping (q = 2, field order p = 2.5, half-circle angles; Sec. III.C) at the paper's
    # parameters (Sec. IV: I J_parallel = 10, I J_perp = 0.1, I h = 1, eta = 1) in its -J cos convention, T
    # crossing the critical value 0.1969 J_parallel; a width that is no multiple of 64
    "si_36x20_fp64": (dict(Lx=36, Ly=20, Jx=-10.0, Jy=-0.1, h=-1.0, gamma=1.0, dt=0.01,
                           schedule=[(0, 2.2), (300, 1.5)], seed=4, replica=3, model="si", p=2.5), 300, 50,
                      "Si(001) model (q = 2, p = 2.5), 36 x 20, Jx = -10, Jy = -0.1, h = -1, gamma = 1, dt = 0.01, "
                      "T 2.2 -> 1.5 over steps 0..300, seed 4, replica 3"),
}

NSITES = 64


def sample_sites(N: int) -> np.ndarray:
    """A fixed spread of linear site indices (stride coprime with N where possible)."""
    stride = 67 if np.gcd(67, N) == 1 else 61
    return (np.arange(NSITES) * stride + 5) % N


def write(name: str) -> str:
    cfg, nsteps, every, desc = CASES[name]
    o = oracle.Oracle(**cfg)
    th0, om0 = o.init_random()
    th, om, samples = o.run(th0, om0, 0, nsteps, every=every)
    sites = sample_sites(o.N)
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write("# %s\n" % desc)
        f.write("# random start from the init stream, omega = 0; %d BBK steps; observables every %d steps\n"
                % (nsteps, every))
        f.write("# written by tests/golden/make_golden.py from the FP64 oracle\n")
        f.write("config %s\n" % repr(cfg))
        f.write("run %d %d\n" % (nsteps, every))
        f.write("samples %d  # step %s\n" % (len(samples), " ".join(OBS)))
        for j, row in enumerate(samples):
            f.write("%d %s\n" % (j * every, " ".join(repr(float(v)) for v in row)))
        f.write("sites %d  # linear index i = y Lx + x, theta, omega at the last step\n" % len(sites))
        for i in sites:
            f.write("%d %r %r\n" % (i, float(th.ravel()[i]), float(om.ravel()[i])))
    return path


def read(name: str) -> dict:
    """Parses a fixture: config (dict), nsteps, every, samples (n x 7: step and
    the observables), sites (int array), theta and omega at those sites."""
    import ast
    out = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        lines = [ln.split("#")[0].strip() for ln in f if not ln.startswith("#")]
    lines = [ln for ln in lines if ln]
    it = iter(lines)
    for ln in it:
        key, _, rest = ln.partition(" ")
        if key == "config":
            out["config"] = ast.literal_eval(rest)
        elif key == "run":
            out["nsteps"], out["every"] = (int(v) for v in rest.split())
        elif key == "samples":
            out["samples"] = np.array([[float(v) for v in next(it).split()] for _ in range(int(rest))])
        elif key == "sites":
            rows = [next(it).split() for _ in range(int(rest))]
            out["sites"] = np.array([int(r[0]) for r in rows])
            out["theta"] = np.array([float(r[1]) for r in rows])
            out["omega"] = np.array([float(r[2]) for r in rows])
    return out


if __name__ == "__main__":
    oracle.build()
    for n in CASES:
        print(write(n))
