"""The FP64 HIP path against the oracle runs stored under tests/golden, through
the C-ABI: the same configuration from the library's own random start (the
init stream), the same number of steps; samples to rtol 1e-10 (XY) or 1e-9
(Si), angles at the stored sites to the FP64 trajectory bar of each model."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden  # noqa: E402

pytestmark = pytest.mark.gpu

BARS = {"xy_64x64_fp64": (1e-12, 1e-10), "si_36x20_fp64": (1e-10, 1e-9)}


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_fp64_path_meets_stored_oracle_run(xyl, name):
    g = make_golden.read(name)
    c = g["config"]
    print("golden", name, flush=True)
    lat = xyl.Lattice(c["Lx"], c["Ly"], dtype="f64", Jx=c["Jx"], Jy=c["Jy"], h=c["h"], gamma=c["gamma"],
                      dt=c["dt"], schedule=c["schedule"], seed=c["seed"], replica=c["replica"], model=c["model"],
                      p=c["p"])
    lat.init_random()
    s = lat.step_measured(g["nsteps"], g["every"])
    th, om, k = lat.get_state()
    lat.close()
    ang, rel = BARS[name]
    assert k == g["nsteps"]
    np.testing.assert_allclose(s, g["samples"][:, 1:], rtol=rel, atol=1e-12)
    period = np.pi if c["model"] == "si" else 2 * np.pi
    d = np.abs(np.remainder(th.ravel()[g["sites"]] - g["theta"] + period / 2, period) - period / 2)
    print("max|dtheta|", d.max(), flush=True)
    assert d.max() <= ang
    np.testing.assert_allclose(om.ravel()[g["sites"]], g["omega"], rtol=0, atol=100 * ang)
