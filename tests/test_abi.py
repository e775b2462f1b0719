"""The C-ABI library (CPU-only checks): it loads, exports every function that
include/xyl.h declares, rejects invalid arguments before touching a device and
its pure-host estimators agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import estimators

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xyl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xyl_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2409_06412_amd as xyl
    return xyl.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 40
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    import re
    with open(os.path.join(ROOT, "include", "xyl.h")) as f:
        want = int(re.search(r"#define XYL_ABI_VERSION (\d+)", f.read()).group(1))
    assert lib.xyl_abi_version() == want


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of xyl_replica_desc and xyl_obs have the C layout
    (sizes and field offsets printed by a program compiled against the header)."""
    import subprocess
    import paper_2409_06412_amd as xyl
    fields = [f for f, _ in xyl.ReplicaDesc._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "xyl.h"\nint main(void) {\n'
                   '  printf("%zu %zu\\n", sizeof(xyl_replica_desc), sizeof(xyl_obs));\n'
                   + "".join('  printf("%%zu\\n", offsetof(xyl_replica_desc, %s));\n' % f for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(xyl.ReplicaDesc)
    assert int(out[1]) == 6 * 8
    for f, off in zip(fields, out[2:]):
        assert getattr(xyl.ReplicaDesc, f).offset == int(off), f


def test_invalid_arguments_are_rejected_without_a_device(lib):
    import paper_2409_06412_amd as xyl
    h = ctypes.c_void_p()
    assert lib.xyl_create(ctypes.byref(h), 1, 8, 0, 0) == -1        # L < 2
    assert b"Lx and Ly" in lib.xyl_last_error()
    assert lib.xyl_create(ctypes.byref(h), 8, 8, 7, 0) == -1        # unknown dtype
    assert lib.xyl_create(ctypes.byref(h), 6, 8, 0, 0) == -5        # Lx not a multiple of 4
    assert lib.xyl_create(ctypes.byref(h), 65536, 32768, 0, 0) == -5  # 2^31 sites: labels overflow int32
    assert b"int32" in lib.xyl_last_error()
    assert lib.xyl_create(ctypes.byref(h), 1 << 20, 1 << 14, 0, 0) == -1  # 2^34 sites
    assert lib.xyl_create(None, 8, 8, 0, 0) == -1
    e = ctypes.c_void_p()
    desc = (xyl.ReplicaDesc * 1)()
    assert lib.xyl_ensemble_create(ctypes.byref(e), desc, 0, 0, 0) == -1   # no replicas
    assert b"at least one replica" in lib.xyl_last_error()
    assert lib.xyl_ensemble_create(ctypes.byref(e), desc, 1, 7, 0) == -1   # unknown dtype
    assert lib.xyl_destroy(None) == 0
    assert lib.xyl_step(None, 1) == -1
    with pytest.raises(xyl.XylError):
        xyl.binder(np.zeros(10))                                    # <m^2> = 0


def test_binder_and_errors_match_oracle_estimators():
    import paper_2409_06412_amd as xyl
    rng = np.random.default_rng(3)
    m = np.empty(4000)
    m[0] = 0.3
    for t in range(1, m.size):
        m[t] = 0.9 * m[t - 1] + 0.1 * rng.standard_normal() + 0.03
    U, se = xyl.binder(m, 800)
    assert U == pytest.approx(estimators.binder(m, 0.2), rel=1e-13)
    assert np.isfinite(se) and se > 0
    mu, e, tau = xyl.mean_error(m, 800)
    mo, eo, to = estimators.mean_and_error(m, 0.2)
    assert mu == pytest.approx(mo, rel=1e-13)
    assert tau == pytest.approx(to, rel=1e-12)
    assert e == pytest.approx(eo, rel=1e-12)


def test_lorentzian_fit_matches_oracle_estimator():
    """The library's Levenberg-Marquardt fit and scipy's curve_fit (oracle)
    agree on noisy peaks; exact Lorentzians are recovered; bad input fails."""
    import paper_2409_06412_amd as xyl
    rng = np.random.default_rng(8)
    N = 1024
    k = np.arange(N // 2 + 1)
    for xi, A in ((4.0, 1.3), (25.0, 0.4), (80.0, 2.0)):
        exact = estimators.lorentzian(k, xi, A, N)
        got, amp = xyl.lorentzian_xi(exact, N, 0, 30)
        assert got == pytest.approx(xi, rel=1e-9) and amp == pytest.approx(A, rel=1e-9)
        noisy = exact * (1 + 0.03 * rng.standard_normal(k.size))
        for k0 in (0, 1):
            g, a = xyl.lorentzian_xi(noisy, N, k0, 40)
            go, ao = estimators.lorentzian_xi(noisy, N, k0, 40)
            assert g == pytest.approx(go, rel=1e-6) and a == pytest.approx(ao, rel=1e-6)
    with pytest.raises(xyl.XylError):
        xyl.lorentzian_xi(np.linspace(1, 2, 20), 64, 0, 10)            # rising: not a peak
    with pytest.raises(xyl.XylError):
        xyl.lorentzian_xi(np.ones(20), 64, 5, 5)                       # one point


def test_binder_relaxation_and_z_collapse_match_oracle_estimators():
    import paper_2409_06412_amd as xyl
    rng = np.random.default_rng(12)
    m = rng.standard_normal((37, 103)) * np.linspace(1.0, 0.2, 103) + 0.3 * np.linspace(0, 1, 103)
    U, se = xyl.binder_relaxation(m, 5)
    np.testing.assert_allclose(U, estimators.binder_relaxation(m, 5), rtol=1e-13)
    assert U.size == 20 and np.all(np.isfinite(se)) and np.all(se > 0)
    f = lambda t: 1.1 + 1.9 * np.exp(-t / 30.0)
    t = np.linspace(0.0, 300.0, 151)
    t2 = np.linspace(0.0, 300.0, 97)
    for z0, L1, L2 in ((2.16, 144, 112), (1.9, 64, 96)):
        U1 = f((L1 / L2) ** (-z0) * t) + 1e-3 * rng.standard_normal(t.size)
        z, c = xyl.z_collapse(t, U1, L1, t2, f(t2), L2, 1.5, 3.0, 0.01)
        zo, co = estimators.z_collapse(t, U1, L1, t2, f(t2), L2, 1.5, 3.0, 0.01)
        assert z == pytest.approx(zo, abs=1e-12) and c == pytest.approx(co, rel=1e-9)
        assert abs(z - z0) < 0.05
    with pytest.raises(xyl.XylError):
        xyl.z_collapse(t, f(t), 64, t, f(t), 64)                    # equal sizes
    with pytest.raises(xyl.XylError):
        xyl.binder_relaxation(np.zeros((3, 4)), 2)                   # <m^2> = 0


def test_oracle_library_is_independent_of_product():
    """The oracle neither links nor imports the HIP library."""
    for f in ("xyo.c", "xyo.h", "__init__.py", "estimators.py"):
        src = open(os.path.join(ROOT, "oracle", f)).read()
        assert not re.search(r"^\s*(import|from)\s+paper_2409_06412_amd", src, flags=re.M), f
        assert "#include" not in src or "xyl" not in "".join(re.findall(r"#include.*", src)), f
    assert oracle.lib() is not None


def test_second_moment_xi_matches_oracle_estimator():
    """The library's second-moment correlation length: exact on the lattice
    Lorentzian, the oracle estimator's value on noisy samples (means before the
    ratio, samples before `discard` dropped, either axis), 0 where F(0) does not
    exceed F(k_min), and bad input refused."""
    import math
    import paper_2409_06412_amd as xyl
    L, xi = 64, 3.0
    S1 = 1.0 / (1 + 4 * xi * xi * math.sin(math.pi / L) ** 2)
    s = np.zeros((5, 6))
    s[:, 3], s[:, 4], s[:, 5] = 1.0, S1, 0.5
    assert xyl.xi_second_moment(s, L) == pytest.approx(xi, rel=1e-12)
    rng = np.random.default_rng(3)
    s = np.abs(rng.normal(1.0, 0.2, size=(40, 6)))
    s[:, 4] *= 0.3
    s[:, 5] *= 0.6
    for axis in (0, 1):
        for discard in (0, 8):
            want = estimators.xi_second_moment(s[discard:, 3].mean(), s[discard:, 4 + axis].mean(), 48)
            assert xyl.xi_second_moment(s, 48, axis, discard) == pytest.approx(want, rel=1e-12)
    flat = np.ones((4, 6))
    assert xyl.xi_second_moment(flat, 32) == 0.0
    with pytest.raises(xyl.XylError):
        xyl.xi_second_moment(np.zeros((4, 6)), 32)                     # <F(k_min)> = 0
    with pytest.raises(xyl.XylError):
        xyl.xi_second_moment(flat, 32, axis=2)
    with pytest.raises(xyl.XylError):
        xyl.xi_second_moment(flat, 32, discard=4)
