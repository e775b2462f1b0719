"""The allocation-free domain labelling (xyl_domains_noalloc, for callers that
cannot allocate device memory) against xyl_domains, through the C-ABI: labels
and (size, count) distributions identical (integer work: bit for bit) on two
calls in a row, the second on a smaller lattice, so that the second call
starts from the first one's leftovers in the shared static scratch.  Also the
largest lattice it takes (2^22 sites) and the refusal beyond it."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def quenched(xyl, Lx, Ly, seed, nsteps, dtype="f32"):
    lat = xyl.Lattice(Lx, Ly, dtype=dtype, schedule=[(0, 1.5), (nsteps // 2, 0.0)], seed=seed)
    lat.init_random()
    lat.step(nsteps)
    return lat


def same(a, b):
    la, sa, ca, nda, mxa = a
    lb, sb, cb, ndb, mxb = b
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(ca, cb)
    assert nda == ndb and mxa == mxb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_domains_equal_domains_two_calls(xyl, dtype):
    big = quenched(xyl, 1024, 512, 3, 400, dtype)
    small = quenched(xyl, 96, 40, 4, 200, dtype)
    try:
        for lat in (big, small):
            got = lat.domains_noalloc()
            want = lat.domains()
            say("noalloc", dtype, lat.Lx, lat.Ly, "domains", got[3], "largest", got[4])
            same(got, want)
            th, _, _ = lat.get_state()
            o = oracle.Oracle(lat.Lx, lat.Ly)
            lab_o, nd_o = o.domains(th, 32 if dtype == "f32" else 64)
            np.testing.assert_array_equal(got[0], lab_o)
            assert got[3] == nd_o
        # without labels, and the small lattice again after the big one
        a = small.domains_noalloc(want_labels=False)
        b = small.domains(want_labels=False)
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[2], b[2])
        assert a[3] == b[3] and a[4] == b[4]
    finally:
        big.close()
        small.close()


def test_noalloc_domains_size_limit(xyl):
    lat = quenched(xyl, 2048, 2048, 7, 200)
    try:
        same(lat.domains_noalloc(), lat.domains())
    finally:
        lat.close()
    lat = xyl.Lattice(2048, 2052, dtype="f32", schedule=[(0, 0.5)], seed=1)
    try:
        lat.init_random()
        with pytest.raises(xyl.XylError) as e:
            lat.domains_noalloc()
        assert e.value.code == -1 and "2^22" in str(e.value)
    finally:
        lat.close()
