"""Pins of the oracle's random numbers (CPU only).

* Philox4x32-10 against an independent implementation: the host/device Philox
  engine that ships as a source header with PyTorch (ATen PhiloxRNGEngine.h),
  compiled here with g++.  Its counter is (offset_lo, offset_hi, subseq_lo,
  subseq_hi) and its key (seed_lo, seed_hi), so any raw (counter, key) block can
  be requested from it.
* The uniform map at its closed-form extremes.
* Box-Muller as polar coordinates: a pair of normals has squared radius
  -2 ln U1 and angle 2 pi U2, which fixes the word-to-site mapping and the
  cosine/sine branch without retyping the formula.
* Moments and a Kolmogorov-Smirnov test of the normals.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.stats

import oracle

HELPER = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long sub = c2 | (c3 << 32);
    unsigned long long off = c0 | (c1 << 32);
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def torch_philox():
    import torch.utils.cpp_extension as ce
    inc = ce.include_paths()[0]
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch Philox header not present")
    d = tempfile.mkdtemp(prefix="philox_pin_")
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(HELPER)
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc, src, "-o", exe], check=True)

    def run(blocks):
        inp = "\n".join(" ".join(str(int(v)) for v in (*c, *k)) for c, k in blocks) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [np.array([int(v) for v in line.split()], dtype=np.uint32) for line in out.strip().split("\n")]

    return run


def test_philox_matches_independent_implementation(torch_philox):
    rng = np.random.default_rng(1234)
    blocks = [((0, 0, 0, 0), (0, 0)),
              ((0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF)),
              ((1, 2, 3, 4), (5, 6)),
              ((0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF), (0, 1))]
    for _ in range(60):
        blocks.append((tuple(int(v) for v in rng.integers(0, 2**32, 4)),
                       tuple(int(v) for v in rng.integers(0, 2**32, 2))))
    ref = torch_philox(blocks)
    for (c, k), r in zip(blocks, ref):
        np.testing.assert_array_equal(oracle.philox(c, k), r)


def test_uniform_extremes():
    assert oracle.uniform(0) == 0.5 * 2.0 ** -23
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -23
    assert oracle.uniform(511) == oracle.uniform(0)          # low 9 bits dropped
    assert oracle.uniform(512) == 1.5 * 2.0 ** -23
    # the uniform is exactly representable in binary32
    for r in (0, 1 << 31, 0xFFFFFFFF, 123456789):
        u = oracle.uniform(r)
        assert float(np.float32(u)) == u


def test_box_muller_polar_identity():
    """For each pair of sites sharing words (2p, 2p+1) of one Philox block,
    n_even^2 + n_odd^2 = -2 ln U(w_2p) and atan2(n_odd, n_even) = 2 pi U(w_2p+1)."""
    o = oracle.Oracle(8, 4, seed=0xDEADBEEF12345678, replica=7)
    for k in (0, 1, 2**33 + 5):
        n = o.normals(k).ravel()
        for i in range(0, o.N, 2):
            r = oracle.philox((i >> 2, 7, k & 0xFFFFFFFF, k >> 32), (0x12345678, 0xDEADBEEF))
            p = (i & 3) >> 1
            u1, u2 = oracle.uniform(r[2 * p]), oracle.uniform(r[2 * p + 1])
            assert math.isclose(n[i] ** 2 + n[i + 1] ** 2, -2.0 * math.log(u1), rel_tol=1e-13)
            ang = math.atan2(n[i + 1], n[i]) % (2 * math.pi)
            assert abs(ang - 2 * math.pi * u2) < 1e-12


def test_normals_distribution():
    o = oracle.Oracle(256, 256, seed=3, replica=1)
    x = np.concatenate([o.normals(k).ravel() for k in range(4)])
    n = len(x)
    assert abs(x.mean()) < 4 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    kurt = np.mean(x ** 4) / np.mean(x ** 2) ** 2
    assert abs(kurt - 3.0) < 4 * math.sqrt(96.0 / n)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3


def test_streams_are_distinct():
    """Different (seed, replica, step) give uncorrelated draws; the init stream differs."""
    a = oracle.Oracle(64, 64, seed=5, replica=0)
    b = oracle.Oracle(64, 64, seed=5, replica=1)
    c = oracle.Oracle(64, 64, seed=6, replica=0)
    xs = [a.normals(10).ravel(), a.normals(11).ravel(), b.normals(10).ravel(), c.normals(10).ravel()]
    for i in range(len(xs)):
        for j in range(i + 1, len(xs)):
            assert abs(np.corrcoef(xs[i], xs[j])[0, 1]) < 5 / math.sqrt(len(xs[i]))


def test_init_stream_uniform():
    o = oracle.Oracle(128, 128, seed=0)
    th, om = o.init_random()
    assert np.all(om == 0.0)
    assert th.min() > -math.pi and th.max() < math.pi
    assert scipy.stats.kstest(th.ravel(), "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    # the init stream is the reserved step counter 2^64 - 1
    r = oracle.philox((0, 0, 0xFFFFFFFF, 0xFFFFFFFF), (0, 0))
    assert th.ravel()[1] == math.pi * (2.0 * oracle.uniform(r[1]) - 1.0)


def test_schedule_piecewise_linear():
    o = oracle.Oracle(4, 4, schedule=[(0, 1.5), (1000, 0.0)])
    assert o.temperature(0) == 1.5
    assert o.temperature(500) == 0.75
    assert o.temperature(1000) == 0.0
    assert o.temperature(10 ** 6) == 0.0
    o2 = oracle.Oracle(4, 4, schedule=[(100, 1.0), (200, 2.0), (400, 0.0)])
    assert o2.temperature(0) == 1.0
    assert o2.temperature(150) == 1.5
    assert o2.temperature(300) == 1.0
    assert o2.temperature(400) == 0.0
    o3 = oracle.Oracle(4, 4, schedule=[(0, 0.7)])
    assert o3.temperature(12345) == 0.7
