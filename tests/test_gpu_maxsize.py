"""Lattices at the largest supported size (just under 2^31 sites, the limit of
int32 domain labels), through the C-ABI: a square one whose rows run as twelve
column tiles in the two-step pass, and one with rows of 2^20 sites (wider than
any tiling, so single steps).  Checked where the oracle can follow:

* the initial angles at sampled sites, up to the last one, bit for bit against
  the oracle's Philox and uniform map (the init stream);
* four steps at T = 0 (no noise) on bands of rows at the top, the middle and
  the bottom (across the periodic seam): the oracle advances each band as its
  own lattice, and the rows at least four away from the band's ends match to
  the FP32 bar;
* the two-step pass and single steps, bit for bit on the same bands;
* the domain size distribution: sizes times counts sum to N, counts to the
  number of domains, and the largest size is the one reported.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SHAPES = [(46336, 46336), (1 << 20, 2046)]
NSTEPS = 4
ROWS = 8          # rows compared per band


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def band_rows(Ly):
    """Row indices of three bands (ROWS rows each plus NSTEPS on each side)."""
    out = []
    for y0 in (0, Ly // 2 - ROWS // 2, Ly - ROWS):
        out.append(np.arange(y0 - NSTEPS, y0 + ROWS + NSTEPS) % Ly)
    return out


def read_rows(lat, rows):
    import torch
    t = lat.theta_tensor()
    idx = torch.as_tensor(rows, device=t.device)
    return t.index_select(0, idx).double().cpu().numpy()


@pytest.mark.parametrize("Lx,Ly", SHAPES)
def test_largest_lattices(xyl, Lx, Ly):
    import torch
    N = Lx * Ly
    assert N < 2 ** 31 - 1
    say("max size", Lx, Ly, N)
    params = dict(Jx=1.0, Jy=-0.1, h=0.5, gamma=1.0, dt=0.01)
    seed, replica = 9, 5
    lat = xyl.Lattice(Lx, Ly, dtype="f32", schedule=[(0, 0.0)], seed=seed, replica=replica, **params)
    try:
        lat.set_fusion(2)
        fused = lat.fusion()[1] > 0
        say("two steps per pass:", fused)
        lat.init_random()
        # initial angles at sampled sites, the last one included
        t = lat.theta_tensor().view(-1)
        rng = np.random.default_rng(1)
        idx = np.unique(np.concatenate([rng.integers(0, N, 200), [0, Lx - 1, N - Lx, N - 1]]))
        got = t.index_select(0, torch.as_tensor(idx, device=t.device)).cpu().numpy()
        want = []
        for i in idx:
            r = oracle.philox([int(i) >> 2, replica, 0xFFFFFFFF, 0xFFFFFFFF], [seed & 0xFFFFFFFF, seed >> 32])
            want.append(np.float32(np.pi * (2.0 * oracle.uniform(int(r[int(i) & 3])) - 1.0)))
        np.testing.assert_array_equal(got, np.array(want, dtype=np.float32))

        bands = band_rows(Ly)
        start = [read_rows(lat, b) for b in bands]
        lat.step(NSTEPS)
        assert lat.step_index == NSTEPS
        after2 = [read_rows(lat, b) for b in bands]
        # the same steps as single steps
        lat.init_random()
        lat.set_fusion(1)
        lat.step(NSTEPS)
        after1 = [read_rows(lat, b) for b in bands]
        for a, b in zip(after2, after1):
            np.testing.assert_array_equal(a, b)
        # the oracle on each band (T = 0: the noise is multiplied by zero)
        worst = 0.0
        for th0, th in zip(start, after2):
            o = oracle.Oracle(Lx, th0.shape[0], schedule=[(0, 0.0)], seed=seed, replica=replica, **params)
            tr, _ = o.run(th0, np.zeros_like(th0), 0, NSTEPS)
            inner = slice(NSTEPS, NSTEPS + ROWS)
            d = np.abs(np.remainder(th[inner] - tr[inner] + np.pi, 2 * np.pi) - np.pi).max()
            worst = max(worst, d)
        say("bands vs oracle max|dtheta|", worst)
        assert worst <= 1e-5

        _, sizes, counts, nd, mx = lat.domains(want_labels=False)
        say("domains", nd, "largest", mx, "distinct sizes", len(sizes))
        assert int(np.sum(sizes.astype(np.float64) * counts)) == N
        assert int(counts.sum()) == nd
        assert int(sizes.max()) == mx
        assert np.all(np.diff(sizes.astype(np.int64)) > 0)
    finally:
        lat.close()
        torch.cuda.empty_cache()
