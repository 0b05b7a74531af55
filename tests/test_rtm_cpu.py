"""Pins of the oracle's RTM image product (the direct-arrival mute and the
5-point Laplacian; oracle/rtm_ref.py) and the host image score (no GPU)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import rtm_ref
from synth import configs
from paper_2403_17518_amd.rtm import image_score


def test_mute_layout_and_ramp():
    wl = configs.ragged_small()
    g, a = wl.grid, wl.acq
    v, pad, taper = 1500.0, 0.02, 0.03
    m = rtm_ref.mute_weights(g, a, v, pad, taper)
    assert m.shape == (a.data_size(g),)
    pos = 0
    for s in range(a.nshots):
        nt, nr = a.nt_of(s, g), a.nrec(s)
        block = m[pos:pos + nt * nr].reshape(nr, nt)
        pos += nt * nr
        t = np.arange(nt) * g.dt
        for k in range(nr):
            r = int(a.rec_ptr[s]) + k
            d = np.hypot((a.rec_x[r] - a.src_x[s]) * g.h, (a.rec_z[r] - a.src_z[s]) * g.h)
            t0 = d / v + pad
            assert np.all(block[k][t <= t0] == 0.0)
            assert np.all(block[k][t >= t0 + taper] == 1.0)
            assert np.all(np.diff(block[k]) >= 0.0)
            mid = (t > t0) & (t < t0 + taper)
            assert np.all((block[k][mid] > 0.0) & (block[k][mid] <= 1.0))
            # half-cosine: the ramp's midpoint weighs 1/2
            u = (t[mid] - t0) / taper
            assert np.allclose(block[k][mid], np.sin(0.5 * np.pi * u) ** 2, rtol=0, atol=1e-14)
    assert pos == m.size


def test_mute_uses_off_grid_offsets():
    wl = configs.ragged_small()
    g, a = wl.grid, wl.acq
    a0 = a.subset([0])
    n = int(a0.rec_ptr[1])
    a1 = a.subset([0])
    a1.src_fz, a1.src_fx = np.zeros(1, np.float32), np.zeros(1, np.float32)
    a1.rec_fz, a1.rec_fx = np.zeros(n, np.float32), np.full(n, 0.5, np.float32)
    m0 = rtm_ref.mute_weights(g, a0, 1500.0, 0.0, 0.02)
    m1 = rtm_ref.mute_weights(g, a1, 1500.0, 0.0, 0.02)
    assert m0.shape == m1.shape and not np.array_equal(m0, m1)
    a1.rec_fx = np.zeros(n, np.float32)
    assert np.array_equal(rtm_ref.mute_weights(g, a1, 1500.0, 0.0, 0.02), m0)


def test_laplacian_of_quadratic_constant_and_impulse():
    z, x = np.meshgrid(np.arange(9.0), np.arange(11.0), indexing="ij")
    L = rtm_ref.laplacian5(z ** 2 + 3.0 * x ** 2)
    assert np.allclose(L[1:-1, 1:-1], -8.0)          # -(2 + 6)
    Lc = rtm_ref.laplacian5(np.full((5, 6), 2.5))
    assert np.allclose(Lc[1:-1, 1:-1], 0.0)
    assert Lc[0, 0] == pytest.approx(5.0)            # two zero neighbours outside
    d = np.zeros((7, 8))
    d[3, 4] = 1.0
    Ld = rtm_ref.laplacian5(d)
    assert Ld[3, 4] == 4.0 and Ld[2, 4] == Ld[4, 4] == Ld[3, 3] == Ld[3, 5] == -1.0
    assert np.count_nonzero(Ld) == 5


def test_laplacian_matches_a_zero_padded_convolution():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((13, 17))
    k = np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])
    assert np.allclose(rtm_ref.laplacian5(y), ndimage.convolve(y, k, mode="constant", cval=0.0), atol=1e-13)


def test_image_score():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((20, 30))
    assert image_score(a, a) == pytest.approx(1.0)
    assert image_score(a, -2.0 * a) == pytest.approx(-1.0)
    b = a.copy()
    b[:5] = rng.standard_normal((5, 30))
    assert image_score(a, b, top=5) == pytest.approx(1.0)
    assert image_score(a, b) < 1.0
    assert image_score(np.zeros_like(a), a) == 0.0
