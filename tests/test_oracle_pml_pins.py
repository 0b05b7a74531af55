"""Pins of the oracle's perfectly matched layer (the grid's `pml` flag).

The paper names the finite-difference method but no boundary; the PML is a
variant of the library's boundary, written in the symmetric form of the
stretched-coordinate wave equation (see the oracle's header). What fixes it:

* absorption: a small box with the layer reproduces the exact free-space 2D
  Green's function (scipy's Hankel function) as well as a box too large for
  any reflection to arrive, in a window where the sponge of the same width
  is visibly reflected; against a far boundary the layer leaves well under
  1% of the trace at 20 cells, over 20x less than the sponge;
* symmetry: the discrete operator is symmetric for every time shift, so
  source-receiver reciprocity holds to round-off in a heterogeneous model,
  also with the layer under a free surface;
* the Born operator is the derivative of the forward map (Taylor ratio 4),
  the migration is its transpose (dot-product test to round-off, regular and
  ragged geometries) and the gradient matches finite differences;
* stability over long records at the CFL limit of the workloads;
* nb = 0 (no layer) is the plain scheme.
A sign error or a dropped term in the edge fields breaks absorption or
symmetry; a wrong imaging term breaks the dot test or the gradient.
"""
from dataclasses import replace

import numpy as np
import pytest
from scipy.special import hankel2

import oracle
from synth import Acquisition, Grid, configs, ricker


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _tiny(seed=0, nz=14, nx=16, nb=5, nt=120, **kw):
    rng = np.random.default_rng(seed)
    grid = Grid(nz=nz, nx=nx, nb=nb, h=10.0, dt=1e-3, nt_max=nt, v_ref=3000.0, pml=True, **kw)
    v = 2000.0 + 500.0 * rng.random((nz, nx))
    acq = Acquisition(src_z=[2, 5], src_x=[3, 10], rec_ptr=[0, 3, 6],
                      rec_z=[1, 7, 2, 3, 3, 12], rec_x=[0, 8, 15, 5, 5, 1],
                      wavelet=ricker(25.0, 1e-3, nt))
    return grid, acq, v, rng


def _trace(half, nb, pml, T=0.8, v=2000.0, h=10.0, dt=1e-3, off=10):
    nt = int(round(T / dt))
    n = 2 * half + 1
    g = Grid(nz=n, nx=n, nb=nb, h=h, dt=dt, nt_max=nt, v_ref=v, pml=pml)
    a = Acquisition(src_z=[half], src_x=[half], rec_ptr=[0, 1],
                    rec_z=[half], rec_x=[half + off], wavelet=ricker(10.0, dt, nt))
    return oracle.forward(g, a, np.full((n, n), v))


def test_layer_absorbs_far_better_than_the_sponge():
    ref = _trace(half=200, nb=0, pml=False)       # boundary 2 km away
    for nb in (10, 20):
        e_pml = _rel(_trace(30, nb, True), ref)
        e_sp = _rel(_trace(30, nb, False), ref)
        print(f"nb={nb}: reflected part PML {e_pml:.2e}, sponge {e_sp:.2e}")
        assert e_pml < e_sp / 20.0
        assert e_pml < (5e-3 if nb == 10 else 2e-3)


def test_small_box_with_layer_matches_the_free_space_green_function():
    """200 m offset, 10 Hz, 0.6 s: in a box of 25 + 20 cells the sponge's
    reflections are inside the window; the layer's trace matches the exact
    Green's function as closely as an unbounded box does."""
    h, dt, T, v, f, off = 10.0, 1e-3, 0.6, 2000.0, 10.0, 200.0
    nt = int(round(T / dt))
    N = 1 << 15
    W = np.fft.rfft(ricker(f, dt, N)) * dt
    om = 2.0 * np.pi * np.fft.rfftfreq(N, dt)
    G = np.zeros_like(W)
    G[1:] = -0.25j * hankel2(0, om[1:] * off / v)
    exact = np.fft.irfft(W * G, N)[1:nt + 1] / dt
    k = int(round(off / h))
    big = _trace(200, 0, False, T=T, off=k)
    e_big = _rel(big, exact)
    e_pml = _rel(_trace(25, 20, True, T=T, off=k), exact)
    e_sp = _rel(_trace(25, 20, False, T=T, off=k), exact)
    print(f"vs exact Green's function: unbounded {e_big:.2e}, PML {e_pml:.2e}, sponge {e_sp:.2e}")
    assert e_pml < 1.2 * e_big + 1e-3
    assert e_sp > 5.0 * e_pml


@pytest.mark.parametrize("free_surface", [False, True])
def test_reciprocity(free_surface):
    grid, _, v, _ = _tiny(seed=3, nz=20, nx=24, nb=6, nt=150, free_surface=free_surface)
    w = ricker(20.0, grid.dt, grid.nt_max)
    a = Acquisition(src_z=[3], src_x=[4], rec_ptr=[0, 1], rec_z=[15], rec_x=[19], wavelet=w)
    b = Acquisition(src_z=[15], src_x=[19], rec_ptr=[0, 1], rec_z=[3], rec_x=[4], wavelet=w)
    da, db = oracle.forward(grid, a, v), oracle.forward(grid, b, v)
    assert np.linalg.norm(da) > 0
    assert _rel(da, db) < 1e-12


def test_layer_changes_the_data_only_through_the_boundary():
    """The layer and the sponge share their damping profile; early samples,
    before any wave reaches the padding, are identical."""
    grid, acq, v, _ = _tiny(seed=1, nz=40, nx=40, nb=8, nt=300)
    acq = Acquisition(src_z=[20], src_x=[20], rec_ptr=[0, 1], rec_z=[20], rec_x=[22],
                      wavelet=ricker(25.0, grid.dt, grid.nt_max))
    dp = oracle.forward(grid, acq, v)
    ds = oracle.forward(replace(grid, pml=False), acq, v)
    # the padding starts 20 cells (200 m) away: at most 2500 m/s, nothing
    # comes back from it within the first 60 ms
    assert np.array_equal(dp[:60], ds[:60])
    assert _rel(dp[60:], ds[60:]) > 1e-3


def test_no_layer_is_the_plain_scheme():
    grid, acq, v, _ = _tiny(seed=2, nb=0)
    assert np.array_equal(oracle.forward(grid, acq, v), oracle.forward(replace(grid, pml=False), acq, v))


@pytest.mark.parametrize("seed", [0, 7])
def test_born_taylor_ratio(seed):
    grid, acq, v, rng = _tiny(seed=seed)
    dv = 50.0 * rng.standard_normal((grid.nz, grid.nx))
    F0 = oracle.forward(grid, acq, v)
    Jdv = oracle.born_demig(grid, acq, v, dv)
    errs = [np.linalg.norm(oracle.forward(grid, acq, v + e * dv) - F0 - e * Jdv) for e in (0.4, 0.2, 0.1)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, (r1, r2)


@pytest.mark.parametrize("case", ["tiny", "ragged", "free_surface"])
def test_dot_product(case):
    if case == "ragged":
        wl = configs.ragged_small(nz=17, nx=60, nb=6, nshots=3, nt_lo=60, nt_hi=90)
        grid, acq, v = replace(wl.grid, pml=True), wl.acq, wl.v0
        rng = np.random.default_rng(5)
    else:
        grid, acq, v, rng = _tiny(seed=5, free_surface=case == "free_surface")
    x = rng.standard_normal((grid.nz, grid.nx))
    y = rng.standard_normal(acq.data_size(grid))
    lhs = np.dot(oracle.born_demig(grid, acq, v, x), y)
    rhs = np.sum(x * oracle.born_mig(grid, acq, v, y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_finite_difference_gradient():
    grid, acq, v, rng = _tiny(seed=6)
    d_obs = oracle.forward(grid, acq, v + 150.0 * rng.random((grid.nz, grid.nx)))
    g, phi, _ = oracle.gradient(grid, acq, v, d_obs)
    dv = rng.standard_normal((grid.nz, grid.nx))
    eps = 1e-2
    fp = oracle.gradient(grid, acq, v + eps * dv, d_obs)[1]
    fm = oracle.gradient(grid, acq, v - eps * dv, d_obs)[1]
    fd = (fp - fm) / (2.0 * eps)
    assert abs(fd - np.sum(g * dv)) < 1e-7 * abs(fd), (fd, np.sum(g * dv))


def test_long_record_decays_at_the_stability_limit():
    """8000 steps at v dt / h = 0.45 in a box of 41 + 2 x 20 cells: the
    wave leaves through the layer and the field dies away."""
    half, nb, T, v = 20, 20, 8.0, 4500.0
    d = _trace(half, nb, True, T=T, v=v, off=5)
    assert np.all(np.isfinite(d))
    peak = np.max(np.abs(d))
    assert np.max(np.abs(d[-500:])) < 1e-5 * peak
