"""Pins of the oracle's off-grid sources and receivers (bilinear weights).

Checked against facts that do not depend on the oracle's own code: the
exact 2D Green's function between off-grid points (second-order convergence
of the interpolated trace), linearity of the wave equation in its source
(an off-grid source is the weighted sum of the four on-grid ones), the
definition of interpolated sampling (an off-grid receiver records the
weighted sum of the four cells' records), exact reduction to the on-grid
operators at zero offsets, and the dot-product test and finite-difference
gradient with off-grid geometry.
"""
import numpy as np
import pytest
from scipy.special import hankel2

import oracle
from synth import Acquisition, Grid, ricker


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _acq(src, recs, nt, src_f=None, rec_f=None):
    """src = (z, x); recs = [(z, x), ...]; fractions as (fz, fx) pairs."""
    return Acquisition(src_z=[src[0]], src_x=[src[1]], rec_ptr=[0, len(recs)],
                       rec_z=[r[0] for r in recs], rec_x=[r[1] for r in recs], wavelet=ricker(25.0, 1e-3, nt),
                       src_fz=None if src_f is None else [src_f[0]], src_fx=None if src_f is None else [src_f[1]],
                       rec_fz=None if rec_f is None else [f[0] for f in rec_f],
                       rec_fx=None if rec_f is None else [f[1] for f in rec_f])


def _f32(*xs):
    """The fractions as the geometry stores them (float32)."""
    return [float(np.float32(x)) for x in xs]


def _model(nz=16, nx=18, seed=0):
    rng = np.random.default_rng(seed)
    return 2000.0 + 500.0 * rng.random((nz, nx)), rng


GRID = Grid(nz=16, nx=18, nb=5, h=10.0, dt=1e-3, nt_max=110, v_ref=3000.0)


def test_zero_offsets_equal_the_on_grid_operators():
    v, rng = _model()
    dv = rng.standard_normal(v.shape)
    on = _acq((3, 4), [(2, 9), (7, 15)], GRID.nt_max)
    off = _acq((3, 4), [(2, 9), (7, 15)], GRID.nt_max, src_f=(0.0, 0.0), rec_f=[(0.0, 0.0), (0.0, 0.0)])
    y = rng.standard_normal(on.data_size(GRID))
    assert np.array_equal(oracle.forward(GRID, on, v), oracle.forward(GRID, off, v))
    assert np.array_equal(oracle.born_demig(GRID, on, v, dv), oracle.born_demig(GRID, off, v, dv))
    assert np.array_equal(oracle.born_mig(GRID, on, v, y), oracle.born_mig(GRID, off, v, y))


@pytest.mark.parametrize("fz,fx", [(0.0, 0.3), (0.625, 0.0), (0.25, 0.75)])
def test_off_grid_receiver_records_the_weighted_cells(fz, fx):
    v, _ = _model(seed=1)
    corners = [(6, 9), (6, 10), (7, 9), (7, 10)]
    z32, x32 = _f32(fz, fx)
    w = [(1 - z32) * (1 - x32), (1 - z32) * x32, z32 * (1 - x32), z32 * x32]
    d4 = oracle.forward(GRID, _acq((3, 4), corners, GRID.nt_max), v).reshape(4, -1)
    d1 = oracle.forward(GRID, _acq((3, 4), [(6, 9)], GRID.nt_max, rec_f=[(fz, fx)]), v)
    ref = sum(wk * d4[k] for k, wk in enumerate(w))
    assert _rel(d1, ref) < 1e-13


@pytest.mark.parametrize("fz,fx", [(0.0, 0.5), (0.375, 0.0), (0.2, 0.9)])
def test_off_grid_source_is_the_weighted_on_grid_sources(fz, fx):
    v, rng = _model(seed=2)
    dv = rng.standard_normal(v.shape)
    recs = [(2, 1), (9, 12), (14, 17)]
    z32, x32 = _f32(fz, fx)
    w = [(1 - z32) * (1 - x32), (1 - z32) * x32, z32 * (1 - x32), z32 * x32]
    corners = [(5, 6), (5, 7), (6, 6), (6, 7)]
    off = _acq((5, 6), recs, GRID.nt_max, src_f=(fz, fx))
    d = oracle.forward(GRID, off, v)
    dd = oracle.born_demig(GRID, off, v, dv)
    ref = sum(wk * oracle.forward(GRID, _acq(c, recs, GRID.nt_max), v) for c, wk in zip(corners, w))
    ref_b = sum(wk * oracle.born_demig(GRID, _acq(c, recs, GRID.nt_max), v, dv) for c, wk in zip(corners, w))
    assert _rel(d, ref) < 1e-13
    assert _rel(dd, ref_b) < 1e-12


def test_dot_product_off_grid():
    v, rng = _model(seed=3)
    acq = Acquisition(src_z=[2, 6], src_x=[3, 11], rec_ptr=[0, 3, 6],
                      rec_z=[1, 7, 2, 3, 3, 12], rec_x=[0, 8, 15, 5, 5, 1], wavelet=ricker(25.0, 1e-3, GRID.nt_max),
                      src_fz=[0.3, 0.0], src_fx=[0.55, 0.25],
                      rec_fz=[0.5, 0.0, 0.125, 0.7, 0.7, 0.0], rec_fx=[0.0, 0.9, 0.5, 0.2, 0.2, 0.0])
    x = rng.standard_normal(v.shape)
    y = rng.standard_normal(acq.data_size(GRID))
    lhs = np.dot(oracle.born_demig(GRID, acq, v, x), y)
    rhs = np.sum(x * oracle.born_mig(GRID, acq, v, y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_finite_difference_gradient_off_grid():
    v, rng = _model(seed=4)
    acq = _acq((4, 5), [(2, 3), (8, 12), (11, 16)], GRID.nt_max, src_f=(0.4, 0.6),
               rec_f=[(0.5, 0.5), (0.0, 0.3), (0.8, 0.0)])
    d_obs = oracle.forward(GRID, acq, v + 150.0 * rng.random(v.shape))
    g, phi, _ = oracle.gradient(GRID, acq, v, d_obs)
    dv = rng.standard_normal(v.shape)
    eps = 1e-2
    fd = (oracle.gradient(GRID, acq, v + eps * dv, d_obs)[1] - oracle.gradient(GRID, acq, v - eps * dv, d_obs)[1])
    fd /= 2.0 * eps
    assert abs(fd - np.sum(g * dv)) < 1e-7 * abs(fd), (fd, np.sum(g * dv))


def _analytic_offgrid(h, dt, half, nb, fs=(0.3, 0.6), fr=(0.7, 0.25), T=0.45, v=2000.0, f=10.0, off=200.0):
    """Oracle trace between off-grid points and the exact 2D Green's trace at
    their true distance."""
    n = 2 * half + 1
    nt = int(round(T / dt))
    grid = Grid(nz=n, nx=n, nb=nb, h=h, dt=dt, nt_max=nt, v_ref=v)
    k = int(round(off / h))
    acq = Acquisition(src_z=[half], src_x=[half], rec_ptr=[0, 1], rec_z=[half], rec_x=[half + k],
                      wavelet=ricker(f, dt, nt), src_fz=[fs[0]], src_fx=[fs[1]], rec_fz=[fr[0]], rec_fx=[fr[1]])
    d = oracle.forward(grid, acq, np.full((n, n), v))
    fs, fr = _f32(*fs), _f32(*fr)
    r = h * np.hypot(fr[0] - fs[0], k + fr[1] - fs[1])
    N = 1 << 15
    W = np.fft.rfft(ricker(f, dt, N)) * dt
    om = 2.0 * np.pi * np.fft.rfftfreq(N, dt)
    G = np.zeros_like(W)
    G[1:] = -0.25j * hankel2(0, om[1:] * r / v)
    u = np.fft.irfft(W * G, N) / dt
    return d, u[1:nt + 1]


def test_off_grid_green_function_converges():
    """Bilinear spreading and sampling are second-order accurate: halving h
    cuts the error against the exact trace at the true positions ~4x."""
    d1, a1 = _analytic_offgrid(10.0, 1e-3, half=50, nb=20)
    d2, a2 = _analytic_offgrid(5.0, 5e-4, half=100, nb=40)
    e1, e2 = _rel(d1, a1), _rel(d2, a2)
    assert e1 < 3e-2, e1
    assert e2 < 0.4 * e1, (e1, e2)
    # and the on-grid-rounded positions are clearly worse at the coarse grid
    d0, _ = _analytic_offgrid(10.0, 1e-3, half=50, nb=20, fs=(0.0, 0.0), fr=(0.0, 0.0))
    assert _rel(d0, a1) > 2.0 * e1
