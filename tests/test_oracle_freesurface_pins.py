"""Pins of the oracle's pressure-free top surface (image method).

Against facts independent of the oracle's code: the exact half-space
Green's function (direct wave minus the wave of the image source mirrored
about the surface) with second-order convergence, the surface row staying
at zero, the dot-product test, the finite-difference gradient, and Pad/Pad^T
adjointness of the layout without top sponge rows.
"""
import numpy as np
import pytest
from scipy.special import hankel2

import oracle
from synth import Acquisition, Grid, ricker


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _green(r, v, f, dt, nt):
    N = 1 << 15
    W = np.fft.rfft(ricker(f, dt, N)) * dt
    om = 2.0 * np.pi * np.fft.rfftfreq(N, dt)
    G = np.zeros_like(W)
    G[1:] = -0.25j * hankel2(0, om[1:] * r / v)
    return (np.fft.irfft(W * G, N) / dt)[1:nt + 1]


def _halfspace(h, dt, zs, zr, half, nb, T=0.45, v=2000.0, f=10.0, off=200.0):
    """Oracle trace under a free surface and the exact half-space trace:
    G(r_direct) - G(r_image), the image source mirrored about row 0."""
    nz, nx = 2 * half + 1, 2 * half + 1
    nt = int(round(T / dt))
    grid = Grid(nz=nz, nx=nx, nb=nb, h=h, dt=dt, nt_max=nt, v_ref=v, free_surface=True)
    k = int(round(off / h))
    acq = Acquisition(src_z=[zs], src_x=[half], rec_ptr=[0, 1], rec_z=[zr], rec_x=[half + k],
                      wavelet=ricker(f, dt, nt))
    d = oracle.forward(grid, acq, np.full((nz, nx), v))
    r1 = h * np.hypot(zr - zs, k)
    r2 = h * np.hypot(zr + zs, k)
    return d, _green(r1, v, f, dt, nt) - _green(r2, v, f, dt, nt)


def test_half_space_green_function_converges():
    # source and receiver 40 m below the surface, 200 m apart
    d1, a1 = _halfspace(10.0, 1e-3, zs=4, zr=4, half=50, nb=20)
    d2, a2 = _halfspace(5.0, 5e-4, zs=8, zr=8, half=100, nb=40)
    e1, e2 = _rel(d1, a1), _rel(d2, a2)
    assert e1 < 2e-2, e1
    assert e2 < 0.5 * e1, (e1, e2)
    # without the image term the same data miss by far more: the surface
    # reflection is really there
    nt = d1.shape[0]
    direct = _green(10.0 * 20, 2000.0, 10.0, 1e-3, nt)
    assert _rel(d1, direct) > 10 * e1


def _small(seed=0, nz=14, nx=16, nb=5, nt=110):
    rng = np.random.default_rng(seed)
    grid = Grid(nz=nz, nx=nx, nb=nb, h=10.0, dt=1e-3, nt_max=nt, v_ref=3000.0, free_surface=True)
    v = 2000.0 + 500.0 * rng.random((nz, nx))
    acq = Acquisition(src_z=[2, 5], src_x=[3, 10], rec_ptr=[0, 3, 6],
                      rec_z=[1, 7, 2, 3, 3, 12], rec_x=[0, 8, 15, 5, 5, 1], wavelet=ricker(25.0, 1e-3, nt))
    return grid, acq, v, rng


def test_surface_row_stays_zero():
    grid, acq, v, _ = _small(seed=1)
    f = oracle.shot_fields(grid, acq, 0, v)
    assert grid.NZ == grid.nz + grid.nb
    assert np.all(f["u"][:, 0, :] == 0.0)
    assert np.abs(f["u"][:, 1, :]).max() > 0.0


def test_dot_product_free_surface():
    grid, acq, v, rng = _small(seed=2)
    x = rng.standard_normal((grid.nz, grid.nx))
    y = rng.standard_normal(acq.data_size(grid))
    lhs = np.dot(oracle.born_demig(grid, acq, v, x), y)
    rhs = np.sum(x * oracle.born_mig(grid, acq, v, y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_finite_difference_gradient_free_surface():
    grid, acq, v, rng = _small(seed=3)
    d_obs = oracle.forward(grid, acq, v + 150.0 * rng.random(v.shape))
    g, _, _ = oracle.gradient(grid, acq, v, d_obs)
    dv = rng.standard_normal(v.shape)
    eps = 1e-2
    fd = (oracle.gradient(grid, acq, v + eps * dv, d_obs)[1] - oracle.gradient(grid, acq, v - eps * dv, d_obs)[1])
    fd /= 2.0 * eps
    assert abs(fd - np.sum(g * dv)) < 1e-7 * abs(fd), (fd, np.sum(g * dv))


@pytest.mark.parametrize("window", [(0, 16), (3, 9)])
def test_pad_adjoint_pair_free_surface(window):
    grid, _, _, rng = _small(seed=4)
    x0, wn = window
    x = rng.standard_normal((grid.nz, grid.nx))
    P = oracle.pad(grid, x, x0, wn)
    assert P.shape == (grid.nz + grid.nb, wn + 2 * grid.nb)
    y = rng.standard_normal(P.shape)
    lhs = np.sum(P * y)
    rhs = np.sum(x * oracle.pad_adjoint(grid, y, x0, wn))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
