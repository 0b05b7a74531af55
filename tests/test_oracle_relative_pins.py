"""Pins of the oracle's relative-perturbation Born operator (section 2.2
eq. 12: the Born operator acts on dm / m_o), J_rel = J diag(v).

Checked against facts that do not depend on the oracle's own code: J_rel
is the derivative of the forward map with respect to ln v (Taylor test
along v exp(eps dm): the remainder is second order, so halving eps divides
it by 4, while a missing or doubled factor v leaves a first-order remainder
that only halves), the gradient it returns is the derivative of the misfit
with respect to ln v (central differences), the migration is its exact
transpose (dot-product test), and the doubly migrated image is symmetric.
"""
from dataclasses import replace

import numpy as np

import oracle
from synth import Acquisition, Grid, ricker

GRID = Grid(nz=14, nx=17, nb=5, h=10.0, dt=1e-3, nt_max=120, v_ref=3000.0)
REL = replace(GRID, relative=True)


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    v = 2000.0 + 600.0 * rng.random((GRID.nz, GRID.nx))
    acq = Acquisition(src_z=[2, 5], src_x=[3, 12], rec_ptr=[0, 3, 7],
                      rec_z=[1, 6, 12, 2, 2, 9, 13], rec_x=[0, 9, 16, 4, 11, 1, 7],
                      wavelet=ricker(25.0, 1e-3, GRID.nt_max))
    return v, acq, rng


def test_relative_born_is_the_log_velocity_derivative():
    v, acq, rng = _setup(0)
    dm = 0.05 * rng.standard_normal(v.shape)
    f0 = oracle.forward(GRID, acq, v)
    lin = oracle.born_demig(REL, acq, v, dm)
    errs = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        errs.append(np.linalg.norm(oracle.forward(GRID, acq, v * np.exp(eps * dm)) - f0 - eps * lin))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, (r1, r2)
    # the absolute operator is not that derivative: its remainder is first order
    lin_abs = oracle.born_demig(GRID, acq, v, dm)
    e_abs = [np.linalg.norm(oracle.forward(GRID, acq, v * np.exp(eps * dm)) - f0 - eps * lin_abs)
             for eps in (5e-2, 2.5e-2)]
    assert e_abs[0] / e_abs[1] < 2.5


def test_relative_born_is_absolute_born_of_v_dm():
    v, acq, rng = _setup(1)
    dm = rng.standard_normal(v.shape)
    a = oracle.born_demig(REL, acq, v, dm)
    b = oracle.born_demig(GRID, acq, v, v * dm)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_dot_product_relative():
    v, acq, rng = _setup(2)
    x = rng.standard_normal(v.shape)
    y = rng.standard_normal(acq.data_size(GRID))
    lhs = np.dot(oracle.born_demig(REL, acq, v, x), y)
    rhs = np.sum(x * oracle.born_mig(REL, acq, v, y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_relative_gradient_is_the_log_velocity_gradient():
    v, acq, rng = _setup(3)
    d_obs = oracle.forward(GRID, acq, v * (1.0 + 0.05 * rng.random(v.shape)))
    g, phi, _ = oracle.gradient(REL, acq, v, d_obs)
    g_abs, phi_abs, _ = oracle.gradient(GRID, acq, v, d_obs)
    assert phi == phi_abs
    x = rng.standard_normal(v.shape)
    eps = 1e-4
    fd = (oracle.gradient(GRID, acq, v * np.exp(eps * x), d_obs)[1]
          - oracle.gradient(GRID, acq, v * np.exp(-eps * x), d_obs)[1]) / (2.0 * eps)
    assert abs(fd - np.sum(g * x)) < 1e-6 * abs(fd), (fd, np.sum(g * x))
    # and not the velocity gradient (they differ by the factor v ~ 2000-2600)
    assert abs(fd - np.sum(g_abs * x)) > 0.5 * abs(fd)


def test_relative_pair_is_symmetric_and_psd():
    v, acq, rng = _setup(4)
    x, y = rng.standard_normal(v.shape), rng.standard_normal(v.shape)
    hx, hy = oracle.born_pair(REL, acq, v, x), oracle.born_pair(REL, acq, v, y)
    a, b = np.sum(y * hx), np.sum(x * hy)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert np.sum(x * hx) > 0.0
