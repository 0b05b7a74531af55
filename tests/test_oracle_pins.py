"""Pins of the FP64 oracle against facts the paper and mathematics fix.

None of these compares the oracle with itself: each checks a closed form
(analytic 2D Green's function, polynomial exactness of the stencil), an
identity that a correct operator must satisfy (reciprocity, Taylor test of
the Born map, dot-product test of the adjoint, finite-difference gradient,
Pad/Pad^T adjointness, Gauss-Newton symmetry/positivity), or a special case
(zero source, linearity, zero residual). A dropped term, a wrong sign, a
transposed index or a missing fold in any oracle routine fails at least one.
"""
import numpy as np
import pytest
from scipy.special import hankel2

import oracle
from synth import Acquisition, Grid, ricker, configs


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _tiny(seed=0, nz=14, nx=16, nb=5, nt=120):
    rng = np.random.default_rng(seed)
    grid = Grid(nz=nz, nx=nx, nb=nb, h=10.0, dt=1e-3, nt_max=nt, v_ref=3000.0)
    v = 2000.0 + 500.0 * rng.random((nz, nx))
    acq = Acquisition(src_z=[2, 5], src_x=[3, 10], rec_ptr=[0, 3, 6],
                      rec_z=[1, 7, 2, 3, 3, 12], rec_x=[0, 8, 15, 5, 5, 1],
                      wavelet=ricker(25.0, 1e-3, nt))
    return grid, acq, v, rng


# --------------------------------------------------------------------------
# C1 forward: closed forms

def _analytic_trace(h, dt, half, nb, T=0.45, v=2000.0, f=10.0, off=200.0):
    """Oracle trace and the exact 2D Green's-function trace.

    For (1/v^2) u_tt - lap u = w(t) delta(x) the exact solution is the
    convolution of w with the 2D Green's function, whose Fourier transform
    (time dependence e^{+i w t}) is (-i/4) H0^(2)(w r / v).
    """
    n = 2 * half + 1
    nt = int(round(T / dt))
    grid = Grid(nz=n, nx=n, nb=nb, h=h, dt=dt, nt_max=nt, v_ref=v)
    k = int(round(off / h))
    acq = Acquisition(src_z=[half], src_x=[half], rec_ptr=[0, 1],
                      rec_z=[half], rec_x=[half + k], wavelet=ricker(f, dt, nt))
    d = oracle.forward(grid, acq, np.full((n, n), v))
    N = 1 << 15
    W = np.fft.rfft(ricker(f, dt, N)) * dt
    om = 2.0 * np.pi * np.fft.rfftfreq(N, dt)
    G = np.zeros_like(W)
    G[1:] = -0.25j * hankel2(0, om[1:] * off / v)
    u = np.fft.irfft(W * G, N) / dt
    # receiver sample n is the field at t_{n+1}
    return d, u[1:nt + 1]


def test_analytic_green_function_converges():
    d1, a1 = _analytic_trace(10.0, 1e-3, half=50, nb=20)
    d2, a2 = _analytic_trace(5.0, 5e-4, half=100, nb=40)
    e1, e2 = _rel(d1, a1), _rel(d2, a2)
    assert e1 < 1e-2, e1
    assert e2 < 0.5 * e1, (e1, e2)          # second order: ~4x smaller


def test_stencil_is_eighth_order_cross():
    """Read the Laplacian weights off a two-step impulse response and check
    they are exact on polynomials up to degree 9 and have no diagonal taps."""
    n, nb, nt = 31, 4, 2
    grid = Grid(nz=n, nx=n, nb=nb, h=7.0, dt=1e-3, nt_max=nt, v_ref=2000.0)
    w = np.zeros(nt)
    w[0] = 1.0
    c0 = 15
    acq = Acquisition(src_z=[c0], src_x=[c0], rec_ptr=[0, 0], rec_z=[],
                      rec_x=[], wavelet=w)
    f = oracle.shot_fields(grid, acq, 0, np.full((n, n), 1800.0))
    u1, u2 = f["u"][1], f["u"][2]
    i = c0 + nb
    cc = f["c"][i, i]
    base = u1[i, i]
    assert np.isclose(base, cc * 1.0 / grid.h ** 2)
    wts = [(u2[i, i] - 2.0 * base) * grid.h ** 2 / (2.0 * cc * base)]
    for k in range(1, 6):
        wx = u2[i, i + k] * grid.h ** 2 / (cc * base)
        wz = u2[i + k, i] * grid.h ** 2 / (cc * base)
        assert np.isclose(wx, wz, rtol=1e-12, atol=1e-15)
        assert np.isclose(u2[i, i - k], u2[i, i + k], rtol=1e-12, atol=1e-30)
        wts.append(wx)
    wts = np.array(wts)
    assert abs(wts[5]) < 1e-14                        # radius 4
    assert abs(u2[i + 1, i + 1]) < 1e-14 * abs(base)  # no diagonal taps
    k = np.arange(1, 5)
    assert abs(wts[0] + 2.0 * wts[1:5].sum()) < 1e-12          # constants
    assert abs(wts[1:5] @ k ** 2 - 1.0) < 1e-12                 # f'' of x^2
    for p in (4, 6, 8):                                          # order 8
        assert abs(wts[1:5] @ k.astype(float) ** p) < 1e-10


def test_sponge_absorbs_boundary_reflections():
    """A small domain with the sponge matches a large domain whose boundary
    is never reached; without the sponge the boundary reflects strongly."""
    h, dt, T, v = 10.0, 1e-3, 0.8, 2000.0
    nt = int(T / dt)
    w = ricker(10.0, dt, nt)

    def trace(half, nb):
        n = 2 * half + 1
        g = Grid(nz=n, nx=n, nb=nb, h=h, dt=dt, nt_max=nt, v_ref=v)
        a = Acquisition(src_z=[half], src_x=[half], rec_ptr=[0, 1],
                        rec_z=[half], rec_x=[half + 10], wavelet=w)
        return oracle.forward(g, a, np.full((n, n), v))

    ref = trace(half=200, nb=0)       # boundary 2 km away: no reflection
    with_sponge = trace(half=30, nb=30)
    without = trace(half=30, nb=0)
    e_s, e_n = _rel(with_sponge, ref), _rel(without, ref)
    # a damping sponge (not a PML) leaves a few percent of reflected energy
    assert e_s < 0.08, e_s
    assert e_n > 10.0 * e_s, (e_s, e_n)


# --------------------------------------------------------------------------
# C1: symmetry and special cases

def test_reciprocity_heterogeneous_model():
    grid, _, v, _ = _tiny(seed=3, nz=20, nx=24, nb=6, nt=150)
    w = ricker(20.0, grid.dt, grid.nt_max)
    a = Acquisition(src_z=[3], src_x=[4], rec_ptr=[0, 1], rec_z=[15], rec_x=[19], wavelet=w)
    b = Acquisition(src_z=[15], src_x=[19], rec_ptr=[0, 1], rec_z=[3], rec_x=[4], wavelet=w)
    da, db = oracle.forward(grid, a, v), oracle.forward(grid, b, v)
    assert np.linalg.norm(da) > 0
    assert _rel(da, db) < 1e-12


def test_zero_source_and_linearity_in_wavelet():
    grid, acq, v, rng = _tiny(seed=1)
    z = Acquisition(**{**acq.__dict__, "wavelet": np.zeros(grid.nt_max)})
    assert np.all(oracle.forward(grid, z, v) == 0.0)
    w1, w2 = rng.standard_normal(grid.nt_max), rng.standard_normal(grid.nt_max)
    A = lambda w: oracle.forward(grid, Acquisition(**{**acq.__dict__, "wavelet": w}), v)
    lhs = A(2.0 * w1 - 3.0 * w2)
    rhs = 2.0 * A(w1) - 3.0 * A(w2)
    assert _rel(lhs, rhs) < 1e-12


def test_zero_residual_gives_zero_misfit_and_gradient():
    grid, acq, v, _ = _tiny(seed=2)
    d = oracle.forward(grid, acq, v)
    g, phi, d_syn = oracle.gradient(grid, acq, v, d)
    assert phi == 0.0
    assert np.all(g == 0.0)
    assert np.array_equal(d_syn, d)


# --------------------------------------------------------------------------
# C2 Born: derivative of the forward map

@pytest.mark.parametrize("seed", [0, 7])
def test_born_taylor_ratio(seed):
    grid, acq, v, rng = _tiny(seed=seed)
    dv = 50.0 * rng.standard_normal((grid.nz, grid.nx))
    F0 = oracle.forward(grid, acq, v)
    Jdv = oracle.born_demig(grid, acq, v, dv)
    errs = [np.linalg.norm(oracle.forward(grid, acq, v + e * dv) - F0 - e * Jdv)
            for e in (0.4, 0.2, 0.1)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, (r1, r2)


def test_born_is_linear_in_perturbation():
    grid, acq, v, rng = _tiny(seed=4)
    x, y = rng.standard_normal((2, grid.nz, grid.nx))
    J = lambda q: oracle.born_demig(grid, acq, v, q)
    assert _rel(J(x + 2.0 * y), J(x) + 2.0 * J(y)) < 1e-12


# --------------------------------------------------------------------------
# C3 adjoint / gradient

@pytest.mark.parametrize("ragged", [False, True])
def test_dot_product(ragged):
    if ragged:
        wl = configs.ragged_small(nz=17, nx=60, nb=6, nshots=3, nt_lo=60, nt_hi=90)
        grid, acq, v = wl.grid, wl.acq, wl.v0
        rng = np.random.default_rng(5)
    else:
        grid, acq, v, rng = _tiny(seed=5)
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


def test_misfit_is_half_squared_residual():
    grid, acq, v, rng = _tiny(seed=8)
    d_obs = rng.standard_normal(acq.data_size(grid)) * 1e-3
    _, phi, d_syn = oracle.gradient(grid, acq, v, d_obs)
    assert np.isclose(phi, 0.5 * np.sum((d_syn - d_obs) ** 2), rtol=1e-13)
    assert _rel(d_syn, oracle.forward(grid, acq, v)) < 1e-12


def test_gradient_is_migration_of_residual():
    grid, acq, v, rng = _tiny(seed=9)
    d_obs = rng.standard_normal(acq.data_size(grid)) * 1e-3
    g, _, d_syn = oracle.gradient(grid, acq, v, d_obs)
    assert _rel(g, oracle.born_mig(grid, acq, v, d_syn - d_obs)) < 1e-13


@pytest.mark.parametrize("window", [(0, 16), (3, 9), (5, 1)])
def test_pad_adjoint_pair(window):
    grid = Grid(nz=7, nx=16, nb=4, h=10.0, dt=1e-3, nt_max=1, v_ref=2000.0)
    rng = np.random.default_rng(10)
    x0, wnx = window
    x = np.zeros((grid.nz, grid.nx))
    x[:, x0:x0 + wnx] = rng.standard_normal((grid.nz, wnx))
    y = rng.standard_normal((grid.nz + 2 * grid.nb, wnx + 2 * grid.nb))
    lhs = np.sum(oracle.pad(grid, x, x0, wnx) * y)
    rhs = np.sum(x * oracle.pad_adjoint(grid, y, x0, wnx))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # Pad is edge replication: corners of the padded box copy corners of the window
    P = oracle.pad(grid, x, x0, wnx)
    assert P[0, 0] == x[0, x0] and P[-1, -1] == x[-1, x0 + wnx - 1]


def test_imaging_condition_equals_second_time_derivative_form():
    """Eq. 11's secondary source is 2 dm/m^3 * d2u/dt2; in the discrete
    scheme V^2 dt^2 (L8 u^n + s^n) equals the damped second difference
    (1 + sigma dt/2) u^{n+1} - 2 u^n + (1 - sigma dt/2) u^{n-1}, so the
    migrated image also equals Pad^T((2/(V^3 dt^2)) sum lam^n * D2u^n)."""
    grid, acq, v, rng = _tiny(seed=11, nt=90)
    one = acq.subset([1])
    res = rng.standard_normal((one.nrec(0), grid.nt_max)) * 1e-3
    f = oracle.shot_fields(grid, one, 0, v, res)
    u, lam, a, b, c = f["u"], f["lam"], f["a"], f["b"], f["c"]
    nt = grid.nt_max
    um1 = np.concatenate([np.zeros((1,) + u.shape[1:]), u[:nt - 1]])
    d2 = u[1:nt + 1] / a - 2.0 * u[:nt] + (b / a) * um1   # (1+sdt/2), (1-sdt/2)
    V3dt2 = (np.sqrt(c) / grid.dt) ** 3 * grid.dt ** 2
    img = oracle.pad_adjoint(grid, (2.0 / V3dt2) * np.sum(lam * d2, axis=0))
    ref = oracle.born_mig(grid, one, v, res.ravel())
    assert _rel(img, ref) < 1e-10


# --------------------------------------------------------------------------
# C4: the Gauss-Newton Hessian J^T J

def test_gauss_newton_hessian_symmetric_psd():
    grid, acq, v, rng = _tiny(seed=12)
    x, y = rng.standard_normal((2, grid.nz, grid.nx))
    Hx = oracle.born_pair(grid, acq, v, x)
    Hy = oracle.born_pair(grid, acq, v, y)
    assert abs(np.sum(y * Hx) - np.sum(x * Hy)) < 1e-11 * abs(np.sum(y * Hx))
    Jx = oracle.born_demig(grid, acq, v, x)
    assert np.isclose(np.sum(x * Hx), np.dot(Jx, Jx), rtol=1e-11)
    assert np.sum(x * Hx) > 0.0


def test_shots_are_independent_and_summed():
    grid, acq, v, rng = _tiny(seed=13)
    y = rng.standard_normal(acq.data_size(grid))
    full = oracle.born_mig(grid, acq, v, y)
    off = acq.trace_offsets(grid)
    parts = sum(oracle.born_mig(grid, acq.subset([s]), v, y[off[s]:off[s + 1]])
                for s in range(acq.nshots))
    assert _rel(full, parts) < 1e-13
