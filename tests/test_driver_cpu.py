"""Host logic of the FWI driver (no GPU): band filter, line search, grids,
time-to-error bookkeeping."""
import numpy as np
import pytest

pytest.importorskip("torch")
from paper_2403_17518_amd import fwi_driver as D  # noqa: E402


def test_lowpass_is_zero_phase_and_cuts_high_frequencies():
    dt = 1e-3
    t = np.arange(2000) * dt
    lo = np.sin(2 * np.pi * 2.0 * t)
    hi = np.sin(2 * np.pi * 40.0 * t)
    y = D.lowpass(lo + hi, dt, 8.0)
    mid = slice(500, 1500)
    assert np.max(np.abs(y[mid] - lo[mid])) < 2e-2          # no phase shift, passband kept
    assert np.max(np.abs(D.lowpass(hi, dt, 8.0)[mid])) < 1e-3


def test_parabola_step_finds_the_minimum_of_a_quadratic():
    f = lambda a: 3.0 * (a - 0.7) ** 2 + 1.0
    a0 = 0.25
    assert abs(D.parabola_step(f(0), f(a0), f(2 * a0), a0) - 0.7) < 1e-12
    # clamped to 4 a0 when the minimum is far
    g = lambda a: (a - 10.0) ** 2
    assert D.parabola_step(g(0), g(a0), g(2 * a0), a0) == 4 * a0
    # concave and uphill: no step
    assert D.parabola_step(1.0, 2.0, 4.0, a0) == 0.0


def test_net_grid_padding():
    assert D.net_grid(200, 600, 3) == (208, 608)
    assert D.net_grid(176, 848, 3) == (184, 856)
    # odd sides: the odd padding cell goes below / right
    assert D.net_grid(175, 848, 3) == (184, 856)
    assert D.net_grid(221, 601, 3) == (224, 608) and D.net_grid(221, 601, 4) == (224, 608)


def test_time_to_error():
    plain = [{"model_error": e, "wall_s": i, "solves": 4 * i} for i, e in enumerate([1.0, 0.9, 0.8])]
    net = [{"model_error": e, "wall_s": 2 * i, "solves": 8 * i} for i, e in enumerate([0.95, 0.79, 0.6])]
    s = D.time_to_error(plain, net)
    assert s["target_model_error"] == 0.8 and s["net_iters"] == 2 and s["net_wall_s"] == 2


def test_bb_short_step_on_quadratics():
    import torch
    # 1-D quadratic f = a x^2 / 2: the two-point step is exactly 1/a
    a = 3.7
    dx = torch.tensor([0.4], dtype=torch.float64)
    assert abs(D.bb_short(dx, a * dx) - 1 / a) < 1e-12
    # diagonal quadratic: alpha_short lies between 1/max(a) and 1/min(a)
    A = torch.tensor([1.0, 2.0, 5.0], dtype=torch.float64)
    dx = torch.tensor([0.3, -0.2, 0.1], dtype=torch.float64)
    al = D.bb_short(dx, A * dx)
    assert 1 / 5.0 <= al <= 1.0
    # negative curvature: no step
    assert D.bb_short(dx, -dx) is None


def test_lbfgs_two_loop_secant_and_quadratic():
    import torch
    rng = np.random.default_rng(0)
    n = 6
    M = rng.standard_normal((n, n))
    A = torch.tensor(M @ M.T + n * np.eye(n))
    # the newest pair satisfies the secant equation H y = s
    s1 = torch.tensor(rng.standard_normal(n))
    s2 = torch.tensor(rng.standard_normal(n))
    pairs = [(s1, A @ s1), (s2, A @ s2)]
    assert torch.allclose(D.lbfgs_two_loop(A @ s2, pairs), s2, atol=1e-10)
    # one pair of a multiple of the identity gives its inverse exactly
    c = 2.5
    g = torch.tensor(rng.standard_normal(n))
    assert torch.allclose(D.lbfgs_two_loop(g, [(s1, c * s1)]), g / c, atol=1e-12)
    # BFGS on a quadratic with exact line searches: after n steps H = A^-1
    x = torch.tensor(rng.standard_normal(n))
    b = torch.tensor(rng.standard_normal(n))
    pairs = []
    gr = A @ x - b
    for _ in range(n):
        d = -(D.lbfgs_two_loop(gr, pairs) if pairs else gr)
        t = -float(gr @ d) / float(d @ A @ d)      # exact minimiser along d
        xn = x + t * d
        gn = A @ xn - b
        pairs.append((xn - x, gn - gr))
        x, gr = xn, gn
    assert torch.allclose(x, torch.linalg.solve(A, b), atol=1e-8)


def test_ssim_properties():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((40, 60)).cumsum(0).cumsum(1)
    r = float(x.max() - x.min())
    assert abs(D.ssim(x, x, r) - 1.0) < 1e-12
    assert abs(D.ssim(x, x + 0.0, r) - D.ssim(x, x, r)) < 1e-15
    y = x + 0.05 * r * rng.standard_normal(x.shape)
    assert abs(D.ssim(x, y, r) - D.ssim(y, x, r)) < 1e-12         # symmetric
    z = x + 0.2 * r * rng.standard_normal(x.shape)
    assert D.ssim(x, z, r) < D.ssim(x, y, r) < 1.0                 # more noise, lower
    # constant images: the luminance term alone, in closed form
    c1 = (0.01 * 10.0) ** 2
    v = D.ssim(np.full((20, 20), 3.0), np.full((20, 20), 5.0), 10.0)
    assert abs(v - (2 * 15 + c1) / (9 + 25 + c1)) < 1e-12


class _QuadCtx:
    """Stand-in for the propagation context: misfit 1/2 ||v - v*||^2."""
    device = "cpu"

    def __init__(self, v_star):
        self.v_star = v_star

    def _phi(self, v):
        return 0.5 * float(((v - self.v_star).double() ** 2).sum())

    def gradient_pair(self, grid, acq, v, d_obs, scale=-1.0):
        g = (v - self.v_star).float()
        return g, self._phi(v), scale * g

    def fwi_gradient(self, grid, acq, v, d_obs):
        return (v - self.v_star).float(), self._phi(v), None

    def fwi_misfit(self, grid, acq, v, d_obs):
        return self._phi(v)

    def stats(self):
        return {"cell_updates": 0.0}


class _Net:
    """Stand-in for the network: a fixed loss history and a direction maker."""

    def __init__(self, loss, direction):
        self.loss, self.direction, self.resets = loss, direction, []

    def deblur_train(self, x, y, steps, lr):
        return np.asarray(self.loss, np.float32)

    def deblur_apply(self, g):
        return self.direction(g)

    def reset(self, seed):
        self.resets.append(seed)


def _run(net, monkeypatch):
    import torch
    monkeypatch.setattr(D, "_sync", lambda: None)
    rng = np.random.default_rng(0)
    v_star = torch.from_numpy((2000.0 + 100.0 * rng.standard_normal((6, 7))).astype(np.float32))
    v0 = (v_star + 50.0 * torch.from_numpy(rng.standard_normal((6, 7)).astype(np.float32))).numpy()
    grid = type("G", (), {"v_ref": 3000.0})()
    run = D.FwiRun(_QuadCtx(v_star), grid, None, v0, D.FwiOptions(method="plain"), v_true=v_star.numpy())
    run._updates_per_pass = 1.0
    run.t0 = 0.0
    run.opts = D.FwiOptions(method="net")
    run.net = net
    return run


def test_network_direction_without_decrease_falls_back_to_the_gradient(monkeypatch):
    """A direction that passes the descent test (a 1e-4 share of the paper's
    gradient g = -grad phi, which the network receives) but is otherwise
    orthogonal to it and large: no trial step lowers the misfit, so the
    iteration takes the plain gradient instead."""
    import torch

    def bad(g):
        g = g.double()
        w = torch.ones_like(g) - (torch.ones_like(g) * g).sum() / (g * g).sum() * g
        return (1e3 * w / torch.linalg.norm(w) + 1e-4 * g).float()
    run = _run(_Net([1.0, 0.5], bad), monkeypatch)
    e_before = run.model_error()
    rec = run.iteration(None, None, 0, 0, 3.0)
    assert rec["fallback"] == "no decrease"
    assert rec["max_dv"] > 0 and run.model_error() < e_before
    assert run.net.resets == []


def test_diverged_training_is_discarded(monkeypatch):
    import torch
    run = _run(_Net([1.0, 1e9], lambda g: g), monkeypatch)
    e_before = run.model_error()
    rec = run.iteration(None, None, 1, 0, 8.0)
    assert rec["fallback"] == "diverged" and len(run.net.resets) == 1
    assert run.model_error() < e_before


def test_good_network_direction_is_taken(monkeypatch):
    run = _run(_Net([1.0, 0.1], lambda g: 2.0 * g), monkeypatch)
    e_before = run.model_error()
    rec = run.iteration(None, None, 0, 0, 3.0)
    assert rec["fallback"] is False and rec["max_dv"] > 0
    assert run.model_error() < e_before
