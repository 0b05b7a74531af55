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
    with pytest.raises(ValueError):
        D.net_grid(175, 848, 3)


def test_time_to_error():
    plain = [{"model_error": e, "wall_s": i, "solves": 4 * i} for i, e in enumerate([1.0, 0.9, 0.8])]
    net = [{"model_error": e, "wall_s": 2 * i, "solves": 8 * i} for i, e in enumerate([0.95, 0.79, 0.6])]
    s = D.time_to_error(plain, net)
    assert s["target_model_error"] == 0.8 and s["net_iters"] == 2 and s["net_wall_s"] == 2
