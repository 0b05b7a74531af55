"""Source time functions (inputs, not part of the propagation)."""
from __future__ import annotations

import numpy as np


def ricker(freq: float, dt: float, nt: int, t0: float | None = None,
           dtype=np.float64) -> np.ndarray:
    """Ricker wavelet ``(1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2)``.

    ``tau = n*dt - t0`` with the delay ``t0 = 1.5 / f`` by default (the
    paper names a Ricker source of a given peak frequency but no delay).
    """
    if t0 is None:
        t0 = 1.5 / freq
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (np.pi * freq * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(dtype)
