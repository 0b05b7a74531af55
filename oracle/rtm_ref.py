"""FP64 CPU reference of the RTM image product (test infrastructure only).

Section 3.3 compares inverted velocity models through the migrated images
they give. The image here is the migration J^T (the oracle's born_mig) of
the observed data with the direct arrival muted, followed by a 5-point
Laplacian that removes the low-wavenumber backscatter of the
cross-correlation imaging condition. The mute and the filter are readings
(the paper names neither): a half-cosine ramp starting at the direct
arrival's time plus a pad, and -(d2/dz2 + d2/dx2) in grid units with zero
outside the image. Plain per-trace and per-cell loops; only tests may import
this module.
"""
from __future__ import annotations

import math

import numpy as np

from . import born_mig


def mute_weights(grid, acq, mute_v: float, mute_pad: float, mute_taper: float) -> np.ndarray:
    """Packed-data weights (shot, receiver, time): 0 while n dt <= t0, a
    half-cosine ramp over mute_taper seconds, then 1, with t0 = source-receiver
    distance / mute_v + mute_pad (off-grid offsets included)."""
    out = []
    for s in range(acq.nshots):
        nt = acq.nt_of(s, grid)
        sz = acq.src_z[s] + (acq.src_fz[s] if acq.src_fz is not None else 0.0)
        sx = acq.src_x[s] + (acq.src_fx[s] if acq.src_fx is not None else 0.0)
        for r in range(int(acq.rec_ptr[s]), int(acq.rec_ptr[s + 1])):
            rz = acq.rec_z[r] + (acq.rec_fz[r] if acq.rec_fz is not None else 0.0)
            rx = acq.rec_x[r] + (acq.rec_fx[r] if acq.rec_fx is not None else 0.0)
            t0 = math.hypot(float(rz) - float(sz), float(rx) - float(sx)) * grid.h / mute_v + mute_pad
            w = np.empty(nt)
            for n in range(nt):
                u = min(max((n * grid.dt - t0) / max(mute_taper, 1e-12), 0.0), 1.0)
                w[n] = 0.5 - 0.5 * math.cos(math.pi * u)
            out.append(w)
    return np.concatenate(out) if out else np.zeros(0)


def laplacian5(img: np.ndarray) -> np.ndarray:
    """4 y[i, j] minus its four neighbours, neighbours outside the image
    taken as zero."""
    y = np.asarray(img, np.float64)
    nz, nx = y.shape
    out = np.empty_like(y)
    for i in range(nz):
        for j in range(nx):
            acc = 4.0 * y[i, j]
            if i > 0:
                acc -= y[i - 1, j]
            if i + 1 < nz:
                acc -= y[i + 1, j]
            if j > 0:
                acc -= y[i, j - 1]
            if j + 1 < nx:
                acc -= y[i, j + 1]
            out[i, j] = acc
    return out


def rtm(grid, acq, v, d_obs, mute_v: float = 0.0, mute_pad: float = 0.0, mute_taper: float = 0.0) -> np.ndarray:
    """Laplacian of the migration of the (muted, if mute_v > 0) data."""
    d = np.asarray(d_obs, np.float64)
    if mute_v > 0.0:
        d = d * mute_weights(grid, acq, mute_v, mute_pad, mute_taper)
    return laplacian5(born_mig(grid, acq, v, d))
