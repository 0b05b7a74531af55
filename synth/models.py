"""Seeded synthetic velocity models (m/s), ``[nz][nx]`` float64.

They stand in for the paper's Marmousi and Volve models, which are not
available: same shape class (layered sediments, faults, a salt body),
velocities in the stated ranges, smooth starting models.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

SEED = 2403


def two_layer_anomaly(nz: int = 100, nx: int = 100, z_if: int = 50,
                      v1: float = 1500.0, v2: float = 2500.0,
                      amp: float = 200.0, zc: float = 30.0, xc: float = 50.0,
                      sigma: float = 8.0) -> tuple[np.ndarray, np.ndarray]:
    """Two-layer model with a Gaussian velocity anomaly.

    Returns ``(v_true, v0)`` where ``v0`` is the two-layer model without
    the anomaly.
    """
    z = np.arange(nz, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    v0 = np.where(z < z_if, v1, v2) * np.ones((1, nx))
    blob = amp * np.exp(-((z - zc) ** 2 + (x - xc) ** 2) / (2.0 * sigma ** 2))
    return v0 + blob, v0


def layered_faulted(nz: int = 200, nx: int = 600, nlayers: int = 10,
                    vmin: float = 1500.0, vmax: float = 4500.0,
                    nfaults: int = 3, seed: int = SEED) -> np.ndarray:
    """Layered model with sinusoidal folds and dipping normal faults.

    Velocities of the ``nlayers`` layers are drawn uniformly in
    ``[vmin, vmax]`` and sorted (top layer forced to ``vmin``). Each
    interface is folded by a sum of three random sinusoids (amplitude at
    most 15 cells, wavelength 100-600 cells). Each fault has a dip of
    50-75 degrees and a throw of 5-15 cells; the hanging wall is shifted
    down.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    vel = np.sort(rng.uniform(vmin, vmax, nlayers))
    vel[0] = vmin
    # interface depths (cells) of the nlayers-1 boundaries
    base = np.sort(rng.uniform(0.08 * nz, 0.95 * nz, nlayers - 1))
    x = np.arange(nx, dtype=np.float64)
    folds = np.zeros(nx)
    for _ in range(3):
        amp = rng.uniform(2.0, 5.0)
        lam = rng.uniform(100.0, 600.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        folds += amp * np.sin(2.0 * np.pi * x / lam + ph)
    # interface z(x) for every boundary; layer index of a cell = number of
    # interfaces above it.
    z = np.arange(nz, dtype=np.float64)[:, None]

    def layer_index(zz, xx_fold):
        idx = np.zeros(zz.shape[:1] + xx_fold.shape, dtype=np.int64)
        for k in range(nlayers - 1):
            idx += (zz >= base[k] + xx_fold[None, :]).astype(np.int64)
        return idx

    idx = layer_index(z, folds)
    # faults: hanging wall (x beyond the fault trace) samples the layer
    # stack shifted up by the throw, i.e. the layers move down.
    for _ in range(nfaults):
        dip = np.deg2rad(rng.uniform(50.0, 75.0))
        throw = rng.uniform(5.0, 15.0)
        x_top = rng.uniform(0.15 * nx, 0.85 * nx)
        sgn = 1.0 if rng.uniform() < 0.5 else -1.0
        trace_x = x_top + sgn * z / np.tan(dip)          # [nz, 1]
        hang = (sgn * (x[None, :] - trace_x) > 0.0)       # [nz, nx]
        shifted = layer_index(z - throw, folds)
        idx = np.where(hang, shifted, idx)
    idx = np.clip(idx, 0, nlayers - 1)
    return vel[idx]


def add_salt(v: np.ndarray, zc: float, xc: float, r0: float,
             vsalt_lo: float = 4500.0, vsalt_hi: float = 4700.0,
             seed: int = SEED + 1) -> np.ndarray:
    """Insert a salt body bounded by a closed random-radius polar curve."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, nx = v.shape
    nharm = 5
    amps = rng.uniform(0.0, 0.25, nharm) / np.arange(1, nharm + 1)
    phs = rng.uniform(0.0, 2.0 * np.pi, nharm)
    z = np.arange(nz, dtype=np.float64)[:, None] - zc
    x = (np.arange(nx, dtype=np.float64)[None, :] - xc) / 2.5  # wide body
    th = np.arctan2(z, x)
    r = np.hypot(z, x)
    rad = r0 * (1.0 + sum(a * np.cos((k + 1) * th + p)
                          for k, (a, p) in enumerate(zip(amps, phs))))
    inside = r <= rad
    vs = vsalt_lo + (vsalt_hi - vsalt_lo) * (1.0 - np.clip(r / np.maximum(rad, 1e-9), 0, 1))
    out = v.copy()
    out[inside] = vs[inside]
    return out


def smooth(v: np.ndarray, sigma: float = 10.0) -> np.ndarray:
    """Starting model: Gaussian smoothing (sigma in cells) of the true model."""
    return gaussian_filter(v, sigma=sigma, mode="nearest")
