"""The seeded workloads (grid + acquisition + models) used by tests and bench.

* ``two_layer()``      - 100x100 grid, 20-cell sponge, 10 m, two layers
  1500/2500 m/s with a +200 m/s Gaussian anomaly (sigma 8 cells), 4 surface
  shots, 100 receivers, 10 Hz Ricker, dt = 1 ms, 1000 steps.
* ``layered_600x200()`` - 200x600 grid, 10 m, layered/folded/faulted model
  1500-4500 m/s, 64 shots, 600 receivers, 15 Hz Ricker, dt = 0.8 ms, 4000
  steps.
* ``salt_1700x350()``   - 350x1700 grid, 10 m, layered + faulted + salt
  1500-4700 m/s, 300 shots of uneven aperture (200-1700 receivers) and record
  length (3-5 s), dt = 1 ms.
* ``salt_full_width()`` - the salt grid with full-width windows and a short
  record: a working set far larger than the last-level cache.
* ``ragged_small()``    - a small ragged case (windows, record lengths,
  co-located receivers) for parity tests.

Sources and receivers sit on physical row 2 ("zero depth" in the paper,
moved two cells down so the source stencil stays out of the sponge).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import models
from .problem import Acquisition, Grid
from .wavelet import ricker


@dataclass
class Workload:
    name: str
    grid: Grid
    acq: Acquisition
    v_true: np.ndarray
    v0: np.ndarray
    freq: float


def _surface_acq(src_x, rec_x, wavelet, z=2, win_x0=None, win_nx=None,
                 nt=None, rec_lists=None) -> Acquisition:
    ns = len(src_x)
    if rec_lists is None:
        rec_lists = [np.asarray(rec_x, dtype=np.int32)] * ns
    ptr = np.zeros(ns + 1, dtype=np.int64)
    for s in range(ns):
        ptr[s + 1] = ptr[s] + len(rec_lists[s])
    rx = np.concatenate(rec_lists).astype(np.int32)
    return Acquisition(
        src_z=np.full(ns, z, np.int32), src_x=np.asarray(src_x, np.int32),
        rec_ptr=ptr, rec_z=np.full(rx.shape[0], z, np.int32), rec_x=rx,
        wavelet=wavelet, win_x0=win_x0, win_nx=win_nx, nt=nt)


def two_layer(nt: int = 1000) -> Workload:
    grid = Grid(nz=100, nx=100, nb=20, h=10.0, dt=1e-3, nt_max=nt,
                v_ref=2700.0)
    v_true, v0 = models.two_layer_anomaly(100, 100)
    acq = _surface_acq([12, 37, 62, 87], np.arange(100),
                       ricker(10.0, grid.dt, nt))
    return Workload("two_layer_100x100", grid, acq, v_true, v0, 10.0)


def layered_600x200(nshots: int = 64, nt: int = 4000) -> Workload:
    grid = Grid(nz=200, nx=600, nb=20, h=10.0, dt=0.8e-3, nt_max=nt,
                v_ref=4500.0)
    v_true = models.layered_faulted(200, 600)
    v0 = models.smooth(v_true, 10.0)
    src_x = np.round((np.arange(nshots) + 0.5) * 600 / nshots).astype(np.int32)
    acq = _surface_acq(src_x, np.arange(600), ricker(15.0, grid.dt, nt))
    return Workload("layered_600x200", grid, acq, v_true, v0, 15.0)


def marmousi_601x221(nt: int = 3000, dt: float = 1.4e-3) -> Workload:
    """The acquisition of the paper's Marmousi example: 601 x 221 grid
    points at 15 m, 30 sources and 300 receivers equally spaced along the
    top row (zero depth), a 5 Hz Ricker wavelet. The Marmousi model itself is
    not available: a seeded layered and faulted model over Marmousi's
    velocity range (1500-5500 m/s) stands in for it, smoothed for the
    starting model. dt keeps v_max dt / h at 0.51; 3000 steps record 4.2 s."""
    grid = Grid(nz=221, nx=601, nb=20, h=15.0, dt=dt, nt_max=nt, v_ref=5500.0)
    v_true = models.layered_faulted(221, 601, vmin=1500.0, vmax=5500.0)
    v0 = models.smooth(v_true, 10.0)
    src_x = np.round((np.arange(30) + 0.5) * 601 / 30).astype(np.int32)
    rec_x = np.round((np.arange(300) + 0.5) * 601 / 300).astype(np.int32)
    acq = _surface_acq(src_x, rec_x, ricker(5.0, dt, nt), z=0)
    return Workload("marmousi_601x221", grid, acq, v_true, v0, 5.0)


def salt_1700x350(nshots: int = 300, dt: float = 1e-3,
                  seed: int = models.SEED, nz: int = 350, nx: int = 1700,
                  h: float = 10.0, margin: int = 50, name: str = "salt_1700x350") -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed + 5))
    v = models.layered_faulted(nz, nx, vmin=1500.0, vmax=4500.0, seed=seed)
    v_true = models.add_salt(v, zc=0.55 * nz, xc=0.5 * nx, r0=0.18 * nz)
    v0 = models.smooth(v_true, 10.0)
    src_x = np.round((np.arange(nshots) + 0.5) * nx / nshots).astype(np.int32)
    rec_lists, wx0, wnx, nts = [], [], [], []
    nt_max = 0
    for s in range(nshots):
        nrec = int(rng.integers(max(2, (200 * nx) // 1700), nx + 1))
        lo = int(src_x[s]) - nrec // 2
        hi = lo + nrec
        lo, hi = max(lo, 0), min(hi, nx)
        rec = np.arange(lo, hi, dtype=np.int32)
        x0 = max(0, min(lo, int(src_x[s])) - margin)
        x1 = min(nx, max(hi, int(src_x[s]) + 1) + margin)
        rec_lists.append(rec)
        wx0.append(x0)
        wnx.append(x1 - x0)
        n = int(round(rng.uniform(3.0, 5.0) / dt))
        nts.append(n)
        nt_max = max(nt_max, n)
    grid = Grid(nz=nz, nx=nx, nb=20, h=h, dt=dt, nt_max=nt_max,
                v_ref=4700.0)
    acq = _surface_acq(src_x, None, ricker(15.0, dt, nt_max),
                       win_x0=np.asarray(wx0), win_nx=np.asarray(wnx),
                       nt=np.asarray(nts), rec_lists=rec_lists)
    return Workload(name, grid, acq, v_true, v0, 15.0)


def salt_full_width(nshots: int = 300, nt: int = 100) -> Workload:
    """The 1700 x 350 salt grid with every shot's window opened to the full
    width (390 x 1740 padded cells per shot) and the record cut to ``nt``
    steps: a working set of several GB per wavefield, far beyond the
    last-level cache, for measuring the stencil kernels against HBM."""
    wl = salt_1700x350(nshots=nshots)
    acq, g = wl.acq, wl.grid
    acq.win_x0 = acq.win_nx = acq.nt = None        # full width, nt steps each
    acq.wavelet = ricker(15.0, g.dt, nt)
    grid = Grid(nz=g.nz, nx=g.nx, nb=g.nb, h=g.h, dt=g.dt, nt_max=nt, v_ref=g.v_ref)
    return Workload("salt_full_width", grid, acq, wl.v_true, wl.v0, 15.0)


def salt_848x176(nshots: int = 100) -> Workload:
    """The salt workload at half resolution (20 m cells, same 17 km x 3.5 km
    extent, 2 ms steps): receivers per shot 100-848, record length 3-5 s."""
    return salt_1700x350(nshots=nshots, dt=2e-3, nz=176, nx=848, h=20.0,
                         margin=25, name="salt_848x176")


def ragged_small(seed: int = models.SEED, nz: int = 37, nx: int = 150,
                 nb: int = 10, nshots: int = 5, nt_lo: int = 150,
                 nt_hi: int = 260, per_shot_wavelet: bool = True) -> Workload:
    """Small ragged workload: per-shot windows, record lengths, co-located
    receivers, receivers at several depths, per-shot wavelets."""
    rng = np.random.Generator(np.random.PCG64(seed + 11))
    v = models.layered_faulted(nz, nx, nlayers=5, vmin=1500.0, vmax=3000.0,
                               nfaults=1, seed=seed)
    v0 = models.smooth(v, 3.0)
    dt, h = 1.5e-3, 10.0
    src_x = rng.integers(5, nx - 5, nshots).astype(np.int32)
    src_z = rng.integers(1, nz - 1, nshots).astype(np.int32)
    rz, rx, ptr, wx0, wnx, nts = [], [], [0], [], [], []
    for s in range(nshots):
        x0 = int(max(0, src_x[s] - rng.integers(10, 60)))
        x1 = int(min(nx, src_x[s] + rng.integers(10, 60)))
        n = int(rng.integers(3, 40))
        xs = rng.integers(x0, x1, n).astype(np.int32)
        zs = rng.integers(0, nz, n).astype(np.int32)
        # make at least one pair co-located
        if n >= 2:
            xs[1], zs[1] = xs[0], zs[0]
        rz.append(zs)
        rx.append(xs)
        ptr.append(ptr[-1] + n)
        wx0.append(x0)
        wnx.append(x1 - x0)
        nts.append(int(rng.integers(nt_lo, nt_hi + 1)))
    nt_max = max(nts)
    grid = Grid(nz=nz, nx=nx, nb=nb, h=h, dt=dt, nt_max=nt_max, v_ref=3000.0)
    if per_shot_wavelet:
        freqs = rng.uniform(8.0, 14.0, nshots)
        wav = np.stack([ricker(f, dt, nt_max) for f in freqs])
    else:
        wav = ricker(10.0, dt, nt_max)
    acq = Acquisition(src_z=src_z, src_x=src_x, rec_ptr=np.asarray(ptr),
                      rec_z=np.concatenate(rz), rec_x=np.concatenate(rx),
                      wavelet=wav, win_x0=np.asarray(wx0),
                      win_nx=np.asarray(wnx), nt=np.asarray(nts))
    return Workload("ragged_small", grid, acq, v, v0, 10.0)
