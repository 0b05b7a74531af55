"""Plain data containers describing one modelling problem.

Grid: the physical model grid, the sponge width and the time stepping.
Acquisition: sources, receivers, per-shot windows, record lengths, wavelets.

Conventions (shared by the oracle and the C-ABI):
* models are ``[nz][nx]`` row-major, z (depth) slow, x fast;
* source/receiver positions are physical cell indices ``(z, x)`` in the
  full model; a shot only sees the columns ``[win_x0, win_x0 + win_nx)``;
* data are packed traces: shot order, then that shot's receiver order,
  time fastest, ``nt[s]`` samples per trace of shot ``s``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Grid:
    nz: int
    nx: int
    nb: int          # sponge width in cells, on all four sides
    h: float         # grid spacing (m), dz == dx
    dt: float        # time step (s)
    nt_max: int      # longest record (samples)
    v_ref: float     # fixed sponge reference velocity (m/s)
    R: float = 1e-3  # nominal sponge reflection coefficient
    ckpt_every: int = 0  # checkpoint interval for the GPU path (0 = auto)
    free_surface: bool = False  # pressure-free top surface on row 0 (no top sponge)
    relative: bool = False  # Born perturbations and images per dv / v (J diag(v)) instead of per dv
    pml: bool = False  # perfectly matched layer in the nb padded cells instead of the sponge

    @property
    def top(self) -> int:
        """Padded rows above physical row 0."""
        return 0 if self.free_surface else self.nb

    @property
    def NZ(self) -> int:
        return self.nz + self.nb + self.top


@dataclass
class Acquisition:
    src_z: np.ndarray            # int32 [nshots]
    src_x: np.ndarray            # int32 [nshots]
    rec_ptr: np.ndarray          # int64 [nshots + 1] (CSR over shots)
    rec_z: np.ndarray            # int32 [nrec_total]
    rec_x: np.ndarray            # int32 [nrec_total]
    wavelet: np.ndarray          # float [nt_max] (shared) or [nshots][nt_max]
    win_x0: np.ndarray | None = None  # int32 [nshots]; None = full width
    win_nx: np.ndarray | None = None  # int32 [nshots]
    nt: np.ndarray | None = None      # int32 [nshots]; None = nt_max for all
    # off-grid positions: fractional offsets in [0, 1) toward +z / +x from
    # (src_z, src_x) and (rec_z, rec_x), float32; None = on the grid
    src_fz: np.ndarray | None = None
    src_fx: np.ndarray | None = None
    rec_fz: np.ndarray | None = None
    rec_fx: np.ndarray | None = None

    def __post_init__(self):
        self.src_z = np.ascontiguousarray(self.src_z, dtype=np.int32)
        self.src_x = np.ascontiguousarray(self.src_x, dtype=np.int32)
        self.rec_ptr = np.ascontiguousarray(self.rec_ptr, dtype=np.int64)
        self.rec_z = np.ascontiguousarray(self.rec_z, dtype=np.int32)
        self.rec_x = np.ascontiguousarray(self.rec_x, dtype=np.int32)
        for name in ("win_x0", "win_nx", "nt"):
            a = getattr(self, name)
            if a is not None:
                setattr(self, name, np.ascontiguousarray(a, dtype=np.int32))
        for name in ("src_fz", "src_fx", "rec_fz", "rec_fx"):
            a = getattr(self, name)
            if a is not None:
                setattr(self, name, np.ascontiguousarray(a, dtype=np.float32))

    @property
    def nshots(self) -> int:
        return int(self.src_z.shape[0])

    @property
    def wavelet_shared(self) -> bool:
        return self.wavelet.ndim == 1

    def nrec(self, s: int) -> int:
        return int(self.rec_ptr[s + 1] - self.rec_ptr[s])

    def nt_of(self, s: int, grid: Grid) -> int:
        return int(grid.nt_max if self.nt is None else self.nt[s])

    def window(self, s: int, grid: Grid) -> tuple[int, int]:
        if self.win_x0 is None:
            return 0, grid.nx
        return int(self.win_x0[s]), int(self.win_nx[s])

    def trace_offsets(self, grid: Grid) -> np.ndarray:
        """int64 [nshots + 1]: start of each shot's block in the packed data."""
        off = np.zeros(self.nshots + 1, dtype=np.int64)
        for s in range(self.nshots):
            off[s + 1] = off[s] + self.nrec(s) * self.nt_of(s, grid)
        return off

    def data_size(self, grid: Grid) -> int:
        return int(self.trace_offsets(grid)[-1])

    def shot_data(self, d: np.ndarray, s: int, grid: Grid) -> np.ndarray:
        """View of shot ``s`` as ``[nrec][nt]`` inside a packed data vector."""
        off = self.trace_offsets(grid)
        return d[off[s]:off[s + 1]].reshape(self.nrec(s), self.nt_of(s, grid))

    def subset(self, shots) -> "Acquisition":
        shots = np.asarray(shots, dtype=np.int64)
        ptr = [0]
        rz, rx, rfz, rfx = [], [], [], []
        for s in shots:
            a, b = self.rec_ptr[s], self.rec_ptr[s + 1]
            rz.append(self.rec_z[a:b])
            rx.append(self.rec_x[a:b])
            if self.rec_fz is not None:
                rfz.append(self.rec_fz[a:b])
                rfx.append(self.rec_fx[a:b])
            ptr.append(ptr[-1] + (b - a))
        wav = self.wavelet if self.wavelet_shared else self.wavelet[shots]
        return Acquisition(
            src_z=self.src_z[shots], src_x=self.src_x[shots],
            rec_ptr=np.asarray(ptr, dtype=np.int64),
            rec_z=np.concatenate(rz) if rz else np.zeros(0, np.int32),
            rec_x=np.concatenate(rx) if rx else np.zeros(0, np.int32),
            wavelet=wav,
            win_x0=None if self.win_x0 is None else self.win_x0[shots],
            win_nx=None if self.win_nx is None else self.win_nx[shots],
            nt=None if self.nt is None else self.nt[shots],
            src_fz=None if self.src_fz is None else self.src_fz[shots],
            src_fx=None if self.src_fx is None else self.src_fx[shots],
            rec_fz=None if self.rec_fz is None else (np.concatenate(rfz) if rfz else np.zeros(0, np.float32)),
            rec_fx=None if self.rec_fx is None else (np.concatenate(rfx) if rfx else np.zeros(0, np.float32)),
        )


def cell_updates(grid: Grid, acq: Acquisition) -> int:
    """Padded-cell time-step updates of one wavefield over all shots.

    One cell-update = one padded cell (sponge included), one time step,
    one shot, one wavefield.
    """
    total = 0
    for s in range(acq.nshots):
        _, wnx = acq.window(s, grid)
        total += grid.NZ * (wnx + 2 * grid.nb) * acq.nt_of(s, grid)
    return total
