"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It is an independent, plain implementation of the
paper's operators (section 2.1 eq. 1-2: forward modelling and misfit, with a damping sponge
or a perfectly matched layer around the model;
section 2.2 eq. 5-12b: Born modelling; section 2.3 eq. 13-15: adjoint /
FWI gradient and the demigration-remigration pair) written in C
(``fwi_oracle.c``) and shares no code with the HIP library.

Functions take a :class:`synth.Grid`, a :class:`synth.Acquisition` and
float64 numpy arrays; inputs that arrive as float32 are promoted, so the
oracle sees exactly the values the GPU sees.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import build as _build, LIB_PATH

_lib = None


class _OgGrid(C.Structure):
    _fields_ = [("nz", C.c_int), ("nx", C.c_int), ("nb", C.c_int),
                ("h", C.c_double), ("dt", C.c_double),
                ("v_ref", C.c_double), ("R", C.c_double),
                ("free_surface", C.c_int), ("relative", C.c_int), ("pml", C.c_int)]


class _OgGeom(C.Structure):
    _fields_ = [("nshots", C.c_int),
                ("src_z", C.c_void_p), ("src_x", C.c_void_p),
                ("win_x0", C.c_void_p), ("win_nx", C.c_void_p),
                ("nt", C.c_void_p), ("nt_max", C.c_int),
                ("rec_ptr", C.c_void_p), ("rec_z", C.c_void_p),
                ("rec_x", C.c_void_p), ("wavelet", C.c_void_p),
                ("wavelet_shared", C.c_int),
                ("src_fz", C.c_void_p), ("src_fx", C.c_void_p),
                ("rec_fz", C.c_void_p), ("rec_fx", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        L = C.CDLL(LIB_PATH)
        for name in ("oracle_forward", "oracle_born_demig", "oracle_born_mig",
                     "oracle_gradient", "oracle_shot_fields", "oracle_set_threads"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (0 = leave as is); returns the count used."""
    return lib().oracle_set_threads(int(n))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Call:
    """Holds ctypes views of one (grid, acquisition) pair for one call."""

    def __init__(self, grid, acq):
        self.keep = []
        self.g = _OgGrid(grid.nz, grid.nx, grid.nb, float(grid.h),
                         float(grid.dt), float(grid.v_ref), float(grid.R),
                         1 if getattr(grid, "free_surface", False) else 0,
                         1 if getattr(grid, "relative", False) else 0,
                         1 if getattr(grid, "pml", False) else 0)

        def ptr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            self.keep.append(a)
            return a.ctypes.data

        wav = _f64(acq.wavelet)
        if wav.shape[-1] < grid.nt_max:
            raise ValueError("wavelet shorter than nt_max")
        self.keep.append(wav)
        self.geo = _OgGeom(
            acq.nshots, ptr(acq.src_z, np.int32), ptr(acq.src_x, np.int32),
            ptr(acq.win_x0, np.int32), ptr(acq.win_nx, np.int32),
            ptr(acq.nt, np.int32), int(grid.nt_max),
            ptr(acq.rec_ptr, np.int64), ptr(acq.rec_z, np.int32),
            ptr(acq.rec_x, np.int32), wav.ctypes.data,
            1 if acq.wavelet_shared else 0,
            ptr(getattr(acq, "src_fz", None), np.float64), ptr(getattr(acq, "src_fx", None), np.float64),
            ptr(getattr(acq, "rec_fz", None), np.float64), ptr(getattr(acq, "rec_fx", None), np.float64))
        if not acq.wavelet_shared and wav.shape[1] != grid.nt_max:
            raise ValueError("per-shot wavelets must be [nshots][nt_max]")


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed (out of memory?)")


def forward(grid, acq, v) -> np.ndarray:
    """d = F(v): packed traces (section 2.1 eq. 1, receivers sample u^{n+1})."""
    c = _Call(grid, acq)
    v = _f64(v)
    d = np.zeros(acq.data_size(grid))
    _check(lib().oracle_forward(C.byref(c.g), C.byref(c.geo),
                                v.ctypes.data_as(C.c_void_p),
                                d.ctypes.data_as(C.c_void_p)), "forward")
    return d


def born_demig(grid, acq, v, dv) -> np.ndarray:
    """dd = J dv: Born modelling (section 2.2 eq. 11-12b); with
    ``grid.relative`` the perturbation is dv / v and the operator J diag(v)
    (eq. 12)."""
    c = _Call(grid, acq)
    v, dv = _f64(v), _f64(dv)
    dd = np.zeros(acq.data_size(grid))
    _check(lib().oracle_born_demig(C.byref(c.g), C.byref(c.geo),
                                   v.ctypes.data_as(C.c_void_p),
                                   dv.ctypes.data_as(C.c_void_p),
                                   dd.ctypes.data_as(C.c_void_p)), "born_demig")
    return dd


def born_mig(grid, acq, v, dd) -> np.ndarray:
    """img = J^T dd: adjoint Born / migration (section 2.3 eq. 13); with
    ``grid.relative``, diag(v) J^T dd."""
    c = _Call(grid, acq)
    v, dd = _f64(v), _f64(dd)
    img = np.zeros((grid.nz, grid.nx))
    _check(lib().oracle_born_mig(C.byref(c.g), C.byref(c.geo),
                                 v.ctypes.data_as(C.c_void_p),
                                 dd.ctypes.data_as(C.c_void_p),
                                 img.ctypes.data_as(C.c_void_p)), "born_mig")
    return img


def gradient(grid, acq, v, d_obs):
    """(grad, misfit, d_syn): grad = J^T (F(v) - d_obs), misfit = 1/2 ||.||^2
    (section 2.1 eq. 2 and section 2.3 eq. 13, with the residual sign
    F(v) - d_obs so that grad is the gradient of the misfit)."""
    c = _Call(grid, acq)
    v, d_obs = _f64(v), _f64(d_obs)
    g = np.zeros((grid.nz, grid.nx))
    d_syn = np.zeros(acq.data_size(grid))
    phi = C.c_double(0.0)
    _check(lib().oracle_gradient(C.byref(c.g), C.byref(c.geo),
                                 v.ctypes.data_as(C.c_void_p),
                                 d_obs.ctypes.data_as(C.c_void_p),
                                 g.ctypes.data_as(C.c_void_p), C.byref(phi),
                                 d_syn.ctypes.data_as(C.c_void_p)), "gradient")
    return g, float(phi.value), d_syn


def born_pair(grid, acq, v, g_in) -> np.ndarray:
    """dm1 = J^T J g_in: the doubly migrated image (section 2.3 eq. 15)."""
    return born_mig(grid, acq, v, born_demig(grid, acq, v, g_in))


def shot_fields(grid, acq, s, v, res_shot=None):
    """Wavefield histories of shot ``s`` for identity tests.

    Returns a dict with ``u`` ([nt+1][NZ][NX], u^0..u^nt), ``lam``
    ([nt][NZ][NX], lam^0..lam^{nt-1}, only if ``res_shot`` is given), and
    the padded ``a``, ``b``, ``c`` arrays.
    """
    c = _Call(grid, acq)
    v = _f64(v)
    nt = acq.nt_of(s, grid)
    _, wnx = acq.window(s, grid)
    NZ, NX = grid.NZ, wnx + 2 * grid.nb
    u = np.zeros((nt + 1, NZ, NX))
    lam = None
    rp = None
    if res_shot is not None:
        res_shot = _f64(res_shot)
        lam = np.zeros((nt, NZ, NX))
        rp = res_shot.ctypes.data_as(C.c_void_p)
    a, b, cc = (np.zeros((NZ, NX)) for _ in range(3))
    _check(lib().oracle_shot_fields(
        C.byref(c.g), C.byref(c.geo), int(s), v.ctypes.data_as(C.c_void_p), rp,
        u.ctypes.data_as(C.c_void_p),
        None if lam is None else lam.ctypes.data_as(C.c_void_p),
        a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
        cc.ctypes.data_as(C.c_void_p)), "shot_fields")
    return {"u": u, "lam": lam, "a": a, "b": b, "c": cc}


def pad(grid, v, x0=0, wnx=None):
    """Pad(v) of one window: edge replication into the sponge."""
    wnx = grid.nx if wnx is None else wnx
    g = _OgGrid(grid.nz, grid.nx, grid.nb, float(grid.h), float(grid.dt),
                float(grid.v_ref), float(grid.R), 1 if getattr(grid, "free_surface", False) else 0)
    v = _f64(v)
    P = np.zeros((grid.NZ, wnx + 2 * grid.nb))
    lib().oracle_pad(C.byref(g), int(x0), int(wnx), v.ctypes.data_as(C.c_void_p),
                     P.ctypes.data_as(C.c_void_p))
    return P


def pad_adjoint(grid, P, x0=0, wnx=None):
    """Pad^T of one window: each padded cell adds onto its source cell."""
    wnx = grid.nx if wnx is None else wnx
    g = _OgGrid(grid.nz, grid.nx, grid.nb, float(grid.h), float(grid.dt),
                float(grid.v_ref), float(grid.R), 1 if getattr(grid, "free_surface", False) else 0)
    P = _f64(P)
    img = np.zeros((grid.nz, grid.nx))
    lib().oracle_pad_adjoint(C.byref(g), int(x0), int(wnx), P.ctypes.data_as(C.c_void_p),
                             img.ctypes.data_as(C.c_void_p))
    return img
