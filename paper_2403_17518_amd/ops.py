"""torch-facing binding of libfwi.so: same names as the C ABI.

torch supplies device memory and the stream; every operator runs in the
library's HIP kernels. There is no CPU fallback: without the built library
or a GPU these functions raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi


def _check(lib, ctx, rc):
    if rc != _abi.FWI_OK:
        msg = lib.fwi_last_error(ctx)
        raise _abi.FwiError(rc, msg.decode() if msg else "")


def _dev_f32(t: torch.Tensor, name: str, device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on {device}")
    return t


class FwiContext:
    """Owns one fwi_ctx: scratch pool, plan cache and kernel statistics."""

    def __init__(self, device: int = 0, mem_budget: int = 0, profiling: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: libfwi.so needs an MI355X")
        self.lib = _abi.load()
        self.device = torch.device("cuda", device)
        with torch.cuda.device(self.device):
            ptr = C.c_void_p()
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(self.lib, None, self.lib.fwi_ctx_create(device, C.c_void_p(stream), C.byref(ptr)))
        self.ctx = ptr
        if mem_budget:
            self.set_mem_budget(mem_budget)
        if profiling:
            self.set_profiling(True)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fwi_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- settings ----------------------------------------------------------
    def set_mem_budget(self, nbytes: int):
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_mem_budget(self.ctx, int(nbytes)))

    def set_ckpt_slots(self, slots: int = -1):
        """Cap the snapshots the adjoint sweeps hold (-1: no cap)."""
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_ckpt_slots(self.ctx, int(slots)))

    def set_profiling(self, on: bool):
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_profiling(self.ctx, 1 if on else 0))

    def set_tiling(self, kernel: int = -1, cols_per_lane: int = 0, rows_per_wave: int = 0,
                   levels_per_launch: int = 0, prefetch_rows: int = 0):
        """Force the step-kernel tiling (kernel 0 fwd, 1 adj, 2 joint Born, 3
        scattered field from a stored history, -1 all; the joint Born kernel
        keeps one level per launch); (0, 0, 0) hands it back to the autotuner."""
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_tiling(self.ctx, kernel, cols_per_lane, rows_per_wave,
                                                               levels_per_launch, prefetch_rows))

    def set_autotune(self, on: bool):
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_autotune(self.ctx, 1 if on else 0))

    def set_graphs(self, on: bool):
        """Capture time loops into HIP graphs and replay them (default on)."""
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_graphs(self.ctx, 1 if on else 0))

    def stats(self) -> dict:
        s = _abi.fwi_stats()
        _check(self.lib, self.ctx, self.lib.fwi_ctx_get_stats(self.ctx, C.byref(s)))
        return s.as_dict()

    def trim(self):
        _check(self.lib, self.ctx, self.lib.fwi_ctx_trim(self.ctx))

    def _prep_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib, self.ctx, self.lib.fwi_ctx_set_stream(self.ctx, C.c_void_p(stream)))

    def _prep(self, grid, acq):
        g = _abi.make_grid(grid)
        gv = _abi.GeomView(acq, grid)
        self._prep_stream()
        return g, gv

    def _data_size(self, grid, acq) -> int:
        nt = np.full(len(acq.src_z), grid.nt_max) if getattr(acq, "nt", None) is None else np.asarray(acq.nt)
        nrec = np.diff(np.asarray(acq.rec_ptr, dtype=np.int64))
        return int(np.sum(nrec * nt))

    def _model(self, t, name, grid):
        t = _dev_f32(t, name, self.device)
        if tuple(t.shape) != (grid.nz, grid.nx):
            raise ValueError(f"{name} must have shape ({grid.nz}, {grid.nx})")
        return t

    def _data(self, t, name, n):
        t = _dev_f32(t, name, self.device)
        if t.numel() != n:
            raise ValueError(f"{name} must hold {n} samples")
        return t

    # -- operators -----------------------------------------------------------
    def fwi_forward(self, grid, acq, v: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """d = F(v): packed traces (shot, receiver, time)."""
        v = self._model(v, "v", grid)
        n = self._data_size(grid, acq)
        d = torch.empty(n, device=self.device, dtype=torch.float32) if out is None else self._data(out, "out", n)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_forward(self.ctx, C.byref(g), C.byref(gv.geom),
                                                        C.c_void_p(v.data_ptr()), C.c_void_p(d.data_ptr())))
        return d

    def fwi_forward_noalloc(self, grid, acq, v: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """d = F(v) into the caller's `out` without any device allocation in
        the library (its scratch is a static 64 MiB device array)."""
        v = self._model(v, "v", grid)
        d = self._data(out, "out", self._data_size(grid, acq))
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_forward_noalloc(self.ctx, C.byref(g), C.byref(gv.geom),
                                                                C.c_void_p(v.data_ptr()), C.c_void_p(d.data_ptr())))
        return d

    def fwi_gradient(self, grid, acq, v, d_obs, want_misfit: bool = True, want_dsyn: bool = False):
        """(g, misfit, d_syn): g = J^T (F(v) - d_obs); misfit = 1/2 ||F(v) - d_obs||^2."""
        v = self._model(v, "v", grid)
        n = self._data_size(grid, acq)
        d_obs = self._data(d_obs, "d_obs", n)
        grad = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        d_syn = torch.empty(n, device=self.device, dtype=torch.float32) if want_dsyn else None
        phi = C.c_double(0.0)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_gradient(
            self.ctx, C.byref(g), C.byref(gv.geom), C.c_void_p(v.data_ptr()),
            C.c_void_p(d_obs.data_ptr()), C.c_void_p(grad.data_ptr()),
            C.byref(phi) if want_misfit else None,
            C.c_void_p(d_syn.data_ptr()) if d_syn is not None else None))
        return grad, (float(phi.value) if want_misfit else None), d_syn

    def fwi_misfit(self, grid, acq, v, d_obs) -> float:
        """phi = 1/2 ||F(v) - d_obs||^2 (forward sweep and residual only)."""
        v = self._model(v, "v", grid)
        d_obs = self._data(d_obs, "d_obs", self._data_size(grid, acq))
        phi = C.c_double(0.0)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_misfit(self.ctx, C.byref(g), C.byref(gv.geom),
                                                       C.c_void_p(v.data_ptr()), C.c_void_p(d_obs.data_ptr()),
                                                       C.byref(phi)))
        return float(phi.value)

    def born_demig(self, grid, acq, v0, dv) -> torch.Tensor:
        """dd = J dv."""
        v0 = self._model(v0, "v0", grid)
        dv = self._model(dv, "dv", grid)
        n = self._data_size(grid, acq)
        dd = torch.empty(n, device=self.device, dtype=torch.float32)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.born_demig(self.ctx, C.byref(g), C.byref(gv.geom),
                                                       C.c_void_p(v0.data_ptr()), C.c_void_p(dv.data_ptr()),
                                                       C.c_void_p(dd.data_ptr())))
        return dd

    def born_mig(self, grid, acq, v0, dd) -> torch.Tensor:
        """img = J^T dd."""
        v0 = self._model(v0, "v0", grid)
        dd = self._data(dd, "dd", self._data_size(grid, acq))
        img = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.born_mig(self.ctx, C.byref(g), C.byref(gv.geom),
                                                     C.c_void_p(v0.data_ptr()), C.c_void_p(dd.data_ptr()),
                                                     C.c_void_p(img.data_ptr())))
        return img

    def rtm(self, grid, acq, v, d_obs, mute_v: float = 0.0, mute_pad: float = 0.0,
            mute_taper: float = 0.0) -> torch.Tensor:
        """RTM image: the 5-point Laplacian (4 x - neighbours) of J^T of the
        observed data with the direct arrival muted (mute_v > 0: zero before
        offset / mute_v + mute_pad, half-cosine ramp over mute_taper s)."""
        v = self._model(v, "v", grid)
        d_obs = self._data(d_obs, "d_obs", self._data_size(grid, acq))
        img = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_rtm(self.ctx, C.byref(g), C.byref(gv.geom),
                                                    C.c_void_p(v.data_ptr()), C.c_void_p(d_obs.data_ptr()),
                                                    float(mute_v), float(mute_pad), float(mute_taper),
                                                    C.c_void_p(img.data_ptr())))
        return img

    def born_pair(self, grid, acq, v0, g_in, want_dd: bool = False):
        """J^T J g_in, the doubly migrated image (paper section 2.3 eq. 15),
        from one joint Born sweep; with want_dd also J g_in: (img, dd)."""
        v0 = self._model(v0, "v0", grid)
        g_in = self._model(g_in, "g_in", grid)
        img = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        dd = torch.empty(self._data_size(grid, acq), device=self.device, dtype=torch.float32) if want_dd else None
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.born_pair(self.ctx, C.byref(g), C.byref(gv.geom),
                                                      C.c_void_p(v0.data_ptr()), C.c_void_p(g_in.data_ptr()),
                                                      C.c_void_p(dd.data_ptr()) if want_dd else None,
                                                      C.c_void_p(img.data_ptr())))
        return (img, dd) if want_dd else img


    def gradient_pair(self, grid, acq, v, d_obs, scale: float = -1.0, want_dd: bool = False):
        """(grad, misfit, img): the FWI gradient and J^T J (scale * grad) at
        the same model in one call (the pair reuses the gradient's stored
        imaging history when it fits in memory); with want_dd also the
        demigrated data J (scale * grad): (grad, misfit, img, dd)."""
        v = self._model(v, "v", grid)
        nd = self._data_size(grid, acq)
        d_obs = self._data(d_obs, "d_obs", nd)
        grad = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        img = torch.empty((grid.nz, grid.nx), device=self.device, dtype=torch.float32)
        dd = torch.empty(nd, device=self.device, dtype=torch.float32) if want_dd else None
        phi = C.c_double()
        g, gv = self._prep(grid, acq)
        _check(self.lib, self.ctx, self.lib.fwi_gradient_pair(
            self.ctx, C.byref(g), C.byref(gv.geom), C.c_void_p(v.data_ptr()), C.c_void_p(d_obs.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.byref(phi), C.c_float(scale), C.c_void_p(img.data_ptr()),
            C.c_void_p(dd.data_ptr()) if want_dd else None))
        return (grad, float(phi.value), img, dd) if want_dd else (grad, float(phi.value), img)


_default: dict = {}


def default_context(device: int = 0) -> FwiContext:
    ctx = _default.get(device)
    if ctx is None:
        ctx = _default[device] = FwiContext(device)
    return ctx


def _ctx_of(t: torch.Tensor) -> FwiContext:
    return default_context(t.device.index or 0)


def fwi_forward(grid, acq, v):
    return _ctx_of(v).fwi_forward(grid, acq, v)


def fwi_gradient(grid, acq, v, d_obs, want_dsyn: bool = False):
    return _ctx_of(v).fwi_gradient(grid, acq, v, d_obs, True, want_dsyn)


def fwi_misfit(grid, acq, v, d_obs):
    return _ctx_of(v).fwi_misfit(grid, acq, v, d_obs)


def born_demig(grid, acq, v0, dv):
    return _ctx_of(v0).born_demig(grid, acq, v0, dv)


def born_mig(grid, acq, v0, dd):
    return _ctx_of(v0).born_mig(grid, acq, v0, dd)


def checkpoint_schedule(nseg: int, slots: int) -> int:
    """Replay the adjoint sweeps' checkpointing schedule for `nseg` segments
    and `slots` snapshot slots on the host (no device needed), checking
    every action; returns the number of segments it recomputes."""
    lib = _abi.load()
    n = C.c_int64(0)
    rc = lib.fwi_checkpoint_schedule(int(nseg), int(slots), C.byref(n))
    if rc != _abi.FWI_OK:
        raise _abi.FwiError(rc, f"checkpoint schedule nseg={nseg} slots={slots}")
    return int(n.value)
