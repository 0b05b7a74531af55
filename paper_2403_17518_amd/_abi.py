"""ctypes view of the C ABI declared in include/fwi.h (argument marshalling
only: every step of the propagation runs in libfwi.so's HIP kernels)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwi.so")

FWI_OK, FWI_EINVAL, FWI_ENOMEM, FWI_EHIP, FWI_ECFL, FWI_ESTATE, FWI_ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {FWI_EINVAL: "FWI_EINVAL", FWI_ENOMEM: "FWI_ENOMEM", FWI_EHIP: "FWI_EHIP",
               FWI_ECFL: "FWI_ECFL", FWI_ESTATE: "FWI_ESTATE", FWI_ENOTIMPL: "FWI_ENOTIMPL"}


class FwiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class fwi_grid(C.Structure):
    _fields_ = [("nz", C.c_int32), ("nx", C.c_int32), ("nb", C.c_int32),
                ("h", C.c_float), ("dt", C.c_float), ("nt_max", C.c_int32),
                ("v_ref", C.c_float), ("R", C.c_float), ("ckpt_every", C.c_int32),
                ("free_surface", C.c_int32), ("relative", C.c_int32), ("pml", C.c_int32)]


class fwi_geom(C.Structure):
    _fields_ = [("nshots", C.c_int32),
                ("src_z", C.c_void_p), ("src_x", C.c_void_p),
                ("win_x0", C.c_void_p), ("win_nx", C.c_void_p),
                ("nt", C.c_void_p), ("rec_ptr", C.c_void_p),
                ("rec_z", C.c_void_p), ("rec_x", C.c_void_p),
                ("wavelet", C.c_void_p), ("wavelet_shared", C.c_int32),
                ("src_fz", C.c_void_p), ("src_fx", C.c_void_p),
                ("rec_fz", C.c_void_p), ("rec_fx", C.c_void_p)]


class fwi_stats(C.Structure):
    _fields_ = [("cell_updates", C.c_double), ("stencil_launches", C.c_int64),
                ("ckpt_every", C.c_int32), ("n_segments", C.c_int32),
                ("scratch_bytes", C.c_int64),
                ("ms_fwd", C.c_double), ("ms_adj", C.c_double),
                ("ms_born", C.c_double), ("ms_other", C.c_double),
                ("n_fwd", C.c_int64), ("n_adj", C.c_int64), ("n_born", C.c_int64),
                ("bytes_fwd", C.c_double), ("bytes_adj", C.c_double),
                ("bytes_born", C.c_double),
                ("tile_cw", C.c_int32 * 4), ("tile_rows", C.c_int32 * 4),
                ("tile_levels", C.c_int32 * 4), ("tile_prefetch", C.c_int32 * 4),
                ("graph_launches", C.c_int64), ("graph_captures", C.c_int64),
                ("recomputed_steps", C.c_int64), ("ckpt_slots", C.c_int32)]

    def as_dict(self) -> dict:
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if k.startswith("tile_") else v
        return out


class deblur_layer_stat(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("pass_", C.c_int32), ("M", C.c_int32), ("N", C.c_int32),
                ("K", C.c_int32), ("calls", C.c_int64), ("flops", C.c_double), ("ms", C.c_double)]


class deblur_cfg(C.Structure):
    _fields_ = [("depth", C.c_int32), ("base_ch", C.c_int32), ("leaky_slope", C.c_float),
                ("in_h", C.c_int32), ("in_w", C.c_int32)]


# exported symbols and their signatures (every one declared in include/*.h)
_P = C.c_void_p
SIGNATURES = {
    "fwi_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "fwi_ctx_destroy": (None, [_P]),
    "fwi_ctx_set_stream": (C.c_int, [_P, _P]),
    "fwi_ctx_set_mem_budget": (C.c_int, [_P, C.c_int64]),
    "fwi_ctx_set_ckpt_slots": (C.c_int, [_P, C.c_int32]),
    "fwi_checkpoint_schedule": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
    "fwi_ctx_set_profiling": (C.c_int, [_P, C.c_int]),
    "fwi_ctx_get_stats": (C.c_int, [_P, C.POINTER(fwi_stats)]),
    "fwi_ctx_set_tiling": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "fwi_ctx_set_autotune": (C.c_int, [_P, C.c_int]),
    "fwi_ctx_set_graphs": (C.c_int, [_P, C.c_int]),
    "fwi_ctx_trim": (C.c_int, [_P]),
    "fwi_last_error": (C.c_char_p, [_P]),
    "fwi_forward": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P]),
    "fwi_forward_noalloc": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P]),
    "fwi_gradient": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, _P,
                               C.POINTER(C.c_double), _P]),
    "fwi_misfit": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, C.POINTER(C.c_double)]),
    "born_demig": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, _P]),
    "born_mig": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, _P]),
    "fwi_rtm": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, C.c_float, C.c_float, C.c_float,
                          _P]),
    "born_pair": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, _P, _P]),
    "fwi_gradient_pair": (C.c_int, [_P, C.POINTER(fwi_grid), C.POINTER(fwi_geom), _P, _P, _P,
                                    C.POINTER(C.c_double), C.c_float, _P, _P]),
    "deblur_create": (C.c_int, [_P, C.POINTER(deblur_cfg), C.c_uint64, C.POINTER(_P)]),
    "deblur_destroy": (None, [_P]),
    "deblur_last_error": (C.c_char_p, [_P]),
    "deblur_num_params": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "deblur_set_params": (C.c_int, [_P, _P, _P]),
    "deblur_get_params": (C.c_int, [_P, _P, _P]),
    "deblur_reset": (C.c_int, [_P, _P, C.c_uint64]),
    "deblur_train": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_float, _P]),
    "deblur_train_range": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_float, _P]),
    "deblur_apply": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
    "deblur_forward_raw": (C.c_int, [_P, _P, _P, _P]),
    "deblur_grad_raw": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_double), _P]),
    "deblur_set_profiling": (C.c_int, [_P, C.c_int]),
    "deblur_layer_stats": (C.c_int, [_P, _P, C.POINTER(deblur_layer_stat), C.c_int32, C.POINTER(C.c_int32)]),
    "deblur_save": (C.c_int, [_P, _P, C.c_char_p]),
    "deblur_load": (C.c_int, [_P, _P, C.c_char_p]),
}

_lib = None


def _hip_runtimes_loaded() -> set:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def load(path: str = LIB_PATH):
    """Load libfwi.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime libfwi.so binds to)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    rts = _hip_runtimes_loaded()
    if len(rts) > 1:
        raise RuntimeError(f"two HIP runtimes loaded in one process: {sorted(rts)}")
    _lib = lib
    return lib


def make_grid(grid) -> fwi_grid:
    return fwi_grid(int(grid.nz), int(grid.nx), int(grid.nb), float(grid.h),
                    float(grid.dt), int(grid.nt_max), float(grid.v_ref),
                    float(getattr(grid, "R", 1e-3)), int(getattr(grid, "ckpt_every", 0)),
                    1 if getattr(grid, "free_surface", False) else 0,
                    1 if getattr(grid, "relative", False) else 0,
                    1 if getattr(grid, "pml", False) else 0)


class GeomView:
    """Holds host arrays alive for the duration of a call."""

    def __init__(self, acq, grid):
        self.keep = []

        def arr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a), dtype=dt)
            self.keep.append(a)
            return a.ctypes.data

        wav = np.ascontiguousarray(np.asarray(acq.wavelet), dtype=np.float32)
        shared = wav.ndim == 1
        if wav.shape[-1] != grid.nt_max:
            wav = np.ascontiguousarray(wav[..., :grid.nt_max]) if wav.shape[-1] > grid.nt_max else None
            if wav is None:
                raise ValueError("wavelet shorter than nt_max")
        self.keep.append(wav)
        ns = int(np.asarray(acq.src_z).shape[0])
        self.geom = fwi_geom(ns, arr(acq.src_z, np.int32), arr(acq.src_x, np.int32),
                             arr(getattr(acq, "win_x0", None), np.int32),
                             arr(getattr(acq, "win_nx", None), np.int32),
                             arr(getattr(acq, "nt", None), np.int32),
                             arr(acq.rec_ptr, np.int64), arr(acq.rec_z, np.int32),
                             arr(acq.rec_x, np.int32), wav.ctypes.data, 1 if shared else 0,
                             arr(getattr(acq, "src_fz", None), np.float32),
                             arr(getattr(acq, "src_fx", None), np.float32),
                             arr(getattr(acq, "rec_fz", None), np.float32),
                             arr(getattr(acq, "rec_fx", None), np.float32))
