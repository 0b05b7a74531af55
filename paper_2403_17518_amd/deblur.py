"""torch-facing binding of the deblurring network in libfwi.so (the learned
inverse-Hessian approximation of paper section 2.3; names follow the C ABI
in include/deblur.h). Every layer runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi
from .ops import FwiContext


@dataclass(frozen=True)
class DeblurConfig:
    depth: int = 3
    base_ch: int = 32
    leaky_slope: float = 0.0
    in_h: int = 208
    in_w: int = 608


class DeblurNet:
    def __init__(self, fctx: FwiContext, cfg: DeblurConfig = DeblurConfig(), seed: int = 2403):
        self.fctx, self.lib, self.cfg = fctx, fctx.lib, cfg
        c = _abi.deblur_cfg(cfg.depth, cfg.base_ch, cfg.leaky_slope, cfg.in_h, cfg.in_w)
        ptr = C.c_void_p()
        rc = self.lib.deblur_create(fctx.ctx, C.byref(c), C.c_uint64(seed), C.byref(ptr))
        if rc != 0:
            raise _abi.FwiError(rc, "deblur_create failed (bad configuration or out of memory)")
        self.net = ptr
        n = C.c_int64()
        self._check(self.lib.deblur_num_params(self.net, C.byref(n)))
        self.nparams = int(n.value)

    def _check(self, rc):
        if rc != 0:
            msg = self.lib.deblur_last_error(self.net)
            raise _abi.FwiError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "net", None):
            self.lib.deblur_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        self.fctx._prep_stream()

    def _img(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or t.device != self.fctx.device or t.dtype != torch.float32 \
                or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must be a contiguous float32 {tuple(shape)} tensor on {self.fctx.device}")
        return t

    # -- per-layer timing -------------------------------------------------------
    def set_profiling(self, on: bool):
        self._check(self.lib.deblur_set_profiling(self.net, 1 if on else 0))

    def layer_stats(self) -> list[dict]:
        """Summed time and flops of every convolution GEMM since profiling
        was switched on: one record per layer and pass."""
        self._sync_stream()
        buf = (_abi.deblur_layer_stat * 512)()
        n = C.c_int32()
        self._check(self.lib.deblur_layer_stats(self.fctx.ctx, self.net, buf, 512, C.byref(n)))
        passes = ("forward", "data_grad", "weight_grad")
        return [{"name": r.name.decode(), "pass": passes[r.pass_], "M": r.M, "N": r.N, "K": r.K,
                 "calls": r.calls, "flops": r.flops, "ms": r.ms} for r in buf[:n.value]]

    # -- parameters ------------------------------------------------------------
    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        self._sync_stream()
        self._check(self.lib.deblur_set_params(self.fctx.ctx, self.net, flat.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        self._sync_stream()
        self._check(self.lib.deblur_get_params(self.fctx.ctx, self.net, out.ctypes.data))
        return out

    def reset(self, seed: int):
        self._sync_stream()
        self._check(self.lib.deblur_reset(self.fctx.ctx, self.net, C.c_uint64(seed)))

    def save(self, path: str):
        self._sync_stream()
        self._check(self.lib.deblur_save(self.fctx.ctx, self.net, path.encode()))

    def load(self, path: str):
        self._sync_stream()
        self._check(self.lib.deblur_load(self.fctx.ctx, self.net, path.encode()))

    # -- compute ---------------------------------------------------------------
    def forward_raw(self, x: torch.Tensor) -> torch.Tensor:
        x = self._img(x, (self.cfg.in_h, self.cfg.in_w), "x")
        y = torch.empty_like(x)
        self._sync_stream()
        self._check(self.lib.deblur_forward_raw(self.fctx.ctx, self.net, C.c_void_p(x.data_ptr()),
                                                C.c_void_p(y.data_ptr())))
        return y

    def grad_raw(self, x: torch.Tensor, t: torch.Tensor):
        x = self._img(x, (self.cfg.in_h, self.cfg.in_w), "x")
        t = self._img(t, (self.cfg.in_h, self.cfg.in_w), "t")
        loss = C.c_double()
        g = np.empty(self.nparams, dtype=np.float32)
        self._sync_stream()
        self._check(self.lib.deblur_grad_raw(self.fctx.ctx, self.net, C.c_void_p(x.data_ptr()),
                                             C.c_void_p(t.data_ptr()), C.byref(loss), g.ctypes.data))
        return float(loss.value), g

    def deblur_train(self, x: torch.Tensor, y: torch.Tensor, steps: int, lr_max: float = 1e-3) -> np.ndarray:
        """Train on (x_blurred -> y_target), [nz][nx]; returns the loss history."""
        x = self._img(x, x.shape, "x")
        y = self._img(y, x.shape, "y")
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        self._sync_stream()
        self._check(self.lib.deblur_train(self.fctx.ctx, self.net, C.c_void_p(x.data_ptr()),
                                          C.c_void_p(y.data_ptr()), int(x.shape[0]), int(x.shape[1]),
                                          int(steps), float(lr_max), hist.ctypes.data))
        return hist[:steps]

    def train_range(self, x: torch.Tensor, y: torch.Tensor, first: int, count: int, total: int,
                    lr_max: float = 1e-3) -> np.ndarray:
        """Steps first .. first+count-1 of a training run of `total` steps
        (first = 0 starts the run; a later call continues it); returns the
        loss history of these steps."""
        x = self._img(x, x.shape, "x")
        y = self._img(y, x.shape, "y")
        hist = np.zeros(max(count, 1), dtype=np.float32)
        self._sync_stream()
        self._check(self.lib.deblur_train_range(self.fctx.ctx, self.net, C.c_void_p(x.data_ptr()),
                                                C.c_void_p(y.data_ptr()), int(x.shape[0]), int(x.shape[1]),
                                                int(first), int(count), int(total), float(lr_max),
                                                hist.ctypes.data))
        return hist[:count]

    def deblur_apply(self, x: torch.Tensor) -> torch.Tensor:
        x = self._img(x, x.shape, "x")
        y = torch.empty_like(x)
        self._sync_stream()
        self._check(self.lib.deblur_apply(self.fctx.ctx, self.net, C.c_void_p(x.data_ptr()),
                                          int(x.shape[0]), int(x.shape[1]), C.c_void_p(y.data_ptr())))
        return y
