"""MI355X-native finite-difference acoustic propagation for deep-Hessian-
deblurred FWI: forward modelling, FWI gradients and Born demigration /
migration as hand-written HIP kernels (libfwi.so), called through a thin
torch binding.

Import is light; the library loads on first use (``ops.FwiContext``).
"""
from __future__ import annotations

__all__ = ["FwiContext", "fwi_forward", "fwi_gradient", "born_demig", "born_mig"]


def __getattr__(name):
    if name in __all__:
        from . import ops
        return getattr(ops, name)
    raise AttributeError(name)
