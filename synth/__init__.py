"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package only *generates inputs*: grids, velocity models, acquisition
geometries and source wavelets. It holds none of the propagation, Born or
imaging arithmetic, so both sides of every parity test can use it without
sharing any part of the method.
"""
from .problem import Grid, Acquisition
from .wavelet import ricker
from . import models, configs

__all__ = ["Grid", "Acquisition", "ricker", "models", "configs"]
