"""Pins of the bf16-storage emulation that the network parity tests take
their tolerances from (tests/bf16_storage.py).

* With rounding off it is the oracle's network (same structure, same
  gradients), so the emulated error is measured on the right network.
* With rounding on, every stored tensor is bf16-representable and the error
  it causes has the size bf16 storage must cause: above the FP64 level and
  below a few percent, with the unit roundoff 2^-8 entering once per layer.
* The derived bounds of the paper-scale gradient case (widths 128-2048,
  LeakyReLU 0.2, 32 x 64, the GPU test's seeds) are printed and stay below
  a level that would let a wrong tap, weight or skip connection through.
"""
import numpy as np
import torch

import bf16_storage as B
from oracle import deblur_ref as R
from synth import netparams


def smooth_field(H, W, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((H, W))
    k = np.exp(-np.arange(-6, 7) ** 2 / 8.0)
    z = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 0, z)
    z = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 1, z)
    return z / np.abs(z).max()


def test_without_rounding_it_is_the_oracle_network():
    depth, base, H, W, slope = 2, 8, 16, 32, 0.2
    ps = netparams.draw(depth, base, seed=3)
    x, t = smooth_field(H, W, 1), smooth_field(H, W, 2)
    l0, g0, y0 = R.loss_and_grads(ps, x, t, depth, slope)
    l1, g1, y1 = B.loss_and_grads(ps, x, t, depth, slope, rounding=False)
    assert abs(l0 - l1) <= 1e-13 * l0
    assert np.max(np.abs(y0 - y1)) <= 1e-13 * np.max(np.abs(y0))
    for a, b in zip(g0, g1):
        assert B.rel(b, a) <= 1e-12


def test_rounding_stores_bf16_values_and_costs_bf16_accuracy():
    depth, base, H, W, slope = 2, 16, 32, 64, 0.0
    ps = netparams.draw(depth, base, seed=11)
    x = torch.as_tensor(smooth_field(H, W, 3))
    v = torch.linspace(-3.0, 3.0, 1001, dtype=torch.float64)
    r = B._rb(v)
    # bf16 keeps 8 significant bits: every rounded value has a zero low half
    # as an FP32 word, and rounding to nearest errs by at most 2^-8 relative
    bits = r.to(torch.float32).view(torch.int32)
    assert torch.all(bits & 0xFFFF == 0)
    assert torch.all(torch.abs(r - v) <= 2.0 ** -8 * torch.abs(v))
    bound, exact = B.forward_bound(ps, x.numpy(), depth, slope)
    e = bound / B.BF16_FACTOR
    print("emulated bf16-storage forward error", e)
    # more than FP64/FP32 round-off, less than bf16 unit roundoff times the
    # layer count
    assert 1e-5 < e < 15 * 2.0 ** -8


def test_paper_scale_gradient_bounds_are_derived_and_meaningful():
    """The case of the GPU paper-scale gradient test: its bound per tensor is
    BF16_FACTOR times the emulated error printed here."""
    depth, base, H, W, slope = 4, 128, 32, 64, 0.2
    ps = netparams.draw(depth, base, seed=17)
    ps32 = [p.astype(np.float32).astype(np.float64) for p in ps]
    x, t = smooth_field(H, W, 7).astype(np.float32), smooth_field(H, W, 8).astype(np.float32)
    _, gref, _ = R.loss_and_grads(ps32, x, t, depth, slope)
    bounds = B.gradient_bounds(ps32, x, t, depth, slope, gref)
    names = [n for n, _ in netparams.param_shapes(depth, base)]
    worst = max(zip(bounds, names))
    print("derived per-tensor gradient bounds: worst", worst,
          "median", float(np.median(bounds)))
    # the deepest block sums a handful of products per weight (2 x 4
    # pixels), so its emulated error is the largest; everything stays well
    # below the order-one errors a wrong layer gives
    assert worst[0] < 0.25
    assert float(np.median(bounds)) < 0.10
