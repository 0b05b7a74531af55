"""Emulation of the deblurring network's bf16 storage (test helper).

The library runs every convolution on the matrix cores with bf16 operands
and FP32 accumulation, and stores activations and back-propagated gradients
in bf16 between layers. Accumulation errors in FP32 are ~1e-7 relative and
negligible next to bf16 rounding (unit roundoff 2^-8 ~ 3.9e-3), so the error
the GPU can be expected to show against the FP64 oracle is the error that
bf16 *storage alone* causes. This module computes it: the network of
paper Appendix A, Table 1 (the oracle's structure) in float64, with values
rounded to bf16 (round to nearest even) exactly where the library stores
bf16 tensors:

  forward    the input image, every weight tensor of a 3x3 or transposed
             convolution, every layer output after its activation, the
             pooled maps and the up-sampled maps; the 1x1 output layer
             reads FP32 weights and writes FP32;
  backward   the gradient at every convolution's pre-activation output (the
             library applies the activation's derivative in the kernel that
             forms the gradient, and stores the product), the gradient of
             every pooled and up-sampled map, and the skip half of a
             concatenation's gradient (stored before the pooling adjoint
             adds the second path to it).

Weight and bias gradients are accumulated without rounding, as the library
accumulates them in FP32. The parity tests derive their tolerances from the
emulated errors (a stated multiple of them) instead of fixed constants. With
rounding switched off the emulation is the oracle's network exactly (pinned
in test_bf16_storage_cpu.py).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def _rb(x: torch.Tensor) -> torch.Tensor:
    return x.to(torch.bfloat16).to(torch.float64)


class _RoundBoth(torch.autograd.Function):
    """bf16 storage of a tensor and of the gradient written for it."""

    @staticmethod
    def forward(ctx, x):
        return _rb(x)

    @staticmethod
    def backward(ctx, g):
        return _rb(g)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; the gradient is stored in bf16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _rb(g)


class _RoundFwd(torch.autograd.Function):
    """bf16 copy of a weight tensor; its gradient reaches the FP32 master
    unrounded."""

    @staticmethod
    def forward(ctx, x):
        return _rb(x)

    @staticmethod
    def backward(ctx, g):
        return g


def _act(x, slope):
    return F.leaky_relu(x, negative_slope=slope) if slope > 0 else F.relu(x)


def forward(params, x, depth: int, slope: float = 0.0, rounding: bool = True):
    """y = N(x) (float64 tensors, parameter-vector order) with bf16 storage
    emulated when `rounding` is set."""
    both = _RoundBoth.apply if rounding else (lambda t: t)
    grad = _RoundGrad.apply if rounding else (lambda t: t)
    wq = _RoundFwd.apply if rounding else (lambda t: t)
    it = iter(params)

    def conv_act(h, w, b):
        z = F.conv2d(h, wq(w), b, padding=1)
        return wq(_act(grad(z), slope))

    def dconv(h):
        w1, b1, w2, b2 = next(it), next(it), next(it), next(it)
        return conv_act(conv_act(h, w1, b1), w2, b2)

    h = both(x[None, None])
    h = dconv(h)
    skips = [h]
    for _ in range(depth):
        h = both(F.avg_pool2d(h, 3, stride=2, padding=1, count_include_pad=True))
        h = dconv(h)
        skips.append(h)
    for lvl in range(depth - 1, -1, -1):
        wt, bt = next(it), next(it)
        h = both(F.conv_transpose2d(h, wq(wt), bt, stride=2))
        h = torch.cat([grad(skips[lvl]), h], dim=1)
        h = dconv(h)
    wo, bo = next(it), next(it)
    return F.conv2d(h, wo, bo)[0, 0]


def loss_and_grads(params_np, x_np, t_np, depth: int, slope: float = 0.0, rounding: bool = True):
    """MSE loss and every parameter gradient under bf16 storage."""
    params = [torch.as_tensor(np.asarray(p, np.float64)).requires_grad_(True) for p in params_np]
    y = forward(params, torch.as_tensor(np.asarray(x_np, np.float64)), depth, slope, rounding)
    loss = torch.mean((y - torch.as_tensor(np.asarray(t_np, np.float64))) ** 2)
    loss.backward()
    return float(loss.detach()), [p.grad.numpy().copy() for p in params], y.detach().numpy()


def rel(a, b) -> float:
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else 0.0


# The GPU's rounding differs from the emulation's in where sums are split
# (FP32 partial sums, gradients accumulated into bf16 buffers in two steps)
# and in which values sit next to a rounding boundary: its error is a second
# draw of the same size, not the same draw. A GPU error within this multiple
# of the emulated one is consistent with bf16 storage; a wrong tap, weight or
# skip connection gives errors of order one.
BF16_FACTOR = 2.0


def forward_bound(params_np, x_np, depth: int, slope: float) -> tuple[float, np.ndarray]:
    """(bound, exact output): BF16_FACTOR times the emulated relative L2
    error of N(x) against the unrounded float64 network."""
    ps = [torch.as_tensor(np.asarray(p, np.float64)) for p in params_np]
    x = torch.as_tensor(np.asarray(x_np, np.float64))
    with torch.no_grad():
        exact = forward(ps, x, depth, slope, rounding=False).numpy()
        emul = forward(ps, x, depth, slope, rounding=True).numpy()
    return BF16_FACTOR * rel(emul, exact), exact


def gradient_bounds(params_np, x_np, t_np, depth: int, slope: float, grads_exact) -> list[float]:
    """Per-tensor bounds: BF16_FACTOR times the emulated relative L2 error of
    every parameter gradient against the exact (oracle) gradients."""
    _, ge, _ = loss_and_grads(params_np, x_np, t_np, depth, slope, rounding=True)
    return [BF16_FACTOR * rel(a, b) for a, b in zip(ge, grads_exact)]
