"""FP64 CPU reference of the deblurring network (test infrastructure only).

Paper section 2.3 / 2.4 and Appendix A (Table 1): a UNet-like network with
an input block of two 3x3 convolutions (stride 1, padding 1) each followed by
the activation, D down blocks (3x3 average pooling with stride 2, then the
same double convolution doubling the channels), D up blocks (a transposed
convolution that halves the channels, then a double convolution) and a 1x1
output convolution to one channel. Readings where the paper is silent (they
are the library's definition): the pooling pads by 1 and counts the padding,
the transposed convolution has kernel 2 and stride 2, the up block
concatenates [encoder features, up-sampled features] as in the cited UNet,
no activation follows the output convolution. Training: MSE loss, Adam with
a cosine-annealed learning rate (section 2.4).

Built from plain PyTorch CPU functional ops in float64; gradients come from
torch autograd. Only tests may import this module.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def act(x, slope):
    return F.leaky_relu(x, negative_slope=slope) if slope > 0 else F.relu(x)


def forward(params, x, depth: int, slope: float = 0.0):
    """y = N(x) for x of shape [H][W] (float64 tensors); params in the
    parameter-vector order (torch layouts)."""
    it = iter(params)

    def dconv(h):
        w1, b1, w2, b2 = next(it), next(it), next(it), next(it)
        h = act(F.conv2d(h, w1, b1, padding=1), slope)
        return act(F.conv2d(h, w2, b2, padding=1), slope)

    h = x[None, None]
    h = dconv(h)
    skips = [h]
    for _ in range(depth):
        h = F.avg_pool2d(h, 3, stride=2, padding=1, count_include_pad=True)
        h = dconv(h)
        skips.append(h)
    for l in range(depth - 1, -1, -1):
        wt, bt = next(it), next(it)
        h = F.conv_transpose2d(h, wt, bt, stride=2)
        h = torch.cat([skips[l], h], dim=1)
        h = dconv(h)
    wo, bo = next(it), next(it)
    return F.conv2d(h, wo, bo)[0, 0]


def loss_and_grads(params_np, x_np, t_np, depth: int, slope: float = 0.0):
    """MSE loss mean((N(x) - t)^2) and its gradient for every parameter."""
    params = [_t(p).requires_grad_(True) for p in params_np]
    y = forward(params, _t(x_np), depth, slope)
    loss = torch.mean((y - _t(t_np)) ** 2)
    loss.backward()
    return float(loss.detach()), [p.grad.numpy().copy() for p in params], y.detach().numpy()


def cosine_lr(lr_max: float, t: int, steps: int) -> float:
    """Learning rate of step t (0-based) annealed from lr_max to 0 over steps."""
    return lr_max * 0.5 * (1.0 + math.cos(math.pi * t / steps))


def adam_step(p, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1) with bias-corrected moments."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(params_np, x_np, t_np, depth: int, steps: int, lr_max: float, slope: float = 0.0):
    """Adam training with the cosine schedule; returns (params, losses)."""
    ps = [np.asarray(p, dtype=np.float64).copy() for p in params_np]
    ms = [np.zeros_like(p) for p in ps]
    vs = [np.zeros_like(p) for p in ps]
    losses = []
    for t in range(steps):
        loss, grads, _ = loss_and_grads(ps, x_np, t_np, depth, slope)
        losses.append(loss)
        lr = cosine_lr(lr_max, t, steps)
        for i in range(len(ps)):
            ps[i], ms[i], vs[i] = adam_step(ps[i], grads[i], ms[i], vs[i], t + 1, lr)
    return ps, losses


def normalise_pad(img, H: int, W: int):
    """img / max|img|, reflect-padded to H x W: floor((H - nz) / 2) rows
    above, the rest below; columns alike."""
    img = np.asarray(img, dtype=np.float64)
    mx = np.max(np.abs(img))
    nz, nx = img.shape
    py, px = (H - nz) // 2, (W - nx) // 2
    return np.pad(img / mx if mx > 0 else img * 0, ((py, H - nz - py), (px, W - nx - px)), mode="reflect"), mx, py, px
