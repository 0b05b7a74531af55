"""Pins of the network oracle: brute-force loops on tiny inputs for every
layer type, the whole network against a loop-only forward, the autograd
gradient against finite differences, Adam and the cosine schedule against
torch's own optimiser and scheduler."""
import math

import numpy as np
import pytest
import torch

from oracle import deblur_ref as R
from synth import netparams


def conv3x3_loops(x, w, b):
    """x [Cin][H][W], w [Cout][Cin][3][3]: zero-padded stride-1 correlation."""
    Cin, H, W = x.shape
    Cout = w.shape[0]
    xp = np.zeros((Cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((Cout, H, W))
    for co in range(Cout):
        for i in range(H):
            for j in range(W):
                y[co, i, j] = b[co] + np.sum(w[co] * xp[:, i:i + 3, j:j + 3])
    return y


def pool_loops(x):
    C, H, W = x.shape
    y = np.zeros((C, H // 2, W // 2))
    for i in range(H // 2):
        for j in range(W // 2):
            s = np.zeros(C)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy, xx = 2 * i + dy, 2 * j + dx
                    if 0 <= yy < H and 0 <= xx < W:
                        s += x[:, yy, xx]
            y[:, i, j] = s / 9.0
    return y


def convt_loops(x, w, b):
    """x [Cin][H][W], w [Cin][Cout][2][2]: out[co][2i+a][2j+b]."""
    Cin, H, W = x.shape
    Cout = w.shape[1]
    y = np.zeros((Cout, 2 * H, 2 * W)) + b[:, None, None]
    for ci in range(Cin):
        for i in range(H):
            for j in range(W):
                for a in range(2):
                    for bb in range(2):
                        y[:, 2 * i + a, 2 * j + bb] += x[ci, i, j] * w[ci, :, a, bb]
    return y


def unet_loops(params, x, depth, slope):
    it = iter(params)
    act = lambda z: np.where(z > 0, z, slope * z)

    def dconv(h):
        w1, b1, w2, b2 = next(it), next(it), next(it), next(it)
        return act(conv3x3_loops(act(conv3x3_loops(h, w1, b1)), w2, b2))

    h = dconv(x[None])
    skips = [h]
    for _ in range(depth):
        h = dconv(pool_loops(h))
        skips.append(h)
    for l in range(depth - 1, -1, -1):
        wt, bt = next(it), next(it)
        h = convt_loops(h, wt, bt)
        h = dconv(np.concatenate([skips[l], h], axis=0))
    wo, bo = next(it), next(it)
    return bo[0] + np.einsum("c,chw->hw", wo[0, :, 0, 0], h)


@pytest.mark.parametrize("slope", [0.0, 0.2])
def test_network_forward_matches_loops(slope):
    depth, base = 2, 8
    ps = netparams.draw(depth, base, seed=3)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((8, 12))
    y = R.forward([torch.as_tensor(p) for p in ps], torch.as_tensor(x), depth, slope).numpy()
    ref = unet_loops(ps, x, depth, slope)
    assert y.shape == x.shape
    assert np.max(np.abs(y - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_gradient_matches_finite_differences():
    depth, base = 1, 8
    ps = netparams.draw(depth, base, seed=5)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6))
    t = rng.standard_normal((4, 6))
    loss, grads, _ = R.loss_and_grads(ps, x, t, depth, 0.2)
    eps = 1e-6
    for k in (0, 5, len(ps) - 4, len(ps) - 2):
        idx = tuple(rng.integers(0, s) for s in ps[k].shape)
        pp = [p.copy() for p in ps]
        pp[k][idx] += eps
        lp = R.loss_and_grads(pp, x, t, depth, 0.2)[0]
        pp[k][idx] -= 2 * eps
        lm = R.loss_and_grads(pp, x, t, depth, 0.2)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grads[k][idx]) < 1e-6 * max(1.0, abs(fd)), (k, fd, grads[k][idx])


def test_adam_and_cosine_match_torch():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(7)
    gs = rng.standard_normal((5, 7))
    steps, lr_max = 5, 3e-3
    tp = torch.nn.Parameter(torch.as_tensor(p0.copy()))
    opt = torch.optim.Adam([tp], lr=lr_max, betas=(0.9, 0.999), eps=1e-8)
    sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=steps, eta_min=0.0)
    p, m, v = p0.copy(), np.zeros(7), np.zeros(7)
    for t in range(steps):
        assert math.isclose(opt.param_groups[0]["lr"], R.cosine_lr(lr_max, t, steps), rel_tol=1e-12)
        tp.grad = torch.as_tensor(gs[t].copy())
        opt.step()
        sch.step()
        p, m, v = R.adam_step(p, gs[t], m, v, t + 1, R.cosine_lr(lr_max, t, steps))
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_parameter_count_of_the_default_network():
    # input block 32, down 64/128/256, up with skips: about 1.93 M parameters
    n = sum(int(np.prod(s)) for _, s in netparams.param_shapes(3, 32))
    assert n == 1925025


def test_normalise_pad_reflects():
    img = np.arange(12.0).reshape(3, 4) - 5
    out, mx, py, px = R.normalise_pad(img, 5, 8)
    assert mx == 6 and (py, px) == (1, 2)
    assert out[1, 2] == img[0, 0] / 6 and out[0, 2] == img[1, 0] / 6 and out[1, 0] == img[0, 2] / 6


def test_odd_padding_puts_the_extra_cell_below_and_right():
    img = np.arange(12.0).reshape(3, 4) + 1
    out, mx, py, px = R.normalise_pad(img, 6, 7)
    assert out.shape == (6, 7) and (py, px) == (1, 1) and mx == 12
    assert np.array_equal(out[1:4, 1:5], img / 12)
    # mirror images about the first and last row / column, edge not repeated
    assert np.array_equal(out[0, 1:5], img[1] / 12)
    assert np.array_equal(out[4, 1:5], img[1] / 12) and np.array_equal(out[5, 1:5], img[0] / 12)
    assert np.array_equal(out[1:4, 5], img[:, 2] / 12) and np.array_equal(out[1:4, 6], img[:, 1] / 12)
