"""GPU parity of the deblurring network (bf16 matrix cores, FP32 accumulation)
against the FP64 network oracle, on weights and inputs drawn by the shared
seeded generators.

Tolerances are derived, not fixed: the library stores activations, weights
and back-propagated gradients in bf16 (unit roundoff 2^-8) and accumulates in
FP32, so the error it can show against the FP64 oracle is the error bf16
storage causes. tests/bf16_storage.py computes that error for each case (the
oracle's network with values rounded to bf16 where the library stores them)
and every bound below is BF16_FACTOR (2) times it: per output for the
forward pass, per tensor for the parameter gradients, and for the loss the
first-order effect of the output error, 2 |dy| / |y - t| + (|dy| / |y - t|)^2.

The optimiser is checked element by element: the weights after each Adam
step of a training run equal the oracle's Adam update (FP64) of the weights
before it, fed the gradient the GPU used, to FP32 rounding.
"""
import os
import tempfile

import numpy as np
import pytest

import bf16_storage as B
from oracle import deblur_ref as R
from synth import netparams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import _abi, ops  # noqa: E402
from paper_2403_17518_amd.deblur import DeblurConfig, DeblurNet  # noqa: E402


def loss_bound(fwd_bound, y_exact, t):
    """Relative loss error that an output error of fwd_bound |y| allows."""
    r = fwd_bound * np.linalg.norm(y_exact) / np.linalg.norm(np.asarray(y_exact) - np.asarray(t, np.float64))
    return 2.0 * r + r * r


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def smooth_field(H, W, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((H, W))
    k = np.exp(-np.arange(-6, 7) ** 2 / 8.0)
    z = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 0, z)
    z = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 1, z)
    return z / np.abs(z).max()


@pytest.fixture(scope="module")
def fctx():
    c = ops.FwiContext(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("depth,base,H,W,slope", [(2, 16, 32, 64, 0.0), (3, 32, 64, 192, 0.2),
                                                  (4, 128, 32, 64, 0.2)])
def test_forward_matches_oracle(fctx, depth, base, H, W, slope):
    print(f"[deblur] forward depth={depth} base={base} {H}x{W}", flush=True)
    cfg = DeblurConfig(depth, base, slope, H, W)
    net = DeblurNet(fctx, cfg)
    ps = netparams.draw(depth, base, seed=7)
    flat = netparams.flatten(ps)
    net.set_params(flat)
    assert np.array_equal(net.get_params(), flat)
    x = smooth_field(H, W, 1)
    y = net.forward_raw(dev(x)).cpu().numpy()
    ps32 = [torch.as_tensor(p.astype(np.float32).astype(np.float64)) for p in ps]
    ref = R.forward(ps32, torch.as_tensor(x.astype(np.float32).astype(np.float64)), depth, slope).numpy()
    bound, _ = B.forward_bound([p.numpy() for p in ps32], x.astype(np.float32), depth, slope)
    e = rel(y, ref)
    print(f"forward rel err {e:.3e}, derived bound {bound:.3e}")
    assert e < bound
    net.close()


def test_full_size_forward(fctx):
    """The configuration trained in FWI: depth 3, widths 32-64-128-256, ReLU,
    208 x 608."""
    cfg = DeblurConfig()
    net = DeblurNet(fctx, cfg)
    ps = netparams.draw(3, 32, seed=9)
    net.set_params(netparams.flatten(ps))
    x = smooth_field(208, 608, 2)
    y = net.forward_raw(dev(x)).cpu().numpy()
    ps32 = [torch.as_tensor(p.astype(np.float32).astype(np.float64)) for p in ps]
    ref = R.forward(ps32, torch.as_tensor(x.astype(np.float32).astype(np.float64)), 3, 0.0).numpy()
    bound, _ = B.forward_bound([p.numpy() for p in ps32], x.astype(np.float32), 3, 0.0)
    e = rel(y, ref)
    print(f"full-size forward rel err {e:.3e}, derived bound {bound:.3e}")
    assert e < bound
    net.close()


def _check_gradients(net, depth, base, slope, ps, x, t, tag):
    loss, g = net.grad_raw(dev(x), dev(t))
    ps32 = [p.astype(np.float32).astype(np.float64) for p in ps]
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    lref, gref, yref = R.loss_and_grads(ps32, x32, t32, depth, slope)
    fb, _ = B.forward_bound(ps32, x32, depth, slope)
    lb = loss_bound(fb, yref, t32)
    print(f"[{tag}] loss rel err {abs(loss - lref) / lref:.3e}, derived bound {lb:.3e}")
    assert abs(loss - lref) <= lb * lref
    bounds = B.gradient_bounds(ps32, x32, t32, depth, slope, gref)
    gg = netparams.unflatten(g, depth, base)
    names = [n for n, _ in netparams.param_shapes(depth, base)]
    worst = (0.0, "", 0.0)
    for name, a, b, bd in zip(names, gg, gref, bounds):
        if np.linalg.norm(b) == 0:
            continue
        e = rel(a, b)
        if e / bd > worst[0]:
            worst = (e / bd, name, e)
        assert e < bd, (name, e, bd)
    print(f"[{tag}] largest gradient error / derived bound: {worst[0]:.2f} ({worst[1]}, {worst[2]:.3e})")


@pytest.mark.parametrize("slope", [0.0, 0.2])
def test_parameter_gradients_match_oracle(fctx, slope):
    depth, base, H, W = 2, 16, 32, 64
    net = DeblurNet(fctx, DeblurConfig(depth, base, slope, H, W))
    ps = netparams.draw(depth, base, seed=11)
    net.set_params(netparams.flatten(ps))
    _check_gradients(net, depth, base, slope, ps, smooth_field(H, W, 3), smooth_field(H, W, 4), f"slope {slope}")
    net.close()


def test_paper_scale_gradients_match_oracle(fctx):
    """The paper's network (four down blocks, widths 128-2048, LeakyReLU 0.2):
    every parameter gradient against the FP64 oracle on a 32 x 64 image. The
    deepest block works on 2 x 4 pixels, so its weight gradients are sums of
    a handful of products of bf16-stored activations and gradients after 23
    layers: its derived bound is the loosest (about 0.14)."""
    depth, base, H, W, slope = 4, 128, 32, 64, 0.2
    net = DeblurNet(fctx, DeblurConfig(depth, base, slope, H, W))
    ps = netparams.draw(depth, base, seed=17)
    net.set_params(netparams.flatten(ps))
    _check_gradients(net, depth, base, slope, ps, smooth_field(H, W, 7), smooth_field(H, W, 8), "paper scale")
    net.close()


def test_adam_steps_match_the_oracle_elementwise(fctx):
    """Adam with bias correction and the cosine-annealed rate (paper section
    2.4): a 3-step run split over three deblur_train_range calls. Before each
    step the gradient at the network's current weights is read with
    deblur_grad_raw (the image fills the grid and is already scaled to
    max |x| = 1, so it is the gradient the training step computes); after it,
    every weight must equal the oracle's FP64 Adam update of the weights
    before it with that gradient and the oracle's moments, within one FP32
    unit in the last place of the weight plus 1e-5 of the step's learning
    rate (the FP32 arithmetic of the update). The split run must give the
    weights of one deblur_train(3) call bit for bit."""
    depth, base, H, W, slope = 2, 16, 32, 64, 0.2
    net = DeblurNet(fctx, DeblurConfig(depth, base, slope, H, W))
    p0 = netparams.flatten(netparams.draw(depth, base, seed=19))
    x, y = dev(smooth_field(H, W, 3)), dev(smooth_field(H, W, 4))
    assert float(x.abs().max()) == 1.0 and float(y.abs().max()) == 1.0
    total, lr_max = 3, 1e-3
    net.set_params(p0)
    net.deblur_train(x, y, total, lr_max)
    p_once = net.get_params()
    net.set_params(p0)
    p = p0.copy()
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    for t in range(total):
        _, g = net.grad_raw(x, y)
        net.train_range(x, y, t, 1, total, lr_max)
        p_new = net.get_params()
        lr = R.cosine_lr(lr_max, t, total)
        ref, m, v = R.adam_step(p.astype(np.float64), g.astype(np.float64), m, v, t + 1, lr)
        err = np.abs(p_new.astype(np.float64) - ref)
        tol = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) + 1e-5 * lr
        k = int(np.argmax(err / tol))
        print(f"[adam] step {t}: lr {lr:.3e}, worst |err| / tol = {err[k] / tol[k]:.3f} "
              f"(update {abs(ref[k] - p[k]):.3e})")
        assert np.all(err <= tol)
        # the step moved every weight with a non-zero gradient by about lr
        moved = np.abs(ref - p) > 0.5 * lr
        assert moved.mean() > 0.5
        p = p_new
    assert np.array_equal(p, p_once)
    net.close()


def test_train_range_refuses_a_broken_run(fctx):
    depth, base, H, W = 2, 8, 16, 32
    net = DeblurNet(fctx, DeblurConfig(depth, base, 0.0, H, W))
    x, y = dev(smooth_field(H, W, 1)), dev(smooth_field(H, W, 2))
    net.train_range(x, y, 0, 2, 5, 1e-3)
    for first, total, lr in ((3, 5, 1e-3), (2, 6, 1e-3), (2, 5, 2e-3)):
        with pytest.raises(_abi.FwiError) as ei:
            net.train_range(x, y, first, 1, total, lr)
        assert ei.value.code == _abi.FWI_ESTATE
    with pytest.raises(_abi.FwiError):
        net.train_range(x, y, 4, 2, 5, 1e-3)        # past the end of the run
    net.train_range(x, y, 2, 3, 5, 1e-3)            # the run continues where it stopped
    net.set_params(net.get_params())                 # new weights end the run
    with pytest.raises(_abi.FwiError):
        net.train_range(x, y, 0 + 1, 1, 5, 1e-3)
    net.close()


def test_training_follows_the_oracle_and_reduces_the_loss(fctx):
    """Adam + cosine schedule on a known blur: the GPU loss curve tracks the
    FP64 oracle's and falls by more than 10x."""
    depth, base, H, W = 2, 16, 32, 64
    cfg = DeblurConfig(depth, base, 0.0, H, W)
    net = DeblurNet(fctx, cfg)
    ps = netparams.draw(depth, base, seed=13)
    net.set_params(netparams.flatten(ps))
    y = smooth_field(H, W, 5)
    k = np.exp(-np.arange(-4, 5) ** 2 / 4.0)
    x = np.apply_along_axis(lambda r: np.convolve(r, k / k.sum(), "same"), 0, y)
    x = np.apply_along_axis(lambda r: np.convolve(r, k / k.sum(), "same"), 1, x)
    steps, lr = 60, 2e-3
    hist = net.deblur_train(dev(x), dev(y), steps, lr)
    # oracle on the same normalised pair (no padding: the image fills the grid)
    xn = (x / np.abs(x).max()).astype(np.float32)
    yn = (y / np.abs(y).max()).astype(np.float32)
    ps32 = [p.astype(np.float32).astype(np.float64) for p in ps]
    _, lref = R.train(ps32, xn, yn, depth, steps, lr)
    fb, y0 = B.forward_bound(ps32, xn, depth, 0.0)
    lb = loss_bound(fb, y0, yn)
    print("loss gpu", hist[0], hist[-1], "oracle", lref[0], lref[-1], "first-loss bound", lb)
    assert abs(hist[0] - lref[0]) <= lb * lref[0]
    assert hist[-1] < hist[0] / 10.0
    assert abs(np.log(hist[-1] / lref[-1])) < np.log(2.0)
    net.close()


def test_apply_scales_pads_and_crops(fctx):
    depth, base = 2, 16
    cfg = DeblurConfig(depth, base, 0.0, 40, 72)
    net = DeblurNet(fctx, cfg)
    g = smooth_field(36, 64, 6) * 3.7
    out = net.deblur_apply(dev(g)).cpu().numpy()
    xp, mx, py, px = R.normalise_pad(g.astype(np.float32), 40, 72)
    raw = net.forward_raw(dev(xp)).cpu().numpy()
    assert (py, px) == (2, 4)
    assert rel(out, mx * raw[py:py + 36, px:px + 64]) < 1e-3
    # odd padding (3 rows, 5 columns): the extra cell below and right
    g = smooth_field(37, 67, 6) * 2.1
    out = net.deblur_apply(dev(g)).cpu().numpy()
    xp, mx, py, px = R.normalise_pad(g.astype(np.float32), 40, 72)
    raw = net.forward_raw(dev(xp)).cpu().numpy()
    assert (py, px) == (1, 2) and out.shape == (37, 67)
    assert rel(out, mx * raw[py:py + 37, px:px + 67]) < 1e-3
    net.close()


def test_layer_stats_cover_every_gemm(fctx):
    """Per-layer timing: every convolution appears with its three passes
    (the input layer without a data gradient), one call per training step,
    and the flops add up to three forward passes less the input layer's
    data gradient."""
    import bench
    depth, base, H, W = 2, 16, 32, 64
    net = DeblurNet(fctx, DeblurConfig(depth, base, 0.0, H, W))
    x, y = dev(smooth_field(H, W, 1)), dev(smooth_field(H, W, 2))
    net.set_profiling(True)
    net.deblur_train(x, y, 2, 1e-3)
    recs = net.layer_stats()
    net.set_profiling(False)
    names = {r["name"] for r in recs}
    assert names == {"inc.1", "inc.2", "down1.1", "down1.2", "down2.1", "down2.2",
                     "up1.T", "up1.1", "up1.2", "up0.T", "up0.1", "up0.2"}
    assert all(r["calls"] == 2 and r["ms"] > 0 for r in recs)
    assert not any(r["name"] == "inc.1" and r["pass"] == "data_grad" for r in recs)
    fwd = sum(r["flops"] for r in recs if r["pass"] == "forward") / 2
    assert abs(fwd - (bench.deblur_flops(H, W, depth, base) - 2 * H * W * base)) < 1.0   # less the 1x1 output conv
    net.close()


def test_save_load_reset(fctx):
    cfg = DeblurConfig(2, 8, 0.0, 16, 32)
    net = DeblurNet(fctx, cfg, seed=1)
    p1 = net.get_params()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "w.bin")
        net.save(path)
        net.reset(2)
        p2 = net.get_params()
        assert not np.array_equal(p1, p2)
        net.load(path)
        assert np.array_equal(net.get_params(), p1)
    net.close()
