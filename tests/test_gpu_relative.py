"""GPU parity of the relative-perturbation Born operator J diag(v) (section
2.2 eq. 12) against the FP64 oracle: Born data, migration, gradient (with
and without checkpointing), the pair and the fused gradient + pair; the
misfit does not depend on the parametrisation; the relative operators are
the velocity ones with dv = v dm and images times v; tilings agree
bitwise; autograd stays with the velocity gradient."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops, autograd  # noqa: E402

TOL_DATA = 1e-4
TOL_IMAGE = 1e-4
TOL_GRAD = 1e-3


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def ctx():
    c = ops.FwiContext(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def wl():
    w = configs.ragged_small()
    w.acq.wavelet = np.asarray(w.acq.wavelet, np.float32)
    return w


@pytest.mark.parametrize("ckpt", [0, 29])
def test_relative_operators_match_oracle(ctx, wl, ckpt):
    g = replace(wl.grid, relative=True, ckpt_every=ckpt)
    acq = wl.acq
    print(f"[relative] ragged ckpt={ckpt}", flush=True)
    vt, v0 = f32(wl.v_true), f32(wl.v0)
    d_obs = f32(oracle.forward(g, acq, vt))
    gr, phi, _ = ctx.fwi_gradient(g, acq, dev(v0), dev(d_obs))
    g_ref, phi_ref, _ = oracle.gradient(g, acq, v0, d_obs)
    e_g = rel(host(gr), g_ref)
    print("gradient rel err", e_g)
    assert e_g < TOL_GRAD
    assert abs(phi - phi_ref) <= 1e-4 * abs(phi_ref)
    if ckpt:
        assert ctx.stats()["n_segments"] > 1
    dm = f32((wl.v_true - wl.v0) / wl.v0)
    dd = host(ctx.born_demig(g, acq, dev(v0), dev(dm)))
    assert rel(dd, oracle.born_demig(g, acq, v0, dm)) < TOL_DATA
    y = f32(np.random.default_rng(6).standard_normal(acq.data_size(g)))
    im = host(ctx.born_mig(g, acq, dev(v0), dev(y)))
    assert rel(im, oracle.born_mig(g, acq, v0, y)) < TOL_IMAGE
    pair = host(ctx.born_pair(g, acq, dev(v0), dev(dm)))
    assert rel(pair, oracle.born_pair(g, acq, v0, dm)) < TOL_IMAGE
    grad, phi2, img = ctx.gradient_pair(g, acq, dev(v0), dev(d_obs), scale=-1.0)
    assert torch.equal(grad, gr) and phi2 == phi
    e_p = rel(host(img), oracle.born_pair(g, acq, v0, -host(grad)))
    print("pair rel err", e_p)
    assert e_p < TOL_IMAGE


def test_relative_is_velocity_operator_rescaled(ctx, wl):
    ga, gr_ = wl.grid, replace(wl.grid, relative=True)
    acq = wl.acq
    v0 = dev(wl.v0)
    d_obs = ctx.fwi_forward(ga, acq, dev(wl.v_true))
    g_abs, phi_a, _ = ctx.fwi_gradient(ga, acq, v0, d_obs)
    g_rel, phi_r, _ = ctx.fwi_gradient(gr_, acq, v0, d_obs)
    assert phi_a == phi_r
    assert rel(host(g_rel), host(v0 * g_abs)) < 1e-6
    dm = dev((wl.v_true - wl.v0) / wl.v0)
    a = ctx.born_demig(gr_, acq, v0, dm)
    b = ctx.born_demig(ga, acq, v0, v0 * dm)
    assert rel(host(a), host(b)) < 1e-5


def test_relative_tilings_bitwise_equal(ctx, wl):
    g = replace(wl.grid, relative=True)
    acq = wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    dm = (vt - v0) / v0
    outs = []
    for t in [(1, 7, 1, 1), (2, 13, 1, 2), (1, 300, 2, 1), (2, 5, 2, 1)]:
        print(f"[relative] tiling {t}", flush=True)
        ctx.set_tiling(-1, *t)
        d = ctx.fwi_forward(g, acq, vt)
        gr = ctx.fwi_gradient(g, acq, v0, d * 0.5)[0]
        dd = ctx.born_demig(g, acq, v0, dm)
        gp = ctx.gradient_pair(g, acq, v0, d * 0.5, scale=-1.0)[2]
        outs.append((d, gr, dd, gp))
    ctx.set_tiling(-1, 0, 0, 0)
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)


def test_autograd_keeps_the_velocity_gradient(ctx, wl):
    ga, gr_ = wl.grid, replace(wl.grid, relative=True)
    acq = wl.acq
    d_obs = ctx.fwi_forward(ga, acq, dev(wl.v_true))
    v = dev(wl.v0).requires_grad_(True)
    autograd.misfit(v, d_obs, gr_, acq, ctx).backward()
    g_abs = ctx.fwi_gradient(ga, acq, dev(wl.v0), d_obs)[0]
    assert torch.equal(v.grad, g_abs)


def test_bad_relative_flag_rejected(ctx, wl):
    import ctypes as C
    v = dev(wl.v0)
    d = torch.empty(wl.acq.data_size(wl.grid), device="cuda", dtype=torch.float32)
    g, gv = ctx._prep(wl.grid, wl.acq)
    g.relative = 2
    rc = ctx.lib.fwi_forward(ctx.ctx, C.byref(g), C.byref(gv.geom), C.c_void_p(v.data_ptr()),
                             C.c_void_p(d.data_ptr()))
    assert rc == -1                               # FWI_EINVAL
    g.relative = 1
    assert ctx.lib.fwi_forward(ctx.ctx, C.byref(g), C.byref(gv.geom), C.c_void_p(v.data_ptr()),
                               C.c_void_p(d.data_ptr())) == 0
