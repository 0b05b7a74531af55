"""GPU parity of the perfectly matched layer (fwi_grid.pml) against the FP64
oracle: forward data, misfit and gradient (whole history stored,
checkpointed with uniform and binomial schedules), Born data, migration,
born_pair and the fused gradient + pair, also under a free surface and on
two-level tilings (the intermediate level's edge fields kept in registers);
the FP32 dot-product test; one- and two-level tilings agree bitwise."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops  # noqa: E402

TOL_DATA = 1e-4
TOL_IMAGE = 1e-4
TOL_GRAD = 1e-3
TOL_DOT = 1e-4


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def ctx():
    c = ops.FwiContext(0)
    yield c
    c.close()


def _ragged(free_surface=False):
    wl = configs.ragged_small()
    wl.grid = replace(wl.grid, pml=True, free_surface=free_surface)
    wl.acq.wavelet = np.asarray(wl.acq.wavelet, np.float32)
    return wl


@pytest.mark.parametrize("free_surface,ckpt,tiling", [(False, 0, None), (False, 29, None), (True, 0, None),
                                                      (False, 0, (2, 24, 2, 1)), (True, 29, (1, 16, 2, 2))])
def test_pml_operators_match_oracle(ctx, free_surface, ckpt, tiling):
    wl = _ragged(free_surface)
    g, acq = replace(wl.grid, ckpt_every=ckpt), wl.acq
    print(f"[pml] ragged free_surface={free_surface} ckpt={ckpt} tiling={tiling}", flush=True)
    ctx.set_tiling(-1, *(tiling or (0, 0, 0)))
    vt = np.asarray(wl.v_true, np.float32).astype(np.float64)
    v0 = np.asarray(wl.v0, np.float32).astype(np.float64)
    d_obs = np.asarray(oracle.forward(g, acq, vt), np.float32).astype(np.float64)
    d = host(ctx.fwi_forward(g, acq, dev(vt)))
    e_d = rel(d, d_obs)
    gr, phi, _ = ctx.fwi_gradient(g, acq, dev(v0), dev(d_obs))
    g_ref, phi_ref, _ = oracle.gradient(g, acq, v0, d_obs)
    e_g = rel(host(gr), g_ref)
    if ckpt:
        assert ctx.stats()["n_segments"] > 1
    dv = np.asarray(wl.v_true - wl.v0, np.float32).astype(np.float64)
    dd = host(ctx.born_demig(g, acq, dev(v0), dev(dv)))
    e_b = rel(dd, oracle.born_demig(g, acq, v0, dv))
    y = np.random.default_rng(4).standard_normal(acq.data_size(g)).astype(np.float32).astype(np.float64)
    im = host(ctx.born_mig(g, acq, dev(v0), dev(y)))
    e_m = rel(im, oracle.born_mig(g, acq, v0, y))
    grad, phi2, img = ctx.gradient_pair(g, acq, dev(v0), dev(d_obs), scale=-1.0)
    pair_ref = oracle.born_pair(g, acq, v0, -host(grad))
    e_p = rel(host(img), pair_ref)
    img_bp = ctx.born_pair(g, acq, dev(v0), -grad)
    e_bp = rel(host(img_bp), pair_ref)
    print(f"forward {e_d:.2e} gradient {e_g:.2e} misfit {abs(phi - phi_ref) / phi_ref:.2e} born {e_b:.2e} "
          f"migration {e_m:.2e} pair {e_p:.2e} born_pair {e_bp:.2e}", flush=True)
    assert e_d < TOL_DATA
    assert e_g < TOL_GRAD
    assert abs(phi - phi_ref) <= 1e-4 * abs(phi_ref)
    assert e_b < TOL_DATA
    assert e_m < TOL_IMAGE
    assert torch.equal(grad, gr) and phi2 == phi
    assert e_p < TOL_IMAGE and e_bp < TOL_IMAGE
    if tiling:
        assert ctx.stats()["tile_levels"][:2] == [2, 2]
    ctx.set_tiling(-1, 0, 0, 0)


def test_pml_dot_product_fp32(ctx):
    wl = _ragged()
    g, acq = wl.grid, wl.acq
    rng = np.random.default_rng(9)
    x = dev(rng.standard_normal((g.nz, g.nx)))
    yv = dev(rng.standard_normal(acq.data_size(g)))
    v0 = dev(wl.v0)
    lhs = float(torch.dot(ctx.born_demig(g, acq, v0, x).double(), yv.double()))
    rhs = float(torch.sum(x.double() * ctx.born_mig(g, acq, v0, yv).double()))
    print(f"[pml] dot test {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
    assert abs(lhs - rhs) <= TOL_DOT * abs(lhs)


def test_pml_checkpoint_schedules_give_the_full_history_bits(ctx):
    """Snapshots carry the layer's edge fields: uniform and binomial
    schedules (3, 1 and 0 snapshots) reproduce the stored-history bits."""
    wl = _ragged()
    g0, acq = wl.grid, wl.acq
    v0 = dev(wl.v0)
    d_obs = ctx.fwi_forward(g0, acq, dev(wl.v_true))
    ref = ctx.fwi_gradient(g0, acq, v0, d_obs)[0]
    assert ctx.stats()["n_segments"] == 1
    ref_bp = ctx.born_pair(g0, acq, v0, ref)
    g = replace(g0, ckpt_every=13)
    for slots in (-1, 3, 1, 0):
        print(f"[pml] checkpoints of 13 steps, snapshot cap {slots}", flush=True)
        ctx.set_ckpt_slots(slots)
        gr = ctx.fwi_gradient(g, acq, v0, d_obs)[0]
        st = ctx.stats()
        assert st["n_segments"] > 1
        assert torch.equal(gr, ref)
        assert torch.equal(ctx.born_pair(g, acq, v0, ref), ref_bp)
    ctx.set_ckpt_slots(-1)


@pytest.mark.parametrize("free_surface", [False, True])
def test_pml_tilings_bitwise_equal(ctx, free_surface):
    wl = _ragged(free_surface)
    g, acq = wl.grid, wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    outs = []
    for t in [(1, 7, 1, 1), (2, 13, 1, 2), (1, 300, 1, 2), (2, 5, 1, 1),
              (1, 24, 2, 1), (2, 13, 2, 2), (1, 300, 2, 2), (2, 48, 2, 1)]:
        print(f"[pml] tiling {t}", flush=True)
        ctx.set_tiling(-1, *t)
        d = ctx.fwi_forward(g, acq, vt)
        gr = ctx.fwi_gradient(g, acq, v0, d * 0.5)[0]
        dd = ctx.born_demig(g, acq, v0, vt - v0)
        gp = ctx.gradient_pair(g, acq, v0, d * 0.5, scale=-1.0)[2]
        outs.append((d, gr, dd, gp))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)
    ctx.set_tiling(-1, 0, 0, 0)
    assert torch.equal(ctx.fwi_forward(g, acq, vt), outs[0][0])   # the autotuner's pick


def test_pml_absorbs_on_the_gpu(ctx):
    """A trace 100 m from the source in a 61 x 61 box with a 20-cell layer
    matches a box too large for reflections to return within the record,
    where the sponge of the same width leaves a visible reflection."""
    from synth import Acquisition, Grid, ricker
    nt, v = 800, 2000.0

    def trace(half, nb, pml):
        n = 2 * half + 1
        g = Grid(nz=n, nx=n, nb=nb, h=10.0, dt=1e-3, nt_max=nt, v_ref=v, pml=pml)
        a = Acquisition(src_z=[half], src_x=[half], rec_ptr=[0, 1], rec_z=[half], rec_x=[half + 10],
                        wavelet=ricker(10.0, 1e-3, nt).astype(np.float32))
        return host(ctx.fwi_forward(g, a, dev(np.full((n, n), v))))

    ref = trace(200, 0, False)
    e_pml, e_sp = rel(trace(30, 20, True), ref), rel(trace(30, 20, False), ref)
    print(f"[pml] reflected part on the GPU: PML {e_pml:.2e}, sponge {e_sp:.2e}", flush=True)
    assert e_pml < 2e-3 and e_sp > 20.0 * e_pml
