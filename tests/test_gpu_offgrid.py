"""GPU parity of off-grid sources and receivers (bilinear spreading and
sampling) against the FP64 oracle: forward data, misfit and gradient, Born
data, migration and the fused gradient + pair, on a ragged geometry with
co-located and cell-sharing receivers; zero offsets reproduce the on-grid
results exactly; every tiling gives the same bits; bad offsets are
rejected."""
import numpy as np
import pytest

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops, _abi  # noqa: E402

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


def offgrid(wl, seed=3):
    """Random offsets on most sources and receivers; zero where the next
    cell would leave the model or the shot's window."""
    g, a = wl.grid, wl.acq
    a.wavelet = np.asarray(a.wavelet, np.float32)
    rng = np.random.default_rng(seed)
    nr = a.rec_z.shape[0]
    fz = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    fx = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    fz[::4] = 0.0
    fx[::6] = 0.0
    sfz = rng.uniform(0.0, 1.0, a.nshots).astype(np.float32)
    sfx = rng.uniform(0.0, 1.0, a.nshots).astype(np.float32)
    for s in range(a.nshots):
        x0, wn = a.window(s, g)
        r0, r1 = a.rec_ptr[s], a.rec_ptr[s + 1]
        fx[r0:r1][a.rec_x[r0:r1] >= x0 + wn - 1] = 0.0
        if a.src_x[s] >= x0 + wn - 1:
            sfx[s] = 0.0
        if a.src_z[s] >= g.nz - 1:
            sfz[s] = 0.0
    fz[a.rec_z >= g.nz - 1] = 0.0
    a.rec_fz, a.rec_fx, a.src_fz, a.src_fx = fz, fx, sfz, sfx
    return wl


@pytest.fixture(scope="module")
def ctx():
    c = ops.FwiContext(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ragged_off():
    wl = offgrid(configs.ragged_small())
    # a receiver pair sharing cells: the first two receivers of shot 0 moved
    # next to each other
    a = wl.acq
    a.rec_x[1] = a.rec_x[0]
    a.rec_z[1] = a.rec_z[0]
    x0, wn = a.window(0, wl.grid)
    a.rec_fx[1] = 0.0 if a.rec_x[0] >= x0 + wn - 1 else (np.float32(0.5) if a.rec_fx[0] != 0.5 else np.float32(0.25))
    return wl


def test_offgrid_operators_match_oracle(ctx, ragged_off):
    wl = ragged_off
    g, acq = wl.grid, wl.acq
    print("[offgrid] ragged forward/gradient/Born/migration/pair", flush=True)
    vt = np.asarray(wl.v_true, np.float32).astype(np.float64)
    v0 = np.asarray(wl.v0, np.float32).astype(np.float64)
    d_obs = np.asarray(oracle.forward(g, acq, vt), np.float32).astype(np.float64)
    d = host(ctx.fwi_forward(g, acq, dev(vt)))
    assert rel(d, d_obs) < TOL_DATA
    gr, phi, _ = ctx.fwi_gradient(g, acq, dev(v0), dev(d_obs))
    g_ref, phi_ref, _ = oracle.gradient(g, acq, v0, d_obs)
    e_g = rel(host(gr), g_ref)
    print("gradient rel err", e_g, "misfit", phi, phi_ref)
    assert e_g < TOL_GRAD
    assert abs(phi - phi_ref) <= 1e-4 * abs(phi_ref)
    dv = np.asarray(wl.v_true - wl.v0, np.float32).astype(np.float64)
    dd = host(ctx.born_demig(g, acq, dev(v0), dev(dv)))
    assert rel(dd, oracle.born_demig(g, acq, v0, dv)) < TOL_DATA
    y = np.random.default_rng(2).standard_normal(acq.data_size(g)).astype(np.float32).astype(np.float64)
    im = host(ctx.born_mig(g, acq, dev(v0), dev(y)))
    assert rel(im, oracle.born_mig(g, acq, v0, y)) < TOL_IMAGE
    grad, phi2, img = ctx.gradient_pair(g, acq, dev(v0), dev(d_obs), scale=-1.0)
    assert torch.equal(grad, gr) and phi2 == phi
    e_p = rel(host(img), oracle.born_pair(g, acq, v0, -host(grad)))
    print("pair rel err", e_p)
    assert e_p < TOL_IMAGE


def test_offgrid_checkpointed_sweeps_give_the_full_history_bits(ctx, ragged_off):
    """Off-grid adjoint sources injected in recomputed segments: uniform and
    binomial snapshot schedules give the full-history bits for the gradient
    and the migration; the fused call's pair (its own joint sweep once
    checkpointed) equals the separate pair and the oracle's."""
    from dataclasses import replace
    wl = ragged_off
    g0, acq = wl.grid, wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    d_obs = ctx.fwi_forward(g0, acq, vt)
    y = dev(np.random.default_rng(4).standard_normal(acq.data_size(g0)))
    gr0, phi0, _ = ctx.fwi_gradient(g0, acq, v0, d_obs)
    im0 = ctx.born_mig(g0, acq, v0, y)
    g = replace(g0, ckpt_every=29)
    try:
        for slots in (-1, 1):
            print(f"[offgrid] checkpointed sweeps, slots={slots}", flush=True)
            ctx.set_ckpt_slots(slots)
            gr, phi, _ = ctx.fwi_gradient(g, acq, v0, d_obs)
            st = ctx.stats()
            assert st["n_segments"] > 3
            assert st["ckpt_slots"] == (st["n_segments"] - 2 if slots < 0 else slots)
            assert torch.equal(gr, gr0) and phi == phi0
            assert torch.equal(ctx.born_mig(g, acq, v0, y), im0)
            grad, phi2, img = ctx.gradient_pair(g, acq, v0, d_obs, scale=-1.0)
            assert torch.equal(grad, gr0) and phi2 == phi0
            assert torch.equal(img, ctx.born_pair(g, acq, v0, -grad))
        e_p = rel(host(img), oracle.born_pair(g0, acq, np.asarray(wl.v0, np.float32).astype(np.float64),
                                              -host(grad)))
        print("checkpointed pair rel err", e_p)
        assert e_p < TOL_IMAGE
    finally:
        ctx.set_ckpt_slots(-1)


def test_zero_offsets_are_the_on_grid_path(ctx):
    wl = configs.ragged_small()
    g, a = wl.grid, wl.acq
    a.wavelet = np.asarray(a.wavelet, np.float32)
    v0, vt = dev(wl.v0), dev(wl.v_true)
    d0 = ctx.fwi_forward(g, a, vt)
    g0 = ctx.fwi_gradient(g, a, v0, d0 * 0.5)[0]
    a.rec_fz = np.zeros(a.rec_z.shape[0], np.float32)
    a.rec_fx = np.zeros(a.rec_z.shape[0], np.float32)
    a.src_fz = np.zeros(a.nshots, np.float32)
    a.src_fx = np.zeros(a.nshots, np.float32)
    d1 = ctx.fwi_forward(g, a, vt)
    g1 = ctx.fwi_gradient(g, a, v0, d0 * 0.5)[0]
    assert torch.equal(d0, d1) and torch.equal(g0, g1)


def test_offgrid_tilings_bitwise_equal(ctx, ragged_off):
    wl = ragged_off
    g, acq = wl.grid, wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    outs = []
    for t in [(1, 7, 1, 1), (2, 13, 1, 2), (1, 300, 2, 1), (2, 5, 2, 1)]:
        print(f"[offgrid] tiling {t}", flush=True)
        ctx.set_tiling(-1, *t)
        d = ctx.fwi_forward(g, acq, vt)
        gr = ctx.fwi_gradient(g, acq, v0, d * 0.5)[0]
        dd = ctx.born_demig(g, acq, v0, vt - v0)
        outs.append((d, gr, dd))
    ctx.set_tiling(-1, 0, 0, 0)
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)


def test_bad_offsets_rejected(ctx):
    wl = configs.ragged_small()
    g, a = wl.grid, wl.acq
    v = dev(wl.v0)
    a.rec_fz = np.zeros(a.rec_z.shape[0], np.float32)
    a.rec_fx = np.zeros(a.rec_z.shape[0], np.float32)
    a.rec_fx[0] = 1.0
    with pytest.raises(_abi.FwiError):
        ctx.fwi_forward(g, a, v)
    a.rec_fx[0] = 0.0
    a.rec_fz[0] = 0.5
    a.rec_z[0] = g.nz - 1                    # no row below the last one
    with pytest.raises(_abi.FwiError):
        ctx.fwi_forward(g, a, v)
