"""GPU parity: every C-ABI operator against the FP64 oracle.

Tolerances (relative L2): 1e-4 on seismograms and migrated images, 1e-3 on
FWI gradients, 1e-4 on the FP32 dot-product test. The oracle is fed the
FP32-rounded inputs the GPU sees, so input rounding does not count.
"""
import numpy as np
import pytest

import oracle
from synth import Acquisition, Grid, configs, ricker

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops, _abi  # noqa: E402

TOL_DATA = 1e-4
TOL_IMAGE = 1e-4
TOL_GRAD = 1e-3


def rel(a, b):
    a, b = np.ravel(np.asarray(a, dtype=np.float64)), np.ravel(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(a):
    return np.asarray(a, dtype=np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(f32(a))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def wl32(wl):
    """Round the workload's wavelet to FP32 for both sides."""
    acq = wl.acq
    acq.wavelet = f32(acq.wavelet)
    return wl


@pytest.fixture(scope="module")
def ctx():
    c = ops.FwiContext(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def two_layer():
    wl = wl32(configs.two_layer())
    v_true = f32(wl.v_true).astype(np.float64)
    v0 = f32(wl.v0).astype(np.float64)
    d_obs = f32(oracle.forward(wl.grid, wl.acq, v_true))
    return wl, v_true, v0, d_obs


@pytest.fixture(scope="module")
def ragged():
    return wl32(configs.ragged_small())


# ---------------------------------------------------------------------------

def test_forward_two_layer(ctx, two_layer):
    wl, v_true, v0, d_obs = two_layer
    print(f"[parity] forward two_layer shots={wl.acq.nshots} nt={wl.grid.nt_max}", flush=True)
    d = host(ctx.fwi_forward(wl.grid, wl.acq, dev(v_true)))
    e = rel(d, d_obs)
    print("forward rel err", e)
    assert e < TOL_DATA


def test_gradient_two_layer(ctx, two_layer):
    wl, v_true, v0, d_obs = two_layer
    print("[parity] gradient two_layer", flush=True)
    g, phi, d_syn = ctx.fwi_gradient(wl.grid, wl.acq, dev(v0), dev(d_obs), want_dsyn=True)
    g_ref, phi_ref, dsyn_ref = oracle.gradient(wl.grid, wl.acq, v0, d_obs.astype(np.float64))
    e_g, e_d = rel(host(g), g_ref), rel(host(d_syn), dsyn_ref)
    print("gradient rel err", e_g, "d_syn", e_d, "misfit", phi, phi_ref)
    assert e_g < TOL_GRAD
    assert e_d < TOL_DATA
    assert abs(phi - phi_ref) < 1e-4 * phi_ref


def test_born_two_layer(ctx, two_layer):
    wl, v_true, v0, _ = two_layer
    print("[parity] born two_layer", flush=True)
    dv = f32(v_true - v0).astype(np.float64)
    dd = ctx.born_demig(wl.grid, wl.acq, dev(v0), dev(dv))
    dd_ref = oracle.born_demig(wl.grid, wl.acq, v0, dv)
    assert rel(host(dd), dd_ref) < TOL_DATA
    dd32 = f32(dd_ref).astype(np.float64)
    img = ctx.born_mig(wl.grid, wl.acq, dev(v0), dev(dd32))
    img_ref = oracle.born_mig(wl.grid, wl.acq, v0, dd32)
    e = rel(host(img), img_ref)
    print("born_mig rel err", e)
    assert e < TOL_IMAGE


def test_ragged_all_operators(ctx, ragged):
    wl = ragged
    g, acq = wl.grid, wl.acq
    print(f"[parity] ragged shots={acq.nshots} nt={list(acq.nt)} win={list(acq.win_nx)}", flush=True)
    v = f32(wl.v_true).astype(np.float64)
    v0 = f32(wl.v0).astype(np.float64)
    d_ref = oracle.forward(g, acq, v)
    assert rel(host(ctx.fwi_forward(g, acq, dev(v))), d_ref) < TOL_DATA
    d_obs = f32(d_ref).astype(np.float64)
    gg, phi, _ = ctx.fwi_gradient(g, acq, dev(v0), dev(d_obs))
    gg_ref, phi_ref, _ = oracle.gradient(g, acq, v0, d_obs)
    assert rel(host(gg), gg_ref) < TOL_GRAD
    assert abs(phi - phi_ref) < 1e-4 * phi_ref
    dv = f32(v - v0).astype(np.float64)
    assert rel(host(ctx.born_demig(g, acq, dev(v0), dev(dv))), oracle.born_demig(g, acq, v0, dv)) < TOL_DATA
    rng = np.random.default_rng(3)
    y = f32(rng.standard_normal(acq.data_size(g))).astype(np.float64)
    assert rel(host(ctx.born_mig(g, acq, dev(v0), dev(y))), oracle.born_mig(g, acq, v0, y)) < TOL_IMAGE


@pytest.mark.parametrize("shared", [True, False])
def test_dot_product_fp32(ctx, shared):
    wl = wl32(configs.ragged_small(per_shot_wavelet=not shared, seed=7))
    g, acq = wl.grid, wl.acq
    rng = np.random.default_rng(11)
    v0 = dev(wl.v0)
    x = rng.standard_normal((g.nz, g.nx))
    y = rng.standard_normal(acq.data_size(g))
    Jx = host(ctx.born_demig(g, acq, v0, dev(x)))
    JTy = host(ctx.born_mig(g, acq, v0, dev(y)))
    lhs, rhs = float(np.dot(Jx, f32(y))), float(np.sum(f32(x) * JTy))
    print("dot", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), abs(rhs))


def test_checkpoint_interval_does_not_change_the_gradient(ctx, two_layer):
    wl, v_true, v0, d_obs = two_layer
    from dataclasses import replace
    g_full = host(ctx.fwi_gradient(wl.grid, wl.acq, dev(v0), dev(d_obs))[0])
    st_full = ctx.stats()
    g37 = replace(wl.grid, ckpt_every=37)
    g_ck = host(ctx.fwi_gradient(g37, wl.acq, dev(v0), dev(d_obs))[0])
    st_ck = ctx.stats()
    assert st_full["n_segments"] == 1
    assert st_ck["n_segments"] == (wl.grid.nt_max + 36) // 37
    assert rel(g_ck, g_full) < 1e-6


def test_repeatable_bitwise(ctx, ragged):
    wl = ragged
    v0 = dev(wl.v0)
    rng = np.random.default_rng(2)
    y = dev(rng.standard_normal(wl.acq.data_size(wl.grid)))
    a = host(ctx.born_mig(wl.grid, wl.acq, v0, y))
    b = host(ctx.born_mig(wl.grid, wl.acq, v0, y))
    assert np.array_equal(a, b)


def test_gradient_equals_migration_of_residual(ctx, two_layer):
    wl, v_true, v0, d_obs = two_layer
    g, _, d_syn = ctx.fwi_gradient(wl.grid, wl.acq, dev(v0), dev(d_obs), want_dsyn=True)
    img = ctx.born_mig(wl.grid, wl.acq, dev(v0), d_syn - dev(d_obs))
    assert rel(host(g), host(img)) < 1e-6


# ---------------------------------------------------------------------------
# error handling and degenerate cases

def _small():
    grid = Grid(nz=20, nx=30, nb=5, h=10.0, dt=1e-3, nt_max=50, v_ref=2500.0)
    acq = Acquisition(src_z=[2], src_x=[5], rec_ptr=[0, 3], rec_z=[2, 2, 10], rec_x=[0, 29, 15],
                      wavelet=f32(ricker(20.0, 1e-3, 50)))
    return grid, acq, np.full((20, 30), 2000.0)


def test_cfl_and_model_errors(ctx):
    from dataclasses import replace
    grid, acq, v = _small()
    with pytest.raises(_abi.FwiError) as e:
        ctx.fwi_forward(replace(grid, v_ref=6000.0), acq, dev(v))
    assert e.value.code == _abi.FWI_ECFL
    vbad = v.copy()
    vbad[3, 4] = 6000.0
    with pytest.raises(_abi.FwiError) as e:
        ctx.fwi_forward(grid, acq, dev(vbad))
    assert e.value.code == _abi.FWI_ECFL
    vbad[3, 4] = np.nan
    with pytest.raises(_abi.FwiError) as e:
        ctx.fwi_forward(grid, acq, dev(vbad))
    assert e.value.code == _abi.FWI_EINVAL
    # the context stays usable after errors
    d = host(ctx.fwi_forward(grid, acq, dev(v)))
    assert rel(d, oracle.forward(grid, acq, v)) < TOL_DATA


def test_geometry_errors(ctx):
    grid, acq, v = _small()
    bad = Acquisition(**{**acq.__dict__, "rec_x": np.array([0, 30, 15])})
    with pytest.raises(_abi.FwiError) as e:
        ctx.fwi_forward(grid, bad, dev(v))
    assert e.value.code == _abi.FWI_EINVAL
    bad = Acquisition(**{**acq.__dict__, "win_x0": np.array([6]), "win_nx": np.array([20])})
    with pytest.raises(_abi.FwiError):    # source at x=5 outside window
        ctx.fwi_forward(grid, bad, dev(v))


def test_empty_and_degenerate(ctx):
    grid, acq, v = _small()
    # a shot without receivers and a shot with zero samples
    acq2 = Acquisition(src_z=[2, 3, 4], src_x=[5, 6, 7], rec_ptr=[0, 0, 3, 5],
                       rec_z=[2, 2, 10, 1, 1], rec_x=[0, 29, 15, 3, 3],
                       wavelet=acq.wavelet, nt=np.array([50, 40, 0]))
    d = host(ctx.fwi_forward(grid, acq2, dev(v)))
    d_ref = oracle.forward(grid, acq2, v)
    assert d.shape == d_ref.shape and rel(d, d_ref) < TOL_DATA
    img = host(ctx.born_mig(grid, acq2, dev(v), dev(d_ref)))
    assert rel(img, oracle.born_mig(grid, acq2, v, f32(d_ref))) < TOL_IMAGE
    # no shots at all: data are empty, images are zero
    none = Acquisition(src_z=[], src_x=[], rec_ptr=[0], rec_z=[], rec_x=[], wavelet=acq.wavelet)
    assert ctx.fwi_forward(grid, none, dev(v)).numel() == 0
    g, phi, _ = ctx.fwi_gradient(grid, none, dev(v), torch.zeros(0, device="cuda"))
    assert phi == 0.0 and float(g.abs().max()) == 0.0
    # no sponge, a one-column window
    from dataclasses import replace
    g0 = replace(grid, nb=0)
    acq3 = Acquisition(src_z=[5], src_x=[12], rec_ptr=[0, 2], rec_z=[0, 19], rec_x=[12, 12],
                       wavelet=acq.wavelet, win_x0=[12], win_nx=[1])
    for gg in (g0, grid):
        d = host(ctx.fwi_forward(gg, acq3, dev(v)))
        assert rel(d, oracle.forward(gg, acq3, v)) < TOL_DATA


@pytest.mark.parametrize("cw,rows,levels,pd", [(1, 7, 1, 1), (2, 13, 1, 1), (1, 300, 1, 1), (2, 5, 1, 1),
                                                (1, 7, 1, 2), (2, 13, 1, 2), (1, 300, 1, 2), (2, 6, 1, 2),
                                                (1, 7, 2, 1), (2, 13, 2, 1), (1, 300, 2, 1), (2, 5, 2, 1),
                                                (2, 33, 2, 1)])
def test_forced_tilings_match_oracle_and_each_other(ctx, ragged, cw, rows, levels, pd):
    """Every tiling computes each cell with the same arithmetic, so results
    are bitwise equal across tilings and match the oracle."""
    wl = ragged
    g, acq = wl.grid, wl.acq
    print(f"[parity] tiling cw={cw} rows={rows} levels={levels} prefetch={pd}", flush=True)
    v = dev(wl.v_true)
    v0 = dev(wl.v0)
    rng = np.random.default_rng(5)
    y = dev(rng.standard_normal(acq.data_size(g)))
    dv = dev(wl.v_true - wl.v0)

    def run():
        d = host(ctx.fwi_forward(g, acq, v))
        gg = host(ctx.fwi_gradient(g, acq, v0, dev(d * 0.5))[0])
        dd = host(ctx.born_demig(g, acq, v0, dv))
        im = host(ctx.born_mig(g, acq, v0, y))
        gp = host(ctx.gradient_pair(g, acq, v0, dev(d * 0.5), scale=-1.0)[2])   # scattered-field kernel
        return d, gg, dd, im, gp

    ctx.set_tiling(-1, 1, 30, 1, 1)
    ref = run()
    ctx.set_tiling(-1, cw, rows, levels, pd)
    got = run()
    st = ctx.stats()
    ctx.set_tiling(-1, 0, 0, 0)
    assert st["tile_cw"] == [cw] * 4 and st["tile_rows"] == [rows] * 4
    assert st["tile_levels"] == [levels, levels, 1, levels]
    assert st["tile_prefetch"][:2] == [pd if levels == 1 else 1] * 2
    assert st["tile_prefetch"][3] == (pd if levels == 1 else 1)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    v64 = f32(wl.v_true).astype(np.float64)
    assert rel(got[0], oracle.forward(g, acq, v64)) < TOL_DATA
    assert rel(got[3], oracle.born_mig(g, acq, f32(wl.v0).astype(np.float64),
                                       host(y))) < TOL_IMAGE


def test_autotuner_picks_a_valid_tiling(ctx, two_layer):
    wl, v_true, v0, d_obs = two_layer
    ctx.set_tiling(-1, 0, 0, 0)
    ctx.set_autotune(True)
    ctx.fwi_forward(wl.grid, wl.acq, dev(v0))
    st = ctx.stats()
    assert all(c in (1, 2) for c in st["tile_cw"])
    assert all(r >= 1 for r in st["tile_rows"])
    assert st["tile_levels"][2] == 1 and all(t in (1, 2) for t in st["tile_levels"])


@pytest.mark.parametrize("case", ["ragged", "two_layer_ckpt"])
def test_born_pair_equals_demig_then_mig(ctx, case):
    """The fused pair (one joint Born sweep feeding the migration) gives
    bitwise the image and data of born_mig(born_demig(.)), with checkpointed
    segments and co-located receivers, and the oracle's J^T J within the
    image tolerance."""
    from dataclasses import replace
    if case == "ragged":
        wl = wl32(configs.ragged_small())
        grid = wl.grid
    else:
        wl = wl32(configs.two_layer(nt=400))
        grid = replace(wl.grid, ckpt_every=37)
    acq = wl.acq
    print(f"[parity] born_pair {case}", flush=True)
    v0 = f32(wl.v0).astype(np.float64)
    dv = f32(wl.v_true - wl.v0).astype(np.float64)
    dd_ref = ctx.born_demig(grid, acq, dev(v0), dev(dv))
    img_ref = ctx.born_mig(grid, acq, dev(v0), dd_ref)
    img, dd = ctx.born_pair(grid, acq, dev(v0), dev(dv), want_dd=True)
    st = ctx.stats()
    assert torch.equal(dd, dd_ref)
    assert torch.equal(img, img_ref)
    if case != "ragged":
        assert st["n_segments"] == (grid.nt_max + 36) // 37
    img2 = ctx.born_pair(grid, acq, dev(v0), dev(dv))
    assert torch.equal(img2, img_ref)
    e = rel(host(img), oracle.born_pair(grid, acq, v0, dv))
    print("born_pair rel err vs oracle", e)
    assert e < TOL_IMAGE


@pytest.mark.parametrize("case", ["ragged", "two_layer", "two_layer_ckpt"])
def test_gradient_pair(ctx, case):
    """Gradient and doubly migrated image in one call: the gradient and
    misfit are those of fwi_gradient bit for bit; the image matches
    born_pair(v, -grad) (bitwise when the history is checkpointed and the
    pair runs its own sweep, to FP32 rounding when the scattered field is
    driven by the stored history) and the oracle's J^T J."""
    from dataclasses import replace
    if case == "ragged":
        wl = wl32(configs.ragged_small())
        grid = wl.grid
    else:
        wl = wl32(configs.two_layer(nt=400))
        grid = replace(wl.grid, ckpt_every=37) if case == "two_layer_ckpt" else wl.grid
    acq = wl.acq
    print(f"[parity] gradient_pair {case}", flush=True)
    v0 = f32(wl.v0).astype(np.float64)
    d_obs = f32(oracle.forward(grid, acq, f32(wl.v_true).astype(np.float64))).astype(np.float64)
    g_ref, phi_ref, _ = ctx.fwi_gradient(grid, acq, dev(v0), dev(d_obs))
    grad, phi, img = ctx.gradient_pair(grid, acq, dev(v0), dev(d_obs), scale=-1.0)
    st = ctx.stats()
    assert torch.equal(grad, g_ref)
    assert phi == phi_ref
    pair = ctx.born_pair(grid, acq, dev(v0), -g_ref)
    if case == "two_layer_ckpt":
        assert st["n_segments"] > 1
        assert torch.equal(img, pair)
    else:
        assert st["n_segments"] == 1
        e = rel(host(img), host(pair))
        print("fused pair vs born_pair", e)
        assert e < 1e-5
    e = rel(host(img), oracle.born_pair(grid, acq, v0, -host(grad)))
    print("gradient_pair image rel err vs oracle", e)
    assert e < TOL_IMAGE
