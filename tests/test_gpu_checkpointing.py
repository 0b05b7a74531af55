"""Checkpointed adjoint sweeps on the GPU. Uniform and binomial snapshot
schedules (Griewank's revolve) give the bits of the full-history sweep for
the gradient, the migration, the pair and the fused gradient + pair, with
one- and two-level tilings and odd segment lengths and record lengths (a
two-level tiling ends a range of odd length with a one-level step, which
runs on the tiling's own one-level wave table); a memory budget too small
for uniform checkpoints falls back to fewer snapshots and more
recomputation with the same bits; the full-history results match the
oracle."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops, _abi  # noqa: E402

TILINGS = [(1, 24, 1, 2), (1, 24, 2, 1), (2, 16, 2, 1)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def rel(a, b):
    a = np.ravel(a.detach().cpu().numpy().astype(np.float64) if isinstance(a, torch.Tensor) else a)
    b = np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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


def _all(ctx, grid, acq, v0, d_obs, dv, y):
    g, phi, _ = ctx.fwi_gradient(grid, acq, v0, d_obs)
    st = ctx.stats()
    im = ctx.born_mig(grid, acq, v0, y)
    pair = ctx.born_pair(grid, acq, v0, dv)
    gp, phi2, img = ctx.gradient_pair(grid, acq, v0, d_obs, scale=-1.0)
    assert torch.equal(gp, g) and phi2 == phi
    return {"g": g, "phi": phi, "im": im, "pair": pair, "gp_img": img}, st


@pytest.mark.parametrize("tiling", TILINGS)
def test_schedules_give_the_full_history_bits(ctx, wl, tiling):
    g0, acq = wl.grid, wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    d_obs = ctx.fwi_forward(g0, acq, vt)
    dv = vt - v0
    y = dev(np.random.default_rng(9).standard_normal(acq.data_size(g0)))
    ctx.set_tiling(-1, *tiling)
    try:
        ctx.set_ckpt_slots(-1)
        ref, st = _all(ctx, g0, acq, v0, d_obs, dv, y)
        assert st["n_segments"] == 1
        for k in (29, 37, 8):
            for slots in (-1, 3, 1, 0):
                print(f"[ckpt] tiling {tiling} k={k} slots={slots}", flush=True)
                ctx.set_ckpt_slots(slots)
                g = replace(g0, ckpt_every=k)
                out, st = _all(ctx, g, acq, v0, d_obs, dv, y)
                nseg = (g0.nt_max + k - 1) // k
                assert st["n_segments"] == nseg
                want = nseg - 2 if slots < 0 else min(slots, nseg - 2)
                assert st["ckpt_slots"] == want
                # recomputed steps: every segment the schedule recomputes, k
                # steps each (the last, shorter one is never recomputed)
                assert st["recomputed_steps"] == k * ops.checkpoint_schedule(nseg, want)
                for name in ("g", "im", "pair"):
                    assert torch.equal(out[name], ref[name]), (name, k, slots)
                assert out["phi"] == ref["phi"]
                # with checkpoints the fused call runs the pair's own joint sweep
                assert torch.equal(out["gp_img"], ctx.born_pair(g, acq, v0, -out["g"]))
    finally:
        ctx.set_ckpt_slots(-1)
        ctx.set_tiling(-1, 0, 0, 0)


def test_tilings_agree_with_an_odd_record(ctx, wl):
    """nt_max odd: every sweep of a two-level tiling ends with a single step."""
    acq = wl.acq
    g = replace(wl.grid, nt_max=wl.grid.nt_max - 1)
    acq = type(acq)(src_z=acq.src_z, src_x=acq.src_x, rec_ptr=acq.rec_ptr, rec_z=acq.rec_z, rec_x=acq.rec_x,
                    wavelet=np.asarray(acq.wavelet)[..., :g.nt_max], win_x0=acq.win_x0, win_nx=acq.win_nx,
                    nt=np.minimum(np.asarray(acq.nt), g.nt_max).astype(np.int32))
    assert g.nt_max % 2 == 1
    v0, vt = dev(wl.v0), dev(wl.v_true)
    outs = []
    for t in TILINGS:
        ctx.set_tiling(-1, *t)
        d = ctx.fwi_forward(g, acq, vt)
        gr, phi, _ = ctx.fwi_gradient(g, acq, v0, d * 0.5)
        outs.append((d, gr, phi))
    ctx.set_tiling(-1, 0, 0, 0)
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1]) and o[2] == outs[0][2]
    g_ref, _, _ = oracle.gradient(g, acq, np.asarray(wl.v0, np.float32).astype(np.float64),
                                  0.5 * outs[0][0].cpu().numpy().astype(np.float64))
    e = rel(outs[0][1], g_ref)
    print("odd record gradient rel err", e)
    assert e < 1e-3


def test_small_budget_falls_back_to_binomial(ctx, wl):
    g0, acq = wl.grid, wl.acq
    v0, vt = dev(wl.v0), dev(wl.v_true)
    d_obs = ctx.fwi_forward(g0, acq, vt)
    g_ref, phi_ref, _ = ctx.fwi_gradient(g0, acq, v0, d_obs)
    budget = ctx.stats()["scratch_bytes"]
    found = None
    try:
        for _ in range(40):
            budget //= 2
            ctx.set_mem_budget(budget)
            try:
                g, phi, _ = ctx.fwi_gradient(g0, acq, v0, d_obs)
            except _abi.FwiError:
                break
            st = ctx.stats()
            assert torch.equal(g, g_ref) and phi == phi_ref
            if st["n_segments"] > 2 and st["ckpt_slots"] < st["n_segments"] - 2:
                found = (budget, st)
                break
    finally:
        ctx.set_mem_budget(0)
    print("binomial at budget", found and found[0], found and {k: found[1][k] for k in
                                                              ("n_segments", "ckpt_slots", "recomputed_steps")})
    assert found is not None


def test_bad_slot_count_rejected(ctx):
    with pytest.raises(_abi.FwiError):
        ctx.set_ckpt_slots(-2)
