"""Captured time loops: every operator run from replayed HIP graphs gives
bitwise the results of direct launches, on the first (capturing) call and on
every replay, with other GPU work and synchronizations between the replays,
and with a new model tensor (the loops read the context's copy of the model,
so the graphs are reused)."""
from dataclasses import replace

import numpy as np
import pytest

from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def run_all(ctx, grid, acq, v, d_obs, dv, y):
    g, phi, d_syn = ctx.fwi_gradient(grid, acq, v, d_obs, want_dsyn=True)
    return [ctx.fwi_forward(grid, acq, v), g, d_syn, torch.tensor([phi]),
            ctx.born_demig(grid, acq, v, dv), ctx.born_mig(grid, acq, v, y)]


@pytest.mark.parametrize("case", ["ragged", "two_layer_ckpt"])
def test_replays_match_direct_launches(case):
    if case == "ragged":
        wl = configs.ragged_small()
        grid = wl.grid
    else:
        wl = configs.two_layer(nt=400)
        grid = replace(wl.grid, ckpt_every=37)
    acq = wl.acq
    acq.wavelet = np.asarray(acq.wavelet, np.float32)
    print(f"[graphs] {case} shots={acq.nshots}", flush=True)
    rng = np.random.default_rng(4)
    v0 = dev(wl.v0)
    d_obs = dev(rng.standard_normal(acq.data_size(grid)) * 1e-3)
    dv = dev(wl.v_true - wl.v0)
    y = dev(rng.standard_normal(acq.data_size(grid)))

    direct = ops.FwiContext(0)
    direct.set_graphs(False)
    ref = [t.cpu() for t in run_all(direct, grid, acq, v0, d_obs, dv, y)]
    assert direct.stats()["graph_launches"] == 0

    cap = ops.FwiContext(0)
    for rep in range(3):
        out = run_all(cap, grid, acq, v0, d_obs, dv, y)
        st = cap.stats()    # statistics of the last call (born_mig)
        assert st["graph_launches"] > 0
        if rep > 0:
            assert st["graph_captures"] == 0
        for a, b in zip(out, ref):
            assert torch.equal(a.cpu(), b), (case, rep)
        # unrelated eager work and a synchronization between replays
        z = torch.randn(1 << 20, device="cuda")
        (z * 2).sum().item()
        direct.fwi_forward(grid, acq, v0)
        torch.cuda.synchronize()

    # a new model tensor (other values, other address): the graphs are
    # replayed and read the new values
    v1 = v0 * 1.01
    ref1 = [t.cpu() for t in run_all(direct, grid, acq, v1, d_obs, dv, y)]
    out1 = run_all(cap, grid, acq, v1, d_obs, dv, y)
    assert cap.stats()["graph_captures"] == 0
    for a, b in zip(out1, ref1):
        assert torch.equal(a.cpu(), b)
    direct.close()
    cap.close()
