"""The allocation-free forward model, fwi_forward_noalloc, through the C ABI.

It runs the forward kernels of fwi_forward with every scratch buffer carved
from a static 64 MiB device array, so its data must be fwi_forward's bit for
bit (every tiling computes each cell with the same arithmetic). Checked on
two calls in a row, the second on a smaller problem (the array keeps the
first call's contents), with the device's free memory unchanged across the
calls; a problem that needs more scratch is refused before any propagation
and leaves the context as it was (its captured loops still replay).
"""
import numpy as np
import pytest

from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import _abi, ops  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _case(wl):
    wl.acq.wavelet = wl.acq.wavelet.astype(np.float32)
    return wl.grid, wl.acq, dev(wl.v_true)


def test_noalloc_forward_equals_fwi_forward_on_two_calls():
    ctx = ops.FwiContext(0)
    try:
        g1, a1, v1 = _case(configs.two_layer(nt=1000))
        g2, a2, v2 = _case(configs.ragged_small(nshots=3, nt_lo=120, nt_hi=160))
        assert a2.data_size(g2) < a1.data_size(g1) and g2.nz * g2.nx < g1.nz * g1.nx
        print("[no_alloc] references from fwi_forward", flush=True)
        ref1 = ctx.fwi_forward(g1, a1, v1)
        ref2 = ctx.fwi_forward(g2, a2, v2)
        out1 = torch.full_like(ref1, float("nan"))
        out2 = torch.full_like(ref2, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        print("[no_alloc] fwi_forward_noalloc, two_layer (4 shots, 1000 steps)", flush=True)
        ctx.fwi_forward_noalloc(g1, a1, v1, out1)
        print("[no_alloc] fwi_forward_noalloc, ragged_small (3 shots, 120-160 steps)", flush=True)
        ctx.fwi_forward_noalloc(g2, a2, v2, out2)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert torch.equal(out1, ref1)
        assert torch.equal(out2, ref2)
        print(f"[no_alloc] free device memory {free0} -> {free1}", flush=True)
        assert free1 == free0
        # and once more on the first problem after the second one
        out1b = torch.full_like(ref1, float("nan"))
        ctx.fwi_forward_noalloc(g1, a1, v1, out1b)
        assert torch.equal(out1b, ref1)
    finally:
        ctx.close()


def test_noalloc_forward_refuses_a_problem_beyond_its_scratch():
    ctx = ops.FwiContext(0)
    try:
        g, a, v = _case(configs.two_layer(nt=1000))
        ref = ctx.fwi_forward(g, a, v)          # captures the context's loops
        big = configs.layered_600x200(nshots=64, nt=1000)
        gb, ab, vb = _case(big)
        out = torch.empty(ab.data_size(gb), device="cuda")
        print("[no_alloc] 600x200, 64 shots, 1000 steps: must be refused", flush=True)
        with pytest.raises(_abi.FwiError) as ei:
            ctx.fwi_forward_noalloc(gb, ab, vb, out)
        assert ei.value.code == _abi.FWI_ENOMEM
        assert "scratch" in str(ei.value)
        # the context is as it was: the same bits, its captured loop replayed
        again = ctx.fwi_forward(g, a, v)
        st = ctx.stats()
        assert torch.equal(again, ref)
        assert st["graph_captures"] == 0 and st["graph_launches"] > 0
    finally:
        ctx.close()
