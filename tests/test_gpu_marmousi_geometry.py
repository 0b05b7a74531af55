"""Parity on the acquisition of the paper's Marmousi example (601 x 221
points at 15 m, 30 sources and 300 receivers on the top row, 5 Hz Ricker;
a seeded layered model stands in for Marmousi), with all 30 shots in one
launch per step and the autotuned tilings. Records are cut to 700 steps
(0.98 s) to keep the oracle within seconds; the oracle runs the sampled
shots only. As in the other full-geometry tests, the gradient is formed
with every other shot's observed data set to the GPU's own synthetic data
(zero residual there) and the sampled shots' to half of it, and the
migration is fed data that is zero outside the sampled shots."""
import numpy as np
import pytest

import oracle
from synth import configs
from synth.problem import Acquisition

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops  # noqa: E402

TOL_DATA = 1e-4
TOL_IMAGE = 1e-4
TOL_GRAD = 1e-3
SAMPLED = [0, 17]
NT = 700


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(a):
    return np.asarray(a, dtype=np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(f32(a))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def marm():
    wl = configs.marmousi_601x221(nt=NT)
    acq = wl.acq
    acq.wavelet = f32(acq.wavelet)
    sub = acq.subset(SAMPLED)
    oracle.set_threads(len(SAMPLED))
    c = ops.FwiContext(0)
    vt, v0 = f32(wl.v_true).astype(np.float64), f32(wl.v0).astype(np.float64)
    print(f"[marmousi] oracle forward of shots {SAMPLED}", flush=True)
    d_ref = oracle.forward(wl.grid, sub, vt)
    yield wl.grid, acq, sub, vt, v0, d_ref, c
    c.close()


def test_forward_sampled_shots(marm):
    grid, acq, sub, vt, v0, d_ref, c = marm
    d = host(c.fwi_forward(grid, acq, dev(vt)))
    e = max(rel(acq.shot_data(d, s, grid), sub.shot_data(d_ref, i, grid)) for i, s in enumerate(SAMPLED))
    print("marmousi-geometry forward worst sampled rel err", e)
    assert e < TOL_DATA


def test_gradient_sampled_shots(marm):
    grid, acq, sub, vt, v0, d_ref, c = marm
    print("[marmousi] gradient", flush=True)
    d_obs = host(c.fwi_forward(grid, acq, dev(v0)))
    off = acq.trace_offsets(grid)
    for s in SAMPLED:
        d_obs[off[s]:off[s + 1]] *= 0.5
    g, phi, _ = c.fwi_gradient(grid, acq, dev(v0), dev(d_obs))
    sub_obs = np.concatenate([f32(d_obs[off[s]:off[s + 1]]) for s in SAMPLED]).astype(np.float64)
    g_ref, phi_ref, _ = oracle.gradient(grid, sub, v0, sub_obs)
    e = rel(host(g), g_ref)
    print("marmousi-geometry gradient rel err", e, "misfit", phi, phi_ref)
    assert e < TOL_GRAD
    assert abs(phi - phi_ref) <= 1e-4 * abs(phi_ref)


def test_migration_and_born_data_of_sampled_shots(marm):
    grid, acq, sub, vt, v0, d_ref, c = marm
    print("[marmousi] migration", flush=True)
    rng = np.random.default_rng(8)
    y = np.zeros(acq.data_size(grid), np.float32)
    parts = []
    off = acq.trace_offsets(grid)
    for s in SAMPLED:
        lo, hi = int(off[s]), int(off[s + 1])
        y[lo:hi] = rng.standard_normal(hi - lo).astype(np.float32)
        parts.append(y[lo:hi])
    im = host(c.born_mig(grid, acq, dev(v0), dev(y)))
    e = rel(im, oracle.born_mig(grid, sub, v0, np.concatenate(parts).astype(np.float64)))
    print("marmousi-geometry migration rel err", e)
    assert e < TOL_IMAGE
    # Born data of the sampled shots
    dv = f32(vt - v0).astype(np.float64)
    dd = host(c.born_demig(grid, acq, dev(v0), dev(dv)))
    dd_ref = oracle.born_demig(grid, sub, v0, dv)
    e = max(rel(acq.shot_data(dd, s, grid), sub.shot_data(dd_ref, i, grid)) for i, s in enumerate(SAMPLED))
    print("marmousi-geometry Born data worst sampled rel err", e)
    assert e < TOL_DATA
