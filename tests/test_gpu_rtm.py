"""RTM image product on the GPU (`fwi_rtm`): the muted, Laplacian-filtered
migration matches the FP64 oracle with and without the mute and with
off-grid receivers; bad mute arguments are rejected; on the two-layer model
the image from the true velocities scores above the one from the initial
model."""
import numpy as np
import pytest

import oracle
from oracle import rtm_ref
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops, _abi  # noqa: E402
from paper_2403_17518_amd.rtm import image_score, rtm_image  # noqa: E402

TOL_IMAGE = 1e-4


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_rtm_two_layer():
    wl = configs.two_layer(nt=600)
    g, a = wl.grid, wl.acq
    a.wavelet = np.asarray(a.wavelet, np.float32)
    c = ops.FwiContext(0)
    vt = torch.from_numpy(wl.v_true.astype(np.float32)).cuda()
    v0 = torch.from_numpy(wl.v0.astype(np.float32)).cuda()
    print("[rtm] two_layer nt=600", flush=True)
    d = c.fwi_forward(g, a, vt)
    mute = (1500.0, 0.12, 0.05)
    img_t = rtm_image(c, g, a, vt, d, *mute)
    img_0 = rtm_image(c, g, a, v0, d, *mute)
    dh = d.double().cpu().numpy()
    v0h = wl.v0.astype(np.float32).astype(np.float64)
    e = rel(img_0.cpu(), rtm_ref.rtm(g, a, v0h, dh, *mute))
    e_nm = rel(c.rtm(g, a, v0, d).cpu(), rtm_ref.rtm(g, a, v0h, dh))
    print(f"rtm vs oracle: muted {e:.2e}, unmuted {e_nm:.2e}", flush=True)
    assert e < TOL_IMAGE and e_nm < TOL_IMAGE
    s_true, s_init = image_score(img_t, img_t, top=10), image_score(img_0, img_t, top=10)
    print("scores true / initial", s_true, s_init)
    assert s_true == pytest.approx(1.0)
    assert s_init < 0.999
    for bad in [(-1.0, 0.0, 0.05), (1500.0, 0.0, -0.1), (float("nan"), 0.0, 0.0)]:
        with pytest.raises(_abi.FwiError):
            c.rtm(g, a, v0, d, *bad)
    c.close()


def test_rtm_ragged_off_grid():
    wl = configs.ragged_small()
    g, a = wl.grid, wl.acq
    a.wavelet = np.asarray(a.wavelet, np.float32)
    rng = np.random.default_rng(11)
    n = int(a.rec_ptr[-1])
    a.rec_fz = (0.9 * rng.random(n)).astype(np.float32)
    a.rec_fx = (0.9 * rng.random(n)).astype(np.float32)
    a.rec_fz[np.asarray(a.rec_z) >= g.nz - 1] = 0.0
    for s in range(a.nshots):            # the next cell must lie inside the shot's window
        x0, wn = a.window(s, g)
        r0, r1 = int(a.rec_ptr[s]), int(a.rec_ptr[s + 1])
        a.rec_fx[r0:r1][np.asarray(a.rec_x[r0:r1]) >= x0 + wn - 1] = 0.0
    a.src_fz = np.zeros(a.nshots, np.float32)
    a.src_fx = np.zeros(a.nshots, np.float32)
    c = ops.FwiContext(0)
    print("[rtm] ragged off-grid", flush=True)
    y = rng.standard_normal(a.data_size(g)).astype(np.float32)
    v0 = wl.v0.astype(np.float32)
    img = c.rtm(g, a, torch.from_numpy(v0).cuda(), torch.from_numpy(y).cuda(), 2000.0, 0.01, 0.02)
    e = rel(img.cpu(), rtm_ref.rtm(g, a, v0.astype(np.float64), y.astype(np.float64), 2000.0, 0.01, 0.02))
    print(f"rtm ragged off-grid vs oracle {e:.2e}", flush=True)
    assert e < TOL_IMAGE
    c.close()
