"""RTM image product on the GPU: the image is the Laplacian of the
migration of the muted data (composition checked bitwise), the migration
matches the FP64 oracle, and on the two-layer model the image from the true
velocities scores above the one from the initial model."""
import numpy as np
import pytest

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2403_17518_amd import ops  # noqa: E402
from paper_2403_17518_amd.rtm import direct_mute, image_score, laplacian, rtm_image  # noqa: E402

TOL_IMAGE = 1e-4


def test_rtm_two_layer():
    wl = configs.two_layer(nt=600)
    g, a = wl.grid, wl.acq
    a.wavelet = np.asarray(a.wavelet, np.float32)
    c = ops.FwiContext(0)
    vt = torch.from_numpy(wl.v_true.astype(np.float32)).cuda()
    v0 = torch.from_numpy(wl.v0.astype(np.float32)).cuda()
    print("[rtm] two_layer nt=600", flush=True)
    d = c.fwi_forward(g, a, vt)
    mask_np = direct_mute(g, a, 1500.0, 0.12, 0.05)
    mask = torch.from_numpy(mask_np).cuda()
    img_t = rtm_image(c, g, a, vt, d, mask)
    img_0 = rtm_image(c, g, a, v0, d, mask)
    assert torch.equal(img_0, laplacian(c.born_mig(g, a, v0, d * mask)))
    # the migration inside against the oracle (same FP32 data on both sides)
    dm = (d * mask).double().cpu().numpy()
    ref = oracle.born_mig(g, a, wl.v0.astype(np.float32).astype(np.float64), dm)
    mig = c.born_mig(g, a, v0, d * mask).double().cpu().numpy()
    e = float(np.linalg.norm(mig - ref) / np.linalg.norm(ref))
    print("rtm migration rel err vs oracle", e)
    assert e < TOL_IMAGE
    s_true, s_init = image_score(img_t, img_t, top=10), image_score(img_0, img_t, top=10)
    print("scores true / initial", s_true, s_init)
    assert s_true == pytest.approx(1.0)
    assert s_init < 0.999
    c.close()
