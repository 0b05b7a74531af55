"""RTM images of the observed data in an inverted model (the paper's imaging
check of its final velocity models, section 3.3, Volve field data: images
from the initial model and from the models of each method are compared).

The image is the migration J^T of the observed data (``born_mig``: the
adjoint wavefield cross-correlated with the background's second time
derivative, section 2.3 eq. 13) after muting the direct arrival, followed
by a 5-point Laplacian that suppresses the low-wavenumber backscatter of
that imaging condition. On the synthetic workloads an image is scored by
its normalised cross-correlation with the image the same data give in the
true model: 1 means reflectors placed and focused as the true velocities
place them.
"""
from __future__ import annotations

import numpy as np
import torch


def direct_mute(grid, acq, v_surface: float, t_pad: float, taper: float) -> np.ndarray:
    """Packed-data mask (shot, receiver, time) that removes the direct
    arrival: 0 before t = |x_r - x_s| h / v_surface + t_pad, a half-cosine
    ramp over `taper` seconds, then 1."""
    nts = [acq.nt_of(s, grid) for s in range(acq.nshots)]
    out = np.empty(sum(acq.nrec(s) * nts[s] for s in range(acq.nshots)), np.float32)
    pos = 0
    for s in range(acq.nshots):
        nt = nts[s]
        t = np.arange(nt) * grid.dt
        r0, r1 = int(acq.rec_ptr[s]), int(acq.rec_ptr[s + 1])
        dist = np.hypot((acq.rec_x[r0:r1] - acq.src_x[s]) * grid.h, (acq.rec_z[r0:r1] - acq.src_z[s]) * grid.h)
        t0 = dist / v_surface + t_pad                          # [nrec]
        u = np.clip((t[None, :] - t0[:, None]) / max(taper, 1e-12), 0.0, 1.0)
        m = 0.5 - 0.5 * np.cos(np.pi * u)
        out[pos:pos + m.size] = m.ravel()
        pos += m.size
    return out


def laplacian(img: torch.Tensor) -> torch.Tensor:
    """-(d2/dz2 + d2/dx2) in grid units, 5-point, zero outside the image."""
    p = torch.nn.functional.pad(img[None, None], (1, 1, 1, 1))[0, 0]
    return 4.0 * img - p[:-2, 1:-1] - p[2:, 1:-1] - p[1:-1, :-2] - p[1:-1, 2:]


def rtm_image(fctx, grid, acq, v: torch.Tensor, d_obs: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """Laplacian-filtered migration of the muted observed data in model v."""
    return laplacian(fctx.born_mig(grid, acq, v, d_obs * mask))


def image_score(img, ref, top: int = 0) -> float:
    """Normalised cross-correlation of two images below row `top`."""
    a = np.asarray(img.detach().cpu() if isinstance(img, torch.Tensor) else img, np.float64)[top:].ravel()
    b = np.asarray(ref.detach().cpu() if isinstance(ref, torch.Tensor) else ref, np.float64)[top:].ravel()
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    if na == 0.0 or nb == 0.0:
        return 0.0
    return float(a @ b / (na * nb))
