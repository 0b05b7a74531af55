"""RTM images of the observed data in an inverted model (the paper's imaging
check of its final velocity models, section 3.3, Volve field data: images
from the initial model and from the models of each method are compared).

The image is computed by the library (`fwi_rtm`): the migration J^T of the
observed data (the adjoint wavefield cross-correlated with the background's
second time derivative, section 2.3 eq. 13) after muting the direct arrival,
followed by a 5-point Laplacian that suppresses the low-wavenumber
backscatter of that imaging condition. On the synthetic workloads an image
is scored by its normalised cross-correlation with the image the same data
give in the true model: 1 means reflectors placed and focused as the true
velocities place them.
"""
from __future__ import annotations

import numpy as np
import torch


def rtm_image(fctx, grid, acq, v: torch.Tensor, d_obs: torch.Tensor, mute_v: float = 0.0,
              mute_pad: float = 0.0, mute_taper: float = 0.0) -> torch.Tensor:
    """Laplacian-filtered migration of the observed data in model v, the
    direct arrival muted when mute_v > 0 (see FwiContext.rtm)."""
    return fctx.rtm(grid, acq, v, d_obs, mute_v, mute_pad, mute_taper)


def image_score(img, ref, top: int = 0) -> float:
    """Normalised cross-correlation of two images below row `top`."""
    a = np.asarray(img.detach().cpu() if isinstance(img, torch.Tensor) else img, np.float64)[top:].ravel()
    b = np.asarray(ref.detach().cpu() if isinstance(ref, torch.Tensor) else ref, np.float64)[top:].ravel()
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    if na == 0.0 or nb == 0.0:
        return 0.0
    return float(a @ b / (na * nb))
