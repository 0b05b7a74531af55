"""Seeded parameter vectors for the deblurring network (inputs shared by the
network oracle and the HIP path; the draws are made here, not by either
side). Layout and order follow the network's parameter vector: every tensor
in PyTorch layout, input block, down blocks 1..D, up blocks D-1..0, output
convolution."""
from __future__ import annotations

import numpy as np


def param_shapes(depth: int, base: int) -> list[tuple[str, tuple[int, ...]]]:
    C = [base << l for l in range(depth + 1)]
    out = [("inc.w1", (C[0], 1, 3, 3)), ("inc.b1", (C[0],)),
           ("inc.w2", (C[0], C[0], 3, 3)), ("inc.b2", (C[0],))]
    for l in range(1, depth + 1):
        out += [(f"down{l}.w1", (C[l], C[l - 1], 3, 3)), (f"down{l}.b1", (C[l],)),
                (f"down{l}.w2", (C[l], C[l], 3, 3)), (f"down{l}.b2", (C[l],))]
    for l in range(depth - 1, -1, -1):
        out += [(f"up{l}.wt", (C[l + 1], C[l], 2, 2)), (f"up{l}.bt", (C[l],)),
                (f"up{l}.w1", (C[l], 2 * C[l], 3, 3)), (f"up{l}.b1", (C[l],)),
                (f"up{l}.w2", (C[l], C[l], 3, 3)), (f"up{l}.b2", (C[l],))]
    out += [("outc.w", (1, C[0], 1, 1)), ("outc.b", (1,))]
    return out


def draw(depth: int, base: int, seed: int = 2403, scale: float = 1.0) -> list[np.ndarray]:
    """Uniform +-scale/sqrt(fan_in) weights and biases (fan_in = Cin*9 for a
    3x3 conv, Cout*4 for the transposed conv, C0 for the output conv)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = param_shapes(depth, base)
    out, fan = [], 1.0
    for name, shp in shapes:
        if len(shp) == 4:
            # [Cout][Cin][k][k] for convs, [Cin][Cout][2][2] for the transposed
            # conv: dimension 1 times the kernel area in both cases
            fan = shp[1] * shp[2] * shp[3]
        bound = scale / np.sqrt(fan)
        out.append(rng.uniform(-bound, bound, shp))
    return out


def flatten(params: list[np.ndarray]) -> np.ndarray:
    return np.concatenate([p.ravel() for p in params]).astype(np.float32)


def unflatten(vec: np.ndarray, depth: int, base: int) -> list[np.ndarray]:
    out, off = [], 0
    for _, shp in param_shapes(depth, base):
        n = int(np.prod(shp))
        out.append(np.asarray(vec[off:off + n]).reshape(shp))
        off += n
    return out
