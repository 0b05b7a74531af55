"""Host helpers of the benchmark: the network flop count against a count
made from the parameter shapes."""
import re

import pytest

import bench
from synth import netparams


@pytest.mark.parametrize("depth,base", [(3, 32), (4, 128), (2, 16)])
def test_deblur_flops_from_parameter_shapes(depth, base):
    H, W = 208, 608
    total = 0
    for name, shp in netparams.param_shapes(depth, base):
        if len(shp) != 4:
            continue
        lvl = int(re.search(r"\d+", name.split(".")[0]).group()) if name[0] in "du" else 0
        pix = (H >> lvl) * (W >> lvl)
        if name.endswith(".wt"):
            # 2x2 stride-2 transposed conv into level lvl: one tap per output pixel
            total += 2 * pix * shp[0] * shp[1]
        else:
            total += 2 * pix * shp[0] * shp[1] * shp[2] * shp[3]
    assert bench.deblur_flops(H, W, depth, base) == total


def test_paper_scale_network_size():
    # the paper's network: 124 M parameters, ~742 GFLOP per 208 x 608 forward
    n = sum(int(__import__("numpy").prod(s)) for _, s in netparams.param_shapes(4, 128))
    assert 123e6 < n < 125e6
    assert abs(bench.deblur_flops(208, 608, 4, 128) / 1e9 - 742.1) < 0.5


@pytest.mark.parametrize("n", ["2", "8", "0"])
def test_more_than_one_gpu_refused(n):
    """The propagation path runs on one GPU: any other count exits with a
    message (before touching a device)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", n],
                       capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
