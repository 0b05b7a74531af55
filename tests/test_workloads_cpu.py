"""The seeded workloads' geometry against what they stand in for."""
import numpy as np

from synth import configs


def test_geometry_is_the_papers():
    wl = configs.marmousi_601x221()
    g, a = wl.grid, wl.acq
    assert (g.nz, g.nx, g.h) == (221, 601, 15.0) and wl.freq == 5.0
    assert a.nshots == 30 and np.all(np.diff(np.asarray(a.rec_ptr)) == 300)
    assert np.all(np.asarray(a.src_z) == 0) and np.all(np.asarray(a.rec_z) == 0)
    # equally spaced to within the rounding to grid points
    for x, n in ((np.asarray(a.src_x), 30), (np.asarray(a.rec_x)[:300], 300)):
        assert np.all(np.abs(np.diff(x) - 601 / n) <= 1.0)
