"""The adjoint sweeps' checkpointing schedule (binomial snapshot placement,
Griewank & Walther's revolve), replayed on the host by the library itself:
every action is checked against the state it tracks (each recomputation
starts from a snapshot of the right segment, the adjoint takes every
segment's fresh history once, last segment first), and the number of
recomputed segments is pinned to facts that do not come from the library:
Griewank's closed form for the minimal number of recomputed steps, a
brute-force minimum over every snapshot placement on small cases, and the
uniform and no-snapshot limits."""
from functools import lru_cache
from math import comb

import pytest

torch = pytest.importorskip("torch")

from paper_2403_17518_amd import ops, _abi  # noqa: E402


def griewank(l: int, s: int) -> int:
    """Fewest advanced steps to reverse l steps with s snapshots (the initial
    state one of them): r l - C(s + r, s + 1), r the least with C(s + r, s) >= l."""
    r = 0
    while comb(s + r, s) < l:
        r += 1
    return r * l - comb(s + r, s + 1)


@lru_cache(None)
def _brute(l: int, s: int, spine: bool) -> int:
    """Minimum over all placements of segments recomputed to reverse l
    segments from a stored root with s snapshots (root included); on the
    first-split path (`spine`) the advances are already done by the forward
    sweep and the last segment's history is kept."""
    if l == 1:
        return 0 if spine else 1
    if s == 1:
        return l * (l - 1) // 2 if spine else l * (l + 1) // 2
    best = None
    for m in range(1, l):
        c = (0 if spine else m) + _brute(l - m, s - 1, spine) + _brute(m, s, False)
        best = c if best is None or c < best else best
    return best


def test_schedule_meets_the_closed_form_minimum():
    for slots in list(range(0, 12)) + [20, 63]:
        for nseg in list(range(1, 160)) + [500, 1999, 4000]:
            assert ops.checkpoint_schedule(nseg, slots) == griewank(nseg, slots + 1), (nseg, slots)


def test_schedule_meets_the_brute_force_minimum():
    for slots in range(0, 5):
        for nseg in range(1, 40):
            assert ops.checkpoint_schedule(nseg, slots) == _brute(nseg, slots + 1, True), (nseg, slots)


def test_uniform_and_no_snapshot_limits():
    for nseg in (1, 2, 3, 17, 300):
        # nseg - 2 snapshots (the zero state is the first): every segment but
        # the last recomputed once; more slots change nothing
        for slots in (max(nseg - 2, 0), nseg, nseg + 5):
            assert ops.checkpoint_schedule(nseg, slots) == nseg - 1
        # no snapshot: segment j recomputed from the start, j + 1 segments
        assert ops.checkpoint_schedule(nseg, 0) == nseg * (nseg - 1) // 2


def test_bad_arguments_rejected():
    for nseg, slots in ((0, 3), (-1, 0), (5, -1)):
        with pytest.raises(_abi.FwiError):
            ops.checkpoint_schedule(nseg, slots)


def test_long_records_do_not_exhaust_the_host_stack():
    """With ample snapshots the splits nest once per segment; the schedule
    keeps its pending work on the heap, so 200000 segments run."""
    assert ops.checkpoint_schedule(200000, 200000) == 199999
    assert ops.checkpoint_schedule(200000, 2) == griewank(200000, 3)
