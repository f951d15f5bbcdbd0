"""Tile placement of the step launch: which workgroup steps which listed
tile (own-segment order when the list is no longer than the launch grid,
with the overflow of longer segments going to idle workgroups; the grid
strided over a longer list) changes no result.  States, clocks and volume
ledgers are compared bitwise across launch grids that force each path, and
one grid against the FP64 oracle (bars of tests/parity.py)."""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1705_00614_amd import scenarios as S
from tests import parity as P

pytestmark = pytest.mark.gpu

swe = pytest.importorskip("paper_1705_00614_amd.swe")


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu] %s" % request.node.nodeid, flush=True)
    sys.stdout.flush()
    yield


def _run(sc, grid, steps, chunk=7):
    g = swe.Solver(sc)
    if grid:
        g.set_launch_grid(grid)
    tiles = []
    for k in range(0, steps, chunk):
        tiles.append(len(g.active_tiles()))
        g.run(min(chunk, steps - k))
    out = (g.state(), g.time(), g.ledger(), g.mass(), tiles)
    g.close()
    return out


CASES = {
    # the front crosses from a few tiles to more than the small grids hold
    "flood": lambda: S.floodplain(n=1024, seed=11),
    # every tile listed from the start (90 tiles of 32x32)
    "random": lambda: S.random_state(300, 260, seed=12),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_results_do_not_depend_on_the_launch_grid(case):
    sc = CASES[case]()
    ref = _run(sc, 0, 60)
    for grid in (8, 24, 64, 96, 200):
        got = _run(sc, grid, 60)
        for x, y in zip(ref[0], got[0]):
            assert np.array_equal(x, y), (case, grid)
        assert ref[1] == got[1] and ref[2] == got[2] and ref[3] == got[3], (case, grid)
        assert ref[4] == got[4], (case, grid)
    # both paths ran: a list longer than the smallest grid, one no longer
    # than the largest
    print("listed tiles per chunk:", ref[4], flush=True)
    assert max(ref[4]) > 8 and 0 < min(ref[4]) <= 200


def test_small_grid_matches_the_oracle():
    sc = S.floodplain(n=512, seed=13, precision=64)
    o = orc.OracleSim(sc)
    g = swe.Solver(sc)
    g.set_launch_grid(8)
    o.run(80)
    g.run(80)
    assert abs(g.time() - o.time()) <= 1e-10 * o.time()
    P.check(g.state(), o.state(), 64, label="grid 8")


def test_launch_grid_bounds():
    g = swe.Solver(S.floodplain(n=256, seed=14))
    d = g.launch_grid()
    for bad in (7, 0, -1, d + 1):
        with pytest.raises(swe.SweError):
            g.set_launch_grid(bad)
    g.set_launch_grid(8)
    assert g.launch_grid() == 8
    g.set_launch_grid(d)
    assert g.launch_grid() == d
