"""The displaced-particle corrector on the GPU (swe_params.sph_displaced):
the corrector's pressure gradient at the particle positions of t_{n+1/2}
(arXiv 1705.00614, Sec. 2.3 stage II, K4-K6), against the FP64 oracle's
sph_displaced reading.  Bars: those of tests/parity.py; dry-tile skipping
changes nothing (bitwise); a lake at rest stays at rest; the variant is
refused where it is not offered."""
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


def _disp(sc, prec):
    return dict(sc, params=dict(sc["params"], sph_displaced=1, precision=prec))


def _compare(sc, steps, prec, held=False, label=""):
    o = orc.OracleSim(sc)
    g = swe.Solver(sc)
    m0 = g.mass()
    if held:
        P.run_held(o, g, steps, prec)
    else:
        o.run(steps)
        g.run(steps)
        assert abs(g.time() - o.time()) <= (1e-10 if prec == 64 else 1e-4) * o.time()
    P.check(g.state(), o.state(), prec, label=label)
    V = g.mass()
    return g, abs(V - m0 - g.inflow() - g.ledger()) / V


@pytest.mark.parametrize("case", ["dam", "flood", "random"])
def test_displaced_fp64_matches_oracle(case):
    sc = {"dam": lambda: S.dam_break(nx=160, ny=40, h=1.0, x_dam=80.0),
          "flood": lambda: S.floodplain(n=128, seed=3),
          "random": lambda: S.random_state(70, 45, seed=8)}[case]()
    g, drift = _compare(_disp(sc, 64), 120, 64, label="disp64 " + case)
    assert drift < 1e-12


def test_displaced_fp32_floodplain_matches_oracle():
    g, drift = _compare(_disp(S.floodplain(n=160, seed=4), 32), 200, 32, label="disp32 flood")
    assert drift <= 1e-6


def test_displaced_fp32_random_state_at_held_steps():
    _compare(_disp(S.random_state(70, 45, seed=9), 32), 200, 32, held=True, label="disp32 random held")


def test_displaced_differs_from_the_lattice_corrector():
    sc = S.dam_break(nx=160, ny=40, h=1.0, x_dam=80.0, precision=64)
    a = swe.Solver(sc)
    b = swe.Solver(_disp(sc, 64))
    a.run(60)
    b.run(60)
    d = np.abs(a.state()[0] - b.state()[0]).sum() / np.abs(a.state()[0]).sum()
    assert 1e-6 < d < 0.02


def test_displaced_skip_dry_is_bitwise_identical():
    sc = _disp(S.floodplain(n=192, seed=5), 32)
    a = swe.Solver(sc, skip_dry=True)
    b = swe.Solver(sc, skip_dry=False)
    a.run(120)
    b.run(120)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()


def test_displaced_lake_at_rest_fp32():
    sc = _disp(S.lake_at_rest(n=96), 32)
    g = swe.Solver(sc)
    g.run(1000)
    H, Qx, Qy = g.state()
    wet = H > 1e-4
    assert np.abs((H + sc["b"].astype(np.float32) - 5.0)[wet]).max() <= 1e-5
    assert (np.hypot(Qx, Qy)[wet] / H[wet]).max() <= 1e-4


def test_displaced_is_refused_where_not_offered():
    sc = _disp(S.floodplain(n=96, seed=6), 32)
    with pytest.raises(swe.SweError):
        swe.Solver(sc, tile=(16, 16))                  # default tile shape only
    with pytest.raises(swe.SweError):
        swe.Batch([sc, sc])
    g = swe.Solver(sc)
    with pytest.raises(swe.SweError):
        g.set_source_field(np.zeros((96, 96)))
    z = np.zeros((3, 96, 96))
    with pytest.raises(swe.SweError):
        g.set_correction(z, z)
