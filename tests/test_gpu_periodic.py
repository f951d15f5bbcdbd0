"""The periodic domain (swe_params.periodic = 1) on the GPU against the FP64
oracle's periodic boundary (the cell one period away, no mirror): parity at
the bars of tests/parity.py, dry-tile skipping bitwise with water crossing
the wrap, momentum conservation on a flat bed (the property the periodic
boundary exists to test: Sec. 2.3's scheme is conservative in flux form),
and the refusals where the variant is not offered."""
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


def _corner_blob(n, prec, h=10.0):
    """Flat bed, a 2 m column of water centred on the domain's corner (so
    it wraps into all four corners), dry elsewhere."""
    x = np.arange(n)
    d = np.minimum(x, n - x)[None, :] ** 2 + np.minimum(x, n - x)[:, None] ** 2
    H0 = np.where(d < 20 ** 2, 2.0, 0.0)
    z = np.zeros((n, n))
    return dict(name="corner-blob", nx=n, ny=n, h=h, b=z.copy(), n_manning=np.full((n, n), 0.03), solid=None,
                H0=H0, Qx0=z.copy(), Qy0=z.copy(), params=S.base_params(precision=prec, periodic=1))


def test_periodic_fp64_matches_oracle():
    sc = S.random_state(96, 64, seed=31, precision=64, periodic=1)
    o = orc.OracleSim(sc)
    g = swe.Solver(sc)
    m0 = g.mass()
    o.run(120)
    g.run(120)
    assert abs(g.time() - o.time()) <= 1e-10 * o.time()
    P.check(g.state(), o.state(), 64, label="periodic64 random")
    V = g.mass()
    assert abs(V - m0 - g.inflow() - g.ledger()) <= 1e-12 * V


def test_periodic_fp32_matches_oracle_at_held_steps():
    sc = S.random_state(128, 96, seed=32, precision=32, periodic=1)
    o = orc.OracleSim(sc)
    g = swe.Solver(sc)
    P.run_held(o, g, 200, 32)
    P.check(g.state(), o.state(), 32, label="periodic32 random held")


@pytest.mark.parametrize("prec", [32, 64])
def test_periodic_water_across_the_wrap(prec):
    """Water crossing the wrap: dry tiles skipped bitwise as without
    skipping, fewer cells processed, and the oracle's result at the oracle's
    steps: the films of a front spreading over a dry bed with friction make
    the choice of the step ill-conditioned (after 150 free steps the clocks
    part by 6e-10 in FP64 and 1.4 % in FP32), as
    tests/test_oracle_conditioning.py shows for rough wet/dry states; the
    step choice itself is tested on loaded oracle layers."""
    n = 192
    sc = _corner_blob(n, prec)
    a = swe.Solver(sc)
    b = swe.Solver(sc, skip_dry=False)
    a.run(150)
    b.run(150)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    assert a.time() == b.time()
    assert a.work()["cell_steps"] < 0.8 * b.work()["cell_steps"]
    H = a.state()[0]
    # the blob is symmetric about the corner in x and in y (cell j mirrors
    # cell -j mod n), and so is its spread, to rounding
    m = (-np.arange(n)) % n
    tol = (1e-12 if prec == 64 else 1e-4) * H.max()
    assert np.abs(H - H[m, :]).max() <= tol and np.abs(H - H[:, m]).max() <= tol
    assert (H[n // 2, :] > 1e-4).sum() < n // 4      # the middle of the domain is still dry
    o = orc.OracleSim(sc)
    g = swe.Solver(sc)
    P.run_held(o, g, 150, prec)
    P.check(g.state(), o.state(), prec, label="periodic%d corner blob held" % prec)


def test_periodic_flat_bed_conserves_momentum_fp64():
    """No friction, viscosity, wind, Coriolis or bed slope on a periodic
    flat bed: the domain sums of Qx and Qy are invariants of the flux-form
    scheme (the oracle pin tests/test_oracle_pins.py checks the same on the
    CPU)."""
    n = 64
    rng = np.random.default_rng(33)
    H0 = 2.0 + rng.uniform(0.0, 0.5, (n, n))
    z = np.zeros((n, n))
    sc = dict(name="periodic-flat", nx=n, ny=n, h=5.0, b=z.copy(), n_manning=z.copy(), solid=None, H0=H0,
              Qx0=H0 * rng.normal(0.0, 0.3, (n, n)), Qy0=H0 * rng.normal(0.0, 0.3, (n, n)),
              params=S.base_params(precision=64, periodic=1))
    g = swe.Solver(sc)
    _, Qx, Qy = g.state()
    px, py, scale = Qx.sum(), Qy.sum(), np.abs(Qx).sum() + np.abs(Qy).sum()
    g.run(200)
    _, Qx, Qy = g.state()
    assert abs(Qx.sum() - px) <= 1e-12 * scale and abs(Qy.sum() - py) <= 1e-12 * scale
    assert np.abs(Qx - sc["Qx0"]).max() > 1e-3          # the flow did evolve


def test_periodic_is_refused_where_not_offered():
    sc = S.random_state(100, 64, seed=34, precision=32, periodic=1)     # 100 is not a multiple of 32
    with pytest.raises(swe.SweError):
        swe.Solver(sc)
    ok = S.random_state(96, 64, seed=34, precision=32, periodic=1)
    with pytest.raises(swe.SweError):
        swe.Solver(ok, tile=(16, 16))
    with pytest.raises(swe.SweError):
        swe.Batch([ok, ok])
    g = swe.Solver(ok)
    with pytest.raises(swe.SweError):
        g.set_source_field(np.zeros((64, 96)))
    z = np.zeros((3, 64, 96))
    with pytest.raises(swe.SweError):
        g.set_correction(z, z)
