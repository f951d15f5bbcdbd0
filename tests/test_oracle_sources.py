"""Pins of the oracle's source rate field sigma(x, y) (arXiv 1705.00614,
Sec. 2.1: the sigma of Eq. (1) stands for precipitation, infiltration and
evaporation as well as inflow).

Reading: a rate adds tau*sigma of depth per step with no momentum (V = 0 in
Eqs. 2-3); a loss (sigma < 0) acts only on cells wet at layer n and takes at
most the water there; the applied depth is summed into the field volume, so
V_N - V_0 = inflow + field + ledger.  Each pin below is a closed form or an
invariant that a plausible slip (rain applied over half a step, a loss on a
dry cell or below zero, momentum given to rain, the field left out of the
budget) breaks.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1705_00614_amd import scenarios as S


def _flat(n, H, sigma, **prm):
    z = np.zeros((n, n))
    prm.setdefault("tau_max", 0.5)
    return dict(nx=n, ny=n, h=2.0, b=z.copy(), n_manning=z.copy(), solid=None,
                H0=np.full((n, n), float(H)), Qx0=z.copy(), Qy0=z.copy(), sigma=sigma,
                params=S.base_params(precision=64, **prm))


def test_uniform_rain_raises_a_lake_uniformly_at_rest():
    """Flat bed, still water, uniform rain: H(t) = H0 + sigma t everywhere
    and the water stays at rest (rain brings no momentum)."""
    n, H0, rate = 24, 1.0, 2e-3
    sim = orc.OracleSim(_flat(n, H0, np.full((n, n), rate)))
    sim.run(60)
    H, Qx, Qy = sim.state()
    t = sim.time()
    assert t > 0
    assert np.abs(H - (H0 + rate * t)).max() <= 1e-13
    assert np.abs(Qx).max() == 0.0 and np.abs(Qy).max() == 0.0
    area = (n * 2.0) ** 2
    assert abs(sim.field_volume() - rate * t * area) <= 1e-12 * rate * t * area
    assert abs(sim.mass() - (H0 + rate * t) * area) <= 1e-12 * sim.mass()


def test_rain_on_dry_ground_wets_it_uniformly():
    """Dry flat ground under uniform rain: depth sigma t, films first, then
    wet water at rest; no clamped volume."""
    n, rate = 16, 1e-5
    sim = orc.OracleSim(_flat(n, 0.0, np.full((n, n), rate), tau_max=4.0))
    sim.run(10)                      # 4e-5 m per step of 4 s: films for two steps, then wet
    H = sim.state()[0]
    assert np.abs(H - rate * sim.time()).max() <= 1e-15
    sim.run(40)
    H, Qx, Qy = sim.state()
    assert np.abs(H - rate * sim.time()).max() <= 1e-15
    assert np.abs(Qx).max() == 0.0 and sim.ledger() == 0.0


def test_uniform_loss_empties_a_lake_exactly():
    """Flat still lake under a uniform loss: the depth falls by tau*|sigma|
    per step and stops at exactly zero (the loss takes what is there, no
    more; no clamped volume), and the field volume is minus the lake."""
    n, H0, rate = 16, 0.3, -4e-3
    sim = orc.OracleSim(_flat(n, H0, np.full((n, n), rate)))
    V0 = sim.mass()
    prev = H0
    for _ in range(400):
        tau = sim.next_tau()
        sim.step()
        H = sim.state()[0]
        assert np.all(H == H[0, 0])
        expect = prev + tau * rate if prev > 1e-4 else prev
        assert abs(H[0, 0] - max(expect, 0.0)) <= 1e-15
        prev = H[0, 0]
    assert prev == 0.0 or prev <= 1e-4
    assert sim.ledger() == 0.0
    assert abs(sim.field_volume() + (V0 - sim.mass())) <= 1e-12 * V0


def test_losses_never_drive_depth_below_zero_and_balance_volume():
    """A strong loss drains a wet patch while water flows in from around it:
    depths stay >= 0 and the budget closes (clamped volume from the flux
    update included)."""
    n = 32
    sc = _flat(n, 0.5, None)
    sc["H0"][8:24, 8:24] = 2.0
    sig = np.zeros((n, n))
    sig[10:22, 10:22] = -0.05         # 0.05 m/s: the patch empties within ~40 s
    sc["sigma"] = sig
    sim = orc.OracleSim(sc)
    V0 = sim.mass()
    for _ in range(150):
        sim.step()
        H = sim.state()[0]
        assert H.min() >= 0.0
    V = sim.mass()
    assert sim.field_volume() < 0.0
    assert abs(V - V0 - sim.field_volume() - sim.inflow() - sim.ledger()) <= 1e-12 * V0
    # the loss cannot take more than the water it found
    assert -sim.field_volume() <= V0


def test_losses_leave_dry_cells_and_films_alone():
    """A loss acts on wet cells only: dry cells and films (0 < H <= eps) keep
    their depth exactly."""
    n = 12
    sc = _flat(n, 0.0, np.full((n, n), -1.0))
    sc["H0"][:, :6] = 5e-5              # films
    sim = orc.OracleSim(sc)
    H0 = sim.state()[0].copy()
    sim.run(20)
    assert np.array_equal(sim.state()[0], H0)
    assert sim.field_volume() == 0.0


def test_field_volume_closes_the_budget_on_a_floodplain():
    """Floodplain flood with inflow, rain over the upstream half and losses
    over the downstream half: V_N - V_0 = inflow + field + ledger to
    rounding, and the field volume is the sum of what the rates could apply
    bounded by the water present."""
    sc = S.floodplain(n=96, seed=4, precision=64)
    sig = np.zeros((96, 96))
    sig[:, :48] = 2e-5
    sig[:, 48:] = -5e-6
    sc["sigma"] = sig
    sim = orc.OracleSim(sc)
    V0 = sim.mass()
    sim.run(200)
    V = sim.mass()
    resid = V - V0 - sim.inflow() - sim.field_volume() - sim.ledger()
    assert abs(resid) <= 1e-12 * V
    area_rain = 96 * 48 * sc["h"] ** 2
    assert sim.field_volume() <= 2e-5 * sim.time() * area_rain * (1 + 1e-12)
    # without the field the same run differs
    sc2 = dict(sc, sigma=None)
    s2 = orc.OracleSim(sc2)
    s2.run(200)
    assert abs(s2.mass() - V) > 1e-3 * V


def test_field_is_rejected_when_not_finite_and_removable():
    sim = orc.OracleSim(_flat(8, 1.0, None))
    bad = np.zeros((8, 8))
    bad[2, 2] = np.nan
    with pytest.raises(ValueError):
        sim.set_source_field(bad)
    sim.set_source_field(np.full((8, 8), 1e-3))
    sim.run(3)
    v = sim.field_volume()
    sim.set_source_field(None)
    sim.run(3)
    assert sim.field_volume() == v > 0


def test_gates_take_no_field():
    sc = _flat(10, 1.0, np.full((10, 10), 1e-3))
    solid = np.zeros((10, 10), np.uint8)
    solid[4, 4] = 1
    sc["solid"] = solid
    sim = orc.OracleSim(sc)
    sim.run(10)
    assert sim.state()[0][4, 4] == 0.0
    assert abs(sim.field_volume() - 1e-3 * sim.time() * 99 * 4.0) <= 1e-12 * sim.field_volume()
