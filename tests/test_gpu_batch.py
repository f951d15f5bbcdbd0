"""Batched ensemble (swe_batch_*): scenarios of uneven sizes in one launch per
step, each with its own time step and clock.  Bars: every scenario equals its
standalone single-grid run bitwise (same tile kernel); FP64 batch against the
oracle <= 1e-10; per-scenario volume balance.  Paper: arXiv 1705.00614 Sec. 1
(hundreds of runs over hydrograph and hydraulic-structure settings), Sec. 2.3.
"""
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


def _small_ensemble(n=6, prec=32, seed0=1000):
    ens = S.ensemble(n=n, seed0=seed0, side_min=48, side_max=160, precision=prec)
    for sc in ens:
        # bring the flood peak into the window of a short test run
        sc["params"].update(t_peak=1800.0, sigma_t=600.0)
    return ens


@pytest.mark.parametrize("tile", [(32, 32), (16, 16)])
def test_batch_scenarios_equal_standalone_runs(tile):
    ens = _small_ensemble()
    assert len({sc["nx"] for sc in ens}) > 3 and any(sc["solid"] is not None for sc in ens)
    b = swe.Batch(ens, tile=tile)
    b.run(70)
    q = b.query()
    assert np.all(q["steps"] == 70)
    assert len(set(np.round(q["time"], 6))) > 1           # each scenario keeps its own clock
    for k, sc in enumerate(ens):
        g = swe.Solver(sc, tile=tile)
        g.run(70)
        a, r = b.state(k), g.state()
        for x, y in zip(a, r):
            assert np.array_equal(x, y), k
        assert q["time"][k] == g.time()
        assert q["mass"][k] == g.mass()
        g.close()


def test_batch_fp64_matches_oracle_and_balances_volume():
    ens = _small_ensemble(n=3, prec=64, seed0=1500)
    b = swe.Batch(ens)
    q0 = b.query()
    b.run(80)
    q = b.query()
    for k, sc in enumerate(ens):
        o = orc.OracleSim(sc)
        o.run(80)
        H, Qx, Qy = b.state(k)
        P.check((H, Qx, Qy), o.state(), 64, label="batch scenario %d" % k)
        assert abs(q["time"][k] - o.time()) <= 1e-12 * o.time()
        V = q["mass"][k]
        assert abs(V - q0["mass"][k] - q["inflow"][k] - q["ledger"][k]) <= 1e-12 * V
        if sc["solid"] is not None:
            assert np.all(H[sc["solid"] == 1] == 0.0)


def test_batch_graph_replay_and_work_counters():
    ens = _small_ensemble(n=4, seed0=1700)
    b1 = swe.Batch(ens)
    b1.run(64)                       # two captured graphs
    b2 = swe.Batch(ens)
    b2.run_timed(64)                 # one launch per step
    for k in range(len(ens)):
        for x, y in zip(b1.state(k), b2.state(k)):
            assert np.array_equal(x, y)
    w = b1.work()
    assert 0 < w["tile_steps"] <= 64 * w["total_tiles"]


def test_batch_rejects_mixed_precision_and_no_skip():
    ens = _small_ensemble(n=2)
    ens[1]["params"] = dict(ens[1]["params"], precision=64)
    with pytest.raises(swe.SweError):
        swe.Batch(ens)


def test_autotuner_times_every_shape_and_changes_no_result():
    """swe_autotune / swe_batch_autotune time every compiled tile shape of
    the precision (fastest first); the chosen shape computes the same state
    as the default one, bit for bit."""
    sc = S.floodplain(n=96, seed=21)
    table = swe.autotune(sc, warmup=2, steps=6)
    shapes = [t for t, _ in table]
    assert sorted(shapes) == sorted([(32, 32), (64, 16), (16, 16)])
    ms = [m for _, m in table]
    assert all(m > 0 for m in ms) and ms == sorted(ms)
    best = swe.Solver(sc, tile=shapes[0])
    ref = swe.Solver(sc)
    best.run(30)
    ref.run(30)
    for x, y in zip(best.state(), ref.state()):
        assert np.array_equal(x, y)
    ens = _small_ensemble(n=3, seed0=77)
    bt = swe.autotune_batch(ens, warmup=1, steps=4)
    assert sorted(t for t, _ in bt) == sorted(shapes)
    tuned = swe.Batch(ens, tile=bt[0][0])
    tuned.run(12)
    for k, scen in enumerate(ens):
        g = swe.Solver(scen, tile=bt[0][0])
        g.run(12)
        for x, y in zip(tuned.state(k), g.state()):
            assert np.array_equal(x, y), k


def test_autotuner_rejects_bad_arguments():
    sc = S.floodplain(n=64, seed=22)
    with pytest.raises(swe.SweError):
        swe.autotune(sc, warmup=0, steps=0)


def test_full_size_ensemble_sampled_scenarios_match_oracle():
    """The 256-scenario ensemble of the benchmark at its full size (sides
    256..2048, 2.65e8 cells) in one batch with the 32x32 tile the autotuner
    picks there, for one 32-step graph replay as the benchmark runs it: the
    three smallest scenarios (which the oracle steps in seconds) against the
    FP64 oracle at the FP32 bar, and every scenario advanced 32 steps with a
    finite, positive clock."""
    ens = S.ensemble(n=256)
    B = swe.Batch(ens, tile=(32, 32))
    B.run(32)
    for k in np.argsort([sc["nx"] * sc["ny"] for sc in ens], kind="stable")[:3]:
        o = orc.OracleSim(ens[k])
        o.run(32)
        P.check(B.state(int(k)), o.state(), 32, label="ensemble scenario %d" % k)
    q = B.query()
    assert np.all(q["steps"] == 32)
    assert np.all(np.isfinite(q["time"])) and np.all(q["time"] > 0)
