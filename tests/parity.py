"""Comparison helpers shared by the GPU parity tests.

Two bars for every comparison of a GPU layer with the oracle's layer:
  * grid-summed relative L1 of H and of (Qx, Qy) together;
  * per cell: max |dH| <= cell_tol * max |H_oracle| and
    max |dQ| <= cell_tol * max |Q_oracle| (both components), so that an error
    confined to a few cells (a tile's halo, a wall row) cannot hide in a sum.

FP64 stencil: the same arithmetic up to rounding order and contraction into
FMAs, each operation agreeing to ~1e-16; over 60-200 steps of a nonlinear
scheme with limiter branches and wet/dry thresholds these differences grow in
rough states (measured up to ~8e-11 of the largest value in a cell of a
nested patch, ~1e-11 on random wet/dry states), so both bars are 1e-10.  A
local defect (a wrong neighbour, halo or wall value) moves the cells it
touches by O(1) of their values, far above 1e-10.  FP32 stencil: the spec bar of 1e-4 relative L1 after 200
steps; the per-cell bar is 2e-4: FP32 rounds every stored value to a relative
6e-8, an error that a stable step carries forward without growth, so 200 steps
accumulate at most ~200 * 6e-8 = 1.2e-5 of the largest value per cell, plus a
wet/dry flip of a cell within rounding of eps (a depth change of ~eps = 1e-4 m,
a discharge change of at most eps * |U|).
"""
import numpy as np

from oracle import oracle as orc

BARS = {64: (1e-10, 1e-10), 32: (1e-4, 2e-4)}


def rel_l1(a, b):
    den = np.abs(b).sum()
    return np.abs(a - b).sum() / (den if den > 0 else 1.0)


def errors(g_state, o_state):
    """(rel L1 of H, rel L1 of HU, max cell |dH| / max H, max cell |dQ| / max |Q|)."""
    H, Qx, Qy = g_state
    Ho, Qxo, Qyo = o_state
    eH = rel_l1(H, Ho)
    eQ = (np.abs(Qx - Qxo).sum() + np.abs(Qy - Qyo).sum()) / max(np.abs(Qxo).sum() + np.abs(Qyo).sum(), 1e-300)
    mH = np.abs(H - Ho).max() / max(np.abs(Ho).max(), 1e-300)
    qmax = max(np.abs(Qxo).max(), np.abs(Qyo).max(), 1e-300)
    mQ = max(np.abs(Qx - Qxo).max(), np.abs(Qy - Qyo).max()) / qmax
    return eH, eQ, mH, mQ


def check(g_state, o_state, prec, l1=None, cell=None, label=""):
    """Assert both bars; returns the four measured errors."""
    bl1, bcell = BARS[prec]
    l1 = bl1 if l1 is None else l1
    cell = bcell if cell is None else cell
    e = errors(g_state, o_state)
    print("[parity] %s prec=%d eH=%.3e eQ=%.3e cellH=%.3e cellQ=%.3e" % ((label, prec) + e), flush=True)
    assert e[0] <= l1 and e[1] <= l1, (label, e)
    assert e[2] <= cell and e[3] <= cell, (label, e)
    return e


def step_tau(o, prec):
    """The oracle's CFL step of its current layer, rounded to the stencil type
    (the GPU stores tau in that type)."""
    tau = o.next_tau()
    return float(np.float32(tau)) if prec == 32 else tau


def run_held(o, g, steps, prec):
    """Advance oracle and GPU `steps` steps with the same time steps: each is
    the oracle's CFL step of its own layer (rounded to the stencil type), held
    on the GPU for that one step."""
    for _ in range(steps):
        tau = step_tau(o, prec)
        g.hold_dt(tau)
        g.step()
        o.step(tau)


def with_precision(sc, prec):
    sc = dict(sc)
    sc["params"] = dict(sc["params"], precision=prec)
    return sc


def oracle_of(sc):
    return orc.OracleSim(sc)


def rounded(state, prec):
    """A layer rounded to the stencil type (as doubles)."""
    if prec == 64:
        return tuple(np.asarray(x, np.float64) for x in state)
    return tuple(np.asarray(x, np.float32).astype(np.float64) for x in state)


def thacker_case(N, prec, L=2.0):
    """Thacker's planar oscillation in a paraboloid bowl (tests/analytic.py)
    at t = 0 on an N x N grid over [-L, L]^2, frictionless, eps = 1e-5."""
    from paper_1705_00614_amd import scenarios as S
    from tests import analytic as A
    th = A.Thacker()
    h = 2 * L / N
    xc = -L + (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(xc, xc)
    H0 = th.depth(X, Y, 0.0)
    u0, v0 = th.velocity(0.0)
    sc = dict(nx=N, ny=N, h=h, b=th.bed(X, Y), n_manning=np.zeros_like(X), solid=None,
              H0=H0, Qx0=H0 * u0, Qy0=H0 * v0, params=S.base_params(eps=1e-5, precision=prec))
    return th, X, Y, sc
