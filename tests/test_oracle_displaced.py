"""Pins of the oracle's displaced-particle corrector (sph_displaced = 1).

arXiv 1705.00614, Sec. 2.3 stage II and kernels K4-K6: the Lagrangian
particles move inside their cells; K4 gives their positions at t_{n+1/2},
K5 the forces there, K6 the corrector.  Reading: particle j at
c_j + (tau/2) U_j^n, the level gradient at particle i the corrected SPH sum
of the cubic B-spline kernel (smoothing length h) over the 5x5 neighbourhood
(exact for linear levels), used by the corrector only.

Pins: with no displacement the gradient is the lattice stencil; for a linear
level it is the exact slope whatever the displacements; it equals a brute-force
sum over every particle of a small domain (the 5x5 truncation loses nothing
within the support); a lake at rest stays at rest; the dam break still
converges to Stoker's solution; mirror symmetry is kept.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1705_00614_amd import scenarios as S
from tests import analytic as A


def _state(n, H, ux, uy, b=None, **prm):
    z = np.zeros((n, n))
    return dict(nx=n, ny=n, h=prm.pop("h", 1.0), b=z.copy() if b is None else b, n_manning=z.copy(), solid=None,
                H0=H, Qx0=H * ux, Qy0=H * uy, params=S.base_params(precision=64, sph_displaced=1, **prm))


def _gradients(sc, tau):
    sim = orc.OracleSim(sc)
    sim.step(tau)
    return (sim.field(orc.F_GX), sim.field(orc.F_GY), sim.field(orc.F_GDX), sim.field(orc.F_GDY))


def test_without_displacement_it_is_the_lattice_stencil():
    rng = np.random.default_rng(3)
    n = 12
    H = 2.0 + rng.uniform(0, 0.5, (n, n))
    z = np.zeros((n, n))
    gx, gy, dx, dy = _gradients(_state(n, H, z, z, b=rng.uniform(-0.3, 0.3, (n, n))), 0.05)
    assert np.abs(dx - gx).max() <= 1e-13 and np.abs(dy - gy).max() <= 1e-13
    assert np.abs(gx).max() > 1e-3


def test_level_linear_in_the_particle_positions_gives_the_exact_slope():
    """Corrected gradient: when the levels the particles carry are a linear
    function a + p x + q y of their displaced positions, the gradient is
    (p, q) exactly, however the particles moved (deep water, so every
    neighbour shows its own level); the lattice stencil is not exact there."""
    rng = np.random.default_rng(4)
    n, h, p, q, tau = 14, 2.0, 0.013, -0.021, 0.25
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    ux, uy = rng.uniform(-3, 3, (n, n)), rng.uniform(-3, 3, (n, n))   # displacements up to 0.19 h
    b = rng.uniform(-1.0, 1.0, (n, n))
    eta = 10.0 + p * (X + 0.5 * tau * ux) + q * (Y + 0.5 * tau * uy)
    H = eta - b
    gx, gy, dx, dy = _gradients(_state(n, H, ux, uy, b=b, h=h), tau)
    inner = (slice(2, -2), slice(2, -2))    # away from the walls' mirror images
    assert np.abs(dx[inner] - p).max() <= 1e-12 and np.abs(dy[inner] - q).max() <= 1e-12
    assert np.abs(gx[inner] - p).max() > 1e-4


def test_matches_a_brute_force_sum_over_every_particle():
    """The 5x5 truncation keeps every particle within the kernel support:
    the oracle's gradient equals the corrected SPH sum taken over all
    particles of a small periodic-free interior, with the kernel slope from
    the B-spline's definition (tests/analytic.py)."""
    rng = np.random.default_rng(5)
    n, tau = 11, 0.3
    b = rng.uniform(-0.5, 0.5, (n, n))
    H = 3.0 + rng.uniform(0, 0.8, (n, n))
    ux, uy = rng.uniform(-1.3, 1.3, (n, n)), rng.uniform(-1.3, 1.3, (n, n))
    sc = _state(n, H, ux, uy, b=b)
    _, _, dx, dy = _gradients(sc, tau)
    eta = H + b
    px = np.arange(n)[None, :] + 0.5 * tau * ux
    py = np.arange(n)[:, None] + 0.5 * tau * uy
    for (j, i) in [(5, 5), (4, 6), (6, 3), (3, 7)]:
        S = np.zeros(2)
        M = np.zeros((2, 2))
        for jj in range(n):
            for ii in range(n):
                if (jj, ii) == (j, i):
                    continue
                r = np.array([px[jj, ii] - px[j, i], py[jj, ii] - py[j, i]])
                d = math.hypot(*r)
                dw = A.cubic_bspline_dw(d)
                if dw == 0.0:
                    continue
                w = dw * r / d
                S += (eta[jj, ii] - eta[j, i]) * w
                M += np.outer(w, r)
        g = np.linalg.solve(M, S)
        assert abs(g[0] - dx[j, i]) <= 1e-12 * max(1.0, abs(g[0]))
        assert abs(g[1] - dy[j, i]) <= 1e-12 * max(1.0, abs(g[1]))


def test_lake_at_rest_stays_at_rest():
    sc = S.lake_at_rest(n=48, precision=64)
    sc["params"] = dict(sc["params"], sph_displaced=1)
    sim = orc.OracleSim(sc)
    sim.run(300)
    H, Qx, Qy = sim.state()
    wet = H > 1e-4
    assert np.abs((H + sc["b"] - 5.0)[wet]).max() <= 1e-12
    assert (np.abs(Qx) + np.abs(Qy))[wet].max() <= 1e-10


def _run_to(sim, T):
    while sim.time() < T - 1e-12:
        sim.step(min(sim.next_tau(), T - sim.time()))


def test_dam_break_still_converges_to_stoker():
    T, errs = 12.0, []
    for nx in (128, 256, 512):
        h = 256.0 / nx
        sc = S.dam_break(nx=nx, ny=2, h=h, h_right=0.5, precision=64)
        sc["params"] = dict(sc["params"], sph_displaced=1)
        sim = orc.OracleSim(sc)
        _run_to(sim, T)
        Hs = sim.state()[0][0]
        x = (np.arange(nx) + 0.5) * h
        he = A.dam_break_depth((x - 128.0) / T, 2.0, 0.5)
        errs.append(np.abs(Hs - he).sum() / np.abs(he).sum())
    assert errs[1] <= 0.02
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


def test_mirror_symmetry_is_kept():
    """A flow symmetric about the grid's diagonal stays symmetric: the
    displaced sums treat x and y alike."""
    n = 24
    rng = np.random.default_rng(6)
    b = rng.uniform(0, 1.0, (n, n))
    b = 0.5 * (b + b.T)
    H = np.maximum(3.0 - b, 0.0)
    H[:8, :8] += 1.0
    sc = _state(n, H, np.zeros((n, n)), np.zeros((n, n)), b=b)
    sim = orc.OracleSim(sc)
    sim.run(60)
    H, Qx, Qy = sim.state()
    assert np.abs(H - H.T).max() <= 1e-12
    assert np.abs(Qx - Qy.T).max() <= 1e-12


def test_changes_the_solution_of_a_moving_flow():
    """The variant is not a no-op: on a moving flow it differs from the
    lattice corrector, by a few per cent of the depth in relative L1 (the
    displacements are a fraction of a cell; both are consistent schemes)."""
    sc = S.dam_break(nx=64, ny=4, h=1.0, x_dam=32.0, precision=64)
    a = orc.OracleSim(sc)
    sc2 = dict(sc, params=dict(sc["params"], sph_displaced=1))
    b = orc.OracleSim(sc2)
    a.run(60)
    b.run(60)
    Ha, Hb = a.state()[0], b.state()[0]
    d = np.abs(Ha - Hb).sum() / np.abs(Ha).sum()
    assert 1e-6 < d < 0.02
