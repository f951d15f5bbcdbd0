"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
solutions (Stoker, Ritter, Thacker, friction/Coriolis/wind ODEs, the discrete
Laplacian eigenvalue), exact invariants (lake at rest, mass balance, momentum
conservation, symmetry), quadrature, and brute force (the K1 wet-block rule).
Paper: arXiv 1705.00614, Sec. 2.1 (Eqs. 1-4), Sec. 2.3 (stages I-IV), Sec. 3
(K1..K8).
"""
import math

import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import oracle as orc
from paper_1705_00614_amd import scenarios as S
from tests import analytic as A


def _uniform(nx, ny, h, H, ux=0.0, uy=0.0, **prm):
    z = np.zeros((ny, nx))
    Hh = np.full((ny, nx), float(H))
    return dict(nx=nx, ny=ny, h=h, b=z.copy(), n_manning=prm.pop("n_manning", z.copy()),
                solid=None, H0=Hh, Qx0=Hh * ux, Qy0=Hh * uy,
                params=S.base_params(precision=64, **prm))


def _run_to(sim, T):
    while sim.time() < T - 1e-12:
        tau = sim.next_tau()
        sim.step(min(tau, T - sim.time()))


# ---------------------------------------------------------------- stage I: SPH gradient

def test_sph_weights_match_cubic_bspline_lattice_sum():
    """The oracle's pressure gradient equals the normalised SPH gradient of the
    cubic B-spline (ell = h) computed here by brute-force lattice summation."""
    w = A.sph_lattice_weights(1.0)
    assert set(w) == {(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)} - {(0, 0)}
    al, be = w[(1, 0)][0], w[(1, 1)][0]
    assert abs(2 * al + 4 * be - 1.0) < 1e-14
    assert abs(al - 1.0 / (12 * math.sqrt(2) - 14)) < 1e-14

    rng = np.random.default_rng(5)
    n, h = 24, 3.0
    b = rng.uniform(-1.0, 1.0, size=(n, n))
    H = 20.0 + rng.uniform(0.0, 1.0, size=(n, n))      # everything wet
    sc = dict(nx=n, ny=n, h=h, b=b, n_manning=np.zeros_like(b), solid=None, H0=H,
              Qx0=np.zeros_like(b), Qy0=np.zeros_like(b), params=S.base_params(precision=64))
    sim = orc.OracleSim(sc)
    sim.step(1e-6)
    Gx, Gy = sim.field(orc.F_GX), sim.field(orc.F_GY)
    eta = H + b
    ex = np.zeros_like(eta)
    ey = np.zeros_like(eta)
    for (di, dj), (wx, wy) in w.items():
        d = np.roll(np.roll(eta, -dj, axis=0), -di, axis=1) - eta
        ex += wx * d
        ey += wy * d
    ex /= h
    ey /= h
    sl = (slice(1, -1), slice(1, -1))
    assert np.allclose(Gx[sl], ex[sl], rtol=0, atol=1e-12)
    assert np.allclose(Gy[sl], ey[sl], rtol=0, atol=1e-12)


def test_sph_gradient_exact_on_linear_level_and_y_uniform_reduction():
    n, h = 16, 2.0
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    for sx, sy in [(0.01, -0.02), (-0.003, 0.0), (0.0, 0.05)]:
        b = sx * X + sy * Y
        sc = dict(nx=n, ny=n, h=h, b=b, n_manning=np.zeros_like(b), solid=None,
                  H0=np.full_like(b, 5.0), Qx0=np.zeros_like(b), Qy0=np.zeros_like(b),
                  params=S.base_params(precision=64))
        sim = orc.OracleSim(sc)
        sim.step(1e-6)
        sl = (slice(1, -1), slice(1, -1))
        assert np.allclose(sim.field(orc.F_GX)[sl], sx, atol=1e-13)
        assert np.allclose(sim.field(orc.F_GY)[sl], sy, atol=1e-13)
    # y-uniform data: G_x is the central difference (eta_E - eta_W)/(2h)
    rng = np.random.default_rng(1)
    prof = 3.0 + rng.uniform(0, 1, size=n)
    H = np.repeat(prof[None, :], n, axis=0)
    sc = _uniform(n, n, h, 1.0)
    sc["H0"] = H
    sim = orc.OracleSim(sc)
    sim.step(1e-6)
    cd = (prof[2:] - prof[:-2]) / (2 * h)
    assert np.allclose(sim.field(orc.F_GX)[:, 1:-1], cd[None, :], atol=1e-13)
    assert np.abs(sim.field(orc.F_GY)).max() < 1e-13


# ---------------------------------------------------------------- well-balancing

def test_lake_at_rest_over_rough_bed_with_islands():
    sc = S.lake_at_rest(n=64, precision=64)
    H0 = sc["H0"]
    assert 0.3 < (H0 > 1e-4).mean() < 0.95          # islands emerge
    sim = orc.OracleSim(sc)
    sim.run(1000)
    H, Qx, Qy = sim.state()
    wet = H > 1e-4
    assert np.abs((H + sc["b"] - 5.0)[wet]).max() <= 1e-12
    assert (np.abs(Qx) + np.abs(Qy))[wet].max() / H[wet].min() <= 1e-10
    assert np.array_equal(H[~wet], H0[~wet])


def test_closed_gates_stay_dry_and_keep_lake_at_rest():
    sc = S.lake_at_rest(n=48, precision=64)
    rng = np.random.default_rng(2)
    solid = np.zeros((48, 48), np.uint8)
    solid[rng.integers(0, 48, 30), rng.integers(0, 48, 30)] = 1
    sc["solid"] = solid
    sim = orc.OracleSim(sc)
    sim.run(300)
    H, Qx, Qy = sim.state()
    assert np.all(H[solid == 1] == 0.0)
    wet = H > 1e-4
    assert np.abs((H + sc["b"] - 5.0)[wet]).max() <= 1e-12
    # moving water against gates: nothing crosses a gate
    sc2 = S.dam_break(nx=40, ny=8, h=1.0, precision=64)
    wall = np.zeros((8, 40), np.uint8)
    wall[:, 25] = 1
    sc2["solid"] = wall
    s2 = orc.OracleSim(sc2)
    m0 = s2.mass()
    right0 = s2.state()[0][:, 26:].sum()
    s2.run(150)
    H2 = s2.state()[0]
    assert abs(H2[:, 26:].sum() - right0) < 1e-12
    assert abs(s2.mass() - m0) < 1e-11 * m0


# ---------------------------------------------------------------- shocks, dry fronts

@pytest.mark.parametrize("h1,first_bar", [(0.5, 0.02), (0.0, 0.03)])
def test_dam_break_converges_to_stoker_and_ritter(h1, first_bar):
    T, errs = 12.0, []
    for nx in (128, 256, 512):
        h = 256.0 / nx
        sc = S.dam_break(nx=nx, ny=2, h=h, h_right=h1, precision=64)
        sim = orc.OracleSim(sc)
        _run_to(sim, T)
        H = sim.state()[0][0]
        x = (np.arange(nx) + 0.5) * h
        he = A.dam_break_depth((x - 128.0) / T, 2.0, h1)
        errs.append(np.abs(H - he).sum() / np.abs(he).sum())
        assert sim.ledger() == 0.0
    assert errs[1] <= first_bar
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


def test_stoker_middle_state_satisfies_jump_conditions():
    """The analytic reference itself: Rankine-Hugoniot and the Riemann invariant."""
    g, h0, h1 = A.G, 2.0, 0.5
    cm, hm, um, s = A.stoker_middle(h0, h1)
    assert abs(um + 2 * cm - 2 * math.sqrt(g * h0)) < 1e-12
    assert abs(s * (hm - h1) - hm * um) < 1e-12                          # mass
    assert abs(s * (hm * um) - (hm * um * um + 0.5 * g * (hm**2 - h1**2))) < 1e-9  # momentum
    assert abs(hm - 1.103494) < 1e-5 and abs(s - 4.166325) < 1e-5


def test_thacker_bowl_moving_shoreline_converges():
    th = A.Thacker()
    # the closed form solves Eqs. (1)-(3): residual by central differences
    x, y, t, d = 0.3, -0.2, 0.7, 1e-5
    Hf = lambda x, y, t: th.eta(x, y, t) - th.bed(x, y)
    u, v = th.velocity(t)
    mass = ((Hf(x, y, t + d) - Hf(x, y, t - d)) / (2 * d) + u * (Hf(x + d, y, t) - Hf(x - d, y, t)) / (2 * d)
            + v * (Hf(x, y + d, t) - Hf(x, y - d, t)) / (2 * d))
    mom = (th.velocity(t + d)[0] - th.velocity(t - d)[0]) / (2 * d) + A.G * (
        th.eta(x + d, y, t) - th.eta(x - d, y, t)) / (2 * d)
    assert abs(mass) < 1e-8 and abs(mom) < 1e-7
    errs = []
    for N in (40, 80):
        L = 2.0
        h = 2 * L / N
        xc = -L + (np.arange(N) + 0.5) * h
        X, Y = np.meshgrid(xc, xc)
        H0 = th.depth(X, Y, 0.0)
        u0, v0 = th.velocity(0.0)
        sc = dict(nx=N, ny=N, h=h, b=th.bed(X, Y), n_manning=np.zeros_like(X), solid=None,
                  H0=H0, Qx0=H0 * u0, Qy0=H0 * v0, params=S.base_params(eps=1e-5, precision=64))
        sim = orc.OracleSim(sc)
        _run_to(sim, th.period)
        He = th.depth(X, Y, th.period)
        errs.append(np.abs(sim.state()[0] - He).sum() / He.sum())
    assert errs[1] < 0.045 and errs[1] < 0.5 * errs[0]


# ---------------------------------------------------------------- sources and mass

def test_hydrograph_volume_matches_quadrature_and_telescopes():
    qb, qp, tp, st = 50.0, 3.0e4, 3600.0, 1200.0
    Q = lambda t: qb + (qp - qb) * math.exp(-(t - tp) ** 2 / (2 * st * st))
    rng = np.random.default_rng(0)
    for _ in range(20):
        t = rng.uniform(0, 8000)
        tau = rng.uniform(0.01, 50.0)
        ref = quad(Q, t, t + tau, epsabs=0, epsrel=1e-12)[0]
        got = orc.hydrograph_volume(qb, qp, tp, st, t, tau)
        assert abs(got - ref) <= 1e-11 * abs(ref)
    # a typical flood step (tau ~ 0.5 s << sigma_t): the erf difference
    # cancels ~4 digits, FP64 keeps the volume to ~1e-12 relative
    ref = quad(Q, 1000.0, 1000.5, epsabs=0, epsrel=1e-12)[0]
    assert abs(orc.hydrograph_volume(qb, qp, tp, st, 1000.0, 0.5) - ref) <= 1e-11 * ref


def test_mass_balance_floodplain_with_inflow():
    sc = S.floodplain(n=128, h=25.0, seed=4, precision=64)
    sim = orc.OracleSim(sc)
    m0 = sim.mass()
    sim.run(400)
    V = sim.mass()
    assert abs(V - m0 - sim.inflow() - sim.ledger()) <= 1e-12 * V
    p = sc["params"]
    Q = lambda t: p["q_base"] + (p["q_peak"] - p["q_base"]) * math.exp(
        -(t - p["t_peak"]) ** 2 / (2 * p["sigma_t"] ** 2))
    ref = quad(Q, 0.0, sim.time(), epsrel=1e-12)[0]
    assert abs(sim.inflow() - ref) <= 1e-10 * ref


def test_uniform_source_raises_level_uniformly_at_rest():
    n = 12
    sc = _uniform(n, n, 10.0, 1.0, inlet=(0, 0, n, n), q_base=2.0, q_peak=2.0)
    sim = orc.OracleSim(sc, periodic=True)
    for _ in range(5):
        sim.step(0.5)
    H, Qx, Qy = sim.state()
    expect = 1.0 + 5 * 0.5 * 2.0 / (n * n * 100.0)
    assert np.allclose(H, expect, rtol=0, atol=1e-14)
    assert np.abs(Qx).max() == 0.0 and np.abs(Qy).max() == 0.0


# ---------------------------------------------------------------- force terms (periodic)

def test_friction_decay_converges_to_manning_ode():
    """Uniform flow under Manning friction alone: dU/dt = -c|U|U/H^(4/3),
    U(t) = U0/(1 + c U0 t/H^(4/3)).  The point-implicit friction factor is
    first-order accurate in tau (it stays L-stable on thin films), so the
    error must halve with tau."""
    H, U0, nM, T = 1.5, 2.0, 0.05, 200.0
    c = A.G * nM * nM / H ** (4.0 / 3.0)
    exact = U0 / (1.0 + c * U0 * T)
    errs = []
    for tau in (2.0, 1.0, 0.5):
        sc = _uniform(6, 6, 10.0, H, ux=U0 * 0.6, uy=U0 * 0.8,
                      n_manning=np.full((6, 6), nM))
        sim = orc.OracleSim(sc, periodic=True)
        for _ in range(int(T / tau)):
            sim.step(tau)
        _, Qx, Qy = sim.state()
        speed = np.hypot(Qx, Qy) / H
        assert np.ptp(speed) < 1e-14
        assert np.allclose(Qy / Qx, 0.8 / 0.6, rtol=1e-12)   # direction kept
        errs.append(abs(speed.mean() - exact) / exact)
    assert errs[0] < 0.01
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def test_coriolis_inertial_circle():
    f, U0, tau = 1e-3, 1.5, 5.0
    sc = _uniform(5, 5, 10.0, 2.0, ux=U0, f_cor=f)
    sim = orc.OracleSim(sc, periodic=True)
    n = 400
    for _ in range(n):
        sim.step(tau)
    _, Qx, Qy = sim.state()
    ux, uy = Qx[0, 0] / 2.0, Qy[0, 0] / 2.0
    t = n * tau
    assert abs(math.hypot(ux, uy) - U0) < 1e-5 * U0
    # dU/dt = f (U_y, -U_x): clockwise rotation at rate f for f > 0
    assert abs(ux - U0 * math.cos(f * t)) < 2e-3 * U0
    assert abs(uy + U0 * math.sin(f * t)) < 2e-3 * U0


def test_wind_drag_matches_ode():
    W, H, kap, tau = 10.0, 0.05, 1e-3, 0.5      # H below h_wind: floor applies
    sc = _uniform(5, 5, 10.0, H, ux=0.0, wind_x=W, wind_kappa=kap, h_wind=0.1)
    sim = orc.OracleSim(sc, periodic=True)
    n = 100
    for _ in range(n):
        sim.step(tau)
    u = sim.state()[1][0, 0] / H
    k = kap / 0.1
    exact = W - W / (1.0 + k * W * n * tau)       # d(W-u)/dt = -k (W-u)^2
    assert abs(u - exact) < 1e-4 * W
    assert abs(sim.state()[2]).max() == 0.0


def test_viscous_shear_mode_lagrangian_stage_eigenvalue():
    """U_x = sin(k y) is an eigenvector of the discrete Laplacian with
    eigenvalue -(2 - 2 cos kh)/h^2; the predictor-corrector then multiplies
    it by 1 + tau lam + (tau lam)^2/2."""
    n, h, nu, tau, H = 32, 2.0, 3.0, 0.1, 1.0
    y = (np.arange(n) + 0.5) * h
    k = 2 * math.pi * 3 / (n * h)
    ux = np.repeat(np.sin(k * y)[:, None], n, axis=1)
    sc = _uniform(n, n, h, H, nu=nu)
    sc["Qx0"] = H * ux
    sim = orc.OracleSim(sc, periodic=True)
    sim.step(tau)
    lam = -nu * (2 - 2 * math.cos(k * h)) / h**2
    ul = sim.field(orc.F_ULX)
    assert np.allclose(ul, ux * (1 + tau * lam + 0.5 * (tau * lam) ** 2), atol=1e-14)
    assert np.abs(sim.field(orc.F_ULY)).max() < 1e-15


# ---------------------------------------------------------------- stage III properties

def test_uniform_flow_fluxes_are_physical_fluxes():
    H, u, v = 1.7, 0.8, -0.3
    sc = _uniform(8, 6, 5.0, H, ux=u, uy=v)
    sim = orc.OracleSim(sc, periodic=True)
    sim.step(0.1)
    FH, Fn, Ft = sim.faces(0)
    assert np.allclose(FH, H * u, atol=1e-14) and np.allclose(Fn, H * u * u, atol=1e-14)
    assert np.allclose(Ft, H * u * v, atol=1e-14)
    FH, Fn, Ft = sim.faces(1)
    assert np.allclose(FH, H * v, atol=1e-14) and np.allclose(Fn, H * v * v, atol=1e-14)
    assert np.allclose(Ft, H * u * v, atol=1e-14)


def test_wall_faces_carry_no_mass():
    sc = S.random_state(20, 14, seed=3, precision=64)
    sim = orc.OracleSim(sc)
    sim.step()
    FH = sim.faces(0)[0]
    assert np.abs(FH[:, 0]).max() == 0.0 and np.abs(FH[:, -1]).max() == 0.0
    FH = sim.faces(1)[0]
    assert np.abs(FH[0, :]).max() == 0.0 and np.abs(FH[-1, :]).max() == 0.0


@pytest.mark.parametrize("lim", [0, 1, 2])
def test_limiters_keep_passive_tangential_velocity_bounded(lim):
    """In 1D flow the tangential velocity is advected passively: a TVD scheme
    creates no new extrema; sharper limiters track the exact shift better."""
    n, h, H, u = 200, 1.0, 1.0, 1.0
    sc = _uniform(n, 1, h, H, ux=u, limiter=lim)
    x = (np.arange(n) + 0.5) * h
    v0 = np.where((x > 40) & (x < 80), 1.0, 0.0) + np.where((x > 100) & (x < 140), np.sin((x - 100) / 40 * np.pi), 0.0)
    sc["Qy0"] = (H * v0)[None, :]
    sim = orc.OracleSim(sc, periodic=True)
    for _ in range(300):
        sim.step(0.1)
    v = sim.state()[2][0] / H
    assert v.max() <= 1.0 + 1e-12 and v.min() >= -1e-12


def _advect_tangential(lim):
    n, h, H, u = 200, 1.0, 1.0, 1.0
    sc = _uniform(n, 1, h, H, ux=u, limiter=lim)
    x = (np.arange(n) + 0.5) * h
    v0 = np.where((x > 40) & (x < 80), 1.0, 0.0) + np.where((x > 100) & (x < 140), np.sin((x - 100) / 40 * np.pi), 0.0)
    sc["Qy0"] = (H * v0)[None, :]
    sim = orc.OracleSim(sc, periodic=True)
    for _ in range(300):
        sim.step(0.1)
    return sim.state()[2][0] / H


def test_limiter_sharpness_order():
    errs = []
    for lim in (0, 1, 2):
        v = _advect_tangential(lim)
        x = (np.arange(200) + 0.5) - 30.0
        ve = np.where((x > 40) & (x < 80), 1.0, 0.0) + np.where((x > 100) & (x < 140), np.sin((x - 100) / 40 * np.pi), 0.0)
        errs.append(np.abs(v - ve).sum())
    assert errs[2] < errs[1] < errs[0]


def test_momentum_conserved_on_periodic_flat_bed():
    rng = np.random.default_rng(7)
    n = 24
    sc = _uniform(n, n, 4.0, 1.0)
    sc["H0"] = 1.0 + 0.5 * rng.uniform(size=(n, n))
    sc["Qx0"] = sc["H0"] * rng.normal(0, 0.3, size=(n, n))
    sc["Qy0"] = sc["H0"] * rng.normal(0, 0.3, size=(n, n))
    sim = orc.OracleSim(sc, periodic=True)
    px0, py0 = sc["Qx0"].sum(), sc["Qy0"].sum()
    m0 = sim.mass()
    sim.run(50)
    H, Qx, Qy = sim.state()
    assert H.min() > 0.1
    assert abs(Qx.sum() - px0) < 1e-11 and abs(Qy.sum() - py0) < 1e-11
    assert abs(sim.mass() - m0) < 1e-12 * m0


def test_transpose_and_mirror_symmetry():
    sc = S.random_state(30, 30, seed=11, precision=64, f_cor=0.0, wind_x=3.0, wind_y=3.0)
    a = orc.OracleSim(sc)
    a.run(40)
    scT = dict(sc)
    for k in ("b", "n_manning", "H0"):
        scT[k] = sc[k].T.copy()
    scT["Qx0"], scT["Qy0"] = sc["Qy0"].T.copy(), sc["Qx0"].T.copy()
    bT = orc.OracleSim(scT)
    bT.run(40)
    Ha, Qxa, Qya = a.state()
    Hb, Qxb, Qyb = bT.state()
    assert np.abs(Ha - Hb.T).max() < 1e-10 and np.abs(Qxa - Qyb.T).max() < 1e-10
    assert np.abs(Qya - Qxb.T).max() < 1e-10
    sc2 = S.random_state(30, 20, seed=12, precision=64, f_cor=0.0, wind_x=0.0, wind_y=2.0)
    c = orc.OracleSim(sc2)
    c.run(40)
    scM = dict(sc2)
    for k in ("b", "n_manning", "H0", "Qy0"):
        scM[k] = sc2[k][:, ::-1].copy()
    scM["Qx0"] = -sc2["Qx0"][:, ::-1]
    d = orc.OracleSim(scM)
    d.run(40)
    Hc, Qxc, Qyc = c.state()
    Hd, Qxd, Qyd = d.state()
    assert np.abs(Hc - Hd[:, ::-1]).max() < 1e-10
    assert np.abs(Qxc + Qxd[:, ::-1]).max() < 1e-10
    assert np.abs(Qyc - Qyd[:, ::-1]).max() < 1e-10


# ---------------------------------------------------------------- time step

def test_time_step_formula_on_hand_built_states():
    g, h, K = A.G, 10.0, 0.4
    sim = orc.OracleSim(_uniform(4, 4, h, 4.0), periodic=True)
    assert abs(sim.next_tau() - K * h / math.sqrt(g * 4.0)) < 1e-14
    sim = orc.OracleSim(_uniform(4, 4, h, 4.0, ux=3.0, uy=-1.0), periodic=True)
    assert abs(sim.next_tau() - K * h / (3.0 + math.sqrt(g * 4.0))) < 1e-14
    # bottom friction is part of F (Eq. 4): F_fric = -(c_f / H^(4/3)) U |U|.
    # Worked by hand: H = 1, c_f = g n_M^2 = 5, U = (-2, 0), h = 10:
    # F = (20, 0), U_p = |-2 + sqrt(10 * 20)| = 10 sqrt2 - 2 > U_s = 2 + sqrt g,
    # tau = K h / U_p = 4 / (10 sqrt2 - 2)
    sim = orc.OracleSim(_uniform(4, 4, h, 1.0, ux=-2.0, n_manning=np.full((4, 4), math.sqrt(5.0 / g))),
                        periodic=True)
    assert abs(sim.next_tau() - 4.0 / (10.0 * math.sqrt(2.0) - 2.0)) < 1e-14
    # H = 1/8 (H^(4/3) = 1/16), c_f = 1/4, U = (0, 3), h = 4: F_y = -4 * 3 * 3 = -36,
    # U_p = |3 - sqrt(4 * 36)| = 9 (the sign of F counts), U_s = 3 + sqrt(g/8),
    # tau = 0.4 * 4 / 9
    nm = np.full((4, 4), math.sqrt(0.25 / g))
    sim = orc.OracleSim(_uniform(4, 4, 4.0, 0.125, uy=3.0, n_manning=nm), periodic=True)
    assert abs(sim.next_tau() - 1.6 / 9.0) < 1e-14
    # the same film moving along x with Coriolis f = 30: F = (-36, -90),
    # U_p = max(|3 - 12|, |0 - sqrt(4 * 90)|) = sqrt(360), tau = 1.6 / sqrt(360)
    sim = orc.OracleSim(_uniform(4, 4, 4.0, 0.125, ux=3.0, n_manning=nm, f_cor=30.0), periodic=True)
    assert abs(sim.next_tau() - 1.6 / math.sqrt(360.0)) < 1e-14
    # wind force F = kappa (W-U)|W-U|/max(H, h_w) enters U_p = |U + sgn(F) sqrt(h|F|)|
    kap, W = 0.05, 30.0
    sim = orc.OracleSim(_uniform(4, 4, h, 0.5, ux=0.5, wind_x=W, wind_kappa=kap), periodic=True)
    F = kap * (W - 0.5) ** 2 / 0.5
    up = 0.5 + math.sqrt(h * F)
    us = 0.5 + math.sqrt(g * 0.5)
    assert up > us
    assert abs(sim.next_tau() - K * h / up) < 1e-13
    # viscous and tau_max caps, dry domain
    sim = orc.OracleSim(_uniform(4, 4, h, 4.0, nu=50.0), periodic=True)
    assert abs(sim.next_tau() - h * h / (4 * 50.0)) < 1e-14
    sc = _uniform(4, 4, h, 0.0, tau_max=2.5)
    assert orc.OracleSim(sc).next_tau() == 2.5


# ---------------------------------------------------------------- K1 wet-block rule

def _brute_active(H, src, tx, ty, eps):
    wet = (H > eps) | src
    dil = wet.copy()
    dil[1:, :] |= wet[:-1, :]
    dil[:-1, :] |= wet[1:, :]
    dil[:, 1:] |= wet[:, :-1]
    dil[:, :-1] |= wet[:, 1:]
    ny, nx = H.shape
    nty, ntx = -(-ny // ty), -(-nx // tx)
    out = np.zeros((nty, ntx), bool)
    for tj in range(nty):
        for ti in range(ntx):
            out[tj, ti] = dil[tj * ty:(tj + 1) * ty, ti * tx:(ti + 1) * tx].any()
    return out


@pytest.mark.parametrize("shape,tile", [((37, 53), (16, 16)), ((64, 64), (32, 8)), ((9, 70), (64, 4))])
def test_k1_rule_matches_brute_force(shape, tile):
    rng = np.random.default_rng(sum(shape))
    for trial in range(10):
        H = np.where(rng.uniform(size=shape) < 0.02, rng.uniform(0, 1e-3, size=shape), 0.0)
        src = rng.uniform(size=shape) < 0.002
        own, ring = orc.tile_flags(H, tile[0], tile[1], 1e-4, src)
        act = _brute_active(H, src, tile[0], tile[1], 1e-4)
        assert np.array_equal((own | ring).astype(bool), act)
        wet = (H > 1e-4) | src
        for tj in range(own.shape[0]):
            for ti in range(own.shape[1]):
                blk = wet[tj * tile[1]:(tj + 1) * tile[1], ti * tile[0]:(ti + 1) * tile[0]]
                assert own[tj, ti] == int(blk.any())


def _golden_k1_cases():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "k1_wet_blocks.txt")
    cases, cur = [], None
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "case":
            cur = dict(name=f[1], H=np.zeros((8, 12)), src=np.zeros((8, 12), bool))
            cases.append(cur)
        elif f[0] == "eps":
            cur["eps"] = float(f[1])
        elif f[0] == "cell":
            cur["H"][int(f[2]), int(f[1])] = float(f[3])
        elif f[0] == "source":
            cur["src"][int(f[2]), int(f[1])] = True
        else:
            cur[f[0]] = np.array([int(v) for v in f[1:]]).reshape(2, 3)
    return cases


def test_k1_rule_matches_hand_worked_golden_cases():
    """Two 12 x 8 grids of 4 x 4 tiles whose own and ring flags were worked
    out by hand from the K1 rule (tests/golden/k1_wet_blocks.txt)."""
    cases = _golden_k1_cases()
    assert [c["name"] for c in cases] == ["A", "B"]
    for c in cases:
        own, ring = orc.tile_flags(c["H"], 4, 4, c["eps"], c["src"])
        assert np.array_equal(own, c["own"]), c["name"]
        assert np.array_equal(ring, c["ring"]), c["name"]


def test_dry_cells_away_from_water_are_untouched():
    """The exactness behind skipping: a cell whose 4 face neighbours and
    itself are dry and not sources is left unchanged by a step."""
    sc = S.floodplain(n=96, h=25.0, seed=9, precision=64)
    sim = orc.OracleSim(sc)
    sim.run(30)
    H0, Qx0, Qy0 = sim.state()
    sim.step()
    H1, Qx1, Qy1 = sim.state()
    wet = (H0 > 1e-4)
    p = sc["params"]["inlet"]
    wet[p[1]:p[1] + p[3], p[0]:p[0] + p[2]] = True
    dil = wet.copy()
    dil[1:] |= wet[:-1]
    dil[:-1] |= wet[1:]
    dil[:, 1:] |= wet[:, :-1]
    dil[:, :-1] |= wet[:, 1:]
    far = ~dil
    assert far.sum() > 1000
    assert np.array_equal(H1[far], H0[far]) and np.all(Qx1[far] == 0) and np.all(Qy1[far] == 0)
