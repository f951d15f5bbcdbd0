"""Pins of the nested-grid oracle (two-way zoom-in, arXiv 1705.00614 Sec. 2.2
and Sec. 5), all on the CPU.  The coupling reading (coarse-first
subcycling, frame from the coarse layers, restriction by the mean, reflux of
the face-flux mismatch) is checked against what it must satisfy:
  - r = 1 with the same bed is the single grid (frame, indices, restriction);
  - the frame carries the coarse velocity at the fine depth;
  - volume is conserved to rounding on a wet domain with inflow (reflux
    signs and targets), and dropping the reflux breaks that;
  - covered coarse cells equal the mean of their fine cells (nothing but
    the restriction writes them);
  - a wet lake at rest stays at rest with a patch over rough fine relief;
  - the transpose symmetry of a symmetric problem survives (x/y mapping of
    the reflux momentum components);
  - inside the patch the nested solution is closer to a fine single grid
    than the coarse grid alone (the patch actually refines).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle.nest import OracleNest
from paper_1705_00614_amd import scenarios as S


def _flat(n, h, H, **prm):
    z = np.zeros((n, n))
    p = S.base_params(precision=64, **prm)
    return dict(name="flat", nx=n, ny=n, h=h, b=z.copy(), n_manning=z.copy(), solid=None,
                H0=np.full((n, n), float(H)), Qx0=z.copy(), Qy0=z.copy(), params=p)


def _hump(n, h, H=2.0, amp=0.5, cx=0.5, cy=0.5, w=0.12):
    sc = _flat(n, h, H)
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    sc["H0"] = H + amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * w * w))
    return sc


def test_r1_same_bed_is_the_single_grid():
    sc = S.random_state(40, 36, seed=21, wet_frac=0.7, precision=64)
    nest = S.nest(sc, [(9, 8, 14, 12)], r=1, detail=0.0)
    assert np.array_equal(nest["coarse"]["b"], sc["b"])
    o = orc.OracleSim(sc)
    tau = 0.8 * o.next_tau()
    N = OracleNest(nest["coarse"], nest["patches"], r=1)
    for _ in range(25):
        o.step(tau)
        N.step(tau)
    a, b = o.state(), N.coarse_state()
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-11 * max(1.0, np.abs(x).max())
    # the patch interior is the same cells
    Hp = N.patch_state(0)[0]
    assert np.abs(Hp - a[0][8:20, 9:23]).max() <= 1e-11 * np.abs(a[0]).max()


def test_frame_carries_the_coarse_velocity():
    """The frame of a patch takes the covering coarse cell's velocity at the
    fine depth H_f = max(0, H_c + b_c - b_f): on a high spot of the fine bed
    (a film of 1 cm under 2 m of coarse water) the discharge is 1 cm times
    the coarse velocity, not the coarse column's discharge, which would move
    that film at 200 times the flow's speed."""
    n, r = 24, 4
    sc = _flat(n, 10.0, 2.0)
    ux, uy = 0.5, -0.2
    sc["Qx0"] = np.full((n, n), 2.0 * ux)
    sc["Qy0"] = np.full((n, n), 2.0 * uy)
    nest = S.nest(sc, [(8, 8, 6, 6)], r=r, detail=0.0)
    P = nest["patches"][0]
    bf = np.zeros_like(P["b"])
    bf[1, 7] = 1.99           # frame rows are 0..4 and the last 5
    bf[3, 2] = 2.5            # above the coarse level: dry
    P["b"] = bf
    N = OracleNest(nest["coarse"], nest["patches"], r=r)
    H0, Qx0, Qy0 = sc["H0"], sc["Qx0"], sc["Qy0"]
    H, Qx, Qy = N._frame(N.P[0], H0, Qx0, Qy0, H0, Qx0, Qy0, 0.0)
    G = 5
    frame = np.ones_like(H, dtype=bool)
    frame[G:-G, G:-G] = False
    assert abs(H[1, 7] - 0.01) < 1e-12 and abs(Qx[1, 7] - 0.01 * ux) < 1e-14 and abs(Qy[1, 7] - 0.01 * uy) < 1e-14
    assert H[3, 2] == 0.0 and Qx[3, 2] == 0.0 and Qy[3, 2] == 0.0
    wet = frame & (H > 0)
    assert np.abs(Qx[wet] / H[wet] - ux).max() < 1e-14 and np.abs(Qy[wet] / H[wet] - uy).max() < 1e-14


def test_ring_update_keeps_momentum_out_of_films():
    """The reflux into a ring cell: depth clamped at 0 (the clamp returned
    for the ledger), discharge zeroed where the cell ends dry, and the
    momentum part weighted from 0 at 5 cm of corrected depth to 1 at 10 cm;
    cells off the ring are untouched."""
    N = _wet_nest()
    H = np.array([[0.0, 0.02, 1.0, 0.3, 2.0, 0.07]])
    Qx = np.array([[0.0, 0.001, 0.5, 0.1, 0.7, 0.01]])
    Qy = -Qx
    dH = np.array([[0.0003, 0.01, 0.01, -0.5, 0.4, 0.005]])
    dQx = np.array([[0.002, 0.003, 0.02, 0.04, 0.05, 0.004]])
    dQy = 2.0 * dQx
    ring = np.array([[True, True, True, True, False, True]])
    H2, X2, Y2, clamped = N.ring_update(H, Qx, Qy, dH, dQx, dQy, ring)
    # a film (3e-4 m after the reflux) keeps no momentum; a 3 cm cell keeps
    # its own but takes none; a 1 m cell takes all; a 7.5 cm cell half; a
    # drained cell is dry
    assert H2[0, 0] == 0.0003 and X2[0, 0] == 0.0 and Y2[0, 0] == 0.0
    assert H2[0, 1] == 0.03 and X2[0, 1] == 0.001 and Y2[0, 1] == -0.001
    assert abs(H2[0, 2] - 1.01) < 1e-15 and abs(X2[0, 2] - 0.52) < 1e-15 and abs(Y2[0, 2] + 0.46) < 1e-15
    assert abs(H2[0, 5] - 0.075) < 1e-15 and abs(X2[0, 5] - 0.012) < 1e-14 and abs(Y2[0, 5] + 0.006) < 1e-14
    assert H2[0, 3] == 0.0 and X2[0, 3] == 0.0 and Y2[0, 3] == 0.0
    assert abs(clamped - 0.2) < 1e-15
    assert H2[0, 4] == 2.0 and X2[0, 4] == 0.7 and Y2[0, 4] == -0.7


def _wet_nest(r=4, feedback=True, reflux=True):
    sc = S.floodplain(n=48, h=50.0, seed=4, q_peak=800.0, t_peak=300.0, sigma_t=200.0,
                      inlet_cells=4, precision=64)
    sc["H0"] = np.maximum(sc["b"].max() + 1.0 - sc["b"], 0.0)     # every cell wet
    nest = S.nest(sc, [(14, 10, 12, 10), (30, 26, 8, 12)], r=r, seed=9)
    N = OracleNest(nest["coarse"], nest["patches"], r=r, feedback=feedback)
    N._reflux = reflux
    return N


def test_volume_conserved_with_inflow():
    N = _wet_nest()
    V0 = N.volume()
    for k in range(30):
        N.step()
        assert min(p["sim"].state()[0].min() for p in N.P) > 0.0
        err = N.volume() - V0 - N.inflow() - N.total_ledger()
        assert abs(err) <= 1e-12 * V0, (k, err / V0)
        # the next coarse step respects the CFL step of the coarse layer after the feedback
        assert N.tau_c <= N.c.next_tau() and N.tau_f == N.tau_c / N.r
    assert N.inflow() > 0.0 and N.total_ledger() == 0.0


def test_volume_not_conserved_without_reflux():
    N = _wet_nest(reflux=False)
    V0 = N.volume()
    N.run(30)
    assert abs(N.volume() - V0 - N.inflow()) > 1e-9 * V0


def test_covered_cells_are_the_mean_of_the_fine_cells():
    N = _wet_nest()
    N.run(10)
    H, Qx, Qy = N.coarse_state()
    for k, P in enumerate(N.P):
        p = P["spec"]
        Hf, Qxf, Qyf = N.patch_state(k)
        r = N.r
        sl = (slice(p["cj0"], p["cj0"] + p["ch"]), slice(p["ci0"], p["ci0"] + p["cw"]))
        for c, f in ((H, Hf), (Qx, Qxf), (Qy, Qyf)):
            m = f.reshape(p["ch"], r, p["cw"], r).mean(axis=(1, 3))
            assert np.array_equal(c[sl], m)


def test_lake_at_rest_with_patch():
    sc = S.lake_at_rest(n=48, h=20.0, seed=6, relief=8.0, eta0=9.5)
    nest = S.nest(sc, [(12, 14, 16, 12)], r=4, seed=2, detail=1.0)
    N = OracleNest(nest["coarse"], nest["patches"], r=4)
    assert min(p["sim"].state()[0][5:-5, 5:-5].min() for p in N.P) > 0.0
    N.run(40)
    H, Qx, Qy = N.coarse_state()
    eta = H + nest["coarse"]["b"]
    assert np.abs(eta - 9.5).max() <= 1e-10
    assert np.abs(Qx).max() <= 1e-10 and np.abs(Qy).max() <= 1e-10
    Hf, Qxf, Qyf = N.patch_state(0)
    bf = nest["patches"][0]["b"][5:-5, 5:-5]
    assert np.abs(Hf + bf - 9.5).max() <= 1e-10
    assert np.abs(Qxf).max() <= 1e-10 and np.abs(Qyf).max() <= 1e-10


def test_transpose_symmetry_survives_nesting():
    sc = _hump(40, 20.0, cx=0.4, cy=0.4)
    nest = S.nest(sc, [(10, 10, 16, 16)], r=2, detail=0.0)
    N = OracleNest(nest["coarse"], nest["patches"], r=2)
    N.run(30)
    H, Qx, Qy = N.coarse_state()
    s = np.abs(H).max()
    assert np.abs(H - H.T).max() <= 1e-12 * s
    q = np.abs(Qx).max()
    assert q > 1e-3
    assert np.abs(Qx - Qy.T).max() <= 1e-11 * q
    Hf, Qxf, Qyf = N.patch_state(0)
    assert np.abs(Qxf - Qyf.T).max() <= 1e-11 * q


def test_patch_refines_towards_the_fine_grid():
    n, h, r = 32, 40.0, 4
    coarse = _hump(n, h, amp=0.8, w=0.08)
    tau = 1.0
    steps = 40
    # fine single grid over the whole domain, same initial function sampled finely
    fine = _hump(n * r, h / r, amp=0.8, w=0.08)
    F = orc.OracleSim(fine)
    for _ in range(steps * r):
        F.step(tau / r)
    Hf_ref = F.state()[0]
    C = orc.OracleSim(coarse)
    for _ in range(steps):
        C.step(tau)
    Hc_only = C.state()[0]
    box = (10, 10, 12, 12)
    nest = S.nest(coarse, [box], r=r, detail=0.0)
    # the patch starts from the finely sampled hump, not the coarse blocks
    ci0, cj0, cw, ch = box
    p = nest["patches"][0]
    p["H0"] = fine["H0"][cj0 * r:(cj0 + ch) * r, ci0 * r:(ci0 + cw) * r].copy()
    nest["coarse"]["H0"][cj0:cj0 + ch, ci0:ci0 + cw] = p["H0"].reshape(ch, r, cw, r).mean(axis=(1, 3))
    N = OracleNest(nest["coarse"], nest["patches"], r=r)
    N.run(steps, tau)
    Hn = N.patch_state(0)[0]
    ref = Hf_ref[cj0 * r:(cj0 + ch) * r, ci0 * r:(ci0 + cw) * r]
    coarse_up = np.kron(Hc_only[cj0:cj0 + ch, ci0:ci0 + cw], np.ones((r, r)))
    e_nest = np.abs(Hn - ref).mean()
    e_coarse = np.abs(coarse_up - ref).mean()
    assert e_nest < 0.5 * e_coarse, (e_nest, e_coarse)


def test_rejects_bad_layouts():
    sc = _flat(30, 10.0, 1.0)
    ok = S.nest(sc, [(4, 4, 6, 6)], r=2, detail=0.0)
    with pytest.raises(ValueError):
        OracleNest(ok["coarse"], [dict(ok["patches"][0], ci0=1)], r=2)          # frame leaves the grid
    two = S.nest(sc, [(4, 4, 6, 6), (10, 4, 6, 6)], r=2, detail=0.0)
    with pytest.raises(ValueError):
        OracleNest(two["coarse"], two["patches"], r=2)                          # no gap between patches
