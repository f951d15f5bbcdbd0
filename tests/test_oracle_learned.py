"""Pins of the learned-correction oracle (CPU): the convolution against its
definition written as loops, back-propagation against central differences,
bfloat16 rounding against hand-worked values, the first Adam step, and the
flux-correction hook of the step oracle against what a face correction must
do to the two cells that share the face."""
import numpy as np
import pytest

from oracle import learned as LN
from oracle import oracle as orc
from paper_1705_00614_amd import scenarios as S


def test_conv_matches_loops():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 6, 2))
    w = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    y = LN.conv3x3(x, w, b)
    assert y.shape == (2, 3, 4, 3)
    for n in range(2):
        for i in range(3):
            for j in range(4):
                for o in range(3):
                    s = b[o]
                    for c in range(2):
                        for dy in range(3):
                            for dx in range(3):
                                s += x[n, i + dy, j + dx, c] * w[o, c, dy, dx]
                    assert abs(y[n, i, j, o] - s) < 1e-12


def test_backward_matches_central_differences():
    rng = np.random.default_rng(2)
    W, b = LN.init_params(3)
    W[-1] = W[-1] * 10.0
    x = rng.normal(size=(2, 11, 11, 6))
    y = rng.normal(size=(2, 3, 3, 6))
    mask = (rng.uniform(size=y.shape) > 0.3).astype(float)

    def loss(Wl, bl):
        out, _ = LN.forward(x, Wl, bl, bf=False)
        return LN.loss_and_grad(out, y, mask)[0]

    out, acts = LN.forward(x, W, b, bf=False)
    _, g = LN.loss_and_grad(out, y, mask)
    dW, db = LN.backward(g, acts, W, bf=False)
    h = 1e-6
    for k in range(4):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W[k].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[k][idx] += h
            Wm[k][idx] -= h
            fd = (loss(Wp, b) - loss(Wm, b)) / (2 * h)
            assert abs(fd - dW[k][idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, idx, fd, dW[k][idx])
        o = int(rng.integers(0, len(b[k])))
        bp = [v.copy() for v in b]
        bm = [v.copy() for v in b]
        bp[k][o] += h
        bm[k][o] -= h
        fd = (loss(W, bp) - loss(W, bm)) / (2 * h)
        assert abs(fd - db[k][o]) <= 1e-6 * max(1e-3, abs(fd))


def test_bf16_rounding_values():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -2.5, 3.0e38, 1e-40])
    r = LN.bf16(v)
    # 8 significant bits: halfway cases go to the even neighbour
    assert r[0] == 1.0
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6
    assert r[4] == -2.5
    assert np.isfinite(r[5])
    assert np.all(np.abs(LN.bf16(np.linspace(-4, 4, 1001)) - np.linspace(-4, 4, 1001)) <= 2 ** -8 * 4)


def test_first_adam_step_moves_by_lr_sign():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    opt = LN.Adam(p, lr=0.01)
    q = opt.step(p, g)[0]
    assert np.allclose(q - p[0], -0.01 * np.sign(g[0]), rtol=1e-4)


def _wet_basin(n=12, seed=3):
    sc = S.random_state(n, n, seed=seed, wet_frac=1.0, precision=64)
    sc["H0"] = sc["H0"] + 0.5
    return sc


def test_zero_correction_changes_nothing():
    sc = _wet_basin()
    a, b = orc.OracleSim(sc), orc.OracleSim(sc)
    z = np.zeros((3, sc["ny"], sc["nx"]))
    b.set_correction(z, z)
    tau = 0.5 * a.next_tau()
    for _ in range(5):
        a.step(tau)
        b.step(tau)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


def test_face_correction_moves_volume_between_the_two_cells():
    sc = _wet_basin()
    n = sc["nx"]
    a, b = orc.OracleSim(sc), orc.OracleSim(sc)
    tau = 0.5 * a.next_tau()
    dE = np.zeros((3, n, n))
    dN = np.zeros((3, n, n))
    dE[0, 4, 5] = 0.01         # east face of cell (j=4, i=5): towards (4, 6)
    dN[0, 7, 2] = -0.02        # north face of (7, 2): from (8, 2) into (7, 2)
    dE[1, 3, 3] = 0.05         # x-momentum through the east face of (3, 3)
    b.set_correction(dE, dN)
    a.step(tau)
    b.step(tau)
    dH = b.state()[0] - a.state()[0]
    dQx = b.state()[1] - a.state()[1]
    r = tau / sc["h"]
    exp = np.zeros((n, n))
    exp[4, 5] -= r * 0.01
    exp[4, 6] += r * 0.01
    exp[7, 2] += r * 0.02
    exp[8, 2] -= r * 0.02
    assert np.abs(dH - exp).max() <= 1e-14
    assert abs(dQx[3, 3] + r * 0.05) <= 1e-14 and abs(dQx[3, 4] - r * 0.05) <= 1e-14
    assert abs(b.mass() - a.mass()) <= 1e-12 * a.mass()


def test_mass_correction_from_a_dry_cell_or_through_a_wall_is_dropped():
    sc = _wet_basin()
    n = sc["nx"]
    sc["H0"][:, 0] = 0.0
    sc["Qx0"][:, 0] = 0.0
    sc["Qy0"][:, 0] = 0.0
    a, b = orc.OracleSim(sc), orc.OracleSim(sc)
    tau = 0.2 * a.next_tau()
    dE = np.zeros((3, n, n))
    dE[0, 5, 0] = 0.01             # out of the dry cell (5, 0): dropped
    dE[0, 6, 0] = -0.01            # into the dry cell from the wet (6, 1): kept
    dE[0, 2, n - 1] = 0.3          # east wall face: no effect
    b.set_correction(dE, None)
    a.step(tau)
    b.step(tau)
    dH = b.state()[0] - a.state()[0]
    r = tau / sc["h"]
    assert dH[5, 0] == 0.0 and dH[5, 1] == 0.0
    assert abs(dH[6, 0] - r * 0.01) <= 1e-14 and abs(dH[6, 1] + r * 0.01) <= 1e-14
    assert np.abs(dH[2, n - 2:]).max() == 0.0


def test_crops_mirror_and_scatter_roundtrip():
    rng = np.random.default_rng(4)
    feat = rng.normal(size=(10, 12, 6))
    c = LN.crops(feat, [(0, 0), (2, 1)], 4)
    assert c.shape == (2, 13, 13, 6)
    # window starts 1 + 4 cells before the tile
    assert np.array_equal(c[0, 5:9, 5:9], feat[0:4, 0:4])
    assert np.array_equal(c[0, 4, 5:9], feat[0, 0:4])          # mirror: cell -1 shows cell 0
    assert np.array_equal(c[0, 0, 5:9], feat[4, 0:4])          # cell -5 shows cell 4
    assert np.array_equal(c[1, 4:9, 4:9], feat[3:8, 7:12])     # tile (2, 1): cells 7.. and 3..
    assert np.array_equal(c[1, 5:9, 9], feat[4:8, 11])          # cell 12 shows 11
    out = rng.normal(size=(2, 5, 5, 6))
    dE, dN = LN.corrections(out, [(0, 0), (2, 1)], 4, 10, 12, np.ones(6))
    assert np.array_equal(dE[1, 3:8, 7:12], out[1, :, :, 1])
    assert np.array_equal(dN[2, 0:4, 0:4], out[0, 1:, 1:, 5])


def test_momentum_correction_needs_both_cells_wet():
    sc = _wet_basin()
    n = sc["nx"]
    sc["H0"][:, 0] = 0.0
    sc["Qx0"][:, 0] = 0.0
    sc["Qy0"][:, 0] = 0.0
    a, b = orc.OracleSim(sc), orc.OracleSim(sc)
    tau = 0.2 * a.next_tau()
    dE = np.zeros((3, n, n))
    dE[1, 5, 0] = 0.05            # x-momentum through the face between dry (5, 0) and wet (5, 1)
    dE[2, 7, 3] = 0.05            # y-momentum through a wet-wet face
    b.set_correction(dE, None)
    a.step(tau)
    b.step(tau)
    r = tau / sc["h"]
    dQx = b.state()[1] - a.state()[1]
    dQy = b.state()[2] - a.state()[2]
    assert dQx[5, 1] == 0.0 and dQx[5, 0] == 0.0
    assert abs(dQy[7, 3] + r * 0.05) <= 1e-14 and abs(dQy[7, 4] - r * 0.05) <= 1e-14


def test_momentum_correction_depth_threshold():
    sc = _wet_basin()
    n = sc["nx"]
    sc["H0"][7, 4] = 0.01          # wet but shallow
    a, b = orc.OracleSim(sc), orc.OracleSim(sc)
    b.set_correction_depth(0.05)
    tau = 0.1 * a.next_tau()
    dE = np.zeros((3, n, n))
    dE[1, 7, 3] = 0.05             # face between (7, 3) (deep) and (7, 4) (shallow): dropped
    dE[1, 2, 3] = 0.05             # deep-deep face: kept
    dE[0, 7, 3] = 0.01             # mass from the deep (7, 3) into the shallow (7, 4): kept
    dE2 = np.zeros((3, n, n))
    dE2[0, 7, 4] = 0.01            # mass out of the shallow (7, 4) through its east face: dropped
    a.set_correction(dE, None)
    b.set_correction(dE, None)
    a.step(tau)
    b.step(tau)
    r = tau / sc["h"]
    c = orc.OracleSim(sc)
    c.step(tau)
    dQa = a.state()[1] - c.state()[1]
    dQb = b.state()[1] - c.state()[1]
    assert abs(dQa[7, 3] + r * 0.05) <= 1e-14          # eps threshold: applied
    assert abs(dQb[7, 3]) <= 1e-14 and abs(dQb[7, 4]) <= 1e-14
    assert abs(dQb[2, 3] + r * 0.05) <= 1e-14
    dHb = b.state()[0] - c.state()[0]
    assert abs(dHb[7, 3] + r * 0.01) <= 1e-14
    d = orc.OracleSim(sc)
    d.set_correction_depth(0.05)
    d.set_correction(dE2, None)
    d.step(tau)
    assert np.array_equal(d.state()[0], c.state()[0])


def test_coarsen_takes_block_means_and_scales_the_inlet():
    """Host logic of the learned leg: the coarse scenario of a fine one has
    the r x r block means of bed, Manning n and state, the cell size times r,
    the step cap times r (the same cap in Courant units) and the inlet
    rectangle divided by r (at least one cell)."""
    from paper_1705_00614_amd import learned as LC
    sc = S.floodplain(n=64, h=25.0, seed=3, q_peak=500.0, t_peak=100.0, sigma_t=80.0, inlet_cells=6)
    sc["params"] = dict(sc["params"], tau_max=2.0)
    c = LC.coarsen(sc, 4)
    assert (c["nx"], c["ny"], c["h"]) == (16, 16, 100.0)
    for k in ("b", "n_manning", "H0", "Qx0", "Qy0"):
        blk = np.asarray(sc[k], dtype=np.float64).reshape(16, 4, 16, 4)
        assert np.allclose(c[k], blk.mean(axis=(1, 3)), rtol=0, atol=1e-12), k
    assert c["params"]["tau_max"] == 8.0
    i0, j0, ni, nj = sc["params"]["inlet"]
    assert c["params"]["inlet"] == (i0 // 4, j0 // 4, max(ni // 4, 1), max(nj // 4, 1))
