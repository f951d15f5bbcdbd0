"""Seeded synthetic inputs for the shallow-water solver.

This module only draws inputs (terrain, roughness, initial water, inlet and
hydrograph parameters); it holds none of the scheme's arithmetic, so both the
GPU library and the CPU oracle used by the tests can take their inputs from
it.  The real inputs of arXiv 1705.00614 (the Volga-Akhtuba digital terrain
model, hydrographs and gauge records, Sec. 2.2 and Sec. 5) are not available;
these generators stand in for them with the shapes the paper describes:
floodplain relief of a few metres cut by a deep meandering river bed, 25-50 m
cells, depths from centimetres to tens of metres, a large inflow from a
hydraulic structure, and a water/land ratio between a few and ~60 %.

Every scenario is a dict with keys
    nx, ny, h              grid and cell size [m]
    b, n_manning           (ny, nx) float64 bed elevation [m] and Manning n
    solid                  (ny, nx) uint8 closed-gate mask or None
    H0, Qx0, Qy0           (ny, nx) float64 initial depth and unit discharge
    params                 dict of physical and numerical constants
Random numbers come from NumPy's PCG64 generator seeded explicitly.
"""
import math

import numpy as np

G = 9.81
# Wind drag coefficient C_a rho_a / rho with C_a = 1.3e-3, rho_a = 1.225,
# rho = 1000 (typical open-water values; the paper names the factors only).
WIND_KAPPA = 1.3e-3 * 1.225 / 1000.0
# Coriolis parameter 2 Omega sin(phi) at about 48.7 N (Volgograd region).
F_COR = 2.0 * 7.2921e-5 * math.sin(math.radians(48.7))


def base_params(**over):
    p = dict(g=G, courant=0.4, eps=1e-4, tau_max=0.0, tau_min=0.0, nu=0.0,
             f_cor=0.0, wind_x=0.0, wind_y=0.0, wind_kappa=0.0, h_wind=0.1,
             limiter=0, inlet=None, q_base=0.0, q_peak=0.0, t_peak=0.0,
             sigma_t=0.0, precision=32)
    p.update(over)
    return p


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def fbm(ny, nx, hurst, seed, relief):
    """Fractional-Brownian relief by spectral synthesis: white noise, Fourier
    amplitudes scaled by |k|^-(hurst+1) with the mean mode removed, inverse
    transform, then scaled to [0, relief] metres."""
    noise = _rng(seed).standard_normal((ny, nx))
    spec = np.fft.rfft2(noise)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    amp[k > 0] = k[k > 0] ** (-(hurst + 1.0))
    z = np.fft.irfft2(spec * amp, s=(ny, nx))
    z -= z.min()
    z *= relief / max(z.max(), 1e-30)
    return z


def _centreline(n, h, rng):
    """Meandering river centre y_c(x) = L/2 + sum_k A_k sin(2 pi x/lambda_k + phi_k)."""
    L = n * h
    A = (rng.uniform(0.10, 0.20) * L, rng.uniform(0.02, 0.05) * L)
    lam = (rng.uniform(0.25, 0.50) * L, rng.uniform(0.08, 0.15) * L)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=2)
    x = (np.arange(n) + 0.5) * h
    yc = 0.5 * L + sum(A[k] * np.sin(2 * math.pi * x / lam[k] + phi[k]) for k in range(2))
    dyc = sum(A[k] * 2 * math.pi / lam[k] * np.cos(2 * math.pi * x / lam[k] + phi[k])
              for k in range(2))
    return yc, dyc


def floodplain_terrain(n, h=25.0, seed=0, relief=15.0, hurst=0.8,
                       channel_depth=8.0, channel_half_width=100.0):
    """fBm floodplain with a carved meandering channel draining in +x.

    Returns (b, n_manning, channel_mask, yc) with the channel bed at the
    running minimum (downstream) of the relief along the centre line minus
    channel_depth."""
    rng = _rng(seed)
    z = fbm(n, n, hurst, rng.integers(2**63), relief)
    yc, dyc = _centreline(n, h, rng)
    y = (np.arange(n) + 0.5) * h
    dist = np.abs(y[:, None] - yc[None, :]) / np.sqrt(1.0 + dyc[None, :] ** 2)
    chan = dist <= channel_half_width
    jc = np.clip(np.floor(yc / h).astype(int), 0, n - 1)
    zc = z[jc, np.arange(n)]
    bed = np.minimum.accumulate(zc) - channel_depth
    b = np.where(chan, np.minimum(z, bed[None, :]), z)
    nm = np.where(chan, 0.03, 0.05)
    return b, nm, chan, yc


def floodplain(n=4096, h=25.0, seed=0, steps=10000, q_peak=3.0e4, t_peak=3600.0,
               sigma_t=1200.0, inlet_cells=40, fill=4.0, precision=32):
    """Synthetic floodplain flood: dry floodplain, channel filled to `fill`
    metres, Gaussian inflow over an inlet_cells^2 inlet on the channel at its
    upstream end, walls all round, wind, Coriolis, turbulent viscosity."""
    b, nm, chan, yc = floodplain_terrain(n, h, seed)
    H0 = np.where(chan, fill, 0.0)
    ni = min(inlet_cells, n)
    jc = int(yc[min(ni // 2, n - 1)] / h)
    j0 = int(np.clip(jc - ni // 2, 0, n - ni))
    prm = base_params(tau_max=2.0, nu=0.5, f_cor=F_COR, wind_x=5.0, wind_y=2.0,
                      wind_kappa=WIND_KAPPA, inlet=(0, j0, ni, ni), q_base=0.0,
                      q_peak=q_peak, t_peak=t_peak, sigma_t=sigma_t, precision=precision)
    return dict(name="floodplain-%d" % n, nx=n, ny=n, h=h, b=b, n_manning=nm, solid=None,
                H0=H0, Qx0=np.zeros_like(b), Qy0=np.zeros_like(b), params=prm, steps=steps)


def floodplain_wet(n=4096, h=25.0, seed=0, percentile=60.0, precision=32):
    """Fully wet control on the same terrain: still water with its level at
    the given percentile of the bed, so that about that share of cells is wet."""
    sc = floodplain(n, h, seed, precision=precision)
    eta0 = float(np.percentile(sc["b"], percentile))
    sc["H0"] = np.maximum(eta0 - sc["b"], 0.0)
    sc["name"] = "floodplain-wet-%d" % n
    return sc


def dam_break(nx=256, ny=256, h=1.0, x_dam=128.0, h_left=2.0, h_right=0.5,
              precision=64):
    """Idealised dam break on a flat frictionless bed, water at rest."""
    x = (np.arange(nx) + 0.5) * h
    H0 = np.where(x < x_dam, h_left, h_right)[None, :].repeat(ny, axis=0)
    z = np.zeros((ny, nx))
    return dict(name="dam-break-%dx%d" % (nx, ny), nx=nx, ny=ny, h=h, b=z.copy(),
                n_manning=z.copy(), solid=None, H0=H0.astype(np.float64),
                Qx0=z.copy(), Qy0=z.copy(), params=base_params(precision=precision),
                steps=200)


def lake_at_rest(n=64, h=10.0, seed=3, relief=8.0, eta0=5.0, precision=64):
    """Still lake over rough fBm relief whose peaks rise above the surface."""
    b = fbm(n, n, 0.8, seed, relief)
    H0 = np.maximum(eta0 - b, 0.0)
    z = np.zeros_like(b)
    return dict(name="lake-%d" % n, nx=n, ny=n, h=h, b=b, n_manning=np.full_like(b, 0.03),
                solid=None, H0=H0, Qx0=z.copy(), Qy0=z.copy(),
                params=base_params(precision=precision, nu=0.5), steps=1000)


def random_state(nx, ny, h=5.0, seed=0, wet_frac=0.6, precision=32, **prm):
    """Rough random wet/dry state with random velocities (stencil stress test)."""
    rng = _rng(seed)
    b = fbm(ny, nx, 0.7, rng.integers(2**63), 4.0)
    eta0 = float(np.quantile(b, wet_frac))
    H0 = np.maximum(eta0 - b, 0.0) * rng.uniform(0.7, 1.3, size=b.shape)
    wet = H0 > 1e-3
    Qx0 = np.where(wet, H0 * rng.normal(0.0, 0.5, size=b.shape), 0.0)
    Qy0 = np.where(wet, H0 * rng.normal(0.0, 0.5, size=b.shape), 0.0)
    nm = rng.uniform(0.02, 0.06, size=b.shape)
    p = base_params(precision=precision, nu=0.5, f_cor=F_COR, wind_x=5.0, wind_y=-3.0,
                    wind_kappa=WIND_KAPPA, tau_max=1.0)
    p.update(prm)
    return dict(name="random-%dx%d" % (nx, ny), nx=nx, ny=ny, h=h, b=b, n_manning=nm,
                solid=None, H0=H0, Qx0=Qx0, Qy0=Qy0, params=p, steps=200)


def ensemble(n=256, seed0=1000, side_min=256, side_max=2048, h=25.0, gates_max=12,
             precision=32):
    """Batched-ensemble stand-in: scenario k (seed seed0 + k) has a square
    grid whose side is drawn log-uniformly from [side_min, side_max], the
    floodplain terrain family, a Gaussian inflow with peak U(5e3, 3e4) m^3/s
    at U(1, 5) days (base flow 0.1 of the peak, sigma = t_peak/3, clock from
    0), and 0..gates_max gate cells on the channel, each closed with
    probability 1/2 (a closed gate is a solid cell)."""
    out = []
    for k in range(n):
        rng = _rng(seed0 + k)
        side = int(round(math.exp(rng.uniform(math.log(side_min), math.log(side_max)))))
        q_peak = float(rng.uniform(5e3, 3e4))
        t_peak = float(rng.uniform(1.0, 5.0)) * 86400.0
        sc = floodplain(n=side, h=h, seed=int(rng.integers(2**31)), q_peak=q_peak, t_peak=t_peak,
                        sigma_t=t_peak / 3.0, precision=precision)
        sc["params"]["q_base"] = 0.1 * q_peak
        ngates = int(rng.integers(0, gates_max + 1))
        solid = np.zeros((side, side), np.uint8)
        i0, j0, ni, nj = sc["params"]["inlet"]
        cand = np.argwhere(sc["H0"] > 0.0)                 # channel cells
        cand = cand[cand[:, 1] >= i0 + ni + 2]             # downstream of the inlet
        if ngates and len(cand):
            pick = cand[rng.choice(len(cand), size=min(ngates, len(cand)), replace=False)]
            closed = rng.uniform(size=len(pick)) < 0.5
            for (j, i), c in zip(pick, closed):
                if c:
                    solid[j, i] = 1
        sc["solid"] = solid if solid.any() else None
        sc["name"] = "ensemble-%d-side%d" % (k, side)
        sc["steps"] = 2000
        out.append(sc)
    return out


def _bilinear_window(z, r, fi0, fj0, nxf, nyf):
    """Cell-centred bilinear interpolation of the coarse field z at the fine
    cells [fi0, fi0+nxf) x [fj0, fj0+nyf) of a grid refined by r (edge
    clamping)."""
    ny, nx = z.shape
    x = (np.arange(fi0, fi0 + nxf) + 0.5) / r - 0.5
    y = (np.arange(fj0, fj0 + nyf) + 0.5) / r - 0.5
    x0 = np.clip(np.floor(x).astype(int), 0, nx - 1)
    y0 = np.clip(np.floor(y).astype(int), 0, ny - 1)
    x1 = np.clip(x0 + 1, 0, nx - 1)
    y1 = np.clip(y0 + 1, 0, ny - 1)
    fx = np.clip(x - x0, 0.0, 1.0)[None, :]
    fy = np.clip(y - y0, 0.0, 1.0)[:, None]
    a = z[np.ix_(y0, x0)] * (1 - fx) + z[np.ix_(y0, x1)] * fx
    b = z[np.ix_(y1, x0)] * (1 - fx) + z[np.ix_(y1, x1)] * fx
    return a * (1 - fy) + b * fy


def nest(coarse, boxes, r=4, seed=0, detail=0.5):
    """Nested-grid inputs: a coarse scenario and refined patches over the
    coarse boxes (ci0, cj0, cw, ch).  The fine bed is the bilinear
    upsampling of the coarse bed plus fBm detail of `detail` metres (drawn
    per patch window); each
    covered coarse cell takes the mean of its r x r fine bed cells, so that
    the coarse grid sees the fine bed's volume.  Fine initial water fills to
    the parent coarse cell's level where that cell is wet (still water); the
    covered coarse cells take the mean fine depth.  A patch carries the
    extended fine grid (frame of NEST_FRAME fine cells round the covered
    area).  Fine cells take their parent's velocity at their own depth where
    they are wet; covered coarse cells take the mean fine discharge."""
    G = NEST_FRAME
    c = dict(coarse)
    bc = np.array(coarse["b"], dtype=np.float64)
    b_orig = bc.copy()
    Hc = np.array(coarse["H0"], dtype=np.float64)
    Qxc = np.array(coarse["Qx0"], dtype=np.float64)
    Qyc = np.array(coarse["Qy0"], dtype=np.float64)
    nmc = np.asarray(coarse["n_manning"], dtype=np.float64)
    rng = _rng(seed)
    eta_c = np.where(Hc > 0.0, Hc + bc, -np.inf)
    patches = []
    for (ci0, cj0, cw, ch) in boxes:
        # extended fine window in global fine indices; fBm detail of its own
        fi0, fj0 = ci0 * r - G, cj0 * r - G
        nxf, nyf = cw * r + 2 * G, ch * r + 2 * G
        d = fbm(nyf, nxf, 0.8, rng.integers(2**63), detail)
        bf = _bilinear_window(b_orig, r, fi0, fj0, nxf, nyf) + d - 0.5 * detail
        par_i = np.floor_divide(np.arange(nxf) + fi0, r)
        par_j = np.floor_divide(np.arange(nyf) + fj0, r)
        PJ, PI = np.meshgrid(par_j, par_i, indexing="ij")
        nmf = nmc[PJ, PI].copy()
        eta = eta_c[PJ, PI]
        Hf = np.where(np.isfinite(eta), np.maximum(eta - bf, 0.0), 0.0)
        Hp = np.where(Hc[PJ, PI] > 0.0, Hc[PJ, PI], 1.0)
        Qxf = np.where(Hf > 0.0, Hf * (Qxc[PJ, PI] / Hp), 0.0)
        Qyf = np.where(Hf > 0.0, Hf * (Qyc[PJ, PI] / Hp), 0.0)
        inner = (slice(G, G + ch * r), slice(G, G + cw * r))
        cov = (slice(cj0, cj0 + ch), slice(ci0, ci0 + cw))
        for fine_f, coarse_f in ((bf, bc), (Hf, Hc), (Qxf, Qxc), (Qyf, Qyc)):
            coarse_f[cov] = fine_f[inner].reshape(ch, r, cw, r).mean(axis=(1, 3))
        patches.append(dict(ci0=ci0, cj0=cj0, cw=cw, ch=ch, b=bf, n_manning=nmf,
                            H0=Hf[inner].copy(), Qx0=Qxf[inner].copy(), Qy0=Qyf[inner].copy()))
    c["b"], c["H0"], c["Qx0"], c["Qy0"] = bc, Hc, Qxc, Qyc
    c["name"] = coarse["name"] + "-nest%d" % len(boxes)
    return dict(coarse=c, patches=patches, r=r)


def nest_reference(coarse, nest_dict, detail_from_patches=True):
    """Uniform fine grid over the whole domain of a nest built by nest():
    the fine bed is the bilinear upsampling of the original coarse bed, with
    each patch's own fine bed (detail included) in its window; water fills to
    the parent coarse cell's level where that cell is wet, with its
    velocity; Manning n and the inlet (scaled by r) from the coarse grid.
    The reference solution a nest approximates inside its patches."""
    r = nest_dict["r"]
    G = NEST_FRAME
    bc = np.asarray(coarse["b"], dtype=np.float64)
    ny, nx = bc.shape
    nyf, nxf = ny * r, nx * r
    bf = _bilinear_window(bc, r, 0, 0, nxf, nyf)
    if detail_from_patches:
        for p in nest_dict["patches"]:
            fi0, fj0 = p["ci0"] * r - G, p["cj0"] * r - G
            pb = np.asarray(p["b"], dtype=np.float64)
            bf[fj0:fj0 + pb.shape[0], fi0:fi0 + pb.shape[1]] = pb
    Hc = np.asarray(coarse["H0"], dtype=np.float64)
    eta_c = np.where(Hc > 0.0, Hc + bc, -np.inf)
    up = lambda a: np.repeat(np.repeat(a, r, axis=0), r, axis=1)
    eta = up(eta_c)
    Hf = np.where(np.isfinite(eta), np.maximum(eta - bf, 0.0), 0.0)
    del eta
    Hp = up(np.where(Hc > 0.0, Hc, 1.0))
    Qxf = np.where(Hf > 0.0, Hf * (up(np.asarray(coarse["Qx0"], dtype=np.float64)) / Hp), 0.0)
    Qyf = np.where(Hf > 0.0, Hf * (up(np.asarray(coarse["Qy0"], dtype=np.float64)) / Hp), 0.0)
    del Hp
    p = dict(coarse["params"])
    if p.get("inlet"):
        i0, j0, ni, nj = p["inlet"]
        p["inlet"] = (i0 * r, j0 * r, ni * r, nj * r)
    return dict(name=coarse["name"] + "-fine%d" % r, nx=nxf, ny=nyf, h=coarse["h"] / r, b=bf,
                n_manning=up(np.asarray(coarse["n_manning"], dtype=np.float64)), solid=None,
                H0=Hf, Qx0=Qxf, Qy0=Qyf, params=p)


# Frame width of a patch in fine cells: one more than the reach of one step
# of the scheme (4 cells).
NEST_FRAME = 5


def nest_floodplain(n=2048, h=50.0, seed=1, r=4, box=512, precision=32):
    """Nested-grid workload: an n^2 floodplain at h metres with two refined
    patches of box^2 coarse cells (ratio r) centred on the two bends of the
    channel with the largest curvature (away from the inlet)."""
    sc = floodplain(n=n, h=h, seed=seed, precision=precision)
    _, _, _, yc = floodplain_terrain(n, h, seed)
    x = np.arange(n)
    curv = np.abs(np.gradient(np.gradient(yc)))
    i0_min = sc["params"]["inlet"][0] + sc["params"]["inlet"][2] + 2
    order = np.argsort(curv)[::-1]
    m = -(-NEST_FRAME // r)
    half = box // 2
    centres = []
    for i in order:
        if i - half < max(i0_min, m) or i + half + m > n:
            continue
        if any(abs(i - c) < box + 1 for c in centres):
            continue
        centres.append(int(i))
        if len(centres) == 2:
            break
    boxes = []
    for i in sorted(centres):
        j = int(np.clip(yc[i] / h - half, m, n - box - m))
        boxes.append((i - half, j, box, box))
    out = nest(sc, boxes, r=r, seed=seed + 7)
    out["coarse"]["name"] = "nest-floodplain-%d-r%d" % (n, r)
    out["source"] = sc          # the coarse scenario before nesting (original bed)
    return out
