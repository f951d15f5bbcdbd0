"""Closed-form solutions of the shallow-water equations used as pins.

Each is derived here from the equations of arXiv 1705.00614 Sec. 2.1
(Eqs. 1-3 without forces) and the textbook results named at each function;
none of them calls the oracle or the GPU library.
"""
import math

import numpy as np
from scipy.optimize import brentq

G = 9.81


def stoker_middle(h0, h1, g=G):
    """Middle state of the wet dam break (Stoker 1957).

    Left rarefaction: u + 2c = 2 c0 (Riemann invariant).  Right shock moving
    into still water of depth h1, from the Rankine-Hugoniot mass and momentum
    jump conditions.  Eliminating the shock speed gives
        8 c1^2 cm^2 (c0 - cm)^2 = (cm^2 - c1^2)^2 (cm^2 + c1^2),  c = sqrt(g h).
    Returns (cm, hm, um, shock_speed)."""
    c0, c1 = math.sqrt(g * h0), math.sqrt(g * h1)

    def f(cm):
        return 8 * c1**2 * cm**2 * (c0 - cm) ** 2 - (cm**2 - c1**2) ** 2 * (cm**2 + c1**2)

    cm = brentq(f, c1 * (1 + 1e-12), c0 * (1 - 1e-12), xtol=1e-15, rtol=1e-15)
    hm = cm * cm / g
    um = 2.0 * (c0 - cm)
    s = hm * um / (hm - h1)
    return cm, hm, um, s


def dam_break_depth(xi, h0, h1, g=G):
    """Depth at similarity coordinate xi = (x - x_dam)/t: Ritter for h1 = 0,
    Stoker otherwise."""
    xi = np.asarray(xi, dtype=np.float64)
    c0 = math.sqrt(g * h0)
    fan = (2.0 * c0 - xi) ** 2 / (9.0 * g)
    if h1 == 0.0:
        return np.where(xi < -c0, h0, np.where(xi < 2.0 * c0, fan, 0.0))
    cm, hm, um, s = stoker_middle(h0, h1, g)
    return np.where(xi < -c0, h0, np.where(xi < um - cm, fan, np.where(xi < s, hm, h1)))


class Thacker:
    """Planar-surface oscillation in a paraboloid bowl (Thacker 1981):
    b = -h0 (1 - r^2/a^2), eta = (sigma h0/a^2)(2x cos wt + 2y sin wt - sigma),
    U = (-sigma w sin wt, sigma w cos wt), w = sqrt(2 g h0)/a."""

    def __init__(self, a=1.0, h0=0.1, sigma=0.5, g=G):
        self.a, self.h0, self.sigma, self.g = a, h0, sigma, g
        self.omega = math.sqrt(2.0 * g * h0) / a
        self.period = 2.0 * math.pi / self.omega

    def bed(self, x, y):
        return -self.h0 * (1.0 - (x * x + y * y) / self.a**2)

    def eta(self, x, y, t):
        w = self.omega
        return (self.sigma * self.h0 / self.a**2) * (
            2 * x * math.cos(w * t) + 2 * y * math.sin(w * t) - self.sigma)

    def velocity(self, t):
        w = self.omega
        return -self.sigma * w * math.sin(w * t), self.sigma * w * math.cos(w * t)

    def depth(self, x, y, t):
        return np.maximum(self.eta(x, y, t) - self.bed(x, y), 0.0)


def cubic_bspline_dw(q):
    """Derivative dW/dq of the 2D cubic B-spline kernel shape (support 2):
    W = 1 - 1.5 q^2 + 0.75 q^3 (q < 1), 0.25 (2 - q)^3 (1 <= q < 2), 0 beyond."""
    q = float(q)
    if q < 1.0:
        return -3.0 * q + 2.25 * q * q
    if q < 2.0:
        return -0.75 * (2.0 - q) ** 2
    return 0.0


def sph_lattice_weights(ell=1.0):
    """Weights w[(di,dj)] of the normalised SPH gradient on a unit square
    lattice with smoothing length ell: G = sum_m w_m (f_m - f_c), normalised
    so that G is exact for linear f.  Computed by summing kernel gradients
    over all lattice neighbours within the support."""
    raw = {}
    R = int(math.ceil(2 * ell)) + 1
    for dj in range(-R, R + 1):
        for di in range(-R, R + 1):
            r = math.hypot(di, dj)
            if r == 0:
                continue
            dw = cubic_bspline_dw(r / ell)
            if dw != 0.0:
                raw[(di, dj)] = (-dw * di / r, -dw * dj / r)   # points along +offset
    # normalisation M_ab = sum_m w_a(m) * offset_b(m); isotropic lattice -> diagonal
    mxx = sum(w[0] * di for (di, dj), w in raw.items())
    myy = sum(w[1] * dj for (di, dj), w in raw.items())
    return {k: (w[0] / mxx, w[1] / myy) for k, w in raw.items()}
