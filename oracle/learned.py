"""FP64 CPU oracle of the learned coarse-grid flux correction.

TEST INFRASTRUCTURE ONLY: imported by the tests and the smoke check, never by
the GPU product path.

The paper has no learned component; this part of the build adds one on top
of its scheme (stage III fluxes of Sec. 2.3): a small convolutional network
reads the coarse state and predicts corrections to the coarse face fluxes so
that a 4x-coarsened grid tracks the fine solution.  Parity with any published
result is unpinned; the functions below are the plain definitions the GPU
kernels are checked against:

  network   four 3x3 "valid" convolutions (no padding) 6 -> 32 -> 32 -> 32 -> 6
            channels, tanh after the first three, linear output; an input
            crop of (S + 9)^2 cells gives the (S + 1)^2 outputs of an S x S
            tile and the cell row and column before it.  Output channels:
            corrections of (mass, x-momentum, y-momentum) flux through the
            east face, then through the north face, of each cell, in units of
            the scale vector the caller applies.
  storage   with bf16=True the values are rounded to bfloat16 (round to
            nearest even) where the GPU stores them: the input features, the
            weights, the hidden activations and the back-propagated
            pre-activation gradients; all sums are exact FP64 here (the GPU
            accumulates in FP32).  With bf16=False nothing is rounded (finite
            difference checks).
  loss      L = 1/2 sum(mask * (out - y)^2) / max(sum(mask), 1) over all
            output elements.
  adam      the standard Adam update (Kingma and Ba) with bias correction.
"""
import numpy as np

LAYERS = ((6, 32), (32, 32), (32, 32), (32, 6))
HALO = len(LAYERS)          # one cell of valid convolution per layer


def bf16(x):
    """Round to bfloat16 (nearest even) and return as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """Seeded weights W[l] (cout, cin, 3, 3) and biases b[l] (cout): uniform
    in +-sqrt(6 / (fan_in + fan_out)) (Glorot), the last layer scaled by 0.1,
    biases zero."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    W, b = [], []
    for k, (ci, co) in enumerate(LAYERS):
        lim = np.sqrt(6.0 / (9 * ci + 9 * co))
        w = rng.uniform(-lim, lim, size=(co, ci, 3, 3))
        if k == len(LAYERS) - 1:
            w *= 0.1
        W.append(w)
        b.append(np.zeros(co))
    return W, b


def conv3x3(x, w, b):
    """Valid 3x3 convolution: x (N, H, W, cin), w (cout, cin, 3, 3), b (cout)
    -> (N, H-2, W-2, cout), y[n,i,j,o] = b[o] + sum x[n,i+dy,j+dx,c] w[o,c,dy,dx]."""
    n, h, wd, _ = x.shape
    y = np.zeros((n, h - 2, wd - 2, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("nijc,oc->nijo", x[:, dy:dy + h - 2, dx:dx + wd - 2, :], w[:, :, dy, dx])
    return y


def conv3x3_grads(x, w, g):
    """Gradients of conv3x3 given dL/dy = g: (dL/dx, dL/dw, dL/db)."""
    n, h, wd, _ = x.shape
    dx_ = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dxx in range(3):
            xs = x[:, dy:dy + h - 2, dxx:dxx + wd - 2, :]
            dw[:, :, dy, dxx] = np.einsum("nijo,nijc->oc", g, xs)
            dx_[:, dy:dy + h - 2, dxx:dxx + wd - 2, :] += np.einsum("nijo,oc->nijc", g, w[:, :, dy, dxx])
    return dx_, dw, g.sum(axis=(0, 1, 2))


def forward(x, W, b, bf=True):
    """Network output and the per-layer inputs kept for the backward pass."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    acts = []
    for k in range(len(LAYERS)):
        acts.append(a)
        z = conv3x3(a, r(W[k]), b[k])
        a = r(np.tanh(z)) if k < len(LAYERS) - 1 else z
    return a, acts


def loss_and_grad(out, y, mask):
    cnt = max(float(mask.sum()), 1.0)
    d = mask * (out - y)
    return 0.5 * float((d * (out - y)).sum()) / cnt, d / cnt


def backward(gout, acts, W, bf=True):
    """Parameter gradients from dL/dout (and the stored layer inputs)."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    dW, db = [None] * len(LAYERS), [None] * len(LAYERS)
    g = r(gout)
    for k in range(len(LAYERS) - 1, -1, -1):
        da, dW[k], db[k] = conv3x3_grads(acts[k], r(W[k]), g)
        if k > 0:
            g = r(da * (1.0 - acts[k] ** 2))     # tanh' from the stored activation
    return dW, db


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for k, (p, g) in enumerate(zip(params, grads)):
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g * g
            out.append(p - self.lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps))
        return out


# ---------------------------------------------------------------- inputs and outputs

def features(H, Qx, Qy, b, n_manning, eps, scale):
    """Six input channels of every coarse cell: H, Ux, Uy, b, n_M, wet, each
    divided by its scale entry (wet is 0/1 and its scale is 1).  U = Q/H
    where H > eps, else 0."""
    wet = H > eps
    Hs = np.where(wet, H, 1.0)
    ux = np.where(wet, Qx / Hs, 0.0)
    uy = np.where(wet, Qy / Hs, 0.0)
    f = np.stack([H, ux, uy, b, n_manning, wet.astype(np.float64)], axis=-1)
    return f / np.asarray(scale, dtype=np.float64)


def mirror_index(i, n):
    """Reflective walls: the cell seen at index i outside [0, n)."""
    i = np.asarray(i)
    i = np.where(i < 0, -1 - i, i)
    return np.where(i >= n, 2 * n - 1 - i, i)


def crops(feat, tiles, S):
    """Input windows (len(tiles), S + 1 + 2*HALO, S + 1 + 2*HALO, 6) of the
    S x S tiles (tx, ty) (tile indices) and the cell row and column before
    each (output cells tx*S - 1 .. tx*S + S - 1), mirrored at the domain
    edges.  A velocity channel is mirrored as the cell's value; walls act
    through the wet/dry and bed channels only."""
    ny, nx, _ = feat.shape
    side = S + 1 + 2 * HALO
    out = np.empty((len(tiles), side, side, feat.shape[2]))
    for k, (tx, ty) in enumerate(tiles):
        ys = mirror_index(np.arange(ty * S - 1 - HALO, ty * S - 1 - HALO + side), ny)
        xs = mirror_index(np.arange(tx * S - 1 - HALO, tx * S - 1 - HALO + side), nx)
        out[k] = feat[np.ix_(ys, xs)]
    return out


def corrections(out, tiles, S, ny, nx, scale):
    """Scatter network outputs (len(tiles), S+1, S+1, 6) of the cells
    tx*S - 1 .. tx*S + S - 1 into east- and north-face corrections (3, ny, nx)
    each, times the output scales (cells outside the grid dropped)."""
    dE = np.zeros((3, ny, nx))
    dN = np.zeros((3, ny, nx))
    o = out * np.asarray(scale, dtype=np.float64)
    for k, (tx, ty) in enumerate(tiles):
        for j in range(S + 1):
            gy = ty * S - 1 + j
            if not 0 <= gy < ny:
                continue
            for i in range(S + 1):
                gx = tx * S - 1 + i
                if not 0 <= gx < nx:
                    continue
                dE[:, gy, gx] = o[k, j, i, 0:3]
                dN[:, gy, gx] = o[k, j, i, 3:6]
    return dE, dN
