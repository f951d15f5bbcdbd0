"""Learned coarse-grid flux correction: training data from fine runs of the
solver, training, and the comparison against the fine solve.

Host orchestration only: every step of the solver, the labels, the network
and its training run in the library's kernels (swe_lc_*); this module picks
time steps, seeds and minibatch sizes and reads back a few scalars.

The coarse grid is the fine grid coarsened by r: bed and Manning n are the
means of r x r fine cells, the state is the restriction of the fine state.
A coarse interval tau_c = min(coarse CFL step, m * fine CFL step) is one
coarse step and m fine steps.
"""
import time

import numpy as np

from . import swe

IN_SCALE = np.array([5.0, 1.0, 1.0, 10.0, 0.05, 1.0])
# depth a face's donor needs before the network's mass correction applies,
# and both of its cells before the momentum correction does: below it a cell
# would gain momentum without the water to carry it.  On the 4096^2 / 1024^2
# floodplain with 64 training runs, 1 m kept the coarse step as long as the
# plain coarse grid's and gave the lowest held-out error of 0.05, 0.5 and 1 m
# (0.05 m: 352 steps instead of 224 over the same interval).
CORR_DEPTH = 1.0


def coarsen(sc, r):
    """Coarse scenario of a fine one: means of r x r cells; the inlet
    rectangle is scaled by 1/r; the step cap tau_max grows with the cell size
    (same cap in Courant units)."""
    ny, nx = sc["ny"] // r, sc["nx"] // r
    R = lambda a: np.asarray(a, dtype=np.float64)[:ny * r, :nx * r].reshape(ny, r, nx, r).mean(axis=(1, 3))
    p = dict(sc["params"])
    if p.get("tau_max"):
        p["tau_max"] = p["tau_max"] * r      # same cap in Courant units
    if p.get("inlet"):
        i0, j0, ni, nj = p["inlet"]
        p["inlet"] = (i0 // r, j0 // r, max(ni // r, 1), max(nj // r, 1))
    return dict(name=sc["name"] + "-coarse%d" % r, nx=nx, ny=ny, h=sc["h"] * r, b=R(sc["b"]),
                n_manning=R(sc["n_manning"]), solid=None, H0=R(sc["H0"]), Qx0=R(sc["Qx0"]), Qy0=R(sc["Qy0"]),
                params=p)


def make_net(tile, max_crops, out_scale=None):
    return swe.Net(tile, max_crops, IN_SCALE, np.ones(6) if out_scale is None else out_scale)


def initial_params(seed=0):
    """Packed starting weights: uniform in +-sqrt(6 / (9 in + 9 out)) per
    layer (Glorot), the output layer scaled by 0.1, biases zero."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    parts = []
    for k, (ci, co) in enumerate(swe.LC_LAYERS):
        lim = np.sqrt(6.0 / (9.0 * (ci + co))) * (0.1 if k == len(swe.LC_LAYERS) - 1 else 1.0)
        parts.append(rng.uniform(-lim, lim, size=co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def collect(net, fine_sc, r, m, intervals, skip=0, gap=0):
    """Run the fine scenario and add the crops and labels of `intervals`
    coarse intervals (after `skip` fine CFL steps, and `gap` more between
    intervals) to the network's data set."""
    f = swe.Solver(fine_sc)
    if skip:
        f.run(skip)
    f.enable_line_taps(r)
    c = swe.Solver(coarsen(fine_sc, r))
    c.enable_line_taps(1)
    taus = []
    for k in range(intervals):
        if gap and k:
            f.run(gap)
        taus.append(net.collect(f, c, r, m))
    f.close()
    c.close()
    return taus


def label_scale(net, max_crops=20000):
    """Per-channel RMS of the collected labels (in current output units), over
    at most max_crops crops spread evenly through the data set."""
    n = net.data_count()
    step = max(1, n // max_crops)
    parts = [net.get_data(k, 1)[1:3] for k in range(0, n, step)] if step > 1 else [net.get_data(0, n)[1:3]]
    y = np.concatenate([p[0] for p in parts])
    mask = np.concatenate([p[1] for p in parts])
    num = (y * y * mask).sum(axis=(0, 1, 2))
    den = np.maximum(mask.sum(axis=(0, 1, 2)), 1.0)
    return np.sqrt(num / den) * net.out_scale


def compare(net, fine_sc, r, m, intervals, skip=0, corr_depth=CORR_DEPTH):
    """Fine solve, plain coarse and learned coarse over the same coarse
    intervals from the same restricted layer; relative L1 depth error of
    both coarse runs against the restricted fine solution at the end."""
    f = swe.Solver(fine_sc)
    if skip:
        f.run(skip)
    csc = coarsen(fine_sc, r)
    plain = swe.Solver(csc)
    lrn = swe.Solver(csc)
    plain.restrict_from(f, r)
    lrn.restrict_from(f, r)
    net.attach(lrn)
    lrn.set_correction_depth(corr_depth)
    for _ in range(intervals):
        tau_c = min(plain.next_dt(), lrn.next_dt(), m * f.next_dt())
        tau_f = tau_c / m
        f.hold_dt(tau_f)
        f.run(m)
        f.hold_dt(0.0)
        for g in (plain, lrn):
            g.hold_dt(tau_f * m)
            g.run(1)
            g.hold_dt(0.0)
    ref = swe.Solver(csc)
    ref.restrict_from(f, r)
    Hr = ref.state()[0]
    Hp, Hl = plain.state()[0], lrn.state()[0]
    net.detach(lrn)
    out = dict(time=f.time(), err_plain=float(np.abs(Hp - Hr).sum() / np.abs(Hr).sum()),
               err_learned=float(np.abs(Hl - Hr).sum() / np.abs(Hr).sum()))
    for g in (f, plain, lrn, ref):
        g.close()
    return out


def timing(net, fine_sc, r, sim_seconds, skip=0, corr_depth=CORR_DEPTH):
    """Wall time of the fine solve, of the learned coarse solve (network
    included) and of the plain coarse solve over the same simulated
    interval, each with its own CFL steps and hipGraph replays.  A first,
    untimed pass counts the steps each solve needs to cover sim_seconds (and
    captures its graphs); the solver is then reset to the starting state and
    time and runs exactly that many steps in one call, timed between two
    synchronisations (no host round trip inside the timed region)."""
    import torch
    f0 = swe.Solver(fine_sc)
    if skip:
        f0.run(skip)
    start, t_start = f0.state(), f0.time()
    csc = coarsen(fine_sc, r)
    res = {}
    for name in ("fine", "learned", "plain"):
        if name == "fine":
            s = swe.Solver(fine_sc)
            reset = lambda s=s: (s.set_state(*start), s.set_time(t_start))
        else:
            s = swe.Solver(csc)
            reset = lambda s=s: s.restrict_from(f0, r)
        reset()
        if name == "learned":
            net.attach(s)
            s.set_correction_depth(corr_depth)
        t0, steps = s.time(), 0
        while s.time() - t0 < sim_seconds:
            s.run(32)
            steps += 32
        reset()
        t0 = s.time()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        s.run(steps)
        torch.cuda.synchronize()
        res[name] = dict(wall=time.perf_counter() - w0, steps=steps, sim=s.time() - t0)
        if name == "learned":
            net.detach(s)
        s.close()
    f0.close()
    return res


def advance_to(g, t_end, frac=0.5, chunk=16, on_run=None):
    """Advance a solver (or a nest, by coarse steps) with its own CFL steps to t_end: runs of at most
    `chunk` steps while the end is far, single steps near it, and a last step
    held to the remaining time (to within the rounding of the step length to
    the stencil type).  A run never passes the end: where the solver has a
    cap on its step (tau_max) a run is at most what is left over that cap;
    without one it covers at most frac of what is left at the current step
    length, and a step that grows faster than that within the run raises.
    on_run(t) is called after every run or step with the solver's time."""
    cap = float(getattr(g, "tau_max", 0.0) or 0.0)
    while True:
        left = t_end - g.time()
        dt = g.next_dt()
        # landed: within a millionth of a step (the held last step is exact
        # to the rounding of its length to the stencil type)
        if left <= 1e-6 * dt:
            if -left > 1e-6 * dt:
                raise RuntimeError("advance_to: overshot %g by %g s" % (t_end, -left))
            return
        # (a step may exceed the cap by the rounding of its length to FP32)
        n = int(left / (max(cap, dt) * (1.0 + 1e-6))) if cap > 0.0 else int(frac * left / dt)
        n = min(n, chunk)
        if n >= 2:
            g.run(n)
        elif dt < left:
            g.step()
        else:
            g.hold_dt(left)
            g.step()
            g.hold_dt(0.0)
            return
        if on_run is not None:
            on_run(g.time())


class GuardedRun:
    """Learned coarse solve with the plain fine solve as its fallback and the
    judge of its error.

    The coarse grid with the attached network advances in windows of
    `window` coarse CFL steps.  After each window a guard reads device
    scalars of the coarse grid: the status of its steps (a non-finite state
    or a collapsed time step stops them), its volume balance over the window
    (V - V_0 - inflow - clamped volume, which the conservative corrections
    keep at rounding level), and the volume the final update had to add by
    clamping negative depths (corrections that drain cells below zero).
    Every `judge_every` windows (0: never) the fine solve is advanced to the
    window's end and judges the coarse depth: relative L1 against the
    restricted fine depth above `err_tol` fails the window.

    A failed window is handed back to the fine solve: it advances from its
    last layer (the start, or the end of the last window it ran or judged)
    to the window's end with its own CFL steps, and the coarse grid restarts
    from the restriction of that layer.  `log` records every window: mode
    ('learned' or 'fine'), the reason of a fallback, the window's end time
    t_end, the coarse clock t after it and the judged error."""

    def __init__(self, net, fine_sc, r, window=32, vol_tol=1e-5, clamp_tol=1e-4, judge_every=0,
                 err_tol=0.02, corr_depth=CORR_DEPTH):
        self.net, self.r, self.window = net, r, int(window)
        self.vol_tol, self.clamp_tol = vol_tol, clamp_tol
        self.judge_every, self.err_tol = int(judge_every), err_tol
        self.fine = swe.Solver(fine_sc)
        self.csc = coarsen(fine_sc, r)
        self.corr_depth = corr_depth
        self.coarse = None
        self._new_coarse()
        self.ref = swe.Solver(self.csc)  # restricted fine layers for the judge
        self.log = []

    def _new_coarse(self):
        """A fresh coarse grid at the fine solve's layer, network attached
        (after a failed window the old grid's clamp ledger may hold the
        diverged steps' volumes, so its bookkeeping is not carried over)."""
        if self.coarse is not None:
            self.net.detach(self.coarse)
            self.coarse.close()
        self.coarse = swe.Solver(self.csc)
        self.coarse.restrict_from(self.fine, self.r)
        self.net.attach(self.coarse)
        self.coarse.set_correction_depth(self.corr_depth)

    def _fallback(self, t_end):
        advance_to(self.fine, t_end)
        self._new_coarse()

    def step_window(self):
        g = self.coarse
        k = len(self.log)
        t0, V0, in0, cl0, dt0 = g.time(), g.mass(), g.inflow(), g.ledger(), g.next_dt()
        rc = g.run_rc(self.window)
        reason, err = None, None
        t_end = g.time()
        if rc != 0:
            reason = "step error %d" % rc
            if not t_end > t0:           # stopped in its first step: a window of the last step length
                t_end = t0 + self.window * dt0
        else:
            V, dV_in, dV_cl = g.mass(), g.inflow() - in0, g.ledger() - cl0
            scale = max(abs(V), abs(V0), 1e-300)
            resid = (V - V0 - dV_in - dV_cl) / scale
            if not abs(resid) <= self.vol_tol:
                reason = "volume balance %.3g" % resid
            elif not abs(dV_cl) <= self.clamp_tol * scale:
                reason = "clamped volume"
        if reason is None and self.judge_every and (k + 1) % self.judge_every == 0:
            advance_to(self.fine, t_end)
            self.ref.restrict_from(self.fine, self.r)
            Hr, Hc = self.ref.state()[0], g.state()[0]
            err = float(np.abs(Hc - Hr).sum() / max(np.abs(Hr).sum(), 1e-300))
            if not err <= self.err_tol:
                reason = "judged error %.3g > %.3g" % (err, self.err_tol)
        if reason is not None:
            self._fallback(t_end)
        self.log.append(dict(window=k, mode="fine" if reason else "learned", reason=reason,
                             t_end=t_end, t=self.coarse.time(), err=err))
        return self.log[-1]

    def run(self, windows):
        for _ in range(int(windows)):
            self.step_window()
        return self.log

    def close(self):
        self.net.detach(self.coarse)
        for g in (self.fine, self.coarse, self.ref):
            g.close()
