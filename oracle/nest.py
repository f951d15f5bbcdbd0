"""FP64 CPU oracle of hierarchical grids with feedback (two-way zoom-in).

TEST INFRASTRUCTURE ONLY: imported by the tests and the smoke check, never by
the GPU product path.

Paper: arXiv 1705.00614, Sec. 2.2 (hierarchical grid system, zoom-in with the
small-scale flow feeding back to the large-scale grid; zoom-in without feedback
is faster but less accurate) and Sec. 5 (a 50 m global grid with a 12.5 m
local grid).  The coupling is not spelled out in the paper; the reading used
here is coarse-first subcycling with conservative flux matching:

  per coarse step
  1. time steps: tau_c = min(tau_coarse, r * min_k tau_k), tau_f = tau_c / r,
     where tau_k is the CFL step of patch k after its last substep (frame
     included) and tau_coarse the CFL step of the largest of two speeds: the
     coarse layer as the coarse step produced it, and the layer after the
     feedback on the covered cells widened by 2 (the cells whose speed the
     feedback can change); at the start, the CFL steps of the initial layers;
  2. the coarse grid advances over the whole domain with tau_c; the fluxes on
     the faces bounding each covered region are recorded (times tau_c);
  3. each patch advances r substeps with tau_f.  A patch is an ordinary grid
     extended by a frame of G = 5 cells, one more than the reach of one step
     of the scheme (4 cells), so the patch interior never sees the frame's
     own outer edge.  Before
     every substep the frame is refilled from the covering coarse cell,
     piecewise constant in space and linear in time between coarse layers n
     and n+1: the coarse depth H_c and Q_c are interpolated, the fine depth
     is H_f = max(0, H_c + b_c - b_fine) and the fine discharge carries the
     coarse velocity, Q_f = H_f (Q_c / H_c), where H_c > eps, else the fine
     cell is dry (copying Q_c itself would put the momentum of the coarse
     column into a fine cell on a high spot of the fine bed: a film moving
     at tens of m/s, whose friction term in U_p then sets the step of the
     whole nest); the fluxes on the boundary faces of the patch
     interior are accumulated (times tau_f);
  4. restriction: covered coarse cells take the mean of their r x r fine
     cells (H, Qx, Qy);
  5. reflux: each uncovered coarse cell next to a covered region gets the
     difference between the recorded coarse flux and the mean of the r fine
     face fluxes over the r substeps (depth clamped at 0 into the ledger, Q
     zeroed where H <= eps, as in the final update); the momentum part with
     a weight rising from 0 at MOMENTUM_DEPTH (5 cm) to 1 at 10 cm of
     corrected depth, as the learned path's corrections keep momentum out of
     films: a film that took the patch flow's
     momentum would set the nest's CFL step through the friction term of
     U_p (1-2 orders of magnitude shorter steps);
  6. the coarse bed under a patch is the mean of the fine bed (an input).
Without feedback (one-way zoom-in) steps 4 and 5 are skipped: the coarse grid
runs as if alone and only drives the patches.  Patches must not touch each
other, the domain edge (ceil(G/r) coarse cells of margin for the frame)
or the inlet.  Parity of this reading with the authors' code is unpinned: the tests
pin it to volume conservation, the lake at rest, the r = 1 case (identical to
the single grid) and the restriction invariant.
"""
import numpy as np

from oracle.oracle import OracleSim

G = 5   # frame width in fine cells: reach of one step (4) plus one
MOMENTUM_DEPTH = 0.05   # [m] ring cells shallower take no momentum reflux, twice as deep all of it


class OracleNest:
    """Coarse grid plus non-overlapping patches refined by r.

    coarse: scenario dict of the coarse grid.
    patches: list of dicts with ci0, cj0, cw, ch (covered coarse cells) and
    the extended fine grid: b (ny_f + 2G, nx_f + 2G), n_manning (same shape),
    H0, Qx0, Qy0 (interior initial state, ny_f x nx_f), with nx_f = r*cw.
    """

    def __init__(self, coarse, patches, r=4, feedback=True):
        self.r = r
        self.feedback = feedback
        self._reflux = True          # tests switch it off to show that conservation needs it
        self.coarse_sc = coarse
        self.c = OracleSim(coarse)
        self.h_c = float(coarse["h"])
        self.h_f = self.h_c / r
        self.eps = coarse["params"]["eps"]
        self.bc = np.asarray(coarse["b"], dtype=np.float64)
        self.ledger = 0.0
        self.P = []
        m = -(-G // r)                    # coarse cells under a frame
        for p in patches:
            nxf, nyf = r * p["cw"], r * p["ch"]
            if not (p["ci0"] >= m and p["cj0"] >= m and p["ci0"] + p["cw"] + m <= coarse["nx"]
                    and p["cj0"] + p["ch"] + m <= coarse["ny"]):
                raise ValueError("patch frame leaves the coarse grid")
            inl = coarse["params"].get("inlet")
            if inl and inl[2] > 0 and not (inl[0] + inl[2] <= p["ci0"] - 1 or inl[0] >= p["ci0"] + p["cw"] + 1
                                           or inl[1] + inl[3] <= p["cj0"] - 1 or inl[1] >= p["cj0"] + p["ch"] + 1):
                raise ValueError("patch covers or touches the inlet")
            ext = dict(nx=nxf + 2 * G, ny=nyf + 2 * G, h=self.h_f, b=p["b"], n_manning=p["n_manning"],
                       solid=None, params=dict(coarse["params"], inlet=None, q_base=0.0, q_peak=0.0))
            H = np.zeros((nyf + 2 * G, nxf + 2 * G))
            Qx, Qy = np.zeros_like(H), np.zeros_like(H)
            H[G:G + nyf, G:G + nxf] = p["H0"]
            Qx[G:G + nyf, G:G + nxf] = p["Qx0"]
            Qy[G:G + nyf, G:G + nxf] = p["Qy0"]
            ext["H0"], ext["Qx0"], ext["Qy0"] = H, Qx, Qy
            sim = OracleSim(ext)
            self.P.append(dict(spec=p, sim=sim, nxf=nxf, nyf=nyf, bf=np.asarray(p["b"], dtype=np.float64)))
        for a in range(len(patches)):
            for b in range(a + 1, len(patches)):
                p, q = patches[a], patches[b]
                if not (p["ci0"] + p["cw"] + 1 <= q["ci0"] or q["ci0"] + q["cw"] + 1 <= p["ci0"]
                        or p["cj0"] + p["ch"] + 1 <= q["cj0"] or q["cj0"] + q["ch"] + 1 <= p["cj0"]):
                    raise ValueError("patches must keep one uncovered coarse cell between them")
        Hc, Qxc, Qyc = self.c.state()
        self._fill_all(Hc, Qxc, Qyc, Hc, Qxc, Qyc, 0.0)
        self.region = np.zeros((coarse["ny"], coarse["nx"]), dtype=bool)
        for p in patches:
            self.region[max(p["cj0"] - 2, 0):p["cj0"] + p["ch"] + 2,
                        max(p["ci0"] - 2, 0):p["ci0"] + p["cw"] + 2] = True
        self._set_taus(self.c.next_tau(), [P["sim"].next_tau() for P in self.P])

    # -------------------------------------------------------------- pieces

    def _frame(self, P, Hc0, Qxc0, Qyc0, Hc1, Qxc1, Qyc1, theta):
        """Extended patch state with the frame from the coarse layers."""
        r, p = self.r, P["spec"]
        H, Qx, Qy = P["sim"].state()
        ny, nx = H.shape
        fi = np.arange(nx) - G
        fj = np.arange(ny) - G
        ci = p["ci0"] + np.floor_divide(fi, r)
        cj = p["cj0"] + np.floor_divide(fj, r)
        CJ, CI = np.meshgrid(cj, ci, indexing="ij")
        Hc = (1.0 - theta) * Hc0[CJ, CI] + theta * Hc1[CJ, CI]
        eta = Hc + self.bc[CJ, CI]
        wet = Hc > self.eps
        Hs = np.where(wet, Hc, 1.0)
        Hf = np.where(wet, np.maximum(0.0, eta - P["bf"]), 0.0)
        # the coarse velocity (interpolated discharge over interpolated
        # depth) carried by the fine depth
        qx = np.where(wet, Hf * (((1.0 - theta) * Qxc0[CJ, CI] + theta * Qxc1[CJ, CI]) / Hs), 0.0)
        qy = np.where(wet, Hf * (((1.0 - theta) * Qyc0[CJ, CI] + theta * Qyc1[CJ, CI]) / Hs), 0.0)
        frame = np.ones_like(H, dtype=bool)
        frame[G:G + P["nyf"], G:G + P["nxf"]] = False
        H = np.where(frame, Hf, H)
        Qx = np.where(frame, qx, Qx)
        Qy = np.where(frame, qy, Qy)
        return H, Qx, Qy

    def _fill_all(self, Hc0, Qxc0, Qyc0, Hc1, Qxc1, Qyc1, theta):
        for P in self.P:
            P["sim"].set_state(*self._frame(P, Hc0, Qxc0, Qyc0, Hc1, Qxc1, Qyc1, theta))

    def _set_taus(self, tau_coarse, tau_patches):
        tau_c = min([tau_coarse] + [self.r * t for t in tau_patches])
        self.tau_c, self.tau_f = tau_c, tau_c / self.r

    def next_taus(self):
        """Coarse and fine time steps of the next coarse step."""
        return self.tau_c, self.tau_f

    # -------------------------------------------------------------- one coarse step

    def step(self, tau_c=None):
        r, h_c = self.r, self.h_c
        if tau_c is None:
            tau_c, tau_f = self.next_taus()
        else:
            tau_f = tau_c / r
        Hc0, Qxc0, Qyc0 = self.c.state()
        self.c.step(tau_c)
        s_pre = self.c.cell_speeds().max()
        # time-integrated coarse face fluxes; x faces (ny, nx+1) carry
        # (H, x-momentum, y-momentum), y faces (ny+1, nx) carry (H, y-momentum, x-momentum)
        cx = [tau_c * f for f in self.c.faces(0)]
        cy = [tau_c * f for f in self.c.faces(1)]
        Hc1, Qxc1, Qyc1 = self.c.state()
        H, Qx, Qy = Hc1.copy(), Qxc1.copy(), Qyc1.copy()
        dH, dQx, dQy = (np.zeros_like(H) for _ in range(3))
        ring = np.zeros(H.shape, dtype=bool)
        tau_k = []
        for P in self.P:
            p, sim = P["spec"], P["sim"]
            nxf, nyf = P["nxf"], P["nyf"]
            fx = [np.zeros((nyf, 2)) for _ in range(3)]   # west / east boundary faces
            fy = [np.zeros((2, nxf)) for _ in range(3)]   # south / north boundary faces
            for s in range(r):
                sim.set_state(*self._frame(P, Hc0, Qxc0, Qyc0, Hc1, Qxc1, Qyc1, s / r))
                sim.step(tau_f)
                Fx, Fy = sim.faces(0), sim.faces(1)
                for q in range(3):
                    fx[q][:, 0] += tau_f * Fx[q][G:G + nyf, G]
                    fx[q][:, 1] += tau_f * Fx[q][G:G + nyf, G + nxf]
                    fy[q][0, :] += tau_f * Fy[q][G, G:G + nxf]
                    fy[q][1, :] += tau_f * Fy[q][G + nyf, G:G + nxf]
            tau_k.append(sim.next_tau())
            if not self.feedback:
                continue
            Hf, Qxf, Qyf = sim.state()
            ci0, cj0, cw, ch = p["ci0"], p["cj0"], p["cw"], p["ch"]
            rows, cols = slice(cj0, cj0 + ch), slice(ci0, ci0 + cw)
            # restriction: mean of the r x r fine cells under each coarse cell
            for src, dst in ((Hf, H), (Qxf, Qx), (Qyf, Qy)):
                blk = src[G:G + nyf, G:G + nxf].reshape(ch, r, cw, r)
                dst[rows, cols] = blk.mean(axis=(1, 3))
            # reflux: (coarse flux - mean of the r fine fluxes through the same
            # coarse face) / h_c, into the uncovered neighbour across that face
            if not self._reflux:
                continue
            fine_x = [fx[q].reshape(ch, r, 2).sum(axis=1) / r for q in range(3)]   # (ch, 2)
            fine_y = [fy[q].reshape(2, cw, r).sum(axis=2) / r for q in range(3)]   # (2, cw)
            for q, tgt in ((0, dH), (1, dQx), (2, dQy)):
                tgt[rows, ci0 - 1] += (cx[q][rows, ci0] - fine_x[q][:, 0]) / h_c
                tgt[rows, ci0 + cw] -= (cx[q][rows, ci0 + cw] - fine_x[q][:, 1]) / h_c
            for q, tgt in ((0, dH), (2, dQx), (1, dQy)):
                tgt[cj0 - 1, cols] += (cy[q][cj0, cols] - fine_y[q][0, :]) / h_c
                tgt[cj0 + ch, cols] -= (cy[q][cj0 + ch, cols] - fine_y[q][1, :]) / h_c
            ring[rows, ci0 - 1] = ring[rows, ci0 + cw] = True
            ring[cj0 - 1, cols] = ring[cj0 + ch, cols] = True
        if self.feedback:
            H, Qx, Qy, clamped = self.ring_update(H, Qx, Qy, dH, dQx, dQy, ring)
            self.ledger += clamped * h_c * h_c
            self.c.set_state(H, Qx, Qy)
            s_post = self.c.cell_speeds()[self.region].max()
            s_pre = max(s_pre, s_post)
        self._set_taus(self.c.tau_from_speed(s_pre), tau_k)

    def ring_update(self, H, Qx, Qy, dH, dQx, dQy, ring):
        """The reflux corrections applied to the ring cells (reading of the
        final update's rules): depth clamped at 0 (the clamped depth is
        returned for the ledger), discharge zeroed where the cell is dry
        after the correction, and the momentum part added with a weight that
        rises from 0 at MOMENTUM_DEPTH to 1 at twice that: the boundary-flux mismatch
        would otherwise give a film at the edge of a box the momentum of the
        patch's flow, and through the friction term of U_p such a film sets
        the CFL step of the whole nest."""
        Hn = H + dH
        Hcl = np.maximum(Hn, 0.0)
        clamped = float((Hcl - Hn)[ring].sum())
        wet = Hcl > self.eps
        # weight of the momentum part: 0 up to MOMENTUM_DEPTH, 1 from twice
        # that, linear between (continuous, so that rounding cannot flip it)
        wgt = np.clip(Hcl / MOMENTUM_DEPTH - 1.0, 0.0, 1.0)
        Qx = np.where(ring, np.where(wet, Qx + wgt * dQx, 0.0), Qx)
        Qy = np.where(ring, np.where(wet, Qy + wgt * dQy, 0.0), Qy)
        return np.where(ring, Hcl, H), Qx, Qy, clamped

    def run(self, n, tau_c=None):
        for _ in range(n):
            self.step(tau_c)

    # -------------------------------------------------------------- queries

    def coarse_state(self):
        return self.c.state()

    def patch_state(self, k):
        P = self.P[k]
        H, Qx, Qy = P["sim"].state()
        sl = (slice(G, G + P["nyf"]), slice(G, G + P["nxf"]))
        return H[sl], Qx[sl], Qy[sl]

    def volume(self):
        """Volume of the nested solution: coarse cells (the covered ones hold
        the restricted fine volume)."""
        return self.c.mass()

    def time(self):
        return self.c.time()

    def inflow(self):
        return self.c.inflow()

    def total_ledger(self):
        return self.c.ledger() + self.ledger
