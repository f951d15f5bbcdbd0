// swe_nest.hpp -- gfx950 kernels of hierarchical (nested) grids.
//
// Method: arXiv 1705.00614, Sec. 2.2 (a hierarchy of grids in which the
// small-scale flow of a zoomed-in area feeds back into the large-scale grid)
// and Sec. 5 (a 50 m global grid with a 12.5 m local grid).  The paper does
// not spell out the coupling; the one implemented here is coarse-first
// subcycling with conservative flux matching.  Per coarse step:
//
//   coarse   one ordinary step of the coarse grid with time step tau_c; the
//            step adds tau_c * flux of the faces bounding every covered box
//            into its taps
//   r times  k_frame fills the frame of every patch (the FRAME cells round
//            its interior, one more than the reach of one step) from the
//            covering coarse cell, linear in time between the coarse layers
//            n and n+1 (depth and discharge interpolated; fine depth
//            H_f = max(0, H_c + b_c - b_fine) and discharge H_f Q_c / H_c
//            where the coarse cell is wet, else dry); then one ordinary
//            step of every patch with tau_c / r,
//            adding tau_f * flux of its interior boundary faces into its taps
//   feedback k_feedback: each covered coarse cell takes the mean of its
//            r x r fine cells; each uncovered cell next to a covered box
//            takes (coarse tap - mean of the r fine taps of the same coarse
//            face) / h_c through that face, with the final update's clamp,
//            ledger and dry rule, the momentum part weighted by the cell's
//            depth after it (NEST_MOMENTUM_DEPTH); then k_nest_close
//            gathers the CFL speed of the changed cells, puts the tiles
//            round the covered boxes on the coarse tile list and clears the
//            taps, its last workgroup setting the steps as below
//   tau      (k_nest_tau without feedback, which also clears the taps)
//            tau_c = min(CFL step of the
//            coarse speeds, r * CFL step of every patch after its last
//            substep), tau_f = tau_c / r, and the coarse hydrograph volume of
//            the next step.
//
// All of it is device work on one stream (capturable in a graph); the host
// only launches.
#pragma once

#include "swe_step.hpp"

namespace swe {

constexpr int NEST_FRAME = 5;   // frame width in fine cells
// patches of a nest at most (the time-step rule reads one per lane of a wave)
constexpr int NEST_MAX_PATCHES = 64;
// ring cells shallower than this [m] after the reflux take its mass but not
// its momentum, twice as deep all of it, linear between (a film moving with
// the patch's flow would set the nest's CFL step through the friction term
// of U_p)
constexpr double NEST_MOMENTUM_DEPTH = 0.05;

template <typename real>
struct NestPatch {
    int ci0, cj0, cw, ch;          // covered coarse box
    int nxe, nye;                  // extended fine grid (interior + frame)
    int frame_base, cov_base;      // prefix sums over the patches: frame cells, covered cells
    int ftap, ctap;                // offsets of the patch's and the coarse box's taps
    real* Hf[2]; real* Qxf[2]; real* Qyf[2];
    const real* bf;
    Ctrl* ctrl;
    const double* mass;            // the patch's per-tile FP64 depth sums
    int ntx, tx, ty;               // its tile columns and tile shape
};

template <typename real>
struct NestArgs {
    const NestPatch<real>* P;
    int np, r, nx, ny;             // patches, refinement, coarse grid
    int nframe, ncov, nring;       // frame cells, covered cells, ring cells (all patches)
    real* Hc[2]; real* Qxc[2]; real* Qyc[2];
    const real* bc;
    real* tap;
    const int* ring_cell;          // coarse cell of each ring cell
    const int* ring_off;           // CSR offsets into ring_face (nring + 1)
    const int* ring_face;          // per face: patch, side (0 W, 1 E, 2 S, 3 N), index along the side
    double* ring_ledger;           // clamp volume per ring cell (accumulated)
    real eps, ih;                  // dry threshold, 1 / h_c
    double h2;                     // h_c^2
    double hold;                   // held coarse step length (0: the CFL rule)
};

__device__ __forceinline__ int floor_div(int a, int r) { return a >= 0 ? a / r : -((-a + r - 1) / r); }

template <typename real>
__device__ __forceinline__ int find_patch(const NestPatch<real>* P, int np, int t, bool frame) {
    int k = 0;
    for (int q = 1; q < np; ++q) k += t >= (frame ? P[q].frame_base : P[q].cov_base);
    return k;
}


// Frame of every patch at time theta in [0, 1) of the coarse step, written to
// the patch buffers pf; the coarse layers n and n+1 are in buffers pc, pc^1.
template <typename real>
__global__ void k_frame(NestArgs<real> n, int pf, int pc, real theta) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n.nframe) return;
    const int k = find_patch(n.P, n.np, t, true);
    const NestPatch<real>& d = n.P[k];
    constexpr int G = NEST_FRAME;
    const int nxe = d.nxe, nye = d.nye;
    int m = t - d.frame_base, fi, fj;
    if (m < G * nxe) {
        fj = m / nxe; fi = m % nxe;
    } else if (m < 2 * G * nxe) {
        m -= G * nxe; fj = nye - G + m / nxe; fi = m % nxe;
    } else {
        m -= 2 * G * nxe;
        fj = G + m / (2 * G);
        const int c = m % (2 * G);
        fi = c < G ? c : nxe - 2 * G + c;
    }
    const int ci = d.ci0 + floor_div(fi - G, n.r), cj = d.cj0 + floor_div(fj - G, n.r);
    const int gc = cj * n.nx + ci, gf = fj * nxe + fi;
    // at theta = 0 the frame is layer n alone (layer n+1 may still be being
    // computed beside this launch): both terms take layer n's value
    const int pn = theta > real(0) ? pc ^ 1 : pc;
    const real u = real(1) - theta;
    const real Hm = u * n.Hc[pc][gc] + theta * n.Hc[pn][gc];
    const bool w = Hm > n.eps;
    const real eta = Hm + n.bc[gc];
    const real Hf = w ? rmax(real(0), eta - d.bf[gf]) : real(0);
    d.Hf[pf][gf] = Hf;
    // the coarse velocity carried by the fine depth (not the coarse
    // discharge, which on a high spot of the fine bed would be a fast film)
    d.Qxf[pf][gf] = w ? Hf * Mth<real>::div(u * n.Qxc[pc][gc] + theta * n.Qxc[pn][gc], Hm) : real(0);
    d.Qyf[pf][gf] = w ? Hf * Mth<real>::div(u * n.Qyc[pc][gc] + theta * n.Qyc[pn][gc], Hm) : real(0);
}

// Restriction of the fine layer (patch buffers pf) into the covered coarse
// cells and the flux correction of the ring cells, both in coarse buffer po.
template <typename real>
__global__ void k_feedback(NestArgs<real> n, int pf, int po) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = n.r;
    if (t < n.ncov) {
        const int k = find_patch(n.P, n.np, t, false);
        const NestPatch<real>& d = n.P[k];
        const int m = t - d.cov_base, cy = m / d.cw, cx = m % d.cw;
        const int gc = (d.cj0 + cy) * n.nx + d.ci0 + cx;
        // a block whose tiles hold no water at all (depth sums exactly 0, so
        // every depth and discharge is +0) restricts to zero without being read
        const int fx0 = NEST_FRAME + cx * r, fy0 = NEST_FRAME + cy * r;
        const int tx0 = fx0 / d.tx, tx1 = (fx0 + r - 1) / d.tx, ty0 = fy0 / d.ty, ty1 = (fy0 + r - 1) / d.ty;
        if (d.mass[ty0 * d.ntx + tx0] == 0.0 && d.mass[ty0 * d.ntx + tx1] == 0.0 &&
            d.mass[ty1 * d.ntx + tx0] == 0.0 && d.mass[ty1 * d.ntx + tx1] == 0.0) {
            n.Hc[po][gc] = real(0);
            n.Qxc[po][gc] = real(0);
            n.Qyc[po][gc] = real(0);
            return;
        }
        double sH = 0.0, sX = 0.0, sY = 0.0;
        for (int jj = 0; jj < r; ++jj)
            for (int ii = 0; ii < r; ++ii) {
                const int gf = (NEST_FRAME + cy * r + jj) * d.nxe + NEST_FRAME + cx * r + ii;
                sH += (double)d.Hf[pf][gf];
                sX += (double)d.Qxf[pf][gf];
                sY += (double)d.Qyf[pf][gf];
            }
        // the restricted cell follows the dry rule of every stored layer: no
        // discharge in a cell with H <= eps (the block mean of a few wet fine
        // cells can leave a dry coarse cell)
        const double inv = 1.0 / (double)(r * r);
        const real Hm = (real)(sH * inv);
        const bool w = Hm > n.eps;
        n.Hc[po][gc] = Hm;
        n.Qxc[po][gc] = w ? (real)(sX * inv) : real(0);
        n.Qyc[po][gc] = w ? (real)(sY * inv) : real(0);
        return;
    }
    const int q = t - n.ncov;
    if (q >= n.nring) return;
    const int gc = n.ring_cell[q];
    real dH = real(0), dQx = real(0), dQy = real(0);
    for (int e = n.ring_off[q]; e < n.ring_off[q + 1]; ++e) {
        const int k = n.ring_face[3 * e], side = n.ring_face[3 * e + 1], idx = n.ring_face[3 * e + 2];
        const NestPatch<real>& d = n.P[k];
        const int nxf = r * d.cw, nyf = r * d.ch;
        const int pc_ = 2 * (d.cw + d.ch), pf_ = 2 * (nxf + nyf);
        const int oc = side == 0 ? idx : side == 1 ? d.ch + idx : side == 2 ? 2 * d.ch + idx : 2 * d.ch + d.cw + idx;
        const int of = side == 0 ? r * idx : side == 1 ? nyf + r * idx
                     : side == 2 ? 2 * nyf + r * idx : 2 * nyf + nxf + r * idx;
        real corr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            real fs = real(0);
            for (int j = 0; j < r; ++j) fs += n.tap[d.ftap + c * pf_ + of + j];
            corr[c] = (n.tap[d.ctap + c * pc_ + oc] - fs / (real)r) * n.ih;
        }
        // the covered box lies east of a W ring cell (its outflow face) and
        // north of an S ring cell
        const real sg = (side == 0 || side == 2) ? real(1) : real(-1);
        dH += sg * corr[0];
        if (side < 2) { dQx += sg * corr[1]; dQy += sg * corr[2]; }
        else { dQy += sg * corr[1]; dQx += sg * corr[2]; }
    }
    const real Hn = n.Hc[po][gc] + dH;
    const real Hcl = rmax(Hn, real(0));
    n.ring_ledger[q] += (double)(Hcl - Hn) * n.h2;
    const bool w = Hcl > n.eps;
    // momentum weight: 0 up to NEST_MOMENTUM_DEPTH, 1 from twice that,
    // linear between (continuous: rounding cannot flip it)
    const real wm = rmin(real(1), rmax(real(0), Hcl / (real)NEST_MOMENTUM_DEPTH - real(1)));
    n.Hc[po][gc] = Hcl;
    n.Qxc[po][gc] = w ? n.Qxc[po][gc] + wm * dQx : real(0);
    n.Qyc[po][gc] = w ? n.Qyc[po][gc] + wm * dQy : real(0);
}

// Cell t of the cells the feedback can change: each covered box widened by
// 2 cells (rects: x0, y0, x1, y1, cell prefix).
__device__ __forceinline__ void region_cell(const int* rects, int nrect, int t, int& gx, int& gy) {
    int k = 0;
    for (int q = 1; q < nrect; ++q) k += t >= rects[5 * q + 4];
    const int* R = rects + 5 * k;
    const int m = t - R[4], w = R[2] - R[0];
    gx = R[0] + m % w;
    gy = R[1] + m / w;
}

// CFL speed of the new coarse layer (buffers of a's input) at cell (gx, gy);
// 0 for a dry cell.
template <typename real>
__device__ real region_speed(const Args<real>& a, int gx, int gy) {
    const real eps = a.eps;
    real Hs[5], ux[5], uy[5];
    const int ox[5] = {0, -1, 1, 0, 0}, oy[5] = {0, 0, 0, -1, 1};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        int fx = 0, fy = 0;
        const int x = mirror(gx + ox[q], a.nx, fx), y = mirror(gy + oy[q], a.ny, fy);
        const int gi = y * a.nx + x;
        const real H = a.Hi[gi];
        real qx = a.Qxi[gi], qy = a.Qyi[gi];
        if (fx & 1) qx = -qx;
        if (fy & 1) qy = -qy;
        const bool wq = H > eps;
        Hs[q] = H;
        ux[q] = wq ? Mth<real>::div(qx, H) : real(0);
        uy[q] = wq ? Mth<real>::div(qy, H) : real(0);
    }
    if (!(Hs[0] > eps)) return real(0);
    Nb4<real> nb;
#pragma unroll
    for (int q = 0; q < 4; ++q) { nb.ux[q] = ux[q + 1]; nb.uy[q] = uy[q + 1]; nb.w[q] = Hs[q + 1] > eps; }
    real fx, fy;
    soft_forces(a, Hs[0], ux[0], uy[0], nb, fx, fy);
    return cfl_speed(a, Hs[0], a.cf[gy * a.nx + gx], ux[0], uy[0], fx, fy);
}

// Lengths of the next coarse step (tc, rounded to the stencil type) and of
// its r substeps; the hydrograph volume of the coarse step follows its clock.
template <typename real>
__device__ void set_nest_steps(const Args<real>& a, const NestArgs<real>& n, double tc) {
    tc = (double)(real)tc;
    set_next_step(a, a.ctrl, tc);
    const double tf = (double)(real)(tc / (double)n.r);
    for (int k = 0; k < n.np; ++k) {
        Ctrl* p = n.P[k].ctrl;
        p->tau = tf;
        p->dV = 0.0;
        p->sdepth = 0.0;
    }
}

// Set the next steps from the host: tc > 0 held, tc = 0 the CFL rule of the
// current layers (speeds recorded by the last coarse step).
template <typename real>
__global__ void k_nest_set_dt(Args<real> a, NestArgs<real> n, double tc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!(tc > 0.0)) {
        tc = cfl_tau_of(a, a.ctrl->speed);
        for (int k = 0; k < n.np; ++k) tc = fmin(tc, (double)n.r * n.P[k].ctrl->tau_cfl);
    }
    set_nest_steps(a, n, tc);
}

// Time steps of the next coarse step and its substeps; errors of any grid
// stop all of them.  `slot` is the coarse list slot of the next step.  Run
// by the first wave of a workgroup (threads 0..63), with every read of the
// control blocks issued before the first write (two memory round trips, not
// one per field and patch): lane k < np reads patch k's CFL step and error,
// lane g < NSEG the coarse list's segment counter g; lane 0 then writes the
// coarse control block and lane k patch k's steps.  With `region`, s_lane is
// a speed maximum gathered besides the control block's, per lane (0 where
// there is none).
template <typename real>
__device__ void nest_tau_rule(const Args<real>& a, const NestArgs<real>& n, int slot, bool region, double s_lane) {
    const int lane = threadIdx.x & 63;
    Ctrl* const c = a.ctrl;
    // reads
    Ctrl* const pc = lane < n.np ? n.P[lane].ctrl : nullptr;
    const double speed = c->speed, prep = prep_speed(c, real(0)), t = c->t;
    const int cerr = c->err;
    const int nseg = a.skip && lane < NSEG ? a.hot[hot_seg(slot, lane)] : 0;
    const double tcf = pc ? (double)n.r * pc->tau_cfl : __builtin_inf();
    const int perr = pc ? pc->err : 0;
    // the rule: tau_c = min(CFL step of the coarse speeds, r * CFL step of
    // every patch), unless held; min and max are exact in any order
    double S = s_lane, tp = tcf;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        S = fmax(S, __shfl_xor(S, o, 64));
        tp = fmin(tp, __shfl_xor(tp, o, 64));
    }
    S = region ? fmax(fmax(speed, prep), S) : fmax(speed, prep);
    const double tc = fmin(cfl_tau_of(a, S), tp);
    const double tcr = (double)(real)(n.hold > 0.0 ? n.hold : tc);
    // the coarse step's scalars (set_next_step's rule) and the substeps'
    const bool bad_step = !(tcr >= a.tau_min) || !(tcr < __builtin_inf());
    double dV = 0.0;
    if (a.nin_h2 > 0.0 && tcr < __builtin_inf())
        dV = hydro_volume(a.q_base, a.q_peak, a.t_peak, a.sigma_t, t, tcr);
    const double tf = (double)(real)(tcr / (double)n.r);
    // the coarse grid's error after the step check, else the first patch's
    int e = bad_step ? -5 : cerr;
    const unsigned long long pm = __ballot(perr != 0);
    const int pe = __shfl(perr, pm ? __ffsll((long long)pm) - 1 : 0, 64);
    if (!e) e = pe;
    int sg[NSEG];
#pragma unroll
    for (int g = 0; g < NSEG; ++g) sg[g] = __shfl(nseg, g, 64);
    // writes
    if (lane == 0) {
        c->prep_speed = 0ull;
        c->speed = S;
        c->tau = tcr;
        c->dV = dV;
        c->sdepth = a.nin_h2 > 0.0 ? (double)(real)(dV / a.nin_h2) : 0.0;
        if (a.skip) close_segments_from(c, sg, slot);
        if (e) { c->err = e; c->err_gate = e; }
    }
    if (pc) {
        pc->tau = tf;
        pc->dV = 0.0;
        pc->sdepth = 0.0;
        if (e) pc->err_gate = e;
    }
}

// The close of a coarse step without feedback: the step rule (first wave
// of block 0) and the taps cleared for the next coarse step (every thread,
// striding; ntap = 0 leaves them).
template <typename real>
__global__ void k_nest_tau(Args<real> a, NestArgs<real> n, int slot, int ntap) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ntap; i += gridDim.x * blockDim.x) n.tap[i] = real(0);
    if (blockIdx.x != 0 || threadIdx.x >= 64) return;
    nest_tau_rule(a, n, slot, false, 0.0);
}

// The close of a two-way coarse step, one launch after k_feedback (at most
// NEST_CLOSE_GRID workgroups of 256 threads, each striding over the work):
// the CFL speed of the new coarse layer on the cells the feedback can change;
// the tiles round the covered boxes put on the coarse list of the next step
// (list `slot`, generation of that list), so that the cells the feedback
// changed are stepped and both buffers of the pair stay consistent; the taps
// cleared for the next coarse step.  The last workgroup to finish sets the
// next steps (k_nest_tau's rule).  Completion uses the coarse grid's group
// words, which are zero between two of its step launches: each workgroup's
// speed maximum and arrival go to its group's words by atomics, the arrival
// issued only once the maximum has returned (so are the workgroup's
// appends, whose results feed its list writes before the barrier), and the
// last arrival of the last group reads and clears them.
constexpr int NEST_CLOSE_GRID = 1024, NEST_CLOSE_CELLS = 4;
template <typename real>
__global__ __launch_bounds__(256) void k_nest_close(Args<real> a, NestArgs<real> n, const int* rects, int nrect,
                                                    int ncells, const int* force, int nforce, int ntap, int slot) {
    constexpr int NT = 256;
    __shared__ real red[NT / 64];
    __shared__ int s_last;
    __shared__ int s_rect[5 * NEST_MAX_PATCHES];
    const int tid = threadIdx.x, G = gridDim.x, grp = blockIdx.x % NSEG;
    for (int i = tid; i < 5 * nrect; i += NT) s_rect[i] = rects[i];
    __syncthreads();
    // the region is mostly dry: the depths of NEST_CLOSE_CELLS cells per
    // thread are loaded together, and only a wet cell loads its neighbours
    real vmax = real(0);
    for (int t0 = blockIdx.x * NT * NEST_CLOSE_CELLS + tid; t0 < ncells; t0 += G * NT * NEST_CLOSE_CELLS) {
        int gx[NEST_CLOSE_CELLS], gy[NEST_CLOSE_CELLS];
        real hc[NEST_CLOSE_CELLS];
#pragma unroll
        for (int u = 0; u < NEST_CLOSE_CELLS; ++u) {
            const int t = t0 + u * NT;
            gx[u] = gy[u] = 0;
            if (t < ncells) region_cell(s_rect, nrect, t, gx[u], gy[u]);
            hc[u] = t < ncells ? a.Hi[gy[u] * a.nx + gx[u]] : real(0);
        }
#pragma unroll
        for (int u = 0; u < NEST_CLOSE_CELLS; ++u)
            if (hc[u] > a.eps) vmax = rmax(vmax, region_speed(a, gx[u], gy[u]));
    }
    const int gen = (int)a.ctrl->step + 1;
    // whole workgroups take each round (the append votes per wave)
    for (int t0 = blockIdx.x * NT; t0 < nforce; t0 += G * NT)
        append_tiles(t0 + tid < nforce ? force[t0 + tid] : -1, 0, 0, gen, a.stamp, a.lists, a.hot, a.ntiles, slot,
                     grp);
    for (int t = blockIdx.x * NT + tid; t < ntap; t += G * NT) n.tap[t] = real(0);
    vmax = wave_max(vmax);
    if ((tid & 63) == 0) red[tid >> 6] = vmax;
    __syncthreads();
    unsigned long long* const h64 = reinterpret_cast<unsigned long long*>(a.hot);
    if (tid == 0) {
        real vm = real(0);
        for (int q = 0; q < NT / 64; ++q) vm = rmax(vm, red[q]);
        const unsigned long long sp = atomicMax(&h64[hot_spd(grp) / 2], (unsigned long long)__double_as_longlong((double)vm));
        const int in_grp = (G - grp + NSEG - 1) / NSEG, ngrp = G < NSEG ? G : NSEG;
        bool last = false;
        if (sp != ~0ull) {        // always (no speed has these bits): waits for the maximum
            const unsigned long long old = atomicAdd(&h64[hot_cnt(grp) / 2], 1ull);
            if ((int)old == in_grp - 1)
                last = atomicAdd((unsigned*)&a.hot[hot_done(NSEG)], 1u) == (unsigned)(ngrp - 1);
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid < 64) {
        const double sg = tid < NSEG ? __longlong_as_double((long long)h64[hot_spd(tid) / 2]) : 0.0;
        nest_tau_rule(a, n, slot, true, sg);
        if (tid < NSEG) { h64[hot_cnt(tid) / 2] = 0ull; h64[hot_spd(tid) / 2] = 0ull; }
        if (tid == 0) a.hot[hot_done(NSEG)] = 0;
    }
}

// Fixed-order sum of a field (volume of the nested solution): per-block
// partials, then k_sum_tiles.
template <typename real>
__global__ void k_field_partials(const real* f, int n, int chunk, double* part) {
    __shared__ double red[256 / 64];
    const int b = blockIdx.x, i0 = b * chunk, i1 = min(n, i0 + chunk);
    double s = 0.0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) s += (double)f[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int q = 0; q < (int)blockDim.x / 64; ++q) v += red[q];
        part[b] = v;
    }
}

}  // namespace swe
