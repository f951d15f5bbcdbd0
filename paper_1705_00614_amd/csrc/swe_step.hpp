// swe_step.hpp -- gfx950 kernels of one CSPH-TVD shallow-water step.
//
// Method: arXiv 1705.00614, Sec. 2.1 (Eqs. 1-4) and Sec. 2.3 (stages I-IV);
// wet-block skipping after Sec. 3 (kernels K1 and K8).  The paper runs eight
// kernels per step, one thread per cell, with every intermediate in global
// memory.  Here one workgroup advances one TX x TY tile through all four
// stages in LDS, so a step reads the state once (H, Qx, Qy, b, c_f) and
// writes it once (H, Qx, Qy):
//
//   load    tile + 5-cell halo of layer n into LDS (mirror images outside the
//           domain = reflective walls)
//   P1      forces at t_n (SPH pressure gradient, viscosity, Coriolis, wind,
//           Manning factor) and the predictor U^{n+1/2} on tile + 4
//   P2      forces at t_{n+1/2}, corrector U^L, sources, post-Lagrangian
//           state on tile + 3
//   FX, FY  limited reconstruction and hydrostatic Rusanov fluxes through the
//           x faces, then the y faces, of tile + 1
//   final   H, Q at t_{n+1} on tile + 1 (written to HBM for the tile)
//   epi     CFL speed of layer n+1 on the tile (needs the ring of tile + 1),
//           wet bits, FP64 volume and clamp partials
//
// The tile list of the next step is built by the workgroups themselves
// (atomic de-duplicated append), and the last workgroup to finish turns the
// maximum speed into the next time step and the next hydrograph volume in
// FP64.  A step is therefore exactly one kernel launch with no host work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

constexpr int HALO = 5;
constexpr double GATE_BED = 1.0e6;

// Device-resident control block of a simulation.
struct Ctrl {
    double t;            // simulated time of the current layer
    double tau;          // time step of the next step (already rounded to the stencil type)
    double dV;           // hydrograph volume of the next step
    double sdepth;       // source depth of the next step (dV / (N_in h^2))
    double inflow;       // hydrograph volume of all completed steps
    double last_tau;     // time step of the last completed step
    unsigned int speed32;          // max speed of the new layer (float bits)
    unsigned int done;             // finished workgroups of the running step
    unsigned long long speed64;    // max speed of the new layer (double bits)
    int count[2];        // tile-list lengths
    int err;             // error raised during the running step
    int err_gate;        // error as of the start of the running step
    long long step;      // completed steps
    long long tiles;     // processed tile-steps
    long long cells;     // processed in-domain cell-steps
};

template <typename real>
struct Args {
    const real* Hi; const real* Qxi; const real* Qyi;   // layer n
    real* Ho; real* Qxo; real* Qyo;                     // layer n+1
    const real* bed; const real* cf;                    // static
    Ctrl* ctrl;
    const int* list_in; int* list_out; int slot;        // tile lists
    int* stamp;                                         // de-duplication stamps
    double* mass;                                       // per-tile sum of H
    double* ledger;                                     // per-tile clamp volume
    int nx, ny, ntx, nty, ntiles, skip, limiter;
    int i0, j0, ni, nj;                                 // inlet rectangle
    real h, ih, g, eps, nuh2, fcor, wx, wy, kw, hw;     // stencil constants
    double h_d, g_d, cfl, tau_max, tau_min, nu_d, nin_h2;
    double q_base, q_peak, t_peak, sigma_t;
};

// ---------------------------------------------------------------- math

template <typename real> struct Mth;
template <> struct Mth<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // x^(-4/3) for x > 0 via the hardware base-2 logarithm and exponential
    static __device__ __forceinline__ float pow_m43(float x) {
        return __builtin_amdgcn_exp2f(-1.33333333f * __builtin_amdgcn_logf(x));
    }
};
template <> struct Mth<double> {
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double pow_m43(double x) { return 1.0 / (x * ::cbrt(x)); }
};

template <typename real> __device__ __forceinline__ real rmax(real a, real b) { return a > b ? a : b; }
template <typename real> __device__ __forceinline__ real rmin(real a, real b) { return a < b ? a : b; }
template <typename real> __device__ __forceinline__ real rabs(real a) { return a < real(0) ? -a : a; }

// Reflect a global index into [0, n) about the end faces; flips counts the
// reflections (odd: the velocity component normal to that wall changes sign).
__device__ __forceinline__ int mirror(int i, int n, int& flips) {
    while (i < 0 || i >= n) {
        i = i < 0 ? -1 - i : 2 * n - 1 - i;
        ++flips;
    }
    return i;
}

// ---------------------------------------------------------------- reductions

template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T u = __shfl_xor(v, o, 64); v = v > u ? v : u; }
    return v;
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- limiter, Riemann

template <typename real>
__device__ __forceinline__ real limit(int kind, real a, real b) {
    if (a * b <= real(0)) return real(0);
    if (kind == 1) return Mth<real>::div(real(2) * a * b, a + b);
    if (kind == 2) {
        real m = rmin(rmin(real(2) * rabs(a), real(2) * rabs(b)), real(0.5) * rabs(a + b));
        return a > real(0) ? m : -m;
    }
    return rabs(a) < rabs(b) ? a : b;
}

template <typename real> struct Face { real H, eta, un, ut; };

// Limited reconstruction on the face of cell c on side `side` (+1: towards
// c+d, -1: towards c-d) from the post-Lagrangian LDS fields.
template <typename real>
__device__ __forceinline__ Face<real> recon(int c, int d, real side, int lim, real eps,
                                            const real* sHt, const real* sEt, const real* sBed,
                                            const real* un, const real* ut) {
    Face<real> f;
    const real Hc = sHt[c];
    if (!(Hc > eps)) {
        f.H = real(0); f.eta = sBed[c]; f.un = real(0); f.ut = real(0);
        return f;
    }
    const int m = c - d, q = c + d;
    const real Hm = sHt[m], Hq = sHt[q];
    const real ec = sEt[c];
    const real sH = limit(lim, Hc - Hm, Hq - Hc);
    const real sE = limit(lim, ec - sEt[m], sEt[q] - ec);
    const bool wm = Hm > eps, wq = Hq > eps;
    const real unc = un[c], utc = ut[c];
    const real sN = limit(lim, wm ? unc - un[m] : real(0), wq ? un[q] - unc : real(0));
    const real sT = limit(lim, wm ? utc - ut[m] : real(0), wq ? ut[q] - utc : real(0));
    const real hs = real(0.5) * side;
    f.H = rmax(real(0), Hc + hs * sH);
    f.eta = ec + hs * sE;
    f.un = unc + hs * sN;
    f.ut = utc + hs * sT;
    return f;
}

template <typename real>
__device__ __forceinline__ void riemann(real g, const Face<real>& L, const Face<real>& R,
                                        real& FH, real& Fn, real& Ft) {
    const real bs = rmax(L.eta - L.H, R.eta - R.H);
    const real hL = rmax(real(0), L.eta - bs), hR = rmax(real(0), R.eta - bs);
    const real a = rmax(rabs(L.un) + Mth<real>::sqrt(g * hL), rabs(R.un) + Mth<real>::sqrt(g * hR));
    const real qL = hL * L.un, qR = hR * R.un;
    FH = real(0.5) * (qL + qR) - real(0.5) * a * (hR - hL);
    Fn = real(0.5) * (qL * L.un + qR * R.un) - real(0.5) * a * (qR - qL);
    Ft = real(0.5) * (qL * L.ut + qR * R.ut) - real(0.5) * a * (hR * R.ut - hL * L.ut);
}

// ---------------------------------------------------------------- forces

// Viscosity over wet face neighbours + Coriolis + wind at cell s for the
// velocity field (ux, uy); H is the cell's depth at layer n.
template <typename real, int W>
__device__ __forceinline__ void soft_forces(const Args<real>& a, int s, const real* ux, const real* uy,
                                            const uint8_t* wet, real H, real& fx, real& fy) {
    const real uxc = ux[s], uyc = uy[s];
    real vx = real(0), vy = real(0);
    if (wet[s - 1]) { vx += ux[s - 1] - uxc; vy += uy[s - 1] - uyc; }
    if (wet[s + 1]) { vx += ux[s + 1] - uxc; vy += uy[s + 1] - uyc; }
    if (wet[s - W]) { vx += ux[s - W] - uxc; vy += uy[s - W] - uyc; }
    if (wet[s + W]) { vx += ux[s + W] - uxc; vy += uy[s + W] - uyc; }
    const real dx = a.wx - uxc, dy = a.wy - uyc;
    const real k = a.kw * Mth<real>::sqrt(dx * dx + dy * dy) * Mth<real>::rcp(rmax(H, a.hw));
    fx = a.nuh2 * vx + a.fcor * uyc + k * dx;
    fy = a.nuh2 * vy - a.fcor * uxc + k * dy;
}

// CFL speed max(U_s, U_p) of a wet cell (Sec. 2.3, stage I).  F is the
// explicitly integrated force (viscosity, Coriolis, wind); the point-implicit
// friction cannot reverse a particle and sets no limit.
template <typename real>
__device__ __forceinline__ real cfl_speed(const Args<real>& a, real H, real ux, real uy,
                                          real fx, real fy) {
    const real us = rmax(rabs(ux), rabs(uy)) + Mth<real>::sqrt(a.g * H);
    const real sx = fx > real(0) ? real(1) : (fx < real(0) ? real(-1) : real(0));
    const real sy = fy > real(0) ? real(1) : (fy < real(0) ? real(-1) : real(0));
    const real upx = rabs(ux + sx * Mth<real>::sqrt(a.h * rabs(fx)));
    const real upy = rabs(uy + sy * Mth<real>::sqrt(a.h * rabs(fy)));
    return rmax(us, rmax(upx, upy));
}

__device__ __forceinline__ void atomic_max_speed(Ctrl* c, float v) {
    atomicMax(&c->speed32, __float_as_uint(v));
}
__device__ __forceinline__ void atomic_max_speed(Ctrl* c, double v) {
    atomicMax(&c->speed64, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ double read_speed(const Ctrl* c, float) { return (double)__uint_as_float(c->speed32); }
__device__ __forceinline__ double read_speed(const Ctrl* c, double) { return __longlong_as_double((long long)c->speed64); }

// Inflow volume over [t, t+tau] of the Gaussian hydrograph (closed form, FP64).
__device__ __forceinline__ double hydro_volume(double qb, double qp, double tp, double st,
                                               double t, double tau) {
    double v = qb * tau;
    if (st > 0.0 && qp != qb) {
        const double k = 1.0 / (st * 1.4142135623730951);
        v += (qp - qb) * st * 1.2533141373155001 /* sqrt(pi/2) */ * (erf((t + tau - tp) * k) - erf((t - tp) * k));
    }
    return v;
}

// Next time step and source from the maximum speed of the new layer.
template <typename real>
__device__ void next_step_scalars(const Args<real>& a, Ctrl* c) {
    const double S = read_speed(c, real(0));
    double tau = a.tau_max > 0.0 ? a.tau_max : __builtin_inf();
    if (S > 0.0) tau = fmin(tau, a.cfl * a.h_d / S);
    if (a.nu_d > 0.0) tau = fmin(tau, a.h_d * a.h_d / (4.0 * a.nu_d));
    tau = (double)(real)tau;
    if (!(tau >= a.tau_min) || !(tau < __builtin_inf())) c->err = -5;
    c->tau = tau;
    double dV = 0.0;
    if (a.nin_h2 > 0.0 && tau < __builtin_inf())
        dV = hydro_volume(a.q_base, a.q_peak, a.t_peak, a.sigma_t, c->t, tau);
    c->dV = dV;
    c->sdepth = a.nin_h2 > 0.0 ? (double)(real)(dV / a.nin_h2) : 0.0;
    c->speed32 = 0u;
    c->speed64 = 0ull;
}

__device__ __forceinline__ void enqueue(int tile, int gen, int* stamp, int* list, int* count) {
    if (atomicMax(&stamp[tile], gen) < gen) list[atomicAdd(count, 1)] = tile;
}

// ---------------------------------------------------------------- step kernel

template <typename real, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step(Args<real> a) {
    constexpr int W = TX + 2 * HALO, HH = TY + 2 * HALO, N = W * HH;
    constexpr int W4 = TX + 8, N4 = W4 * (TY + 8);
    constexpr int W3 = TX + 6, N3 = W3 * (TY + 6);
    constexpr int W1 = TX + 2, N1 = W1 * (TY + 2);
    constexpr int M1 = (N1 + NT - 1) / NT;   // R1 cells per thread
    constexpr int NWAVE = NT / 64;

    // LDS, all arrays share the halo-5 layout: cell (lx, ly) at (ly+5)*W + lx+5
    __shared__ real A0[N];   // H^n             -> eta_t
    __shared__ real A1[N];   // b               -> H^{n+1}
    __shared__ real A2[N];   // Ux^n            -> H_t
    __shared__ real A3[N];   // Uy^n            -> Ux_t
    __shared__ real A4[N];   // Ux^{n+1/2}      -> flux F_H
    __shared__ real A5[N];   // Uy^{n+1/2}      -> flux F normal
    __shared__ real A6[N];   // G_x             -> Qx_t -> Ux^{n+1}
    __shared__ real A7[N];   // G_y             -> Qy_t -> Uy^{n+1}
    __shared__ real A8[N];   // c_f/H^(4/3)     -> flux F tangential
    __shared__ real A9[N];   // Uy_t
    __shared__ uint8_t WET[N];
    __shared__ double red_d[2][NWAVE];
    __shared__ int red_i[NWAVE];
    __shared__ int s_last;

    Ctrl* const ctrl = a.ctrl;
    if (ctrl->err_gate) return;
    const int tid = threadIdx.x;
    const int count = a.skip ? ctrl->count[a.slot] : a.ntiles;
    const real tau = (real)ctrl->tau;
    const real sdep = (real)ctrl->sdepth;
    const real half_tau = real(0.5) * tau;
    const real r = tau * a.ih;
    const int gen = (int)ctrl->step + 2;
    const int nx = a.nx, ny = a.ny;
    const real eps = a.eps;
    // normalised cubic-B-spline SPH gradient weights (smoothing length h):
    // al = 1/(12 sqrt2 - 14), be = (3 sqrt2 - 4)/(12 sqrt2 - 14), 2 al + 4 be = 1
    const real al = real(0.33663655161388173), be = real(0.08168172419305914);

    real vmax = real(0);
    bool bad = false;
    long long ncells = 0;

    for (int p = blockIdx.x; p < count; p += gridDim.x) {
        const int tile = a.skip ? a.list_in[p] : p;
        const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
        ncells += (long long)min(TX, nx - tx0) * min(TY, ny - ty0);
        const bool edge = tx0 < HALO || ty0 < HALO || tx0 + TX + HALO > nx || ty0 + TY + HALO > ny;
        __syncthreads();   // LDS of the previous tile is free

        // ---- load tile + 5 (mirror images outside the domain)
        int act_n = 0;
        for (int k = tid; k < N; k += NT) {
            const int lx = k % W - HALO, ly = k / W - HALO;
            int fx = 0, fy = 0;
            const int gx = mirror(tx0 + lx, nx, fx), gy = mirror(ty0 + ly, ny, fy);
            const long gi = (long)gy * nx + gx;
            const real H = a.Hi[gi];
            real qx = a.Qxi[gi], qy = a.Qyi[gi];
            if (fx & 1) qx = -qx;
            if (fy & 1) qy = -qy;
            const bool w = H > eps;
            const real iH = w ? Mth<real>::rcp(H) : real(0);
            A0[k] = H;
            A1[k] = a.bed[gi];
            A2[k] = qx * iH;
            A3[k] = qy * iH;
            WET[k] = (uint8_t)w;
            // K1 rule at layer n: own cells and outer face neighbours (no corners)
            const bool in_tile = lx >= 0 && lx < TX && ly >= 0 && ly < TY;
            const bool ring = ((lx == -1 || lx == TX) && ly >= 0 && ly < TY) ||
                              ((ly == -1 || ly == TY) && lx >= 0 && lx < TX);
            const int gxr = tx0 + lx, gyr = ty0 + ly;
            const bool in_dom = gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny;
            if ((in_tile || ring) && in_dom) {
                const bool src = (unsigned)(gxr - a.i0) < (unsigned)a.ni && (unsigned)(gyr - a.j0) < (unsigned)a.nj;
                if (w || src) act_n = 1;
            }
        }
        act_n = __syncthreads_or(act_n);

        // ---- P1: forces at t_n and predictor on tile + 4
        for (int k = tid; k < N4; k += NT) {
            const int lx = k % W4 - 4, ly = k / W4 - 4;
            const int gx = tx0 + lx, gy = ty0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            const int s = (ly + HALO) * W + lx + HALO;
            if (!WET[s]) {
                A4[s] = real(0); A5[s] = real(0); A6[s] = real(0); A7[s] = real(0); A8[s] = real(0);
                continue;
            }
            const real Hc = A0[s], bc = A1[s], ec = Hc + bc;
            real e[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                // level a neighbour shows: it pushes with at most its own depth
                // above the own surface and never from below the own bed (a dry
                // neighbour has depth 0 and level = its bed)
                const int m = s + (q / 3 - 1) * W + (q % 3 - 1);
                const bool wm = WET[m];
                const real Hm = wm ? A0[m] : real(0);
                const real em = wm ? A0[m] + A1[m] : A1[m];
                e[q] = rmax(bc, rmin(em, ec + Hm));
            }
            // e: 0 SW 1 S 2 SE 3 W 4 C 5 E 6 NW 7 N 8 NE
            const real Gx = (al * (e[5] - e[3]) + be * ((e[8] - e[6]) + (e[2] - e[0]))) * a.ih;
            const real Gy = (al * (e[7] - e[1]) + be * ((e[8] - e[2]) + (e[6] - e[0]))) * a.ih;
            const long gi = (long)gy * nx + gx;
            const real lam0 = a.cf[gi] * Mth<real>::pow_m43(Hc);
            real fx, fy;
            soft_forces<real, W>(a, s, A2, A3, WET, Hc, fx, fy);
            const real ux = A2[s], uy = A3[s];
            const real ax = -a.g * Gx + fx, ay = -a.g * Gy + fy;
            const real lam = lam0 * Mth<real>::sqrt(ux * ux + uy * uy);
            const real id = Mth<real>::rcp(real(1) + half_tau * lam);
            A4[s] = (ux + half_tau * ax) * id;
            A5[s] = (uy + half_tau * ay) * id;
            A6[s] = Gx;
            A7[s] = Gy;
            A8[s] = lam0;
        }
        __syncthreads();
        if (edge) {   // mirror images of U^{n+1/2} outside the domain
            for (int k = tid; k < N4; k += NT) {
                const int lx = k % W4 - 4, ly = k / W4 - 4;
                const int gx = tx0 + lx, gy = ty0 + ly;
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) continue;
                int fx = 0, fy = 0;
                const int mx = mirror(gx, nx, fx) - tx0, my = mirror(gy, ny, fy) - ty0;
                const int s = (ly + HALO) * W + lx + HALO, m = (my + HALO) * W + mx + HALO;
                A4[s] = (fx & 1) ? -A4[m] : A4[m];
                A5[s] = (fy & 1) ? -A5[m] : A5[m];
            }
            __syncthreads();
        }

        // ---- P2: forces at t_{n+1/2}, corrector, sources on tile + 3
        for (int k = tid; k < N3; k += NT) {
            const int lx = k % W3 - 3, ly = k / W3 - 3;
            const int gx = tx0 + lx, gy = ty0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            const int s = (ly + HALO) * W + lx + HALO;
            const real Hc = A0[s];
            real qx = real(0), qy = real(0);
            if (WET[s]) {
                real fx, fy;
                soft_forces<real, W>(a, s, A4, A5, WET, Hc, fx, fy);
                const real hx = A4[s], hy = A5[s];
                const real ax = -a.g * A6[s] + fx, ay = -a.g * A7[s] + fy;
                const real lam = A8[s] * Mth<real>::sqrt(hx * hx + hy * hy);
                const real id = Mth<real>::rcp(real(1) + tau * lam);
                qx = Hc * ((A2[s] + tau * ax) * id);
                qy = Hc * ((A3[s] + tau * ay) * id);
            }
            const bool src = (unsigned)(gx - a.i0) < (unsigned)a.ni && (unsigned)(gy - a.j0) < (unsigned)a.nj;
            const real Ht = src ? Hc + sdep : Hc;
            const bool wt = Ht > eps;
            const real iH = wt ? Mth<real>::rcp(Ht) : real(0);
            A0[s] = Ht + A1[s];   // eta_t
            A2[s] = Ht;
            A3[s] = qx * iH;
            A9[s] = qy * iH;
            A6[s] = qx;
            A7[s] = qy;
        }
        __syncthreads();
        if (edge) {   // mirror images of the post-Lagrangian fields
            for (int k = tid; k < N3; k += NT) {
                const int lx = k % W3 - 3, ly = k / W3 - 3;
                const int gx = tx0 + lx, gy = ty0 + ly;
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) continue;
                int fx = 0, fy = 0;
                const int mx = mirror(gx, nx, fx) - tx0, my = mirror(gy, ny, fy) - ty0;
                const int s = (ly + HALO) * W + lx + HALO, m = (my + HALO) * W + mx + HALO;
                A0[s] = A0[m];
                A2[s] = A2[m];
                A3[s] = (fx & 1) ? -A3[m] : A3[m];
                A9[s] = (fy & 1) ? -A9[m] : A9[m];
            }
            __syncthreads();
        }

        // ---- FX: x faces of rows -1..TY, face i between cells i-1 and i
        constexpr int NFX = (W1 + 1) * (TY + 2);
        for (int k = tid; k < NFX; k += NT) {
            const int lx = k % (W1 + 1) - 1, ly = k / (W1 + 1) - 1;
            const int s = (ly + HALO) * W + lx + HALO;
            const Face<real> L = recon<real>(s - 1, 1, real(1), a.limiter, eps, A2, A0, A1, A3, A9);
            const Face<real> R = recon<real>(s, 1, real(-1), a.limiter, eps, A2, A0, A1, A3, A9);
            real FH, Fn, Ft;
            riemann<real>(a.g, L, R, FH, Fn, Ft);
            A4[s] = FH; A5[s] = Fn; A8[s] = Ft;
        }
        __syncthreads();
        real dH[M1], dQx[M1], dQy[M1];
#pragma unroll
        for (int m = 0; m < M1; ++m) {
            const int k = tid + m * NT;
            if (k < N1) {
                const int lx = k % W1 - 1, ly = k / W1 - 1;
                const int s = (ly + HALO) * W + lx + HALO;
                dH[m] = A4[s] - A4[s + 1];
                dQx[m] = A5[s] - A5[s + 1];
                dQy[m] = A8[s] - A8[s + 1];
            }
        }
        __syncthreads();

        // ---- FY: y faces of columns -1..TX, face j between cells j-1 and j
        constexpr int NFY = W1 * (TY + 3);
        for (int k = tid; k < NFY; k += NT) {
            const int lx = k % W1 - 1, ly = k / W1 - 1;
            const int s = (ly + HALO) * W + lx + HALO;
            const Face<real> L = recon<real>(s - W, W, real(1), a.limiter, eps, A2, A0, A1, A9, A3);
            const Face<real> R = recon<real>(s, W, real(-1), a.limiter, eps, A2, A0, A1, A9, A3);
            real FH, Fn, Ft;
            riemann<real>(a.g, L, R, FH, Fn, Ft);
            A4[s] = FH; A5[s] = Fn; A8[s] = Ft;
        }
        __syncthreads();

        // ---- final update on tile + 1
        double msum = 0.0, lsum = 0.0;
#pragma unroll
        for (int m = 0; m < M1; ++m) {
            const int k = tid + m * NT;
            if (k >= N1) continue;
            const int lx = k % W1 - 1, ly = k / W1 - 1;
            const int gx = tx0 + lx, gy = ty0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            const int s = (ly + HALO) * W + lx + HALO;
            const real Hn = A2[s] + r * (dH[m] + (A4[s] - A4[s + W]));
            const real qx = A6[s] + r * (dQx[m] + (A8[s] - A8[s + W]));
            const real qy = A7[s] + r * (dQy[m] + (A5[s] - A5[s + W]));
            const real Hc = rmax(Hn, real(0));
            const bool w = Hc > eps;
            const real iH = w ? Mth<real>::rcp(Hc) : real(0);
            const real qxo = w ? qx : real(0), qyo = w ? qy : real(0);
            A1[s] = Hc;
            A6[s] = qxo * iH;
            A7[s] = qyo * iH;
            if (lx >= 0 && lx < TX && ly >= 0 && ly < TY) {
                const long gi = (long)gy * nx + gx;
                a.Ho[gi] = Hc;
                a.Qxo[gi] = qxo;
                a.Qyo[gi] = qyo;
                msum += (double)Hc;
                lsum += (double)(Hc - Hn);
                bad |= !(rabs(Hc) < real(1e30)) || !(rabs(qxo) < real(1e30)) || !(rabs(qyo) < real(1e30));
            }
        }
        __syncthreads();
        if (edge) {   // mirror images of the new layer on the ring
            for (int k = tid; k < N1; k += NT) {
                const int lx = k % W1 - 1, ly = k / W1 - 1;
                const int gx = tx0 + lx, gy = ty0 + ly;
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) continue;
                int fx = 0, fy = 0;
                const int mx = mirror(gx, nx, fx) - tx0, my = mirror(gy, ny, fy) - ty0;
                const int s = (ly + HALO) * W + lx + HALO, m = (my + HALO) * W + mx + HALO;
                A1[s] = A1[m];
                A6[s] = (fx & 1) ? -A6[m] : A6[m];
                A7[s] = (fy & 1) ? -A7[m] : A7[m];
            }
            __syncthreads();
        }
        // wet flags of layer n+1 on tile + 1 for the epilogue
        for (int k = tid; k < N1; k += NT) {
            const int lx = k % W1 - 1, ly = k / W1 - 1;
            const int s = (ly + HALO) * W + lx + HALO;
            WET[s] = (uint8_t)(A1[s] > eps);
        }
        __syncthreads();

        // ---- epilogue on the tile: CFL speed of layer n+1 and flags
        int own = 0, eW = 0, eE = 0, eS = 0, eN = 0, ringf = 0;
        for (int k = tid; k < N1; k += NT) {
            const int lx = k % W1 - 1, ly = k / W1 - 1;
            const int gx = tx0 + lx, gy = ty0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            const int s = (ly + HALO) * W + lx + HALO;
            const bool w = WET[s];
            const bool src = (unsigned)(gx - a.i0) < (unsigned)a.ni && (unsigned)(gy - a.j0) < (unsigned)a.nj;
            const bool in_tile = lx >= 0 && lx < TX && ly >= 0 && ly < TY;
            if (!in_tile) {   // ring cell: outer face neighbour, corners excluded
                const bool corner = (lx < 0 || lx >= TX) && (ly < 0 || ly >= TY);
                if (!corner && (w || src)) ringf = 1;
                continue;
            }
            if (w || src) {
                own = 1;
                if (lx == 0) eW = 1;
                if (lx == TX - 1) eE = 1;
                if (ly == 0) eS = 1;
                if (ly == TY - 1) eN = 1;
            }
            if (w) {
                const real H = A1[s];
                real fx, fy;
                soft_forces<real, W>(a, s, A6, A7, WET, H, fx, fy);
                vmax = rmax(vmax, cfl_speed(a, H, A6[s], A7[s], fx, fy));
            }
        }
        // block reductions: flags, volume and ledger partials
        const int lane = tid & 63, wv = tid >> 6;
        int bits = own | (eW << 1) | (eE << 2) | (eS << 3) | (eN << 4) | (ringf << 5);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bits |= __shfl_xor(bits, o, 64);
        msum = wave_sum(msum);
        lsum = wave_sum(lsum);
        if (lane == 0) { red_i[wv] = bits; red_d[0][wv] = msum; red_d[1][wv] = lsum; }
        __syncthreads();
        if (tid == 0) {
            int bb = 0;
            double ms = 0.0, ls = 0.0;
            for (int q = 0; q < NWAVE; ++q) { bb |= red_i[q]; ms += red_d[0][q]; ls += red_d[1][q]; }
            a.mass[tile] = ms;
            a.ledger[tile] += ls * a.h_d * a.h_d;
            if (a.skip) {
                const int ti = tile % a.ntx, tj = tile / a.ntx;
                int* cnt = &ctrl->count[a.slot ^ 1];
                if (act_n || (bb & 1) || (bb & 32)) enqueue(tile, gen, a.stamp, a.list_out, cnt);
                if ((bb & 2) && ti > 0) enqueue(tile - 1, gen, a.stamp, a.list_out, cnt);
                if ((bb & 4) && ti < a.ntx - 1) enqueue(tile + 1, gen, a.stamp, a.list_out, cnt);
                if ((bb & 8) && tj > 0) enqueue(tile - a.ntx, gen, a.stamp, a.list_out, cnt);
                if ((bb & 16) && tj < a.nty - 1) enqueue(tile + a.ntx, gen, a.stamp, a.list_out, cnt);
            }
        }
    }

    // ---- completion: maximum speed, error flag, last workgroup finalises
    vmax = wave_max(vmax);
    const int lane = tid & 63, wv = tid >> 6;
    __syncthreads();
    if (lane == 0) red_d[0][wv] = (double)vmax;
    int anybad = __syncthreads_or((int)bad);
    if (tid == 0) {
        double vm = 0.0;
        for (int q = 0; q < NWAVE; ++q) vm = fmax(vm, red_d[0][q]);
        if (vm > 0.0) atomic_max_speed(ctrl, (real)vm);
        if (anybad) atomicCAS(&ctrl->err, 0, -4);
        if (ncells) atomicAdd((unsigned long long*)&ctrl->cells, (unsigned long long)ncells);
        __threadfence();
        const unsigned prev = atomicAdd(&ctrl->done, 1u);
        s_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && tid == 0) {
        __threadfence();
        const double tau_done = ctrl->tau;
        ctrl->t += tau_done;
        ctrl->inflow += ctrl->dV;
        ctrl->last_tau = tau_done;
        ctrl->step += 1;
        ctrl->tiles += count;
        if (a.skip) ctrl->count[a.slot] = 0;
        next_step_scalars(a, ctrl);
        ctrl->done = 0u;
        if (ctrl->err) ctrl->err_gate = ctrl->err;
        __threadfence();
    }
}

// ---------------------------------------------------------------- preparation kernel
// Layer-0 (or restored layer) bookkeeping: CFL speed, wet tiles, volume
// partials.  One workgroup per tile; needs only a 1-cell ring.
template <typename real, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_prepare(Args<real> a) {
    constexpr int W = TX + 2, N = W * (TY + 2);
    constexpr int NWAVE = NT / 64;
    __shared__ real sH[N], sUx[N], sUy[N];
    __shared__ uint8_t WET[N];
    __shared__ double red_d[NWAVE];
    __shared__ real red_v[NWAVE];
    __shared__ int red_i[NWAVE];
    const int tid = threadIdx.x, tile = blockIdx.x;
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    const int nx = a.nx, ny = a.ny;
    for (int k = tid; k < N; k += NT) {
        const int lx = k % W - 1, ly = k / W - 1;
        int fx = 0, fy = 0;
        const int gx = mirror(tx0 + lx, nx, fx), gy = mirror(ty0 + ly, ny, fy);
        const long gi = (long)gy * nx + gx;
        const real H = a.Hi[gi];
        real qx = a.Qxi[gi], qy = a.Qyi[gi];
        if (fx & 1) qx = -qx;
        if (fy & 1) qy = -qy;
        const bool w = H > a.eps;
        const real iH = w ? Mth<real>::rcp(H) : real(0);
        sH[k] = H; sUx[k] = qx * iH; sUy[k] = qy * iH; WET[k] = (uint8_t)w;
    }
    __syncthreads();
    real vmax = real(0);
    double msum = 0.0;
    int act = 0;
    for (int k = tid; k < N; k += NT) {
        const int lx = k % W - 1, ly = k / W - 1;
        const int gx = tx0 + lx, gy = ty0 + ly;
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
        const bool in_tile = lx >= 0 && lx < TX && ly >= 0 && ly < TY;
        const bool corner = (lx < 0 || lx >= TX) && (ly < 0 || ly >= TY);
        if (corner) continue;
        const bool src = (unsigned)(gx - a.i0) < (unsigned)a.ni && (unsigned)(gy - a.j0) < (unsigned)a.nj;
        if (WET[k] || src) act = 1;
        if (!in_tile) continue;
        const real H = sH[k];
        msum += (double)H;
        if (WET[k]) {
            real fx, fy;
            soft_forces<real, W>(a, k, sUx, sUy, WET, H, fx, fy);
            vmax = rmax(vmax, cfl_speed(a, H, sUx[k], sUy[k], fx, fy));
        }
    }
    vmax = wave_max(vmax);
    msum = wave_sum(msum);
    int any = act;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) any |= __shfl_xor(any, o, 64);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) { red_v[wv] = vmax; red_d[wv] = msum; red_i[wv] = any; }
    __syncthreads();
    if (tid == 0) {
        real vm = real(0);
        double ms = 0.0;
        int ac = 0;
        for (int q = 0; q < NWAVE; ++q) { vm = rmax(vm, red_v[q]); ms += red_d[q]; ac |= red_i[q]; }
        a.mass[tile] = ms;
        if (vm > real(0)) atomic_max_speed(a.ctrl, vm);
        if (a.skip && ac) enqueue(tile, (int)a.ctrl->step + 1, a.stamp, a.list_out, &a.ctrl->count[a.slot]);
    }
}

template <typename real>
__global__ void k_prepare_finish(Args<real> a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctrl* c = a.ctrl;
        c->err = 0;
        c->err_gate = 0;
        c->done = 0u;
        next_step_scalars(a, c);
        if (c->err) c->err_gate = c->err;
    }
}

// Fixed-order FP64 sum of per-tile partials (one workgroup of 1024 threads).
__global__ void k_sum_tiles(const double* part, int n, double* out);

}  // namespace swe
