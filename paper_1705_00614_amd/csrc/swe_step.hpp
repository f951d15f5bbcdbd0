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
//   FX      limited reconstruction and hydrostatic Rusanov fluxes through the
//           x faces of tile + 1
//   FY      the same through the y faces, fused with the final update of
//           tile + 1 (written to HBM for the tile)
//   epi     CFL speed of layer n+1 on the tile (needs the ring of tile + 1),
//           wet bits, FP64 volume and clamp partials
//
// Work layout: in P1, P2 and FX a thread owns a run of cells along x, in FY
// a run along y (2-4 cells, per stage and precision), so neighbour values and
// limited slopes are loaded and computed once per run instead of once per
// use.  Lanes of a wave stride
// LDS rows (row pitch odd) or columns, which keeps LDS accesses free of bank
// conflicts.  Wet/dry decisions are selects, not branches.
//
// The tile list of the next step is built by the workgroups themselves
// (atomic de-duplicated append), and the last workgroup to finish turns the
// maximum speed into the next time step and the next hydrograph volume in
// FP64.  A step is therefore exactly one kernel launch with no host work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

namespace swe {

constexpr int HALO = 5;
constexpr double GATE_BED = 1.0e6;

// Tile lists and completion counters.  Same-address device atomics
// serialise (~11 ns each on this part), so nothing per workgroup goes to one
// address: the workgroups of a step form NSEG groups, each with its own
// completion counter and its own segment of the next tile list, every counter
// on its own 256-byte line; per-workgroup maxima are plain stores reduced by
// the last workgroup.
constexpr int NSEG = 8;
constexpr int LINE = 64;   // ints per 256-byte line
__host__ __device__ constexpr int hot_done(int g) { return g * LINE; }          // g < NSEG; NSEG: all groups
__host__ __device__ constexpr int hot_seg(int slot, int g) { return (NSEG + 1 + slot * NSEG + g) * LINE; }
// Completion of a single-grid step, per group g: a 64-bit word that counts
// arrivals (low 11 bits) and sums processed cells (above), and a 64-bit
// maximum of the workgroups' speeds (bits of a non-negative double).
constexpr int CNT_BITS = 11;
__host__ __device__ constexpr int hot_cnt(int g) { return (NSEG + 1 + 2 * NSEG + g) * LINE; }
__host__ __device__ constexpr int hot_spd(int g) { return (NSEG + 1 + 3 * NSEG + g) * LINE; }
constexpr int HOT_INTS = (NSEG + 1 + 4 * NSEG) * LINE;

// Device-resident control block of a simulation.
struct Ctrl {
    double t;            // simulated time of the current layer
    double tau;          // time step of the next step (already rounded to the stencil type)
    double dV;           // hydrograph volume of the next step
    double sdepth;       // source depth of the next step (dV / (N_in h^2))
    double inflow;       // hydrograph volume of all completed steps
    double last_tau;     // time step of the last completed step
    unsigned long long prep_speed;  // max speed of the new layer gathered by atomics (preparation
                                    // kernel; batch step), bits of the stencil type
    int seg_off[2][NSEG + 1];       // prefix offsets of the list segments, per list slot
    int err;             // error raised during the running step
    int err_gate;        // error as of the start of the running step
    long long step;      // completed steps
    long long tiles;     // processed tile-steps
    long long cells;     // processed in-domain cell-steps
    double speed;        // maximum CFL speed of the current layer
    double tau_cfl;      // CFL time step of the current layer (rounded to the stencil type)
};

// A tile-list entry packs the scenario of a batch (0 for a single grid) above
// the tile index of that scenario's grid.
constexpr int TILE_BITS = 20;
__host__ __device__ constexpr int pack_entry(int sid, int tile) { return (sid << TILE_BITS) | tile; }
__host__ __device__ constexpr int entry_sid(int e) { return e >> TILE_BITS; }
__host__ __device__ constexpr int entry_tile(int e) { return e & ((1 << TILE_BITS) - 1); }

template <typename real>
struct Args {
    const real* Hi; const real* Qxi; const real* Qyi;   // layer n
    real* Ho; real* Qxo; real* Qyo;                     // layer n+1
    const real* bed; const real* cf;                    // static
    Ctrl* ctrl;                                         // this grid: clock, time step, source, errors
    Ctrl* lctrl;                                        // the tile lists (the batch's for an ensemble)
    int sid, tile_base;                                 // scenario index; its first stamp
    int* hot;                                           // counters, one per 256-byte line
    int* lists;                                         // [2 slots][NSEG segments][ntiles]
    int slot;                                           // list slot read by this step
    int* stamp;                                         // de-duplication stamps
    real* wg_speed;                                     // per-workgroup maximum speed
    long long* wg_cells;                                // per-workgroup processed cells
    double* mass;                                       // per-tile sum of H
    double* ledger;                                     // per-tile clamp volume
    int nx, ny, ntx, nty, ntiles, skip, limiter;
    int periodic;                                       // 1: the domain wraps in x and y (no walls)
    int list_cap;                                       // capacity of one list segment
    int i0, j0, ni, nj;                                 // inlet rectangle
    real h, ih, g, eps, nuh2, fcor, wx, wy, kw, hw;     // stencil constants
    double h_d, g_d, cfl, tau_max, tau_min, nu_d, nin_h2;
    double q_base, q_peak, t_peak, sigma_t;
    // nested grids: the step leaves tau, dV and sdepth to the nest (hold);
    // tap rectangles [x0, y0, x1, y1, offset] whose boundary-face fluxes
    // (times tau) the step adds into tap (TAP kernels only)
    int hold, ntap;
    const int* tap_rect;
    real* tap;
    // learned flux corrections through the east and north face of each cell,
    // 3 planes (mass, x-momentum, y-momentum) of nx*ny (CORR kernels only)
    const real* corrE;
    const real* corrN;
    real corr_hmin;      // correction depth (>= eps): upwind cell for mass, both cells for momentum
    // face taps on the lines of a grid coarsened by tap_r (TAP kernels with
    // tap_r > 0): tau * flux of the x faces at columns that are multiples of
    // tap_r, per row, in tapx [3][ny][nx/tap_r + 1], and of the y faces at
    // rows that are multiples of tap_r, per column, in tapy [3][ny/tap_r + 1][nx]
    int tap_r;
    real* tapx;
    real* tapy;
    // tiles stepped every step of a skipping grid whatever the list holds
    // (patches of a nest: the tiles holding the frame, which the nest
    // rewrites between steps): ring_tiles[nring], and the bounds that make
    // a tile one of them (column <= ring_x0 or >= ring_x1, row <= ring_y0 or
    // >= ring_y1); such tiles are never put on the list
    const int* ring_tiles;
    int nring, ring_x0, ring_x1, ring_y0, ring_y1;
    // source rate field sigma(x, y) [m/s] (rain > 0, losses < 0; null: none),
    // per tile the K1 source bits of its cells with sigma > 0 (own 1, edge
    // cells W 2, E 4, S 8, N 16, outer face neighbours 32), and per tile the
    // field volume applied so far [m^3]
    const real* sigma;
    const unsigned char* fmask;
    double* fvol;
};

template <typename real>
__device__ __forceinline__ bool ring_tile(const Args<real>& a, int tile) {
    if (a.nring == 0) return false;
    const int ti = tile % a.ntx, tj = tile / a.ntx;
    return ti <= a.ring_x0 || ti >= a.ring_x1 || tj <= a.ring_y0 || tj >= a.ring_y1;
}

// Variants of the step kernel: plain, with flux taps (nested grids), with
// learned flux corrections, with a source rate field, with the corrector's
// pressure gradient at the displaced particle positions.
constexpr int MODE_PLAIN = 0, MODE_TAP = 1, MODE_CORR = 2, MODE_FIELD = 3, MODE_DISP = 4, MODE_PERIODIC = 5;

// ---------------------------------------------------------------- math

template <typename real> struct Mth;
template <> struct Mth<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // c_f / H^(4/3) for H > 0 via the hardware base-2 logarithm and exponential
    static __device__ __forceinline__ float friction(float cf, float H) {
        return cf * __builtin_amdgcn_exp2f(-1.33333333f * __builtin_amdgcn_logf(H));
    }
};
template <> struct Mth<double> {
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double friction(double cf, double H) { return cf / (H * ::cbrt(H)); }
};

// fmax/fmin/fabs map to single v_max/v_min instructions and a free abs
// operand modifier (a ternary would cost a compare and a select each)
__device__ __forceinline__ float rmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float rmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float rabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double rmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double rmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double rabs(double a) { return __builtin_fabs(a); }
// false for NaN and +-inf (compare against the largest finite value)
__device__ __forceinline__ bool finite(float a) { return rabs(a) <= 3.40282347e38f; }
__device__ __forceinline__ bool finite(double a) { return rabs(a) <= 1.7976931348623157e308; }

// Stochastic rounding of the depth update (FP32 state).  Round to nearest
// drops every change below half an ulp: a deep cell losing a trickle to a
// shallow neighbour keeps its depth while the neighbour gains, so on a
// rising flood the stored volume creeps up step after step (6e-6 of the
// volume over a 10 000-step 4096^2 flood).  Rounding s = fl(a + d) to its
// neighbour toward the exact remainder e = (a + d) - s (two-sum) with
// probability |e| / gap makes the stored depth unbiased, so the volume error
// is a random walk at the rounding level.  The decision is a hash of the
// cell's global index and the step's clock: the same wherever the cell is
// computed (its own tile, a neighbour's ring, a batch, any tile shape, a run
// resumed from a checkpoint).
__device__ __forceinline__ unsigned cell_hash(unsigned cell, unsigned clk) {
    // MurmurHash3's 32-bit finalizer (Appleby) of the cell index mixed with
    // the step's clock bits by the golden-ratio constant
    unsigned h = cell ^ (clk * 0x9E3779B9u);
    h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
    return h;
}
__device__ __forceinline__ float round_stochastic(float a, float d, float s, unsigned h) {
    const float bb = s - a;
    const float e = (a - (s - bb)) + (d - bb);
    if (!(e != 0.0f)) return s;
    const unsigned bits = __float_as_uint(s);
    const bool away = (e > 0.0f) == (s > 0.0f);
    const float nb = s == 0.0f ? (e > 0.0f ? 1.4e-45f : -1.4e-45f) : __uint_as_float(away ? bits + 1u : bits - 1u);
    const float p = e * __builtin_amdgcn_rcpf(nb - s);   // in [0, 1]; the gap nb - s is exact
    return (float)(h >> 8) * 5.9604645e-8f < p ? nb : s;
}

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

// Limited slope from the backward and forward differences (0 minmod,
// 1 van Leer, 2 monotonised central).
template <typename real, int LIM>
__device__ __forceinline__ real limit(real a, real b) {
    const bool same = a * b > real(0);
    real m;
    if constexpr (LIM == 1) {
        m = Mth<real>::div(real(2) * a * b, a + b);
    } else if constexpr (LIM == 2) {
        const real mm = rmin(rmin(real(2) * rabs(a), real(2) * rabs(b)), real(0.5) * rabs(a + b));
        m = a > real(0) ? mm : -mm;
    } else {
        m = rabs(a) < rabs(b) ? a : b;
    }
    return same ? m : real(0);
}

template <typename real> struct Face { real H, eta, un, ut; };

// Post-Lagrangian values of one cell for reconstruction along one axis.
template <typename real> struct Cell { real H, b, un, ut; };

// Limited reconstruction of cell c on its low (towards m) and high (towards
// q) faces.  A dry cell (H_t <= eps) shows H = 0, U = 0, eta = b; a dry
// neighbour contributes a zero velocity difference; face depth >= 0.
template <typename real, int LIM>
__device__ __forceinline__ void recon(real eps, const Cell<real>& m, const Cell<real>& c,
                                      const Cell<real>& q, Face<real>& lo, Face<real>& hi) {
    const real em = m.H + m.b, ec = c.H + c.b, eq = q.H + q.b;   // eta_t = H_t + b
    const real sH = limit<real, LIM>(c.H - m.H, q.H - c.H);
    const real sE = limit<real, LIM>(ec - em, eq - ec);
    const bool wm = m.H > eps, wq = q.H > eps, wc = c.H > eps;
    const real sN = limit<real, LIM>(wm ? c.un - m.un : real(0), wq ? q.un - c.un : real(0));
    const real sT = limit<real, LIM>(wm ? c.ut - m.ut : real(0), wq ? q.ut - c.ut : real(0));
    const real hH = real(0.5) * sH, hE = real(0.5) * sE, hN = real(0.5) * sN, hT = real(0.5) * sT;
    hi.H = wc ? rmax(real(0), c.H + hH) : real(0);
    lo.H = wc ? rmax(real(0), c.H - hH) : real(0);
    hi.eta = wc ? ec + hE : c.b;
    lo.eta = wc ? ec - hE : c.b;
    hi.un = wc ? c.un + hN : real(0);
    lo.un = wc ? c.un - hN : real(0);
    hi.ut = wc ? c.ut + hT : real(0);
    lo.ut = wc ? c.ut - hT : real(0);
}

// Hydrostatic reconstruction over b* = max(bL, bR) and the Rusanov flux of
// mass, normal and tangential momentum; L is the lower-index side.
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

// Velocities of the four face neighbours (order W, E, S, N) and whether each
// is wet.
template <typename real> struct Nb4 { real ux[4], uy[4]; bool w[4]; };

// 1 for wet, 0 for dry: a dry neighbour (velocity 0, finite) then adds
// 0 * (u_m - u_c) = +-0 to the viscous sum, the same as leaving it out.
template <typename real> __device__ __forceinline__ real mask(bool w) { return w ? real(1) : real(0); }

// Viscosity over wet face neighbours + Coriolis + wind at a cell with depth
// H (layer n) and velocity (uxc, uyc).
template <typename real>
__device__ __forceinline__ void soft_forces(const Args<real>& a, real H, real uxc, real uyc,
                                            const Nb4<real>& nb, real& fx, real& fy) {
    real vx = real(0), vy = real(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real m = mask<real>(nb.w[k]);
        vx += m * (nb.ux[k] - uxc);
        vy += m * (nb.uy[k] - uyc);
    }
    const real dx = a.wx - uxc, dy = a.wy - uyc;
    const real k = Mth<real>::div(a.kw * Mth<real>::sqrt(dx * dx + dy * dy), rmax(H, a.hw));
    fx = a.nuh2 * vx + a.fcor * uyc + k * dx;
    fy = a.nuh2 * vy - a.fcor * uxc + k * dy;
}

// CFL speed max(U_s, U_p) of a wet cell (Sec. 2.3, stage I) of depth H,
// velocity (ux, uy) and Manning coefficient c_f = g n_M^2.  F is the force
// density of Eq. (4) without the pressure gradient: viscosity, Coriolis and
// wind (fx, fy) plus bottom friction -(c_f / H^(4/3)) U |U|.
template <typename real>
__device__ __forceinline__ real cfl_speed(const Args<real>& a, real H, real cf, real ux, real uy,
                                          real fx, real fy) {
    const real fr = Mth<real>::friction(cf, H) * Mth<real>::sqrt(ux * ux + uy * uy);
    fx -= fr * ux;
    fy -= fr * uy;
    const real us = rmax(rabs(ux), rabs(uy)) + Mth<real>::sqrt(a.g * H);
    const real sx = fx > real(0) ? real(1) : (fx < real(0) ? real(-1) : real(0));
    const real sy = fy > real(0) ? real(1) : (fy < real(0) ? real(-1) : real(0));
    const real upx = rabs(ux + sx * Mth<real>::sqrt(a.h * rabs(fx)));
    const real upy = rabs(uy + sy * Mth<real>::sqrt(a.h * rabs(fy)));
    return rmax(us, rmax(upx, upy));
}

__device__ __forceinline__ void atomic_max_prep(Ctrl* c, float v) {
    atomicMax((unsigned int*)&c->prep_speed, __float_as_uint(v));
}
__device__ __forceinline__ void atomic_max_prep(Ctrl* c, double v) {
    atomicMax(&c->prep_speed, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ double prep_speed(const Ctrl* c, float) {
    return (double)__uint_as_float(*(const unsigned int*)&c->prep_speed);
}
__device__ __forceinline__ double prep_speed(const Ctrl* c, double) {
    return __longlong_as_double((long long)c->prep_speed);
}

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

// CFL time step from the maximum speed S of a layer (Sec. 2.3, stage I),
// rounded to the stencil type.
template <typename real>
__device__ double cfl_tau_of(const Args<real>& a, double S) {
    double tau = a.tau_max > 0.0 ? a.tau_max : __builtin_inf();
    if (S > 0.0) tau = fmin(tau, a.cfl * a.h_d / S);
    if (a.nu_d > 0.0) tau = fmin(tau, a.h_d * a.h_d / (4.0 * a.nu_d));
    return (double)(real)tau;
}

// Time step tau of the next step and its hydrograph volume and source depth.
template <typename real>
__device__ __forceinline__ void set_next_step(const Args<real>& a, Ctrl* c, double tau) {
    if (!(tau >= a.tau_min) || !(tau < __builtin_inf())) c->err = -5;
    c->tau = tau;
    double dV = 0.0;
    if (a.nin_h2 > 0.0 && tau < __builtin_inf())
        dV = hydro_volume(a.q_base, a.q_peak, a.t_peak, a.sigma_t, c->t, tau);
    c->dV = dV;
    c->sdepth = a.nin_h2 > 0.0 ? (double)(real)(dV / a.nin_h2) : 0.0;
}

// Bookkeeping of a new layer with maximum speed S: its CFL step and the next
// step's scalars (with hold, the step length set from outside is kept).
template <typename real>
__device__ __forceinline__ void next_step_scalars(const Args<real>& a, Ctrl* c, double S) {
    const double tau = cfl_tau_of(a, S);
    c->speed = S;
    c->tau_cfl = tau;
    // a held step keeps its length; its hydrograph volume moves with the clock
    set_next_step(a, c, a.hold ? c->tau : tau);
}

// Prefix offsets of the list segments of `slot` from their counters.
__device__ __forceinline__ void close_segments(Ctrl* c, int* hot, int slot) {
    int off = 0;
    c->seg_off[slot][0] = 0;
    for (int g = 0; g < NSEG; ++g) {
        off += hot[hot_seg(slot, g)];
        c->seg_off[slot][g + 1] = off;
    }
}

// The same from segment counters already read (stores only).
__device__ __forceinline__ void close_segments_from(Ctrl* c, const int (&n)[NSEG], int slot) {
    int off = 0;
    c->seg_off[slot][0] = 0;
#pragma unroll
    for (int g = 0; g < NSEG; ++g) {
        off += n[g];
        c->seg_off[slot][g + 1] = off;
    }
}

// Entry p of the list in `slot` (segments concatenated in order); cap is the
// capacity of one segment.
__device__ __forceinline__ int list_entry(const Ctrl* c, const int* lists, int cap, int slot, int p) {
    int g = 0;
#pragma unroll
    for (int q = 1; q < NSEG; ++q) g += p >= c->seg_off[slot][q];
    return lists[(slot * NSEG + g) * cap + p - c->seg_off[slot][g]];
}

// The list entry of workgroup b when the list in `slot` is no longer than
// the grid G, each workgroup then stepping at most one tile (own-segment
// order): entry b / NSEG of segment b % NSEG -- the segment its own XCD
// filled (workgroup b runs on XCD b % NSEG under round-robin dispatch), a
// tile that XCD stepped or one facing it -- when that segment is that long;
// the entries of a longer segment beyond the G / NSEG its workgroups take go,
// in segment order, to the workgroups left without one, by rank.  Every
// entry goes to exactly one workgroup (the list has at most G entries).
// Returns the entry, or -1 when workgroup b has none.  The order only
// places the tiles: the results do not depend on it.
__device__ __forceinline__ int list_entry_own(const Ctrl* c, const int* lists, int cap, int slot, int b, int G) {
    int n[NSEG];
#pragma unroll
    for (int g = 0; g < NSEG; ++g) n[g] = c->seg_off[slot][g + 1] - c->seg_off[slot][g];
    const int g0 = b % NSEG, i0 = b / NSEG;
    if (i0 < n[g0]) return lists[(slot * NSEG + g0) * cap + i0];
    int rank = i0 - n[g0];   // among the workgroups left without an entry
#pragma unroll
    for (int g = 0; g < NSEG; ++g)
        if (g < g0) rank += max(0, (G - g + NSEG - 1) / NSEG - n[g]);
#pragma unroll
    for (int g = 0; g < NSEG; ++g) {
        const int taken = (G - g + NSEG - 1) / NSEG, over = max(0, n[g] - taken);
        if (rank < over) return lists[(slot * NSEG + g) * cap + taken + rank];
        rank -= over;
    }
    return -1;
}

// Append the candidate tiles of lanes 0..4 of one wave (cand < 0: none) of
// scenario `sid` to segment `grp` of list `slot`: stamps de-duplicate across
// the grid (one generation per list), one counter update per call reserves
// the slots.
__device__ __forceinline__ void append_tiles(int cand, int sid, int tile_base, int gen, int* stamp,
                                             int* lists, int* hot, int cap, int slot, int grp) {
    const int lane = threadIdx.x & 63;
    const bool ok = cand >= 0 && atomicMax(&stamp[tile_base + cand], gen) < gen;
    const unsigned long long m = __ballot(ok);
    const int n = __popcll(m);
    if (n == 0) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(&hot[hot_seg(slot, grp)], n);
    base = __shfl(base, 0, 64);
    // set bits of the ballot below this lane (no 64-bit lane mask held live)
    const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (ok) lists[(slot * NSEG + grp) * cap + base + below] = pack_entry(sid, cand);
}

// Next-list bookkeeping of the tile being stepped (grids that skip dry
// tiles).  Its atomics are interleaved with the stages of the tile so that
// their latency hides behind the arithmetic: a tile K1-active at layer n
// appends itself right after the load stage, and the stamps of its four
// neighbours are read before the last flux pass, so that at the end only
// neighbours not yet in the list cost an atomic.
struct ListCtx {
    int* stamp; int* lists; int* hot;
    int cap, slot, grp, gen, sid, tile_base, tile, ntx, nty;
    bool on;
    unsigned clk;   // the step's clock mixed to 32 bits (stochastic rounding)
};

// The clock t at the start of a step, mixed to 32 bits: distinct for every
// step of a run and restored with the clock (a resumed run rounds as the
// original did).
__device__ __forceinline__ unsigned clock_bits(double t) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(t);
    return (unsigned)b ^ ((unsigned)(b >> 32) * 0x9E3779B9u);
}

template <typename real>
__device__ __forceinline__ bool is_src(const Args<real>& a, int gx, int gy) {
    return (unsigned)(gx - a.i0) < (unsigned)a.ni && (unsigned)(gy - a.j0) < (unsigned)a.nj;
}

// Flux taps of nested grids.  A tap rectangle [x0, x1) x [y0, y1) of cells
// owns 2(y1-y0) + 2(x1-x0) boundary faces, stored side by side (west x faces
// at x0, east x faces at x1, south y faces at y0, north y faces at y1) in
// three component planes: depth, normal momentum, tangential momentum.  Cell
// (gx, gy) adds tau * flux of its west face (fluxes xH, xN, xT) and its south
// face (yH, yN, yT) where they are tap faces.
template <typename real>
__device__ __forceinline__ void tap_faces(const Args<real>& a, int gx, int gy, real tau, real xH, real xN,
                                          real xT, real yH, real yN, real yT) {
    for (int q = 0; q < a.ntap; ++q) {
        const int* R = a.tap_rect + 5 * q;
        const int w = R[2] - R[0], hh = R[3] - R[1], per = 2 * (w + hh);
        real* T = a.tap + R[4];
        if ((gx == R[0] || gx == R[2]) && gy >= R[1] && gy < R[3]) {
            const int k = (gx == R[0] ? 0 : hh) + gy - R[1];
            T[k] += tau * xH;
            T[per + k] += tau * xN;
            T[2 * per + k] += tau * xT;
        }
        if ((gy == R[1] || gy == R[3]) && gx >= R[0] && gx < R[2]) {
            const int k = 2 * hh + (gy == R[1] ? 0 : w) + gx - R[0];
            T[k] += tau * yH;
            T[per + k] += tau * yN;
            T[2 * per + k] += tau * yT;
        }
    }
}

// ---------------------------------------------------------------- LDS of a tile

// Row pitch is odd so that lanes walking down a column hit distinct banks.
template <int TX, int TY>
struct Geo {
    static constexpr int W = (TX + 2 * HALO) | 1;
    static constexpr int H = TY + 2 * HALO;
    static constexpr int N = W * H;
    static __device__ __forceinline__ int at(int x, int y) { return (y + HALO) * W + x + HALO; }
};

// Ten arrays in one layout, reused across the stages:
//   H   H^n            -> x-flux F_t (y-momentum)
//   B   b
//   UX  Ux^n           -> H_t
//   UY  Uy^n           -> Ux_t
//   HX  Ux^{n+1/2}     -> x-flux F_H
//   HY  Uy^{n+1/2}     -> x-flux F_n (x-momentum)
//   GX  G_x            -> Qx_t -> Ux^{n+1}
//   GY  G_y            -> Qy_t -> Uy^{n+1}
//   LM  c_f/H^(4/3)    -> Uy_t
//   NH  H^{n+1}
template <typename real, int TX, int TY>
struct Lds {
    real H[Geo<TX, TY>::N], B[Geo<TX, TY>::N], UX[Geo<TX, TY>::N], UY[Geo<TX, TY>::N];
    real HX[Geo<TX, TY>::N], HY[Geo<TX, TY>::N], GX[Geo<TX, TY>::N], GY[Geo<TX, TY>::N];
    real LM[Geo<TX, TY>::N], NH[Geo<TX, TY>::N];
};

// Copy mirror images into the positions of [x0, x1) x [y0, y1) (tile
// coordinates) that lie outside the domain.  Bit q of sgx / sgy marks array
// q as the x / y component of a vector (its sign flips across that wall).
template <typename real, int TX, int TY, int NT>
__device__ void fill_ghosts(int tx0, int ty0, int nx, int ny, int x0, int x1, int y0, int y1,
                            real* f0, real* f1, real* f2, int sgx, int sgy) {
    using G = Geo<TX, TY>;
    const int w = x1 - x0, n = w * (y1 - y0);
    for (int k = threadIdx.x; k < n; k += NT) {
        const int x = x0 + k % w, y = y0 + k / w;
        const int gx = tx0 + x, gy = ty0 + y;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) continue;
        int fx = 0, fy = 0;
        const int mx = mirror(gx, nx, fx) - tx0, my = mirror(gy, ny, fy) - ty0;
        const int s = G::at(x, y), m = G::at(mx, my);
        real* fs[3] = {f0, f1, f2};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (!fs[q]) continue;
            const bool neg = (((sgx >> q) & 1) && (fx & 1)) != (((sgy >> q) & 1) && (fy & 1));
            const real v = fs[q][m];
            fs[q][s] = neg ? -v : v;
        }
    }
}

// ---------------------------------------------------------------- one tile

// bits: 1 own wet, 2 W edge, 4 E edge, 8 S edge, 16 N edge (layer n+1),
// 32 ring wet (layer n+1), 64 K1-active at layer n
// Line taps: cell (gx, gy) adds tau * flux of its west face when gx is a
// multiple of tap_r and of its south face when gy is (planes: depth, normal
// momentum, tangential momentum, as for tap rectangles).
template <typename real>
__device__ __forceinline__ void tap_lines(const Args<real>& a, int gx, int gy, real tau, real xH, real xN, real xT,
                                          real yH, real yN, real yT) {
    const int r = a.tap_r;
    if (gx % r == 0) {
        const int w = a.nx / r + 1, pl = a.ny * w, k = gy * w + gx / r;
        a.tapx[k] += tau * xH;
        a.tapx[pl + k] += tau * xN;
        a.tapx[2 * pl + k] += tau * xT;
    }
    if (gy % r == 0) {
        const int pl = (a.ny / r + 1) * a.nx, k = (gy / r) * a.nx + gx;
        a.tapy[k] += tau * yH;
        a.tapy[pl + k] += tau * yN;
        a.tapy[2 * pl + k] += tau * yT;
    }
}

// Learned flux correction of one face (mass, x-momentum, y-momentum planes of
// corr at cell index k), with the correction depth corr_hmin (>= eps) after
// the Lagrangian stage: the mass part only where its upwind cell (lo side for
// a positive correction, else hi side) is deeper, the momentum part only
// where both cells are.  A face dry on both sides takes none, so the dry-wave
// shortcuts of the flux passes stay exact.
template <typename real>
__device__ __forceinline__ void add_correction(const Args<real>& a, const real* corr, int k, real Hlo, real Hhi,
                                               real& FH, real& Fn, real& Ft, bool xface) {
    const int n = a.nx * a.ny;
    const real dH = corr[k], dX = corr[n + k], dY = corr[2 * n + k];
    const real Hd = dH > real(0) ? Hlo : Hhi;
    const bool both = Hlo > a.corr_hmin && Hhi > a.corr_hmin;
    FH += Hd > a.corr_hmin ? dH : real(0);
    Fn += both ? (xface ? dX : dY) : real(0);
    Ft += both ? (xface ? dY : dX) : real(0);
}

// Slope dW/dq of the 2D cubic B-spline kernel shape (support q < 2); its
// normalisation cancels in the corrected gradient.
template <typename real>
__device__ __forceinline__ real bspline_dw(real q) {
    const real u = real(2) - q;
    return q < real(1) ? q * (real(2.25) * q - real(3)) : (q < real(2) ? real(-0.75) * u * u : real(0));
}

// Level gradient at the particle of LDS cell s displaced to its position of
// t_{n+1/2} (cell centre + tau/2 U^n), as the corrected SPH sum over the
// particles of its 5x5 neighbourhood (Sec. 2.3 stage II, K4-K6):
// G = M^{-1} sum_j (eta*_j - eta_i) w_ij, M = sum_j w_ij r_ij^T,
// w_ij = W'(|r_ij|) r_ij / |r_ij|, positions in cell units; eta*_j is the
// level a neighbour shows to the cell (the rule of the lattice stencil).
template <typename real, int W>
__device__ __forceinline__ void displaced_gradient(const real* LH, const real* LB, const real* UX, const real* UY,
                                                   int s, real eps, real half_tau_ih, real ih, real& gx,
                                                   real& gy) {
    const real Hc = LH[s], bc = LB[s], ec = Hc + bc;
    const real pxi = half_tau_ih * UX[s], pyi = half_tau_ih * UY[s];
    real Sx = real(0), Sy = real(0), mxx = real(0), mxy = real(0), myx = real(0), myy = real(0);
    // one row of the neighbourhood at a time keeps the live loads few
#pragma unroll 1
    for (int dj = -2; dj <= 2; ++dj)
#pragma unroll
        for (int di = -2; di <= 2; ++di) {
            if (di == 0 && dj == 0) continue;
            const int m = s + dj * W + di;
            const real rx = real(di) + half_tau_ih * UX[m] - pxi;
            const real ry = real(dj) + half_tau_ih * UY[m] - pyi;
            const real r = Mth<real>::sqrt(rx * rx + ry * ry);
            const real dw = bspline_dw(r);
            const real Hm = LH[m];
            const bool wm = Hm > eps;
            const real em = wm ? Hm + LB[m] : LB[m];
            const real es = rmax(bc, rmin(em, ec + (wm ? Hm : real(0))));
            const real k = Mth<real>::div(dw, r);
            const real wx = k * rx, wy = k * ry;
            Sx += (es - ec) * wx;
            Sy += (es - ec) * wy;
            mxx += wx * rx;
            mxy += wx * ry;
            myx += wy * rx;
            myy += wy * ry;
        }
    const real idet = Mth<real>::div(ih, mxx * myy - mxy * myx);
    gx = (myy * Sx - mxy * Sy) * idet;
    gy = (mxx * Sy - myx * Sx) * idet;
}

// Depth after the source rate field at cell (gx, gy) of tile coordinates
// (x, y), from Hs (depth with the inlet source): rain adds tau*sigma; a loss
// acts only on a cell wet at layer n and takes at most its water.  The depth
// applied on the tile's own cells goes to fsum.
template <typename real, int TX, int TY>
__device__ __forceinline__ real field_depth_t(const Args<real>& a, int gx, int gy, real tau, real Hs, bool wet,
                                              int x, int y, double& fsum) {
    const real sg = a.sigma[gy * a.nx + gx];
    const real Ht = sg > real(0) ? Hs + tau * sg : (sg < real(0) && wet ? rmax(Hs + tau * sg, real(0)) : Hs);
    if (x >= 0 && x < TX && y >= 0 && y < TY) fsum += (double)(Ht - Hs);
    return Ht;
}

template <typename real, int TX, int TY, int NT, int LIM, bool EDGE, int MODE>
__device__ void tile_step(const Args<real>& a, Lds<real, TX, TY>& L, int tx0, int ty0,
                          real tau, real sdep, real& vmax, bool& bad, double& msum, double& lsum,
                          double& fsum, int fm, int& bits, const ListCtx& lx, int& nbst) {
    using G = Geo<TX, TY>;
    constexpr int W = G::W;
    constexpr bool TAP = MODE == MODE_TAP, CORR = MODE == MODE_CORR, FLD = MODE == MODE_FIELD;
    constexpr bool DISP = MODE == MODE_DISP;
    // periodic domain (tests of conservation): a halo cell is the cell one
    // period away, computed there exactly as in its own tile, so the walls'
    // ghost fills are not needed; nx and ny are multiples of the tile shape
    constexpr bool PER = MODE == MODE_PERIODIC;
    const int tid = threadIdx.x, nx = a.nx, ny = a.ny;
    auto wrapx = [&](int g) { if constexpr (PER) { g %= nx; if (g < 0) g += nx; } return g; };
    auto wrapy = [&](int g) { if constexpr (PER) { g %= ny; if (g < 0) g += ny; } return g; };
    const real eps = a.eps, half_tau = real(0.5) * tau, r = tau * a.ih;
    // normalised cubic-B-spline SPH gradient weights (smoothing length h):
    // al = 1/(12 sqrt2 - 14), be = (3 sqrt2 - 4)/(12 sqrt2 - 14), 2 al + 4 be = 1
    const real al = real(0.33663655161388173), be = real(0.08168172419305914);
    // Cells per thread along the run of each stage.  FP32 kernels run four
    // waves per SIMD (128 VGPRs), which short runs fit without spilling:
    // 2 in P1/P2, 3 in FX/FY where the face count divides, so that one pass
    // of a 512-thread workgroup covers a 32-wide tile.  FP64 keeps runs of 4.
    constexpr bool F32 = sizeof(real) == 4;
    constexpr int RP = F32 ? 2 : 4;
    constexpr int RFX = F32 ? ((TX + 4) % 3 == 0 ? 3 : 2) : 4;
    constexpr int RFY = F32 ? 3 : 4;
    static_assert((TX + 8) % RP == 0 && (TX + 4) % RFX == 0, "run lengths must tile the stage rows");
    auto inside = [&](int x, int y) {
        if constexpr (!EDGE || PER) return true;
        const int gx = tx0 + x, gy = ty0 + y;
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    };

    // ---- load tile + 5: every load of the thread is issued before any is
    // used (one memory round trip, not one per row of the loop); c_f goes to
    // LM, where P1 reads it and leaves its friction factor
    {
        constexpr int RW = TX + 2 * HALO, NL = RW * G::H, J = (NL + NT - 1) / NT;
        real vH[J], vX[J], vY[J], vB[J], vC[J];
        int vf[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * NT;
            if (k >= NL) continue;
            const int x = k % RW - HALO, y = k / RW - HALO;
            int gx = tx0 + x, gy = ty0 + y, fx = 0, fy = 0;
            if constexpr (PER) { gx = wrapx(gx); gy = wrapy(gy); }
            else if constexpr (EDGE) { gx = mirror(gx, nx, fx); gy = mirror(gy, ny, fy); }
            const int gi = gy * nx + gx;
            vH[j] = a.Hi[gi];
            vX[j] = a.Qxi[gi];
            vY[j] = a.Qyi[gi];
            vB[j] = a.bed[gi];
            vC[j] = a.cf[gi];
            vf[j] = (fx & 1) | ((fy & 1) << 1);
        }
        int act = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * NT;
            if (k >= NL) continue;
            const int x = k % RW - HALO, y = k / RW - HALO;
            const real H = vH[j];
            real qx = vX[j], qy = vY[j];
            if constexpr (EDGE) { if (vf[j] & 1) qx = -qx; if (vf[j] & 2) qy = -qy; }
            const bool w = H > eps;
            const int s = G::at(x, y);
            L.H[s] = H;
            L.B[s] = vB[j];
            L.LM[s] = vC[j];
            L.UX[s] = w ? Mth<real>::div(qx, H) : real(0);
            L.UY[s] = w ? Mth<real>::div(qy, H) : real(0);
            // K1 rule at layer n: own cells and outer face neighbours (no corners)
            const bool own = x >= 0 && x < TX && y >= 0 && y < TY;
            const bool ring = ((x == -1 || x == TX) && y >= 0 && y < TY) || ((y == -1 || y == TY) && x >= 0 && x < TX);
            if ((own || ring) && inside(x, y) && (w || is_src(a, wrapx(tx0 + x), wrapy(ty0 + y)))) act = 1;
        }
        if (__syncthreads_or(act) || (FLD && (fm & 33))) bits |= 64;
    }
    // self-append of a tile K1-active at layer n: stamp now, slot after P1,
    // entry after P2 (thread 0)
    const bool early = lx.on && tid == 0 && (bits & 64);
    int e_old = lx.gen, e_base = 0;
    if (early) e_old = atomicMax(&lx.stamp[lx.tile_base + lx.tile], lx.gen);

    // ---- P1: forces at t_n and predictor on tile + 4, runs of 4 along x
    {
        constexpr int NRW = (TX + 8) / RP, NRH = TY + 8, NR = NRW * NRH;
        for (int k = tid; k < NR; k += NT) {
            const int y = k % NRH - 4, x0 = (k / NRH) * RP - 4;
            // 3 x 6 patch of effective depth and level: a dry cell shows depth 0
            // and its bed as level
            real He[3][RP + 2], Le[3][RP + 2], Bc[RP + 2];
            bool any = false;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < RP + 2; ++i) {
                    const int s = G::at(x0 - 1 + i, y - 1 + j);
                    const real H = L.H[s], b = L.B[s];
                    const bool w = H > eps;
                    He[j][i] = w ? H : real(0);
                    Le[j][i] = b + He[j][i];
                    if (j == 1) { Bc[i] = b; if (i >= 1 && i <= RP) any |= w; }
                }
            if (!__any(any)) {   // the whole wave is dry here: U^{n+1/2} = 0
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    if (!inside(x0 + i, y)) continue;
                    const int s = G::at(x0 + i, y);
                    L.HX[s] = real(0);
                    L.HY[s] = real(0);
                }
                continue;
            }
            real ux[RP + 2], uy[RP + 2], uxs[RP], uys[RP], uxn[RP], uyn[RP];
#pragma unroll
            for (int i = 0; i < RP + 2; ++i) {
                const int s = G::at(x0 - 1 + i, y);
                ux[i] = L.UX[s]; uy[i] = L.UY[s];
            }
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const int ss = G::at(x0 + i, y - 1), sn = G::at(x0 + i, y + 1);
                uxs[i] = L.UX[ss]; uys[i] = L.UY[ss];
                uxn[i] = L.UX[sn]; uyn[i] = L.UY[sn];
            }
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const int c = i + 1;
                const real Hc = He[1][c], bc = Bc[c], ec = Le[1][c];
                const bool wc = Hc > real(0);
                real e[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        e[j][d] = rmax(bc, rmin(Le[j][c - 1 + d], ec + He[j][c - 1 + d]));
                // e[j][d]: j = 0 south row, 2 north row; d = 0 west column, 2 east
                const real Gx = (al * (e[1][2] - e[1][0]) + be * ((e[2][2] - e[2][0]) + (e[0][2] - e[0][0]))) * a.ih;
                const real Gy = (al * (e[2][1] - e[0][1]) + be * ((e[2][2] - e[0][2]) + (e[2][0] - e[0][0]))) * a.ih;
                const bool ins = inside(x0 + i, y);
                const real cf = ins ? L.LM[G::at(x0 + i, y)] : real(0);
                const real lam0 = Mth<real>::friction(cf, wc ? Hc : real(1));
                Nb4<real> nb;
                nb.ux[0] = ux[c - 1]; nb.uy[0] = uy[c - 1]; nb.w[0] = He[1][c - 1] > real(0);
                nb.ux[1] = ux[c + 1]; nb.uy[1] = uy[c + 1]; nb.w[1] = He[1][c + 1] > real(0);
                nb.ux[2] = uxs[i]; nb.uy[2] = uys[i]; nb.w[2] = He[0][c] > real(0);
                nb.ux[3] = uxn[i]; nb.uy[3] = uyn[i]; nb.w[3] = He[2][c] > real(0);
                real fx, fy;
                soft_forces(a, Hc, ux[c], uy[c], nb, fx, fy);
                const real ax = -a.g * Gx + fx, ay = -a.g * Gy + fy;
                const real lam = lam0 * Mth<real>::sqrt(ux[c] * ux[c] + uy[c] * uy[c]);
                const real d = real(1) + half_tau * lam;
                const int s = G::at(x0 + i, y);
                if (ins) {
                    L.HX[s] = wc ? Mth<real>::div(ux[c] + half_tau * ax, d) : real(0);
                    L.HY[s] = wc ? Mth<real>::div(uy[c] + half_tau * ay, d) : real(0);
                    L.GX[s] = Gx;
                    L.GY[s] = Gy;
                    L.LM[s] = lam0;
                }
            }
        }
        __syncthreads();
        if (early && e_old < lx.gen) e_base = atomicAdd(&lx.hot[hot_seg(lx.slot, lx.grp)], 1);
        if constexpr (EDGE && !PER) {
            fill_ghosts<real, TX, TY, NT>(tx0, ty0, nx, ny, -4, TX + 4, -4, TY + 4, L.HX, L.HY, nullptr,
                                          /*sgx*/ 1, /*sgy*/ 2);
            __syncthreads();
        }
    }

    // ---- PD (displaced-particle corrector only): the corrector's pressure
    // gradient at the particle positions of t_{n+1/2} on tile + 3, from
    // H, b and U^n of tile + 5; it replaces the lattice gradient P2 reads
    if constexpr (DISP) {
        constexpr int NW3 = TX + 6, NC3 = NW3 * (TY + 6);
        const real hti = half_tau * a.ih;
        for (int k = tid; k < NC3; k += NT) {
            const int x = k % NW3 - 3, y = k / NW3 - 3;
            const int s = G::at(x, y);
            if (!(L.H[s] > eps)) continue;
            real gx, gy;
            displaced_gradient<real, W>(L.H, L.B, L.UX, L.UY, s, eps, hti, a.ih, gx, gy);
            L.GX[s] = gx;
            L.GY[s] = gy;
        }
        __syncthreads();
    }

    // ---- P2: forces at t_{n+1/2}, corrector, sources on tile + 3
    {
        constexpr int NRW = (TX + 8) / RP, NRH = TY + 6, NR = NRW * NRH;
        for (int k = tid; k < NR; k += NT) {
            const int y = k % NRH - 3, x0 = (k / NRH) * RP - 4;
            real hx[RP + 2], hy[RP + 2], Hr[RP + 2];
            bool wr[RP + 2];
#pragma unroll
            for (int i = 0; i < RP + 2; ++i) {
                const int s = G::at(x0 - 1 + i, y);
                hx[i] = L.HX[s]; hy[i] = L.HY[s]; Hr[i] = L.H[s]; wr[i] = Hr[i] > eps;
            }
            real hxs[RP], hys[RP], hxn[RP], hyn[RP];
            bool ws[RP], wn[RP];
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const int ss = G::at(x0 + i, y - 1), sn = G::at(x0 + i, y + 1);
                hxs[i] = L.HX[ss]; hys[i] = L.HY[ss]; ws[i] = L.H[ss] > eps;
                hxn[i] = L.HX[sn]; hyn[i] = L.HY[sn]; wn[i] = L.H[sn] > eps;
            }
            real out[RP][5];
            bool anyw = false;
#pragma unroll
            for (int i = 0; i < RP; ++i) anyw |= wr[i + 1];
            if (!__any(anyw)) {   // the whole wave is dry: no forces, Q_t = 0
#pragma unroll
                for (int i = 0; i < RP; ++i) {
                    const int x = x0 + i;
                    if (!inside(x, y)) continue;
                    const int s = G::at(x, y);
                    const real Hs = is_src(a, wrapx(tx0 + x), wrapy(ty0 + y)) ? Hr[i + 1] + sdep : Hr[i + 1];
                    if constexpr (FLD)
                        L.UX[s] = field_depth_t<real, TX, TY>(a, tx0 + x, ty0 + y, tau, Hs, false, x, y, fsum);
                    else
                        L.UX[s] = Hs;
                    L.UY[s] = real(0);
                    L.LM[s] = real(0);
                    L.GX[s] = real(0);
                    L.GY[s] = real(0);
                }
                continue;
            }
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                const int c = i + 1, x = x0 + i;
                const int s = G::at(x, y);
                const real Hc = Hr[c];
                const bool wc = wr[c];
                const real ux = L.UX[s], uy = L.UY[s], gxv = L.GX[s], gyv = L.GY[s], lam0 = L.LM[s];
                Nb4<real> nb;
                nb.ux[0] = hx[c - 1]; nb.uy[0] = hy[c - 1]; nb.w[0] = wr[c - 1];
                nb.ux[1] = hx[c + 1]; nb.uy[1] = hy[c + 1]; nb.w[1] = wr[c + 1];
                nb.ux[2] = hxs[i]; nb.uy[2] = hys[i]; nb.w[2] = ws[i];
                nb.ux[3] = hxn[i]; nb.uy[3] = hyn[i]; nb.w[3] = wn[i];
                real fx, fy;
                soft_forces(a, Hc, hx[c], hy[c], nb, fx, fy);
                const real ax = -a.g * gxv + fx, ay = -a.g * gyv + fy;
                const real lam = lam0 * Mth<real>::sqrt(hx[c] * hx[c] + hy[c] * hy[c]);
                const real d = real(1) + tau * lam;
                const real qx = wc ? Hc * Mth<real>::div(ux + tau * ax, d) : real(0);
                const real qy = wc ? Hc * Mth<real>::div(uy + tau * ay, d) : real(0);
                const real Hs = is_src(a, wrapx(tx0 + x), wrapy(ty0 + y)) ? Hc + sdep : Hc;
                real Ht = Hs;
                if constexpr (FLD)
                    if (inside(x, y)) Ht = field_depth_t<real, TX, TY>(a, tx0 + x, ty0 + y, tau, Hs, wc, x, y, fsum);
                const bool wt = Ht > eps;
                out[i][0] = Ht;
                out[i][1] = wt ? Mth<real>::div(qx, Ht) : real(0);
                out[i][2] = wt ? Mth<real>::div(qy, Ht) : real(0);
                out[i][3] = qx;
                out[i][4] = qy;
            }
            // own-cell stores after all own-cell reads of the run
#pragma unroll
            for (int i = 0; i < RP; ++i) {
                if (!inside(x0 + i, y)) continue;
                const int s = G::at(x0 + i, y);
                L.UX[s] = out[i][0];
                L.UY[s] = out[i][1];
                L.LM[s] = out[i][2];
                L.GX[s] = out[i][3];
                L.GY[s] = out[i][4];
            }
        }
        __syncthreads();
        if (early && e_old < lx.gen)
            lx.lists[(lx.slot * NSEG + lx.grp) * lx.cap + e_base] = pack_entry(lx.sid, lx.tile);
        if constexpr (EDGE && !PER) {
            fill_ghosts<real, TX, TY, NT>(tx0, ty0, nx, ny, -3, TX + 3, -3, TY + 3, L.UX, L.UY, L.LM,
                                          /*sgx*/ 2, /*sgy*/ 4);
            __syncthreads();
        }
    }

    // ---- FX: x faces of rows -1..TY, face x between cells x-1 and x
    {
        constexpr int NRW = (TX + 4) / RFX, NRH = TY + 2, NR = NRW * NRH;
        for (int k = tid; k < NR; k += NT) {
            const int y = k % NRH - 1, x0 = (k / NRH) * RFX - 1;
            Cell<real> cl[RFX + 3];
#pragma unroll
            for (int i = 0; i < RFX + 3; ++i) {
                const int s = G::at(x0 - 2 + i, y);
                cl[i].H = L.UX[s]; cl[i].b = L.B[s]; cl[i].un = L.UY[s]; cl[i].ut = L.LM[s];
            }
            bool anyw = false;
#pragma unroll
            for (int i = 1; i < RFX + 2; ++i) anyw |= cl[i].H > eps;
            if (!__any(anyw)) {   // dry on both sides of every face: zero fluxes
#pragma unroll
                for (int f = 0; f < RFX; ++f) {
                    const int s = G::at(x0 + f, y);
                    L.HX[s] = real(0); L.HY[s] = real(0); L.H[s] = real(0);
                }
                continue;
            }
            Face<real> lo[RFX + 1], hi[RFX + 1];
#pragma unroll
            for (int i = 0; i < RFX + 1; ++i) recon<real, LIM>(eps, cl[i], cl[i + 1], cl[i + 2], lo[i], hi[i]);
            // recon index i is cell x0 - 1 + i; face x0 + f sits between cells f and f+1
#pragma unroll
            for (int f = 0; f < RFX; ++f) {
                real FH, Fn, Ft;
                riemann<real>(a.g, hi[f], lo[f + 1], FH, Fn, Ft);
                if constexpr (CORR) {
                    // face between cells gx-1 and gx: the east face of gx-1
                    const int gx = tx0 + x0 + f, gy = ty0 + y;
                    if (gx >= 1 && gx < nx && gy >= 0 && gy < ny)
                        add_correction(a, a.corrE, gy * nx + gx - 1, cl[f + 1].H, cl[f + 2].H, FH, Fn, Ft, true);
                }
                const int s = G::at(x0 + f, y);
                L.HX[s] = FH; L.HY[s] = Fn; L.H[s] = Ft;
            }
        }
        __syncthreads();
    }

    // stamps of the four neighbours (lanes 1..4 of wave 0: W, E, S, N); a
    // stale value only costs an atomic at the end
    nbst = lx.gen;
    if (lx.on && tid >= 1 && tid <= 4) {
        const int ti = lx.tile % lx.ntx, tj = lx.tile / lx.ntx;
        const int nb = tid == 1 ? (ti > 0 ? lx.tile - 1 : PER ? lx.tile + lx.ntx - 1 : -1)
                     : tid == 2 ? (ti < lx.ntx - 1 ? lx.tile + 1 : PER ? lx.tile - lx.ntx + 1 : -1)
                     : tid == 3 ? (tj > 0 ? lx.tile - lx.ntx : PER ? lx.tile + (lx.nty - 1) * lx.ntx : -1)
                                : (tj < lx.nty - 1 ? lx.tile + lx.ntx : PER ? lx.tile - (lx.nty - 1) * lx.ntx : -1);
        if (nb >= 0) nbst = lx.stamp[lx.tile_base + nb];
    }

    // ---- FY + final update: columns -1..TX, runs of 4 cells along y
    {
        constexpr int NC = TX + 2, NRY = (TY + 2 + RFY - 1) / RFY, NR = NC * NRY;
        // tap faces in this tile: a face belongs to the tile of the cell east
        // (x face) or north (y face) of it
        bool tap_here = false;
        if constexpr (TAP) {
            tap_here = a.tap_r > 0;
            for (int q = 0; q < a.ntap; ++q) {
                const int* R = a.tap_rect + 5 * q;
                const bool xs = ty0 < R[3] && ty0 + TY > R[1] &&
                                ((R[0] >= tx0 && R[0] < tx0 + TX) || (R[2] >= tx0 && R[2] < tx0 + TX));
                const bool ys = tx0 < R[2] && tx0 + TX > R[0] &&
                                ((R[1] >= ty0 && R[1] < ty0 + TY) || (R[3] >= ty0 && R[3] < ty0 + TY));
                tap_here |= xs || ys;
            }
        }
        for (int k = tid; k < NR; k += NT) {
            const int x = k % NC - 1, y0 = (k / NC) * RFY - 1;
            Cell<real> cl[RFY + 4];
#pragma unroll
            for (int i = 0; i < RFY + 4; ++i) {
                const int s = G::at(x, y0 - 2 + i);
                cl[i].H = L.UX[s]; cl[i].b = L.B[s]; cl[i].un = L.LM[s]; cl[i].ut = L.UY[s];
            }
            real FH[RFY + 1], Fn[RFY + 1], Ft[RFY + 1];
            bool anyw = false;
#pragma unroll
            for (int i = 1; i < RFY + 3; ++i) anyw |= cl[i].H > eps;
            if (__any(anyw)) {
                Face<real> lo[RFY + 2], hi[RFY + 2];
#pragma unroll
                for (int i = 0; i < RFY + 2; ++i) recon<real, LIM>(eps, cl[i], cl[i + 1], cl[i + 2], lo[i], hi[i]);
                // recon index i is cell y0 - 1 + i; face y0 + f between cells f and f+1
#pragma unroll
                for (int f = 0; f < RFY + 1; ++f) {
                    riemann<real>(a.g, hi[f], lo[f + 1], FH[f], Fn[f], Ft[f]);
                    if constexpr (CORR) {
                        // face between cells gy-1 and gy: the north face of gy-1
                        const int gx = tx0 + x, gy = ty0 + y0 + f;
                        if (gy >= 1 && gy < ny && gx >= 0 && gx < nx)
                            add_correction(a, a.corrN, (gy - 1) * nx + gx, cl[f + 1].H, cl[f + 2].H, FH[f], Fn[f],
                                           Ft[f], false);
                    }
                }
            } else {   // dry on both sides of every face of the run: zero fluxes
#pragma unroll
                for (int f = 0; f < RFY + 1; ++f) { FH[f] = real(0); Fn[f] = real(0); Ft[f] = real(0); }
            }
#pragma unroll
            for (int i = 0; i < RFY; ++i) {
                const int y = y0 + i;
                if (y > TY || !inside(x, y)) continue;
                const int s = G::at(x, y);
                const real dxH = L.HX[s] - L.HX[s + 1];
                const real dxQx = L.HY[s] - L.HY[s + 1];
                const real dxQy = L.H[s] - L.H[s + 1];
                const real Ht = cl[i + 2].H, dH = r * (dxH + (FH[i] - FH[i + 1]));
                real Hn = Ht + dH;
                if constexpr (F32)
                    Hn = round_stochastic(Ht, dH, Hn, cell_hash((unsigned)((ty0 + y) * nx + tx0 + x), lx.clk));
                const real qx = L.GX[s] + r * (dxQx + (Ft[i] - Ft[i + 1]));
                const real qy = L.GY[s] + r * (dxQy + (Fn[i] - Fn[i + 1]));
                const real Hc = rmax(Hn, real(0));
                const bool w = Hc > eps;
                const real qxo = w ? qx : real(0), qyo = w ? qy : real(0);
                L.NH[s] = Hc;
                L.GX[s] = w ? Mth<real>::div(qxo, Hc) : real(0);
                L.GY[s] = w ? Mth<real>::div(qyo, Hc) : real(0);
                if (x >= 0 && x < TX && y >= 0 && y < TY) {
                    const int gi = (ty0 + y) * nx + tx0 + x;
                    a.Ho[gi] = Hc;
                    a.Qxo[gi] = qxo;
                    a.Qyo[gi] = qyo;
                    msum += (double)Hc;
                    lsum += (double)(Hc - Hn);
                    bad |= !finite(Hn) || !finite(qx) || !finite(qy);
                    if constexpr (TAP) {
                        if (tap_here) {
                            if (a.tap_r > 0)
                                tap_lines(a, tx0 + x, ty0 + y, tau, L.HX[s], L.HY[s], L.H[s], FH[i], Fn[i], Ft[i]);
                            else
                                tap_faces(a, tx0 + x, ty0 + y, tau, L.HX[s], L.HY[s], L.H[s], FH[i], Fn[i], Ft[i]);
                        }
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (EDGE && !PER) {
            fill_ghosts<real, TX, TY, NT>(tx0, ty0, nx, ny, -1, TX + 1, -1, TY + 1, L.NH, L.GX, L.GY,
                                          /*sgx*/ 2, /*sgy*/ 4);
            __syncthreads();
        }
    }

    // ---- epilogue: CFL speed of layer n+1 on the tile, K1 bits of layer n+1
    {
        constexpr int NT_CELLS = TX * TY, NRING = 2 * (TX + TY);
        int own = 0, eW = 0, eE = 0, eS = 0, eN = 0, rg = 0;
        for (int k = tid; k < NT_CELLS + NRING; k += NT) {
            int x, y;
            if (k < NT_CELLS) {
                x = k % TX; y = k / TX;
            } else {
                const int q = k - NT_CELLS;   // ring: S row, N row, W column, E column
                if (q < TX) { x = q; y = -1; }
                else if (q < 2 * TX) { x = q - TX; y = TY; }
                else if (q < 2 * TX + TY) { x = -1; y = q - 2 * TX; }
                else { x = TX; y = q - 2 * TX - TY; }
            }
            if (!inside(x, y)) continue;
            const int s = G::at(x, y);
            const real H = L.NH[s];
            const bool w = H > eps;
            const bool ws = w || is_src(a, wrapx(tx0 + x), wrapy(ty0 + y));
            if (k >= NT_CELLS) { rg |= ws; continue; }
            if (ws) {
                own = 1;
                eW |= x == 0; eE |= x == TX - 1; eS |= y == 0; eN |= y == TY - 1;
            }
            if (w) {
                Nb4<real> nb;
                const int sn[4] = {s - 1, s + 1, s - W, s + W};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    nb.ux[q] = L.GX[sn[q]]; nb.uy[q] = L.GY[sn[q]]; nb.w[q] = L.NH[sn[q]] > eps;
                }
                const real ux = L.GX[s], uy = L.GY[s];
                // c_f again from memory (L2): P1 overwrote its LDS copy
                const real cf = a.cf[(ty0 + y) * nx + tx0 + x];
                real fx, fy;
                soft_forces(a, H, ux, uy, nb, fx, fy);
                vmax = rmax(vmax, cfl_speed(a, H, cf, ux, uy, fx, fy));
            }
        }
        bits |= own | (eW << 1) | (eE << 2) | (eS << 3) | (eN << 4) | (rg << 5);
    }
}

// ---------------------------------------------------------------- step kernel

// Waves per SIMD the step kernels are compiled for: the register budget per
// lane is 512 / WAVES_PER_SIMD.  A budget below the kernel's live state spills
// to scratch memory, which every launch then writes and reads through HBM.
#ifndef SWE_WAVES_PER_SIMD_F32
#define SWE_WAVES_PER_SIMD_F32 4
#endif
#ifndef SWE_WAVES_PER_SIMD_F64
#define SWE_WAVES_PER_SIMD_F64 2
#endif
template <typename real> constexpr int waves_per_simd() {
    return sizeof(real) == 4 ? SWE_WAVES_PER_SIMD_F32 : SWE_WAVES_PER_SIMD_F64;
}

template <typename real, int TX, int TY, int NT, int LIM, int MODE>
__global__ __launch_bounds__(NT, waves_per_simd<real>()) void k_step(Args<real> a) {
    constexpr int NWAVE = NT / 64;
    __shared__ Lds<real, TX, TY> L;
    __shared__ double red_d[MODE == MODE_FIELD ? 3 : 2][NWAVE];
    __shared__ int red_i[NWAVE];
    __shared__ int s_last;

    Ctrl* const ctrl = a.ctrl;
    // The workgroup's own-segment entry is read beside the list's counts
    // (one memory round trip before the tile load, not two); it is used when
    // the list is no longer than the grid and its segment is long enough.
    constexpr bool RING = MODE == MODE_TAP;
    const int b0 = blockIdx.x;
    const bool spec_in = !RING && a.skip && b0 / NSEG < a.ntiles;
    const int spec = spec_in ? a.lists[(a.slot * NSEG + b0 % NSEG) * a.ntiles + b0 / NSEG] : 0;
    if (ctrl->err_gate) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int G = gridDim.x, grp = blockIdx.x % NSEG;
    // only the patches of a nest (tapping grids) carry ring tiles; the other
    // variants compile without them (no registers held for their bounds)
    const int nlist = a.skip ? ctrl->seg_off[a.slot][NSEG] : a.ntiles;
    const int count = nlist + (RING && a.skip ? a.nring : 0);   // list entries, then the ring tiles
    const real tau = (real)ctrl->tau;
    const real sdep = (real)ctrl->sdepth;
    const int gen = (int)ctrl->step + 2;
    const unsigned clk = clock_bits(ctrl->t);
    const int nx = a.nx, ny = a.ny;
    // a list no longer than the grid: one tile or none per workgroup, in
    // own-segment order; a longer one: plain order, strided by the grid
    const bool own = !RING && a.skip && count <= G;
    int first = -1;
    if (own) {
        const int g0 = b0 % NSEG, n0 = ctrl->seg_off[a.slot][g0 + 1] - ctrl->seg_off[a.slot][g0];
        const int e = spec_in && b0 / NSEG < n0 ? spec : list_entry_own(ctrl, a.lists, a.ntiles, a.slot, b0, G);
        first = e < 0 ? -1 : entry_tile(e);
    }
    const int npos = own ? (first >= 0 ? b0 + 1 : 0) : count;

    real vmax = real(0);
    bool bad = false;
    long long ncells = 0;

    for (int p = blockIdx.x; p < npos; p += G) {
        const int tile = !a.skip ? p
                         : first >= 0 ? first
                         : RING && p >= nlist ? a.ring_tiles[p - nlist]
                                              : entry_tile(list_entry(ctrl, a.lists, a.ntiles, a.slot, p));
        const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
        ncells += (long long)min(TX, nx - tx0) * min(TY, ny - ty0);
        const bool edge = tx0 < HALO || ty0 < HALO || tx0 + TX + HALO > nx || ty0 + TY + HALO > ny;
        constexpr bool FLD = MODE == MODE_FIELD;
        double msum = 0.0, lsum = 0.0, fsum = 0.0;
        int bits = 0, nbst = gen;
        const int fm = FLD ? (int)a.fmask[tile] : 0;
        // the tile's clamp ledger (and field volume) are read now and written
        // back at the end
        const double led = tid == 0 ? a.ledger[tile] : 0.0;
        const double fvo = FLD && tid == 0 ? a.fvol[tile] : 0.0;
        const ListCtx lx{a.stamp, a.lists, a.hot, a.ntiles, a.slot ^ 1, grp, gen, 0, 0, tile, a.ntx, a.nty,
                         a.skip != 0 && !(RING && ring_tile(a, tile)), clk};
        __syncthreads();   // LDS of the previous tile is free
        if (edge)
            tile_step<real, TX, TY, NT, LIM, true, MODE>(a, L, tx0, ty0, tau, sdep, vmax, bad, msum, lsum, fsum,
                                                         fm, bits, lx, nbst);
        else
            tile_step<real, TX, TY, NT, LIM, false, MODE>(a, L, tx0, ty0, tau, sdep, vmax, bad, msum, lsum, fsum,
                                                          fm, bits, lx, nbst);
        if constexpr (FLD) bits |= fm & 63;   // cells with rain are sources of the K1 rule
        // block reductions: flags, volume and ledger partials
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bits |= __shfl_xor(bits, o, 64);
        msum = wave_sum(msum);
        lsum = wave_sum(lsum);
        if constexpr (FLD) fsum = wave_sum(fsum);
        if (lane == 0) {
            red_i[wv] = bits; red_d[0][wv] = msum; red_d[1][wv] = lsum;
            if constexpr (FLD) red_d[2][wv] = fsum;
        }
        __syncthreads();
        if (wv == 0) {
            int bb = 0;
#pragma unroll
            for (int q = 0; q < NWAVE; ++q) bb |= red_i[q];
            if (lane == 0) {
                double ms = 0.0, ls = 0.0;
                for (int q = 0; q < NWAVE; ++q) { ms += red_d[0][q]; ls += red_d[1][q]; }
                a.mass[tile] = ms;
                a.ledger[tile] = led + ls * a.h_d * a.h_d;
                if constexpr (FLD) {
                    double fs = 0.0;
                    for (int q = 0; q < NWAVE; ++q) fs += red_d[2][q];
                    a.fvol[tile] = fvo + fs * a.h_d * a.h_d;
                }
            }
            if (a.skip) {
                // next list: this tile if K1-active at layer n (appended
                // already) or n+1, and the neighbours facing its wet edges
                // (layer n+1) unless their stamps show them listed
                const int ti = tile % a.ntx, tj = tile / a.ntx;
                const bool fresh = nbst < gen;
                int cand = -1;
                if (lane == 0 && !(bb & 64) && (bb & (1 | 32))) cand = tile;
                constexpr bool PER = MODE == MODE_PERIODIC;   // neighbours wrap round the domain
                if (lane == 1 && (bb & 2) && fresh && (ti > 0 || PER)) cand = ti > 0 ? tile - 1 : tile + a.ntx - 1;
                if (lane == 2 && (bb & 4) && fresh && (ti < a.ntx - 1 || PER))
                    cand = ti < a.ntx - 1 ? tile + 1 : tile - a.ntx + 1;
                if (lane == 3 && (bb & 8) && fresh && (tj > 0 || PER))
                    cand = tj > 0 ? tile - a.ntx : tile + (a.nty - 1) * a.ntx;
                if (lane == 4 && (bb & 16) && fresh && (tj < a.nty - 1 || PER))
                    cand = tj < a.nty - 1 ? tile + a.ntx : tile - (a.nty - 1) * a.ntx;
                if (RING && cand >= 0 && ring_tile(a, cand)) cand = -1;
                append_tiles(cand, 0, 0, gen, a.stamp, a.lists, a.hot, a.ntiles, a.slot ^ 1, grp);
            }
        }
    }

    // ---- completion.  The workgroup's error, speed maximum and cell count go
    // to its group's words by atomics, each issued only once the previous one
    // has returned (its result feeds the next one's condition), and its
    // arrival is counted with the cells: when the count completes, every
    // workgroup's contributions have been performed, and no memory fence is
    // needed on the way (the tile outputs and list entries are for the next
    // launch).  The last arrival of the last group finalises.
    vmax = wave_max(vmax);
    __syncthreads();
    if (lane == 0) red_d[0][wv] = (double)vmax;
    const int anybad = __syncthreads_or((int)bad);
    if (tid == 0) {
        double vm = 0.0;
        for (int q = 0; q < NWAVE; ++q) vm = fmax(vm, red_d[0][q]);
        unsigned long long* const h64 = reinterpret_cast<unsigned long long*>(a.hot);
        const int err_was = anybad ? atomicCAS(&ctrl->err, 0, -4) : 0;
        unsigned long long sp = 0;
        if (err_was != INT_MIN)   // always: waits for the error
            sp = atomicMax(&h64[hot_spd(grp) / 2], (unsigned long long)__double_as_longlong(vm));
        const int in_grp = (G - grp + NSEG - 1) / NSEG, ngrp = G < NSEG ? G : NSEG;
        bool last = false;
        if (sp != ~0ull) {        // always (no speed has these bits): waits for the maximum
            const unsigned long long old =
                atomicAdd(&h64[hot_cnt(grp) / 2], ((unsigned long long)ncells << CNT_BITS) | 1ull);
            if ((int)(old & ((1ull << CNT_BITS) - 1)) == in_grp - 1)
                last = atomicAdd((unsigned*)&a.hot[hot_done(NSEG)], 1u) == (unsigned)(ngrp - 1);
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    // acquire only: the group words, segment counters and errors were
    // performed by atomics; nothing this workgroup wrote needs to be made
    // visible before the kernel ends (a full fence would also write back
    // every dirty line of this XCD's L2, microseconds on the critical path)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) {
        // every read of the bookkeeping is issued before the first write, so
        // the reads cost one memory round trip, not one each
        Ctrl c = *ctrl;
        int nseg[NSEG];
#pragma unroll
        for (int g = 0; g < NSEG; ++g) nseg[g] = a.skip ? a.hot[hot_seg(a.slot ^ 1, g)] : 0;
        unsigned long long* const h64 = reinterpret_cast<unsigned long long*>(a.hot);
        double S = 0.0;
        long long cells = 0;
#pragma unroll
        for (int g = 0; g < NSEG; ++g) {
            S = fmax(S, __longlong_as_double((long long)h64[hot_spd(g) / 2]));
            cells += (long long)(h64[hot_cnt(g) / 2] >> CNT_BITS);
        }
        const double tau_done = c.tau;
        c.t += tau_done;
        c.inflow += c.dV;
        c.last_tau = tau_done;
        c.step += 1;
        // tiles of the step: the list's (read again: the step does not
        // change the counts of the list it runs) and the ring tiles
        c.tiles += a.skip ? ctrl->seg_off[a.slot][NSEG] + (RING ? a.nring : 0) : a.ntiles;
        c.cells += cells;
        next_step_scalars(a, &c, S);
        if (c.err) c.err_gate = c.err;
        *ctrl = c;
        if (a.skip) close_segments_from(ctrl, nseg, a.slot ^ 1);
        if (a.skip)
            for (int g = 0; g < NSEG; ++g) a.hot[hot_seg(a.slot, g)] = 0;
        for (int g = 0; g < NSEG; ++g) { h64[hot_cnt(g) / 2] = 0ull; h64[hot_spd(g) / 2] = 0ull; }
        a.hot[hot_done(NSEG)] = 0;
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
    __shared__ double red_d[NWAVE];
    __shared__ real red_v[NWAVE];
    __shared__ int red_i[NWAVE];
    const int tid = threadIdx.x, tile = blockIdx.x;
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    const int nx = a.nx, ny = a.ny;
    const real eps = a.eps;
    for (int k = tid; k < N; k += NT) {
        const int lx = k % W - 1, ly = k / W - 1;
        int fx = 0, fy = 0, gx, gy;
        if (a.periodic) {   // the cell one period away, as it is
            gx = (tx0 + lx + nx) % nx;
            gy = (ty0 + ly + ny) % ny;
        } else {
            gx = mirror(tx0 + lx, nx, fx);
            gy = mirror(ty0 + ly, ny, fy);
        }
        const int gi = gy * nx + gx;
        const real H = a.Hi[gi];
        real qx = a.Qxi[gi], qy = a.Qyi[gi];
        if (fx & 1) qx = -qx;
        if (fy & 1) qy = -qy;
        const bool w = H > eps;
        sH[k] = H;
        sUx[k] = w ? Mth<real>::div(qx, H) : real(0);
        sUy[k] = w ? Mth<real>::div(qy, H) : real(0);
    }
    __syncthreads();
    real vmax = real(0);
    double msum = 0.0;
    int act = 0;
    for (int k = tid; k < N; k += NT) {
        const int lx = k % W - 1, ly = k / W - 1;
        int gx = tx0 + lx, gy = ty0 + ly;
        if (a.periodic) { gx = (gx + nx) % nx; gy = (gy + ny) % ny; }
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
        const bool in_tile = lx >= 0 && lx < TX && ly >= 0 && ly < TY;
        const bool corner = (lx < 0 || lx >= TX) && (ly < 0 || ly >= TY);
        if (corner) continue;
        const bool w = sH[k] > eps;
        if (w || is_src(a, gx, gy) || (a.sigma && a.sigma[gy * nx + gx] > real(0))) act = 1;
        if (!in_tile) continue;
        const real H = sH[k];
        msum += (double)H;
        if (w) {
            Nb4<real> nb;
            const int sn[4] = {k - 1, k + 1, k - W, k + W};
#pragma unroll
            for (int q = 0; q < 4; ++q) { nb.ux[q] = sUx[sn[q]]; nb.uy[q] = sUy[sn[q]]; nb.w[q] = sH[sn[q]] > eps; }
            real fx, fy;
            soft_forces(a, H, sUx[k], sUy[k], nb, fx, fy);
            vmax = rmax(vmax, cfl_speed(a, H, a.cf[gy * nx + gx], sUx[k], sUy[k], fx, fy));
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
        if (vm > real(0)) atomic_max_prep(a.ctrl, vm);
    }
    if (a.skip && wv == 0) {
        int ac0 = 0;
#pragma unroll
        for (int q = 0; q < NWAVE; ++q) ac0 |= red_i[q];
        append_tiles(lane == 0 && ac0 && !ring_tile(a, tile) ? tile : -1, a.sid, a.tile_base, (int)a.lctrl->step + 1,
                     a.stamp, a.lists, a.hot, a.list_cap, a.slot, blockIdx.x % NSEG);
    }
}

// Set the length of the next step (held steps; tau <= 0: the recorded CFL
// step of the current layer) and its hydrograph scalars.  The tile list is
// left alone.
template <typename real>
__global__ void k_set_dt(Args<real> a, double tau) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        set_next_step(a, a.ctrl, tau > 0.0 ? (double)(real)tau : a.ctrl->tau_cfl);
}

// Coarse layer = means of r x r fine cells (H, Qx, Qy), written to both
// coarse buffers.
template <typename real>
__global__ void k_restrict(const real* __restrict__ H, const real* __restrict__ Qx, const real* __restrict__ Qy,
                           int nxf, int r, real* H0, real* Qx0, real* Qy0, real* H1, real* Qx1, real* Qy1,
                           int nxc, int nyc) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nxc * nyc; k += gridDim.x * blockDim.x) {
        const int I = k % nxc, J = k / nxc;
        double sh = 0.0, sx = 0.0, sy = 0.0;
        for (int jj = 0; jj < r; ++jj)
            for (int ii = 0; ii < r; ++ii) {
                const int f = (J * r + jj) * nxf + I * r + ii;
                sh += (double)H[f];
                sx += (double)Qx[f];
                sy += (double)Qy[f];
            }
        const double inv = 1.0 / (double)(r * r);
        H0[k] = H1[k] = (real)(sh * inv);
        Qx0[k] = Qx1[k] = (real)(sx * inv);
        Qy0[k] = Qy1[k] = (real)(sy * inv);
    }
}

template <typename real>
__global__ void k_fill(real* p, long n, real v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

template <typename real>
__global__ void k_prepare_finish(Args<real> a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctrl* c = a.ctrl;
        c->err = 0;
        c->err_gate = 0;
        next_step_scalars(a, c, prep_speed(c, real(0)));
        c->prep_speed = 0ull;
        if (a.skip) close_segments(a.lctrl, a.hot, a.slot);
        if (c->err) c->err_gate = c->err;
    }
}

// ---------------------------------------------------------------- batched ensemble
// Independent scenarios of uneven grid sizes advanced together: one launch per
// step processes the active tiles of every scenario from one shared list
// (entries tagged with the scenario), each scenario with its own time step,
// clock, hydrograph and error state (Sec. 1: hundreds of runs over hydrograph
// and hydraulic-structure settings).  The tile work is the same tile_step as
// a single grid, so a scenario in a batch equals its standalone run bitwise.
template <typename real>
struct BatchArgs {
    const Args<real>* scen;   // per scenario, buffers of this step's parity
    int n;                    // scenarios
    Ctrl* lctrl;              // list control of the batch
    int* hot;
    int* lists;
    int list_cap;             // capacity of one list segment (all tiles of the batch)
    int slot;                 // list slot read by this step
    long long* wg_cells;
};

template <typename real, int TX, int TY, int NT, int LIM>
__global__ __launch_bounds__(NT, waves_per_simd<real>()) void k_batch_step(BatchArgs<real> ba) {
    constexpr int NWAVE = NT / 64;
    __shared__ Lds<real, TX, TY> L;
    __shared__ double red_d[3][NWAVE];
    __shared__ int red_i[NWAVE];
    __shared__ long long red_l[NWAVE];
    __shared__ int s_last;

    Ctrl* const lc = ba.lctrl;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int G = gridDim.x, grp = blockIdx.x % NSEG;
    const int count = lc->seg_off[ba.slot][NSEG];
    const int gen = (int)lc->step + 2;
    long long ncells = 0;

    for (int p = blockIdx.x; p < count; p += G) {
        const int e = list_entry(lc, ba.lists, ba.list_cap, ba.slot, p);
        const int sid = entry_sid(e), tile = entry_tile(e);
        const Args<real>& a = ba.scen[sid];
        Ctrl* const c = a.ctrl;
        if (c->err_gate) continue;   // a stopped scenario drops out of the lists
        const real tau = (real)c->tau, sdep = (real)c->sdepth;
        const int nx = a.nx, ny = a.ny;
        const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
        ncells += (long long)min(TX, nx - tx0) * min(TY, ny - ty0);
        const bool edge = tx0 < HALO || ty0 < HALO || tx0 + TX + HALO > nx || ty0 + TY + HALO > ny;
        real vt = real(0);
        bool bad = false;
        double msum = 0.0, lsum = 0.0, fnone = 0.0;   // scenarios of a batch carry no rate field
        int bits = 0, nbst = gen;
        const double led = tid == 0 ? a.ledger[tile] : 0.0;
        const ListCtx lx{a.stamp, ba.lists, ba.hot, ba.list_cap, ba.slot ^ 1, grp, gen, sid, a.tile_base, tile,
                         a.ntx, a.nty, a.skip != 0, clock_bits(a.ctrl->t)};
        __syncthreads();   // LDS of the previous tile is free
        if (edge)
            tile_step<real, TX, TY, NT, LIM, true, MODE_PLAIN>(a, L, tx0, ty0, tau, sdep, vt, bad, msum, lsum, fnone,
                                                               0, bits, lx, nbst);
        else
            tile_step<real, TX, TY, NT, LIM, false, MODE_PLAIN>(a, L, tx0, ty0, tau, sdep, vt, bad, msum, lsum, fnone,
                                                                0, bits, lx, nbst);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bits |= __shfl_xor(bits, o, 64);
        bits |= __any(bad) ? 128 : 0;
        msum = wave_sum(msum);
        lsum = wave_sum(lsum);
        vt = wave_max(vt);
        if (lane == 0) { red_i[wv] = bits; red_d[0][wv] = msum; red_d[1][wv] = lsum; red_d[2][wv] = (double)vt; }
        __syncthreads();
        if (wv == 0) {
            int bb = 0;
#pragma unroll
            for (int q = 0; q < NWAVE; ++q) bb |= red_i[q];
            if (lane == 0) {
                double ms = 0.0, ls = 0.0, vm = 0.0;
                for (int q = 0; q < NWAVE; ++q) { ms += red_d[0][q]; ls += red_d[1][q]; vm = fmax(vm, red_d[2][q]); }
                a.mass[tile] = ms;
                a.ledger[tile] = led + ls * a.h_d * a.h_d;
                if (vm > 0.0) atomic_max_prep(c, (real)vm);
                if (bb & 128) atomicCAS(&c->err, 0, -4);
            }
            if (a.skip) {
                const int ti = tile % a.ntx, tj = tile / a.ntx;
                const bool fresh = nbst < gen;
                int cand = -1;
                if (lane == 0 && !(bb & 64) && (bb & (1 | 32))) cand = tile;
                if (lane == 1 && (bb & 2) && ti > 0 && fresh) cand = tile - 1;
                if (lane == 2 && (bb & 4) && ti < a.ntx - 1 && fresh) cand = tile + 1;
                if (lane == 3 && (bb & 8) && tj > 0 && fresh) cand = tile - a.ntx;
                if (lane == 4 && (bb & 16) && tj < a.nty - 1 && fresh) cand = tile + a.ntx;
                append_tiles(cand, sid, a.tile_base, gen, a.stamp, ba.lists, ba.hot, ba.list_cap, ba.slot ^ 1, grp);
            }
        }
    }

    // ---- completion: two-level counter; the last workgroup finalises every scenario
    if (tid == 0) {
        ba.wg_cells[blockIdx.x] = ncells;
        __threadfence();
        const int in_grp = (G - grp + NSEG - 1) / NSEG, ngrp = G < NSEG ? G : NSEG;
        bool last = false;
        if (atomicAdd((unsigned*)&ba.hot[hot_done(grp)], 1u) == (unsigned)(in_grp - 1))
            last = atomicAdd((unsigned*)&ba.hot[hot_done(NSEG)], 1u) == (unsigned)(ngrp - 1);
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    long long cs = 0;
    for (int k = tid; k < G; k += NT) cs += ba.wg_cells[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cs += __shfl_xor(cs, o, 64);
    if (lane == 0) red_l[wv] = cs;
    for (int k = tid; k < ba.n; k += NT) {
        const Args<real>& a = ba.scen[k];
        Ctrl c = *a.ctrl;   // all reads first, one write-back
        if (c.err_gate) continue;
        const double tau_done = c.tau;
        c.t += tau_done;
        c.inflow += c.dV;
        c.last_tau = tau_done;
        c.step += 1;
        next_step_scalars(a, &c, prep_speed(&c, real(0)));
        c.prep_speed = 0ull;
        if (c.err) c.err_gate = c.err;
        *a.ctrl = c;
    }
    __syncthreads();
    if (tid == 0) {
        Ctrl c = *lc;
        int nseg[NSEG];
#pragma unroll
        for (int g = 0; g < NSEG; ++g) nseg[g] = ba.hot[hot_seg(ba.slot ^ 1, g)];
        long long cells = 0;
        for (int q = 0; q < NWAVE; ++q) cells += red_l[q];
        c.step += 1;
        c.tiles += count;
        c.cells += cells;
        *lc = c;
        close_segments_from(lc, nseg, ba.slot ^ 1);
        for (int g = 0; g < NSEG; ++g) ba.hot[hot_seg(ba.slot, g)] = 0;
        for (int g = 0; g <= NSEG; ++g) ba.hot[hot_done(g)] = 0;
    }
    __threadfence();
}

// After the per-scenario preparation kernels: first time steps and list offsets.
template <typename real>
__global__ void k_batch_prepare_finish(BatchArgs<real> ba) {
    for (int k = threadIdx.x; k < ba.n; k += blockDim.x) {
        const Args<real>& a = ba.scen[k];
        Ctrl* const c = a.ctrl;
        c->err = 0;
        c->err_gate = 0;
        next_step_scalars(a, c, prep_speed(c, real(0)));
        c->prep_speed = 0ull;
        if (c->err) c->err_gate = c->err;
    }
    if (threadIdx.x == 0) close_segments(ba.lctrl, ba.hot, ba.slot);
}

// Fixed-order FP64 sum of per-tile partials (one workgroup of 1024 threads).
__global__ void k_sum_tiles(const double* part, int n, double* out);

}  // namespace swe
