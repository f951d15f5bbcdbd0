/*
 * swe_oracle.c -- plain FP64 CPU oracle of the CSPH-TVD shallow-water step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU product path.
 *
 * Written from arXiv 1705.00614 (Dyakonova, Khoperskov, Khrapov).  The paper's
 * scheme figure is lost, so where it is silent the reading used is stated at
 * the function that applies it.  Everything runs in IEEE FP64 with libm
 * sqrt/cbrt/erf; build with -ffp-contract=off.  Every cell is computed every
 * step (no dry skipping): the skipping rule of K1 is checked separately.
 *
 * Layout: every field is stored padded with a ghost frame of NG cells, index
 * P(i,j) = (j+NG)*px + (i+NG), px = nx+2NG.  After each stage the ghost frame
 * of its output is refilled: with reflective walls a ghost cell holds the
 * mirror image (about the wall face) of an interior cell, with the velocity
 * component normal to that wall negated; with the periodic test boundary it
 * holds the wrapped cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "swe_oracle.h"

#define NG 2
/* Bed of a closed-gate cell: far above any water level, so the cell stays
 * dry, the hydrostatic face depths beside it are zero and the pressure
 * stencil sees the own level there. */
#define GATE_BED 1.0e6

/* SPH pressure-gradient weights.  Reading: cubic B-spline kernel with
 * smoothing length equal to the cell size h, particles at cell centres,
 * gradient normalised so that it is exact for linear fields.  Only the 4 face
 * and 4 diagonal neighbours fall inside the kernel support with a nonzero
 * kernel slope; the weights are
 *   alpha = 1/(12*sqrt2 - 14),  beta = (3*sqrt2 - 4)/(12*sqrt2 - 14),
 * with 2*alpha + 4*beta = 1. */
static double sph_alpha(void) { return 1.0 / (12.0 * sqrt(2.0) - 14.0); }
static double sph_beta(void)  { return (3.0 * sqrt(2.0) - 4.0) / (12.0 * sqrt(2.0) - 14.0); }

struct orc_sim {
    int nx, ny, px, py;
    long ncell_pad;
    double h;
    orc_params p;
    double *b, *cf;                 /* static: bed, g*n_M^2 */
    unsigned char *src;             /* inlet cells (interior only) */
    unsigned char *solid;           /* closed gates (interior only) */
    long n_src;
    double *H, *Qx, *Qy;            /* state at layer n */
    unsigned char *wet;             /* H > eps at layer n */
    double *Ux, *Uy, *eta;          /* derived at layer n */
    double *Gx, *Gy, *lam0;         /* pressure gradient, c_f / H^(4/3) */
    double *Gdx, *Gdy;              /* gradient at the displaced positions (corrector) */
    double *Uhx, *Uhy;              /* U at t_{n+1/2} */
    double *ULx, *ULy;              /* Lagrangian U at t_{n+1} */
    double *Ht, *Qtx, *Qty;         /* post-Lagrangian state */
    unsigned char *wett;            /* Ht > eps */
    double *Utx, *Uty, *etat;       /* post-Lagrangian velocity and level */
    double *FxH, *FxQn, *FxQt;      /* x-faces (nx+1)*ny */
    double *FyH, *FyQn, *FyQt;      /* y-faces nx*(ny+1) */
    double *sigma;                  /* source rate field [m/s] (rain > 0, losses < 0) or NULL */
    double *corrE, *corrN;          /* flux corrections (3 planes of nx*ny) or NULL */
    double corr_hmin;               /* depth both cells need for momentum corrections */
    double t, tau_last, ledger, inflow, field;
    long steps;
};

static inline long P(const orc_sim* s, int i, int j)
{
    return (long)(j + NG) * s->px + (i + NG);
}

/* ------------------------------------------------------------------ */
/* Ghost frame                                                         */
/* ------------------------------------------------------------------ */

/* Reflect index i into [0, n) about the end faces, counting reflections. */
static int reflect(int i, int n, int* flips)
{
    while (i < 0 || i >= n) {
        if (i < 0) i = -1 - i;
        else       i = 2 * n - 1 - i;
        (*flips)++;
    }
    return i;
}

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Refill the ghost frame of a padded field.  sx (sy) multiplies the value
 * once per reflection across an x (y) wall: -1 for the x (y) component of a
 * vector, +1 for scalars.  Corner ghosts take both reflections. */
static void fill_ghost(const orc_sim* s, double* f, double sx, double sy)
{
    for (int j = -NG; j < s->ny + NG; ++j) {
        for (int i = -NG; i < s->nx + NG; ++i) {
            if (i >= 0 && i < s->nx && j >= 0 && j < s->ny) continue;
            int si, sj;
            double sign = 1.0;
            if (s->p.periodic) {
                si = wrap(i, s->nx);
                sj = wrap(j, s->ny);
            } else {
                int fx = 0, fy = 0;
                si = reflect(i, s->nx, &fx);
                sj = reflect(j, s->ny, &fy);
                if (fx & 1) sign *= sx;
                if (fy & 1) sign *= sy;
            }
            f[P(s, i, j)] = sign * f[P(s, si, sj)];
        }
    }
}

static void fill_ghost_u8(const orc_sim* s, unsigned char* f)
{
    for (int j = -NG; j < s->ny + NG; ++j) {
        for (int i = -NG; i < s->nx + NG; ++i) {
            if (i >= 0 && i < s->nx && j >= 0 && j < s->ny) continue;
            int si, sj;
            if (s->p.periodic) {
                si = wrap(i, s->nx);
                sj = wrap(j, s->ny);
            } else {
                int fx = 0, fy = 0;
                si = reflect(i, s->nx, &fx);
                sj = reflect(j, s->ny, &fy);
            }
            f[P(s, i, j)] = f[P(s, si, sj)];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Creation                                                            */
/* ------------------------------------------------------------------ */

static double* zalloc(long n)
{
    return (double*)calloc((size_t)n, sizeof(double));
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    double** fields[] = {&s->b, &s->cf, &s->H, &s->Qx, &s->Qy, &s->Ux, &s->Uy,
                         &s->eta, &s->Gx, &s->Gy, &s->lam0, &s->Uhx, &s->Uhy,
                         &s->ULx, &s->ULy, &s->Ht, &s->Qtx, &s->Qty, &s->Utx,
                         &s->Uty, &s->etat, &s->FxH, &s->FxQn, &s->FxQt,
                         &s->FyH, &s->FyQn, &s->FyQt, &s->Gdx, &s->Gdy};
    for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k) free(*fields[k]);
    free(s->src);
    free(s->solid);
    free(s->wet);
    free(s->wett);
    free(s->corrE);
    free(s->corrN);
    free(s->sigma);
    free(s);
}

/* Derived fields of layer n on the whole padded range (Sec. 2.1: eta = H+b,
 * U = Q/H on wet cells; dry cells are at rest). */
static void derive_layer(orc_sim* s)
{
    fill_ghost(s, s->H, 1.0, 1.0);
    fill_ghost(s, s->Qx, -1.0, 1.0);
    fill_ghost(s, s->Qy, 1.0, -1.0);
    for (long k = 0; k < s->ncell_pad; ++k) {
        int w = s->H[k] > s->p.eps;
        s->wet[k] = (unsigned char)w;
        s->Ux[k] = w ? s->Qx[k] / s->H[k] : 0.0;
        s->Uy[k] = w ? s->Qy[k] / s->H[k] : 0.0;
        s->eta[k] = s->H[k] + s->b[k];
    }
}

static int finite_state(const orc_sim* s)
{
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long k = P(s, i, j);
            if (!isfinite(s->H[k]) || !isfinite(s->Qx[k]) || !isfinite(s->Qy[k]))
                return 0;
        }
    return 1;
}

/* Load a state; a closed gate is forced dry, dry cells are put at rest. */
static int load_state(orc_sim* s, const double* H, const double* Qx, const double* Qy)
{
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long a = (long)j * s->nx + i, k = P(s, i, j);
            double hh = H ? H[a] : 0.0, qx = Qx ? Qx[a] : 0.0, qy = Qy ? Qy[a] : 0.0;
            if (!isfinite(hh) || !isfinite(qx) || !isfinite(qy) || hh < 0.0)
                return ORC_EINVAL;
            if (s->solid[k]) hh = qx = qy = 0.0;
            if (!(hh > s->p.eps)) qx = qy = 0.0;
            s->H[k] = hh;
            s->Qx[k] = qx;
            s->Qy[k] = qy;
        }
    return 0;
}

orc_sim* orc_create(int nx, int ny, double h, const double* b,
                    const double* n_manning, const unsigned char* solid,
                    const double* H0, const double* Qx0, const double* Qy0,
                    const orc_params* p)
{
    if (nx < 1 || ny < 1 || !(h > 0.0) || !isfinite(h) || !p) return NULL;
    if (!(p->g > 0.0) || !(p->courant > 0.0) || !(p->courant < 1.0) || !(p->eps > 0.0))
        return NULL;
    if (p->nu < 0.0 || p->limiter < 0 || p->limiter > 2) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->nx = nx;
    s->ny = ny;
    s->px = nx + 2 * NG;
    s->py = ny + 2 * NG;
    s->ncell_pad = (long)s->px * s->py;
    s->h = h;
    s->p = *p;
    long n = s->ncell_pad;
    double** fields[] = {&s->b, &s->cf, &s->H, &s->Qx, &s->Qy, &s->Ux, &s->Uy,
                         &s->eta, &s->Gx, &s->Gy, &s->lam0, &s->Uhx, &s->Uhy,
                         &s->ULx, &s->ULy, &s->Ht, &s->Qtx, &s->Qty, &s->Utx,
                         &s->Uty, &s->etat, &s->Gdx, &s->Gdy};
    for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k) {
        *fields[k] = zalloc(n);
        if (!*fields[k]) { orc_destroy(s); return NULL; }
    }
    long nfx = (long)(nx + 1) * ny, nfy = (long)nx * (ny + 1);
    s->FxH = zalloc(nfx); s->FxQn = zalloc(nfx); s->FxQt = zalloc(nfx);
    s->FyH = zalloc(nfy); s->FyQn = zalloc(nfy); s->FyQt = zalloc(nfy);
    s->src = (unsigned char*)calloc((size_t)n, 1);
    s->solid = (unsigned char*)calloc((size_t)n, 1);
    s->wet = (unsigned char*)calloc((size_t)n, 1);
    s->wett = (unsigned char*)calloc((size_t)n, 1);
    if (!s->FxH || !s->FxQn || !s->FxQt || !s->FyH || !s->FyQn || !s->FyQt ||
        !s->src || !s->solid || !s->wet || !s->wett) {
        orc_destroy(s);
        return NULL;
    }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            long a = (long)j * nx + i, k = P(s, i, j);
            double bb = b ? b[a] : 0.0, nm = n_manning ? n_manning[a] : 0.0;
            if (!isfinite(bb) || !isfinite(nm) || nm < 0.0) { orc_destroy(s); return NULL; }
            s->solid[k] = (unsigned char)(solid && solid[a]);
            s->b[k] = s->solid[k] ? GATE_BED : bb;
            /* Manning: lambda/2 = g n_M^2 / H^(4/3) (Sec. 2.1, F_fric). */
            s->cf[k] = s->solid[k] ? 0.0 : p->g * nm * nm;
        }
    fill_ghost(s, s->b, 1.0, 1.0);
    fill_ghost(s, s->cf, 1.0, 1.0);
    if (p->in_ni > 0 && p->in_nj > 0) {
        if (p->in_i0 < 0 || p->in_j0 < 0 || p->in_i0 + p->in_ni > nx ||
            p->in_j0 + p->in_nj > ny) { orc_destroy(s); return NULL; }
        for (int j = p->in_j0; j < p->in_j0 + p->in_nj; ++j)
            for (int i = p->in_i0; i < p->in_i0 + p->in_ni; ++i)
                if (!s->solid[P(s, i, j)]) { s->src[P(s, i, j)] = 1; s->n_src++; }
    }
    if (load_state(s, H0, Qx0, Qy0) != 0) { orc_destroy(s); return NULL; }
    return s;
}

/* ------------------------------------------------------------------ */
/* Stage I: forces and time step                                       */
/* ------------------------------------------------------------------ */

/* Pressure gradient G = grad(eta*) at every interior wet cell (SPH stage,
 * Sec. 2.3).  Reading of the level eta*_m that a neighbour m shows to a wet
 * cell c, after the hydrostatic-reconstruction principle behind the paper's
 * regularisation-free wet/dry fronts: a neighbour pushes with at most its own
 * depth above c's surface and never from below c's bed,
 *     eta*_m = max(b_c, min(eta_m, eta_c + H_m)),
 * with H_m = 0, eta_m = b_m for a dry neighbour (which gives
 * min(eta_c, max(b_m, b_c)): a dry bank above the surface exerts no push, a
 * dry cell below the own bed counts as the own bed).  Over a flat bed and in
 * a lake at rest eta*_m = eta_m; a film on a high bank pushes with its film
 * depth only, so the force is continuous as the film crosses eps. */
static void pressure_gradient(orc_sim* s)
{
    const double al = sph_alpha(), be = sph_beta(), ih = 1.0 / s->h;
    const long px = s->px;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            if (!s->wet[c]) { s->Gx[c] = s->Gy[c] = 0.0; continue; }
            const double ec = s->eta[c], bc = s->b[c];
            double e[9];
            int q = 0;
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    long m = c + dj * px + di;
                    double Hm = s->wet[m] ? s->H[m] : 0.0;
                    double em = s->wet[m] ? s->eta[m] : s->b[m];
                    e[q] = fmax(bc, fmin(em, ec + Hm));
                    ++q;
                }
            /* e[0]=SW e[1]=S e[2]=SE e[3]=W e[4]=C e[5]=E e[6]=NW e[7]=N e[8]=NE */
            s->Gx[c] = (al * (e[5] - e[3]) + be * ((e[8] - e[6]) + (e[2] - e[0]))) * ih;
            s->Gy[c] = (al * (e[7] - e[1]) + be * ((e[8] - e[2]) + (e[6] - e[0]))) * ih;
        }
}

/* c_f / H^(4/3) on wet cells (Manning, Sec. 2.1), H^(4/3) = H*cbrt(H). */
static void friction_factor(orc_sim* s)
{
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            double H = s->H[c];
            s->lam0[c] = s->wet[c] ? s->cf[c] / (H * cbrt(H)) : 0.0;
        }
}

/* Force density without pressure and without friction at cell c for the
 * velocity field (ux, uy) (Eq. 4 and Sec. 2.1):
 *   viscosity  nu * Laplacian(U) over the wet face neighbours (reading: the
 *              printed scalar sum is the vector Laplacian; a dry neighbour
 *              takes no part);
 *   Coriolis   2 [U x Omega] -> f (U_y, -U_x);
 *   wind       C_a rho_a/(rho H) (W-U)|W-U|, with H floored at h_wind. */
static void soft_forces(const orc_sim* s, long c, const double* ux, const double* uy,
                        double* fx, double* fy)
{
    const orc_params* p = &s->p;
    double vx = 0.0, vy = 0.0;
    if (p->nu != 0.0) {
        const long nb[4] = {c - 1, c + 1, c - s->px, c + s->px};
        for (int k = 0; k < 4; ++k) {
            long m = nb[k];
            if (s->wet[m]) {
                vx += ux[m] - ux[c];
                vy += uy[m] - uy[c];
            }
        }
        double k2 = p->nu / (s->h * s->h);
        vx *= k2;
        vy *= k2;
    }
    double cx = p->f_cor * uy[c];
    double cy = -p->f_cor * ux[c];
    double dx = p->wind_x - ux[c], dy = p->wind_y - uy[c];
    double wm = sqrt(dx * dx + dy * dy);
    double kw = p->wind_kappa * wm / fmax(s->H[c], p->h_wind);
    *fx = vx + cx + kw * dx;
    *fy = vy + cy + kw * dy;
}

static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* Time step from layer n (Sec. 2.3, stage I):
 *   U_s = max(|Ux|, |Uy|) + sqrt(g H),
 *   U_p = max(|Ux + sgn(Fx) sqrt(h|Fx|)|, |Uy + sgn(Fy) sqrt(h|Fy|)|),
 * maximum over wet cells, tau = min(tau_max, K h / max(U_s, U_p),
 * h^2/(4 nu)); a bound whose divisor is zero is left out.  F is the whole
 * force density of Eq. (4) at layer n without the pressure gradient:
 * viscosity, Coriolis, wind and bottom friction F_fric = -(lambda/2) U|U|,
 * lambda/2 = c_f / H^(4/3).  The printed sqrt(h F) is read as
 * sgn(F) sqrt(h|F|). */
static double cell_speed(const orc_sim* s, long c)
{
    const orc_params* p = &s->p;
    if (!s->wet[c]) return 0.0;
    double ux = s->Ux[c], uy = s->Uy[c];
    double fx, fy;
    soft_forces(s, c, s->Ux, s->Uy, &fx, &fy);
    double fr = s->lam0[c] * sqrt(ux * ux + uy * uy);
    fx -= fr * ux;
    fy -= fr * uy;
    double us = fmax(fabs(ux), fabs(uy)) + sqrt(p->g * s->H[c]);
    double upx = fabs(ux + sgn(fx) * sqrt(s->h * fabs(fx)));
    double upy = fabs(uy + sgn(fy) * sqrt(s->h * fabs(fy)));
    return fmax(us, fmax(upx, upy));
}

static double tau_from_speed(const orc_sim* s, double smax)
{
    const orc_params* p = &s->p;
    double tau = p->tau_max > 0.0 ? p->tau_max : INFINITY;
    if (smax > 0.0) tau = fmin(tau, p->courant * s->h / smax);
    if (p->nu > 0.0) tau = fmin(tau, s->h * s->h / (4.0 * p->nu));
    return tau;
}

static double cfl_tau(orc_sim* s)
{
    double smax = 0.0;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            double sp = cell_speed(s, P(s, i, j));
            if (sp > smax) smax = sp;
        }
    return tau_from_speed(s, smax);
}

/* ------------------------------------------------------------------ */
/* Stage II: Lagrangian predictor-corrector                            */
/* ------------------------------------------------------------------ */

/* Derivative dW/dq of the 2D cubic B-spline kernel shape (support q < 2):
 * W = 1 - 3/2 q^2 + 3/4 q^3 for q < 1, 1/4 (2 - q)^3 for 1 <= q < 2.  Its
 * normalisation constant cancels in the corrected gradient below. */
static double bspline_dw(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) return -0.75 * (2.0 - q) * (2.0 - q);
    return 0.0;
}

/* Pressure gradient at the displaced particle positions of t_{n+1/2}
 * (Sec. 2.3 stage II and kernels K4-K6: the particles move inside the cells;
 * the corrector takes the forces at the positions of the half step).
 * Reading: particle j sits at its cell centre c_j + (tau/2) U_j^n (dry
 * particles at rest); the level gradient at a wet particle i is the
 * corrected SPH sum of the cubic B-spline kernel with smoothing length h over
 * the particles of its 5x5 neighbourhood (with |tau U| <= K h < h every
 * particle within the support 2h of i is among them):
 *   w_ij = W'(|r_ij|/h) r_ij / |r_ij|,  r_ij = p_j - p_i,
 *   S    = sum_j (eta*_j - eta_i) w_ij,  M = sum_j w_ij r_ij^T,
 *   G_i  = M^{-1} S,
 * exact for a linear level whatever the displacements; with no
 * displacement it is the lattice stencil of pressure_gradient.  eta*_j is the
 * level particle j shows to i (the rule of pressure_gradient). */
static void displaced_gradient(orc_sim* s, double tau)
{
    const double h = s->h;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            if (!s->wet[c]) { s->Gdx[c] = s->Gdy[c] = 0.0; continue; }
            double ec = s->eta[c], bc = s->b[c];
            double pxi = 0.5 * tau * s->Ux[c] / h, pyi = 0.5 * tau * s->Uy[c] / h;
            double Sx = 0.0, Sy = 0.0, mxx = 0.0, mxy = 0.0, myx = 0.0, myy = 0.0;
            for (int dj = -2; dj <= 2; ++dj)
                for (int di = -2; di <= 2; ++di) {
                    if (!di && !dj) continue;
                    long m = c + (long)dj * s->px + di;
                    double rx = di + 0.5 * tau * s->Ux[m] / h - pxi;
                    double ry = dj + 0.5 * tau * s->Uy[m] / h - pyi;
                    double r = sqrt(rx * rx + ry * ry);
                    double dw = bspline_dw(r);
                    if (dw == 0.0) continue;
                    double Hm = s->wet[m] ? s->H[m] : 0.0;
                    double em = s->wet[m] ? s->eta[m] : s->b[m];
                    double es = fmax(bc, fmin(em, ec + Hm));
                    double wx = dw * rx / r, wy = dw * ry / r;
                    Sx += (es - ec) * wx;
                    Sy += (es - ec) * wy;
                    mxx += wx * rx;
                    mxy += wx * ry;
                    myx += wy * rx;
                    myy += wy * ry;
                }
            double det = mxx * myy - mxy * myx;
            s->Gdx[c] = (myy * Sx - mxy * Sy) / det / h;
            s->Gdy[c] = (mxx * Sy - myx * Sx) / det / h;
        }
}

/* Reading of the predictor-corrector (Sec. 2.3, stage II; K4-K6): midpoint
 * rule with the pressure gradient of layer n and friction point-implicit:
 *   U^{n+1/2} = (U + tau/2 A(U)) / (1 + tau/2 Lambda(U)),
 *   U^L       = (U + tau   A(U^{n+1/2})) / (1 + tau Lambda(U^{n+1/2})),
 * A(U) = -g G + F_visc(U) + F_cor(U) + F_wind(U), Lambda(U) = c_f|U|/H^(4/3).
 * The particle displacement tau*U^L is carried by the fluxes of stage III.
 * G is the lattice gradient of layer n in both halves, or (sph_displaced) in
 * the corrector the gradient at the displaced positions of t_{n+1/2}. */
static void lagrangian(orc_sim* s, double tau)
{
    const double g = s->p.g;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            if (!s->wet[c]) { s->Uhx[c] = s->Uhy[c] = 0.0; continue; }
            double ux = s->Ux[c], uy = s->Uy[c], fx, fy;
            soft_forces(s, c, s->Ux, s->Uy, &fx, &fy);
            double ax = -g * s->Gx[c] + fx, ay = -g * s->Gy[c] + fy;
            double lam = s->lam0[c] * sqrt(ux * ux + uy * uy);
            double d = 1.0 + 0.5 * tau * lam;
            s->Uhx[c] = (ux + 0.5 * tau * ax) / d;
            s->Uhy[c] = (uy + 0.5 * tau * ay) / d;
        }
    fill_ghost(s, s->Uhx, -1.0, 1.0);
    fill_ghost(s, s->Uhy, 1.0, -1.0);
    const double *Gcx = s->Gx, *Gcy = s->Gy;
    if (s->p.sph_displaced) {
        displaced_gradient(s, tau);
        Gcx = s->Gdx;
        Gcy = s->Gdy;
    }
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            if (!s->wet[c]) { s->ULx[c] = s->ULy[c] = 0.0; continue; }
            double hx = s->Uhx[c], hy = s->Uhy[c], fx, fy;
            soft_forces(s, c, s->Uhx, s->Uhy, &fx, &fy);
            double ax = -g * Gcx[c] + fx, ay = -g * Gcy[c] + fy;
            double lam = s->lam0[c] * sqrt(hx * hx + hy * hy);
            double d = 1.0 + tau * lam;
            s->ULx[c] = (s->Ux[c] + tau * ax) / d;
            s->ULy[c] = (s->Uy[c] + tau * ay) / d;
        }
}

/* Sources (Eq. 1 sigma; Sec. 2.3 stage I) and the post-Lagrangian state.
 * Reading: the inflow velocity V of Eqs. (2)-(3) is zero, so in conservative
 * form the source adds mass only: Ht = H + s, Qt = H U^L.  Two kinds of
 * sigma: the hydrograph spread over the inlet cells (depth sdepth per step),
 * and a rate field sigma(x, y) [m/s] for the spatial factors of Sec. 2.1
 * (precipitation > 0; infiltration and evaporation < 0).  Over a step of
 * length tau a rate adds tau*sigma of depth; a loss acts only on a cell wet
 * at layer n (films are inert) and takes at most the water it holds,
 * Ht = max(Ht + tau*sigma, 0).  The depth the field applied is summed into
 * the field volume, which closes the volume balance
 * V_N - V_0 = inflow + field + ledger. */
static void post_lagrangian(orc_sim* s, double sdepth, double tau)
{
    const double eps = s->p.eps;
    double field = 0.0;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long c = P(s, i, j);
            double Ht = s->H[c] + (s->src[c] ? sdepth : 0.0);
            if (s->sigma) {
                double sg = s->sigma[(long)j * s->nx + i], H1 = Ht;
                if (sg > 0.0)
                    H1 = Ht + tau * sg;
                else if (sg < 0.0 && s->wet[c])
                    H1 = fmax(Ht + tau * sg, 0.0);
                field += H1 - Ht;
                Ht = H1;
            }
            double qx = s->wet[c] ? s->H[c] * s->ULx[c] : 0.0;
            double qy = s->wet[c] ? s->H[c] * s->ULy[c] : 0.0;
            s->Ht[c] = Ht;
            s->Qtx[c] = qx;
            s->Qty[c] = qy;
            int w = Ht > eps;
            s->wett[c] = (unsigned char)w;
            s->Utx[c] = w ? qx / Ht : 0.0;
            s->Uty[c] = w ? qy / Ht : 0.0;
            s->etat[c] = Ht + s->b[c];
        }
    s->field += field * s->h * s->h;
    fill_ghost(s, s->Ht, 1.0, 1.0);
    fill_ghost(s, s->Utx, -1.0, 1.0);
    fill_ghost(s, s->Uty, 1.0, -1.0);
    fill_ghost(s, s->etat, 1.0, 1.0);
    fill_ghost_u8(s, s->wett);
}

/* ------------------------------------------------------------------ */
/* Stage III: TVD reconstruction and Riemann fluxes                    */
/* ------------------------------------------------------------------ */

static double limiter(int kind, double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    if (kind == 1) return 2.0 * a * b / (a + b);                 /* van Leer */
    if (kind == 2) {                                            /* MC */
        double m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
        return a > 0.0 ? m : -m;
    }
    return fabs(a) < fabs(b) ? a : b;                           /* minmod */
}

typedef struct { double H, eta, un, ut; } face_state;

/* Limited linear reconstruction of cell c on its face in direction +d (side
 * = +1) or -d (side = -1), stride d = 1 (x) or px (y).  un/ut are the normal
 * and tangential velocity fields for that direction.  Reading: a dry cell
 * (Ht <= eps) shows H = 0, U = 0, eta = b on its faces; for a wet cell the
 * slopes of Ht, eta_t, un, ut are limited, a dry neighbour contributes a zero
 * velocity difference, the face depth is clamped at zero. */
static face_state reconstruct(const orc_sim* s, long c, long d, int side,
                              const double* un, const double* ut)
{
    face_state f;
    if (!s->wett[c]) {
        f.H = 0.0; f.eta = s->b[c]; f.un = 0.0; f.ut = 0.0;
        return f;
    }
    const int lim = s->p.limiter;
    long m = c - d, q = c + d;
    double sH = limiter(lim, s->Ht[c] - s->Ht[m], s->Ht[q] - s->Ht[c]);
    double sE = limiter(lim, s->etat[c] - s->etat[m], s->etat[q] - s->etat[c]);
    double dm_n = s->wett[m] ? un[c] - un[m] : 0.0, dq_n = s->wett[q] ? un[q] - un[c] : 0.0;
    double dm_t = s->wett[m] ? ut[c] - ut[m] : 0.0, dq_t = s->wett[q] ? ut[q] - ut[c] : 0.0;
    double sN = limiter(lim, dm_n, dq_n);
    double sT = limiter(lim, dm_t, dq_t);
    double hs = 0.5 * side;
    f.H = fmax(0.0, s->Ht[c] + hs * sH);
    f.eta = s->etat[c] + hs * sE;
    f.un = un[c] + hs * sN;
    f.ut = ut[c] + hs * sT;
    return f;
}

/* Approximate Riemann solver at one face (Sec. 2.3, stage III).  Reading:
 * hydrostatic reconstruction of the face depths over b* = max(bL, bR) and the
 * local Lax-Friedrichs (Rusanov) flux of the advective part; pressure acted
 * in the Lagrangian stage.  L is the lower-index side. */
static void riemann(double g, face_state L, face_state R,
                    double* FH, double* Fqn, double* Fqt)
{
    double bL = L.eta - L.H, bR = R.eta - R.H;
    double bs = fmax(bL, bR);
    double hL = fmax(0.0, L.eta - bs), hR = fmax(0.0, R.eta - bs);
    double a = fmax(fabs(L.un) + sqrt(g * hL), fabs(R.un) + sqrt(g * hR));
    *FH = 0.5 * (hL * L.un + hR * R.un) - 0.5 * a * (hR - hL);
    *Fqn = 0.5 * (hL * L.un * L.un + hR * R.un * R.un) - 0.5 * a * (hR * R.un - hL * L.un);
    *Fqt = 0.5 * (hL * L.un * L.ut + hR * R.un * R.ut) - 0.5 * a * (hR * R.ut - hL * L.ut);
}

/* Learned flux correction (added to the stage III fluxes before the final
 * update): planes [mass, x-momentum, y-momentum] of the correction through
 * the east (or north) face of cell k, which lies between cells cl and cr.
 * With the correction depth hc = max(eps, corr_hmin) after the Lagrangian
 * stage, the mass correction needs a donor (upwind) cell deeper than hc, the
 * momentum correction two cells deeper than hc (a film would otherwise gain
 * momentum without water, or lose water but keep its momentum); wall faces
 * take none. */
static void add_correction(const orc_sim* s, const double* corr, long k, long cl, long cr,
                           double* fH, double* fN, double* fT, int xface)
{
    const long n = (long)s->nx * s->ny;
    const double dH = corr[k], dX = corr[n + k], dY = corr[2 * n + k];
    const long donor = dH > 0.0 ? cl : cr;
    const double hm = s->corr_hmin > s->p.eps ? s->corr_hmin : s->p.eps;
    if (s->Ht[donor] > hm) *fH += dH;
    if (s->Ht[cl] > hm && s->Ht[cr] > hm) {
        *fN += xface ? dX : dY;
        *fT += xface ? dY : dX;
    }
}

static void fluxes(orc_sim* s)
{
    const double g = s->p.g;
    const long px = s->px;
    /* x-faces: face i-1/2 between cells i-1 and i, i = 0..nx */
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i <= s->nx; ++i) {
            long cl = P(s, i - 1, j), cr = P(s, i, j);
            face_state L = reconstruct(s, cl, 1, +1, s->Utx, s->Uty);
            face_state R = reconstruct(s, cr, 1, -1, s->Utx, s->Uty);
            long f = (long)j * (s->nx + 1) + i;
            riemann(g, L, R, &s->FxH[f], &s->FxQn[f], &s->FxQt[f]);
            if (s->corrE && i >= 1 && i <= s->nx - 1)
                add_correction(s, s->corrE, (long)j * s->nx + i - 1, cl, cr,
                               &s->FxH[f], &s->FxQn[f], &s->FxQt[f], 1);
        }
    /* y-faces: face j-1/2 between cells j-1 and j, j = 0..ny */
    for (int j = 0; j <= s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long cl = P(s, i, j - 1), cr = P(s, i, j);
            face_state L = reconstruct(s, cl, px, +1, s->Uty, s->Utx);
            face_state R = reconstruct(s, cr, px, -1, s->Uty, s->Utx);
            long f = (long)j * s->nx + i;
            riemann(g, L, R, &s->FyH[f], &s->FyQn[f], &s->FyQt[f]);
            if (s->corrN && j >= 1 && j <= s->ny - 1)
                add_correction(s, s->corrN, (long)(j - 1) * s->nx + i, cl, cr,
                               &s->FyH[f], &s->FyQn[f], &s->FyQt[f], 0);
        }
}

/* ------------------------------------------------------------------ */
/* Stage IV: final update (K8)                                         */
/* ------------------------------------------------------------------ */

/* H' = Ht + tau/h (net inflow through the 4 faces), H = max(H', 0) with the
 * clamp booked in the ledger; Q = Qt + tau/h (net momentum inflow) where
 * H > eps, else 0 (K8 fragment: dev_h, dev_hv; reading of their bodies).
 * Returns 1 if any updated value was NaN or infinite before the clamps. */
static int final_update(orc_sim* s, double tau)
{
    const double r = tau / s->h, eps = s->p.eps, h2 = s->h * s->h;
    const int nx = s->nx;
    double ledger = 0.0;
    int bad = 0;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < nx; ++i) {
            long c = P(s, i, j);
            long fw = (long)j * (nx + 1) + i, fe = fw + 1;
            long fs = (long)j * nx + i, fn = fs + nx;
            double Hn = s->Ht[c] + r * ((s->FxH[fw] - s->FxH[fe]) + (s->FyH[fs] - s->FyH[fn]));
            double qx = s->Qtx[c] + r * ((s->FxQn[fw] - s->FxQn[fe]) + (s->FyQt[fs] - s->FyQt[fn]));
            double qy = s->Qty[c] + r * ((s->FxQt[fw] - s->FxQt[fe]) + (s->FyQn[fs] - s->FyQn[fn]));
            if (!isfinite(Hn) || !isfinite(qx) || !isfinite(qy)) bad = 1;
            double Hc = fmax(Hn, 0.0);
            ledger += h2 * (Hc - Hn);
            int w = Hc > eps;
            s->H[c] = Hc;
            s->Qx[c] = w ? qx : 0.0;
            s->Qy[c] = w ? qy : 0.0;
        }
    s->ledger += ledger;
    return bad;
}

/* ------------------------------------------------------------------ */
/* Driver                                                              */
/* ------------------------------------------------------------------ */

double orc_hydrograph_volume(double q_base, double q_peak, double t_peak,
                             double sigma_t, double t, double tau)
{
    /* integral over [t, t+tau] of q_base + (q_peak-q_base) exp(-(t-t_p)^2/(2 sigma^2)) */
    double v = q_base * tau;
    if (sigma_t > 0.0 && q_peak != q_base) {
        double k = 1.0 / (sigma_t * sqrt(2.0));
        v += (q_peak - q_base) * sigma_t * sqrt(2.0 * atan(1.0)) * /* sqrt(pi/2) */
             (erf((t + tau - t_peak) * k) - erf((t - t_peak) * k));
    }
    return v;
}

static void prepare_layer(orc_sim* s)
{
    derive_layer(s);
    friction_factor(s);
    fill_ghost(s, s->lam0, 1.0, 1.0);
}

double orc_next_tau(orc_sim* s)
{
    if (!s) return NAN;
    prepare_layer(s);
    return cfl_tau(s);
}

int orc_cell_speeds(orc_sim* s, double* out)
{
    if (!s || !out) return ORC_EINVAL;
    prepare_layer(s);
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) out[(long)j * s->nx + i] = cell_speed(s, P(s, i, j));
    return 0;
}

double orc_tau_from_speed(const orc_sim* s, double smax)
{
    return s ? tau_from_speed(s, smax) : NAN;
}

static int step_with(orc_sim* s, double tau)
{
    if (!(tau > 0.0) || !isfinite(tau)) return ORC_EDTCOLLAPSE;
    pressure_gradient(s);
    lagrangian(s, tau);
    double dV = 0.0, sdepth = 0.0;
    if (s->n_src > 0) {
        dV = orc_hydrograph_volume(s->p.q_base, s->p.q_peak, s->p.t_peak,
                                   s->p.sigma_t, s->t, tau);
        sdepth = dV / ((double)s->n_src * s->h * s->h);
    }
    post_lagrangian(s, sdepth, tau);
    fluxes(s);
    int bad = final_update(s, tau);
    s->t += tau;
    s->inflow += dV;
    s->tau_last = tau;
    s->steps++;
    return (!bad && finite_state(s)) ? 0 : ORC_ENONFINITE;
}

int orc_step(orc_sim* s)
{
    if (!s) return ORC_EINVAL;
    prepare_layer(s);
    double tau = cfl_tau(s);
    if (!(tau >= s->p.tau_min) || !isfinite(tau)) return ORC_EDTCOLLAPSE;
    return step_with(s, tau);
}

int orc_step_tau(orc_sim* s, double tau)
{
    if (!s) return ORC_EINVAL;
    prepare_layer(s);
    return step_with(s, tau);
}

int orc_run(orc_sim* s, long n)
{
    if (!s || n < 0) return ORC_EINVAL;
    for (long k = 0; k < n; ++k) {
        int rc = orc_step(s);
        if (rc) return rc;
    }
    return 0;
}

double orc_mass(const orc_sim* s)
{
    if (!s) return NAN;
    /* Neumaier compensated sum */
    double sum = 0.0, comp = 0.0;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            double x = s->H[P(s, i, j)];
            double t = sum + x;
            if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
            else comp += (x - t) + sum;
            sum = t;
        }
    return (sum + comp) * s->h * s->h;
}

double orc_time(const orc_sim* s) { return s ? s->t : NAN; }
double orc_last_tau(const orc_sim* s) { return s ? s->tau_last : NAN; }
double orc_ledger(const orc_sim* s) { return s ? s->ledger : NAN; }
double orc_inflow(const orc_sim* s) { return s ? s->inflow : NAN; }
double orc_field_volume(const orc_sim* s) { return s ? s->field : NAN; }

int orc_set_source_field(orc_sim* s, const double* sigma)
{
    if (!s) return ORC_EINVAL;
    if (!sigma) {
        free(s->sigma);
        s->sigma = NULL;
        return 0;
    }
    long n = (long)s->nx * s->ny;
    for (long k = 0; k < n; ++k)
        if (!isfinite(sigma[k])) return ORC_EINVAL;
    if (!s->sigma) s->sigma = zalloc(n);
    if (!s->sigma) return ORC_EINVAL;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long a = (long)j * s->nx + i;
            /* a closed gate holds no water: no field there */
            s->sigma[a] = s->solid[P(s, i, j)] ? 0.0 : sigma[a];
        }
    return 0;
}
long   orc_steps(const orc_sim* s) { return s ? s->steps : -1; }

int orc_get_state(const orc_sim* s, double* H, double* Qx, double* Qy)
{
    if (!s) return ORC_EINVAL;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            long a = (long)j * s->nx + i, k = P(s, i, j);
            if (H) H[a] = s->H[k];
            if (Qx) Qx[a] = s->Qx[k];
            if (Qy) Qy[a] = s->Qy[k];
        }
    return 0;
}

int orc_set_state(orc_sim* s, const double* H, const double* Qx, const double* Qy)
{
    if (!s || !H) return ORC_EINVAL;
    return load_state(s, H, Qx, Qy);
}

int orc_get_field(const orc_sim* s, int which, double* out)
{
    if (!s || !out || which < 0 || which >= ORC_F_COUNT) return ORC_EINVAL;
    const double* f[ORC_F_COUNT] = {s->Gx, s->Gy, s->Uhx, s->Uhy, s->ULx, s->ULy,
                                    s->Ht, s->Qtx, s->Qty, s->Gdx, s->Gdy};
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) out[(long)j * s->nx + i] = f[which][P(s, i, j)];
    return 0;
}

int orc_get_faces(const orc_sim* s, int dir, double* FH, double* Fqn, double* Fqt)
{
    if (!s || (dir != 0 && dir != 1)) return ORC_EINVAL;
    long n = dir == 0 ? (long)(s->nx + 1) * s->ny : (long)s->nx * (s->ny + 1);
    const double* a = dir == 0 ? s->FxH : s->FyH;
    const double* b = dir == 0 ? s->FxQn : s->FyQn;
    const double* c = dir == 0 ? s->FxQt : s->FyQt;
    if (FH) memcpy(FH, a, (size_t)n * sizeof(double));
    if (Fqn) memcpy(Fqn, b, (size_t)n * sizeof(double));
    if (Fqt) memcpy(Fqt, c, (size_t)n * sizeof(double));
    return 0;
}

int orc_set_correction_depth(orc_sim* s, double hmin)
{
    if (!s || !(hmin >= 0.0)) return ORC_EINVAL;
    s->corr_hmin = hmin;
    return 0;
}

int orc_set_correction(orc_sim* s, const double* dE, const double* dN)
{
    if (!s) return ORC_EINVAL;
    const long n = 3L * s->nx * s->ny;
    free(s->corrE); free(s->corrN);
    s->corrE = s->corrN = NULL;
    if (!dE && !dN) return 0;
    s->corrE = zalloc(n);
    s->corrN = zalloc(n);
    if (!s->corrE || !s->corrN) return ORC_ENOMEM;
    if (dE) memcpy(s->corrE, dE, (size_t)n * sizeof(double));
    if (dN) memcpy(s->corrN, dN, (size_t)n * sizeof(double));
    return 0;
}

/* K1 wet-block rule (Sec. 3, K1 fragment), written from its definition. */
int orc_tile_flags(int nx, int ny, int tx, int ty, const double* H,
                   const unsigned char* source, double eps, int* own, int* ring)
{
    if (nx < 1 || ny < 1 || tx < 1 || ty < 1 || !H || !own || !ring) return ORC_EINVAL;
    int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty;
    for (int tj = 0; tj < nty; ++tj)
        for (int ti = 0; ti < ntx; ++ti) {
            int k = tj * ntx + ti, o = 0, r = 0;
            int i0 = ti * tx, j0 = tj * ty;
            int i1 = i0 + tx < nx ? i0 + tx : nx, j1 = j0 + ty < ny ? j0 + ty : ny;
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    long a = (long)j * nx + i;
                    if (H[a] > eps || (source && source[a])) o = 1;
                    /* outer face neighbours of edge cells of the tile */
                    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
                    int edge[4] = {i == i0, i == i1 - 1, j == j0, j == j1 - 1};
                    for (int q = 0; q < 4; ++q) {
                        if (!edge[q]) continue;
                        int ii = nb[q][0], jj = nb[q][1];
                        if (ii < 0 || ii >= nx) ii = i;   /* domain edge: self */
                        if (jj < 0 || jj >= ny) jj = j;
                        long m = (long)jj * nx + ii;
                        if (H[m] > eps || (source && source[m])) r = 1;
                    }
                }
            own[k] = o;
            ring[k] = r;
        }
    return 0;
}
