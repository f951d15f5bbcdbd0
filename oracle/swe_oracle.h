/*
 * swe_oracle.h -- plain FP64 CPU oracle of one CSPH-TVD shallow-water step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path never links, calls or falls back to it, and the two share no code,
 * header, table or constant.
 *
 * What it computes follows Dyakonova, Khoperskov & Khrapov, "Numerical Model
 * of Shallow Water: the Use of NVIDIA CUDA Graphics Processors" (arXiv
 * 1705.00614):
 *   - Saint-Venant equations and force terms: Sec. 2.1, Eqs. (1)-(4);
 *   - four-stage CSPH-TVD step (forces and time step, Lagrangian
 *     predictor-corrector, Riemann fluxes through Euler-cell faces, final
 *     update with the particles put back at the cell centres): Sec. 2.3;
 *   - order of the device stages K1..K8 and the wet-block rule of K1:
 *     Sec. 3 (kernel list and the two code fragments).
 * The paper's scheme figure is not available, so the discrete formulas are a
 * documented reading of that text (stated at each function in the .c file).
 *
 * Conventions: arrays are FP64, row-major with x fastest, index j*nx+i, cell
 * centres at ((i+1/2)h, (j+1/2)h).  The caller owns every array it passes;
 * the library copies what it keeps.
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

typedef struct {
    double g;          /* gravitational acceleration [m/s^2] */
    double courant;    /* Courant number K, 0 < K < 1 */
    double eps;        /* wet threshold: a cell is wet iff H > eps [m] */
    double tau_max;    /* upper bound of the time step [s] (<= 0: none) */
    double tau_min;    /* a CFL step below this is an error [s] */
    double nu;         /* turbulent viscosity [m^2/s] */
    double f_cor;      /* Coriolis parameter 2*Omega*sin(latitude) [1/s] */
    double wind_x, wind_y;  /* wind velocity W [m/s] */
    double wind_kappa; /* C_a * rho_a / rho */
    double h_wind;     /* depth floor in the wind term [m] */
    int limiter;       /* 0 minmod, 1 van Leer, 2 monotonised central */
    int periodic;      /* 0 reflective walls, 1 periodic wrap (tests) */
    int in_i0, in_j0, in_ni, in_nj;   /* inlet rectangle of source cells */
    double q_base, q_peak, t_peak, sigma_t; /* Gaussian hydrograph [m^3/s], [s] */
    int sph_displaced; /* 1: corrector pressure gradient at the displaced
                          particle positions of t_{n+1/2} (SPH sum over the
                          5x5 neighbourhood, corrected); 0: lattice stencil */
} orc_params;

/* Error codes (negative). */
#define ORC_EINVAL      (-1)
#define ORC_ENOMEM      (-2)
#define ORC_ENONFINITE  (-4)
#define ORC_EDTCOLLAPSE (-5)

/* Create a simulation.  b, n_manning, solid, H0, Qx0, Qy0 may be NULL
 * (flat bed, no friction, no closed gates, dry, at rest).  A closed gate
 * (solid != 0) is a permanently dry cell whose bed is far above any level.
 * Returns NULL on invalid arguments or allocation failure. */
orc_sim* orc_create(int nx, int ny, double h, const double* b,
                    const double* n_manning, const unsigned char* solid,
                    const double* H0, const double* Qx0, const double* Qy0,
                    const orc_params* p);
void   orc_destroy(orc_sim* s);

/* One step with the CFL time step of the current layer; 0 or ORC_E*. */
int    orc_step(orc_sim* s);
/* One step with a prescribed time step tau (unit tests). */
int    orc_step_tau(orc_sim* s, double tau);
/* n steps; stops at the first error and returns it. */
int    orc_run(orc_sim* s, long n);

/* The CFL time step the next step would take (Sec. 2.3, stage I). */
double orc_next_tau(orc_sim* s);
/* CFL speed max(U_s, U_p) of every cell of the current layer (0 where dry),
 * row-major nx*ny; and the time step that a maximum speed gives. */
int    orc_cell_speeds(orc_sim* s, double* out);
/* Flux corrections added to every later step's stage III fluxes: dE through
 * the east face and dN through the north face of each cell, 3 planes of
 * nx*ny each (mass, x-momentum, y-momentum); after the Lagrangian stage the
 * mass part needs an upwind cell deeper than the correction depth (eps
 * unless set), the momentum part two such cells; wall faces take none.
 * Both NULL clears them. */
int    orc_set_correction(orc_sim* s, const double* dE, const double* dN);
/* Correction depth (default and minimum: eps). */
int    orc_set_correction_depth(orc_sim* s, double hmin);
double orc_tau_from_speed(const orc_sim* s, double smax);

double orc_mass(const orc_sim* s);      /* h^2 * sum H, compensated FP64 sum */
double orc_time(const orc_sim* s);      /* simulated time */
double orc_last_tau(const orc_sim* s);  /* time step of the last step */
double orc_ledger(const orc_sim* s);    /* volume added by depth clamps */
double orc_inflow(const orc_sim* s);    /* sum of hydrograph volumes */
/* Rate field sigma(x, y) [m/s] (nx*ny, row-major; rain > 0, infiltration and
 * evaporation < 0; copied; NULL removes it) and the volume it has applied. */
int    orc_set_source_field(orc_sim* s, const double* sigma);
double orc_field_volume(const orc_sim* s);
long   orc_steps(const orc_sim* s);

int    orc_get_state(const orc_sim* s, double* H, double* Qx, double* Qy);
int    orc_set_state(orc_sim* s, const double* H, const double* Qx,
                     const double* Qy);

/* Intermediate fields of the last step (nx*ny each), for stage-level pins. */
enum {
    ORC_F_GX = 0, ORC_F_GY,     /* SPH pressure gradient of eta at layer n  */
    ORC_F_UHX, ORC_F_UHY,       /* predictor velocity at t_{n+1/2}          */
    ORC_F_ULX, ORC_F_ULY,       /* corrector (Lagrangian) velocity          */
    ORC_F_HT, ORC_F_QTX, ORC_F_QTY, /* post-Lagrangian depth and momentum   */
    ORC_F_GDX, ORC_F_GDY,       /* gradient at the displaced positions of
                                   t_{n+1/2} (sph_displaced only)           */
    ORC_F_COUNT
};
int    orc_get_field(const orc_sim* s, int which, double* out);
/* Face fluxes of the last step.  dir 0: x-faces, (nx+1)*ny, face i-1/2 of
 * row j at j*(nx+1)+i; dir 1: y-faces, nx*(ny+1), face j-1/2 of column i at
 * j*nx+i.  Each of FH, Fqn (normal momentum), Fqt (tangential) may be NULL. */
int    orc_get_faces(const orc_sim* s, int dir, double* FH, double* Fqn,
                     double* Fqt);

/* Volume delivered by the Gaussian hydrograph over [t, t+tau] (closed form). */
double orc_hydrograph_volume(double q_base, double q_peak, double t_peak,
                             double sigma_t, double t, double tau);

/* Wet-block rule of kernel K1 (Sec. 3, K1 fragment) on tiles of tx*ty cells:
 * own[k]  = 1 iff some cell of tile k has H > eps or is a source;
 * ring[k] = 1 iff some outer face-neighbour of an edge cell (no diagonal
 *           corners; at the domain edge the cell itself) has H > eps or is a
 *           source.
 * Tiles are numbered row-major, ceil(nx/tx) per row.  source may be NULL. */
int    orc_tile_flags(int nx, int ny, int tx, int ty, const double* H,
                      const unsigned char* source, double eps,
                      int* own, int* ring);

#ifdef __cplusplus
}
#endif
#endif
