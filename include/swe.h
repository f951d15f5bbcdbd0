/*
 * swe.h -- C ABI of the MI355X (gfx950) CSPH-TVD shallow-water library
 * (libswe_hip.so).
 *
 * The library advances the Saint-Venant equations of arXiv 1705.00614
 * (Sec. 2.1, Eqs. 1-4: continuity with sources sigma, momentum with the
 * free-surface gradient, Manning bottom friction, turbulent viscosity,
 * Coriolis and wind forces) with the four-stage CSPH-TVD step of Sec. 2.3:
 *   I   forces at t_n and the CFL time step tau_n,
 *   II  Lagrangian predictor-corrector of the cell-centred particles,
 *   III TVD reconstruction and approximate-Riemann mass and momentum fluxes
 *       through the Euler-cell faces,
 *   IV  final update with the particles put back at the cell centres,
 * skipping tiles without water (Sec. 3, kernels K1 and K8).  All of it runs
 * in hand-written HIP kernels on the GPU; the host only launches them.
 *
 * Conventions
 *   - Host arrays are FP64, row-major with x fastest: cell (i, j) at index
 *     j*nx + i, centre at ((i+1/2) dx, (j+1/2) dx).  The caller owns every
 *     array and the params struct; swe_create copies what it needs and keeps
 *     no caller pointer.
 *   - The handle is owned by the library until swe_destroy.  One handle is
 *     used by one host thread at a time; all its GPU work is ordered on the
 *     stream given at creation (the caller's hipStream_t, e.g. torch's
 *     current stream; NULL means a stream the library creates).
 *   - The state lives in device memory (HBM) between calls; only the get/set
 *     calls and the scalar queries copy to or from the host.
 *   - Errors: functions returning int give 0 or a negative SWE_E* code;
 *     swe_create returns NULL; the message is in swe_last_error().  After a
 *     device-side error (non-finite state, time-step collapse) the handle
 *     stops advancing until swe_set_state installs a new state.
 *   - Domain edges are reflective walls.  A closed gate (solid cell) is a
 *     permanently dry cell whose bed is far above any water level.
 */
#ifndef SWE_H
#define SWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_OK            0
#define SWE_EINVAL      (-1)   /* invalid argument */
#define SWE_ENOMEM      (-2)   /* device or host allocation failed */
#define SWE_EHIP        (-3)   /* a HIP runtime call failed */
#define SWE_ENONFINITE  (-4)   /* the state became NaN or infinite */
#define SWE_EDTCOLLAPSE (-5)   /* the CFL time step fell below dt_min */

typedef struct swe_s swe_t;

typedef struct {
    int    precision;    /* 32: FP32 stencil, 64: FP64 stencil.  Volume,
                            time and the hydrograph integral are FP64 always. */
    double g;            /* gravitational acceleration [m/s^2] */
    double cfl;          /* Courant number K, 0 < K < 1 (Sec. 2.3) */
    double eps;          /* wet threshold: a cell is wet iff H > eps [m] */
    double dt_max;       /* upper bound of tau [s]; <= 0: none */
    double dt_min;       /* a CFL step below this is SWE_EDTCOLLAPSE [s] */
    double nu;           /* turbulent viscosity [m^2/s] */
    double f_coriolis;   /* 2 Omega sin(latitude) [1/s] */
    double wind_x, wind_y; /* wind velocity W [m/s] */
    double wind_kappa;   /* C_a rho_a / rho of the wind force */
    double h_wind;       /* depth floor of the wind force [m] */
    int    limiter;      /* 0 minmod, 1 van Leer, 2 monotonised central */
    int    skip_dry;     /* 1: skip tiles without water (results identical) */
    int    tile_x, tile_y; /* tile shape; 0,0 = default for the precision */
    int    inlet_i0, inlet_j0, inlet_ni, inlet_nj; /* source rectangle; ni or
                            nj = 0: no source.  Must lie inside the grid and
                            contain no closed gate. */
    double q_base, q_peak, t_peak, sigma_t; /* Gaussian hydrograph
                            Q(t) = q_base + (q_peak-q_base) exp(-(t-t_peak)^2/(2 sigma_t^2))
                            [m^3/s], [s]; spread evenly over the inlet cells */
    const uint8_t* solid;  /* nx*ny closed-gate mask or NULL (copied) */
    const double* H0;      /* nx*ny initial depth >= 0, or NULL: dry */
    const double* Qx0;     /* nx*ny initial unit discharge H*Ux or NULL */
    const double* Qy0;     /* nx*ny initial unit discharge H*Uy or NULL */
    void*  stream;         /* hipStream_t owned by the caller, or NULL */
} swe_params;

/* Create a solver on an nx x ny grid of cell size dx [m] with bed elevation
 * b [m] and Manning coefficient n_M (both nx*ny, host FP64; n_M may be NULL
 * for no friction).  Allocates the state in device memory, uploads the
 * inputs, and computes the wet tiles and the first time step from layer 0.
 * Returns NULL on error (see swe_last_error). */
swe_t* swe_create(int nx, int ny, double dx, const double* b, const double* n_M,
                  const swe_params* p);

/* Advance one CSPH-TVD step (Sec. 2.3 stages I-IV).  Synchronises the
 * stream.  Returns 0 or SWE_E*. */
int    swe_step(swe_t* s);

/* Advance nsteps steps: device-side time step, no host round trip inside,
 * steps replayed from a captured hipGraph.  Synchronises at the end.  Stops
 * advancing at the first device error and returns it. */
int    swe_run(swe_t* s, long nsteps);

/* Water volume dx^2 * sum(H) [m^3], reduced on the GPU in FP64 in a fixed
 * order; NaN on error. */
double swe_mass(swe_t* s);

/* Free the handle and its device memory.  NULL-safe. */
void   swe_destroy(swe_t* s);

/* Copy the current state to host FP64 arrays (nx*ny each; any may be NULL). */
int    swe_get_state(swe_t* s, double* H, double* Qx, double* Qy);

/* Install a new state (H >= 0; Qx, Qy may be NULL for rest), e.g. a
 * checkpoint.  Clears a device error and recomputes the wet tiles and the
 * next time step.  Time, step count, inflow and ledger are kept. */
int    swe_set_state(swe_t* s, const double* H, const double* Qx, const double* Qy);

/* Set the simulated clock (restoring a checkpoint together with
 * swe_set_state); recomputes the next hydrograph volume.  t finite. */
int    swe_set_time(swe_t* s, double t);

double swe_time(swe_t* s);     /* simulated time [s] (FP64) */
double swe_last_dt(swe_t* s);  /* time step of the last completed step [s] */
double swe_next_dt(swe_t* s);  /* time step the next step will take [s] */
double swe_ledger(swe_t* s);   /* volume added by clamping negative depths [m^3] */
double swe_inflow(swe_t* s);   /* volume delivered by the hydrograph [m^3] (FP64) */
long   swe_steps(swe_t* s);    /* completed steps */

/* Work counters since creation: processed tile-steps, processed in-domain
 * cell-steps and tile count of the grid.  Any pointer may be NULL. */
int    swe_work(swe_t* s, long long* tile_steps, long long* cell_steps,
                int* ntiles, int* tile_x, int* tile_y);

/* Tiles the next step will process (row-major tile indices, unordered),
 * at most cap entries; returns the count or SWE_E*. */
int    swe_active_tiles(swe_t* s, int* out, int cap);

/* nsteps steps launched one by one with a HIP event pair around each step
 * kernel on the handle's stream; *kernel_ms receives the summed kernel time
 * [ms].  For measurement. */
int    swe_run_timed(swe_t* s, long nsteps, double* kernel_ms);

/* ------------------------------------------------------------------ batches
 * A batch advances n independent scenarios together -- the paper's use case
 * of hundreds of runs over hydrograph and hydraulic-structure settings
 * (Sec. 1) -- with uneven grid sizes, one kernel launch per step for all of
 * them, each scenario with its own time step, clock, hydrograph and error
 * state.  Scenario k has an nx[k] x ny[k] grid of cell size dx[k], bed b[k],
 * Manning n_M[k] (n_M or n_M[k] may be NULL) and parameters p[k] (closed
 * gates through p[k].solid, initial state through p[k].H0/Qx0/Qy0; all
 * copied).  precision, limiter and the tile shape come from p[0] and must
 * agree; every p[k].skip_dry must be 1; the stream is p[0].stream.  A
 * scenario computes bit for bit what a single handle with the same inputs
 * and tile shape computes.  Returns NULL on error. */
typedef struct swe_batch_s swe_batch_t;
swe_batch_t* swe_batch_create(int n, const int* nx, const int* ny, const double* dx,
                              const double* const* b, const double* const* n_M,
                              const swe_params* p);

/* Advance every scenario nsteps steps (hipGraph replay, one launch per step
 * for the whole batch); a scenario that hits an error stops while the others
 * continue.  Synchronises; returns 0 or the first scenario's SWE_E* code. */
int    swe_batch_run(swe_batch_t* b, long nsteps);

/* As swe_batch_run with a HIP event pair around every step kernel; the summed
 * kernel time goes to *kernel_ms. */
int    swe_batch_run_timed(swe_batch_t* b, long nsteps, double* kernel_ms);

/* Per-scenario clock [s], FP64 volume [m^3], hydrograph volume [m^3], clamp
 * ledger [m^3] and completed steps; arrays of n, any may be NULL. */
int    swe_batch_query(swe_batch_t* b, double* t, double* mass, double* inflow,
                       double* ledger, long* steps);

/* Host FP64 copy of scenario k's state (nx[k]*ny[k] each; any may be NULL). */
int    swe_batch_get_state(swe_batch_t* b, int k, double* H, double* Qx, double* Qy);

/* Processed tile-steps and in-domain cell-steps of the batch, total tiles. */
int    swe_batch_work(swe_batch_t* b, long long* tile_steps, long long* cell_steps,
                      int* total_tiles);

/* Free the batch and its device memory.  NULL-safe. */
void   swe_batch_destroy(swe_batch_t* b);

/* ------------------------------------------------------------------ nests
 * Hierarchical grids (Sec. 2.2: the small-scale flow of zoomed-in areas fed
 * back into the large-scale grid; Sec. 5: a 50 m grid with a 12.5 m local
 * grid): one coarse grid and patches refined by r over boxes of coarse
 * cells.  Per coarse step the coarse grid steps with tau_c, every patch takes
 * r substeps of tau_c / r inside a frame of SWE_NEST_FRAME fine cells filled
 * from the coarse layers n and n+1 (linear in time; fine depth
 * max(0, H_c + b_c - b_fine) where the coarse cell is wet, else dry), and
 * with feedback the covered coarse cells take the mean of their fine cells
 * while the uncovered cells next to a box take the mismatch between the
 * coarse and the summed fine fluxes through their shared face (clamped as in
 * the final update).  tau_c = min(CFL step of the coarse layer as stepped and
 * of the cells the feedback changed, r * CFL step of every patch after its
 * last substep).  Without feedback (one-way zoom-in) the coarse grid runs as
 * if alone and drives the patches.  The paper names the method, not the
 * coupling; this is the reading implemented. */
#define SWE_NEST_FRAME 5

typedef struct {
    int ci0, cj0, cw, ch;       /* covered coarse cells [ci0, ci0+cw) x [cj0, cj0+ch) */
    /* fine bed [m] and Manning n over the extended patch, row-major
     * (r*ch + 2*SWE_NEST_FRAME) x (r*cw + 2*SWE_NEST_FRAME); n may be NULL */
    const double* b;
    const double* n_M;
    /* initial interior state, (r*ch) x (r*cw) row-major; NULL = 0 */
    const double* H0;
    const double* Qx0;
    const double* Qy0;
} swe_patch;

typedef struct swe_nest_s swe_nest_t;

/* Create a nest: the coarse grid as for swe_create (p: its parameters, the
 * patches inherit the physics; tile_x = tile_y = 0 required), refinement
 * 1 <= r <= 16 and npatch >= 1 patches.  Every box keeps
 * ceil(SWE_NEST_FRAME / r) coarse cells from the domain edge, one uncovered
 * cell from every other box and from the inlet, and holds no closed gate
 * in it or its frame.  The coarse bed under a box should be the mean of the
 * fine bed (it is taken as given).  Patches step every tile (no dry
 * skipping).  NULL on error. */
swe_nest_t* swe_nest_create(int nx, int ny, double dx, const double* b, const double* n_M,
                            const swe_params* p, int r, int feedback, int npatch,
                            const swe_patch* patches);

/* Advance n coarse steps (each with its r substeps; hipGraph replay).
 * Synchronises; returns 0 or an SWE_E* code. */
int    swe_nest_run(swe_nest_t* n, long coarse_steps);

/* As swe_nest_run with a HIP event pair around every coarse step (all its
 * launches); the summed time goes to *kernel_ms. */
int    swe_nest_run_timed(swe_nest_t* n, long coarse_steps, double* kernel_ms);

/* Clock [s], volume of the nested solution (FP64 sum of the coarse depths,
 * covered cells holding the fine mean) [m^3], hydrograph volume [m^3], clamp
 * ledger (coarse grid plus feedback) [m^3], completed coarse steps, and the
 * time steps of the next coarse step and substeps [s].  Any may be NULL. */
int    swe_nest_query(swe_nest_t* n, double* t, double* volume, double* inflow, double* ledger,
                      long* steps, double* dt_coarse, double* dt_fine);

/* Host FP64 copy of the coarse state (nx*ny each) or of patch k's interior
 * ((r*ch) x (r*cw) each); any may be NULL. */
int    swe_nest_get_coarse(swe_nest_t* n, double* H, double* Qx, double* Qy);
int    swe_nest_get_patch(swe_nest_t* n, int k, double* H, double* Qx, double* Qy);

/* Free the nest and its device memory.  NULL-safe. */
void   swe_nest_destroy(swe_nest_t* n);

/* Message of the last error on this host thread ("" if none). */
const char* swe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
