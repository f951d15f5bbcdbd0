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
 *   - Domain edges are reflective walls (periodic in x and y with
 *     swe_params.periodic).  A closed gate (solid cell) is a permanently
 *     dry cell whose bed is far above any water level.
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
    int    sph_displaced;  /* 1: the corrector takes the pressure gradient at
                            the particle positions of t_{n+1/2} (Sec. 2.3
                            stage II, K4-K6): cell centre + (tau/2) U^n, the
                            corrected SPH sum of the cubic B-spline kernel
                            over the 5x5 neighbourhood; 0: the lattice
                            stencil at the centres (default).  Single grids
                            with the default tile shape; not with nests,
                            batches, corrections, networks, taps or fields. */
    int    periodic;       /* boundary: 0 reflective walls at the domain edges
                            (default; mirror ghost cells, normal velocity
                            negated); 1 periodic in x and y, for tests of
                            conservation (the cell one period away).
                            Periodic: single grids with the default tile
                            shape, nx and ny multiples of it, no solid
                            cells, the lattice corrector; not with nests,
                            batches, fields, corrections, networks, taps,
                            the autotuner or swe_step_noalloc (SWE_EINVAL /
                            NULL from swe_create). */
} swe_params;

/* Create a solver on an nx x ny grid of cell size dx [m] with bed elevation
 * b [m] and Manning coefficient n_M (both nx*ny, host FP64; n_M may be NULL
 * for no friction).  Allocates the state in device memory, uploads the
 * inputs, and computes the wet tiles and the first time step from layer 0.
 * Limits: nx*ny < 2^31 cells and fewer than 2^20 tiles of the tile shape
 * (with 32 x 32 tiles up to about 1.07e9 cells).  Returns NULL on error
 * (see swe_last_error). */
swe_t* swe_create(int nx, int ny, double dx, const double* b, const double* n_M,
                  const swe_params* p);

/* Advance one CSPH-TVD step (Sec. 2.3 stages I-IV).  Synchronises the
 * stream.  Returns 0 or SWE_E*. */
int    swe_step(swe_t* s);

/* Advance nsteps steps: device-side time step, no host round trip inside,
 * steps replayed from a captured hipGraph.  Synchronises at the end.  Stops
 * advancing at the first device error and returns it. */
int    swe_run(swe_t* s, long nsteps);

/* As swe_run, but only queues the steps on the stream and returns without
 * waiting (host-side errors only).  Device errors of the queued steps are
 * reported by the next synchronising call (swe_run(s, 0), swe_step, a
 * query).  For callers that overlap host work with the steps, and for
 * timing the steps alone with events on the stream. */
int    swe_enqueue(swe_t* s, long nsteps);

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

/* Source rate field sigma(x, y) [m/s] of the continuity equation (Sec. 2.1,
 * Eq. 1: precipitation > 0; infiltration and evaporation < 0), nx*ny host
 * FP64, row-major, copied; zero on closed gates; NULL removes it.  Each step
 * of length tau adds tau*sigma of depth with no momentum (stage I sources);
 * a loss acts only on cells wet at layer n and takes at most the water
 * there.  Cells with sigma > 0 are sources of the wet-tile rule (their tiles
 * and the tiles facing them are stepped).  The volume the field applied is
 * accumulated in FP64 per tile: swe_field_volume returns it [m^3], so that
 * V_N - V_0 = swe_inflow + swe_field_volume + swe_ledger.  Default tile
 * shapes only; not for grids of a nest, nor together with flux corrections,
 * an attached network or line taps (SWE_EINVAL).  Re-lists the active tiles
 * of the current layer; 0 or SWE_E*. */
int    swe_set_source_field(swe_t* s, const double* sigma);
double swe_field_volume(swe_t* s);

/* Workgroups of one step launch: the resident count of the step kernel
 * (compute units x workgroups per unit), fewer only without dry skipping
 * when the grid has fewer tiles.  The tile list is strided over them, so a
 * step with more listed tiles gives some workgroups several.  Returns the
 * count, or SWE_EINVAL for a NULL handle. */
int    swe_launch_grid(swe_t* s);

/* Set the workgroups of the following step launches to `grid`, from 8 up to
 * the default count swe_launch_grid reports for a new handle.  A list no
 * longer than the grid gives each workgroup one tile or none (first the
 * entry its own XCD appended, then the overflow of longer segments); a
 * longer list is strided over the workgroups.  The results do not depend on
 * the grid: it places the work (tests and measurements of that placement).
 * Waits for queued steps.  0, SWE_EINVAL (NULL handle, grid out of range, a
 * grid of a nest) or SWE_EHIP. */
int    swe_set_launch_grid(swe_t* s, int grid);

/* Tiles the next step will process (row-major tile indices, unordered),
 * at most cap entries; returns the count or SWE_E*. */
int    swe_active_tiles(swe_t* s, int* out, int cap);

/* nsteps steps launched one by one with a HIP event pair around each step
 * kernel on the handle's stream; *kernel_ms receives the summed kernel time
 * [ms].  For measurement. */
int    swe_run_timed(swe_t* s, long nsteps, double* kernel_ms);

/* Flux corrections added to the stage III fluxes (Sec. 2.3) of every later
 * step, before the final update: dE through the east face and dN through the
 * north face of each cell, each 3 planes of nx*ny (mass, x-momentum,
 * y-momentum) row-major, FP64 on the host, copied.  After the Lagrangian
 * stage, the mass part needs the face's upwind cell to be deeper than the
 * correction depth (eps unless set, see below), the momentum part both
 * cells; wall faces take none.  One of them NULL means zeros there; both NULL switch the
 * corrections off.  Default tile shapes only; not for grids of a nest. */
int    swe_set_correction(swe_t* s, const double* dE, const double* dN);

/* Correction depth (default and minimum: eps).  A cell just above eps that
 * takes a momentum correction, or loses water to a mass correction but keeps
 * its momentum, gets a velocity Q/H that can set an arbitrarily small CFL
 * step. */
int    swe_set_correction_depth(swe_t* s, double hmin);

/* Hold the step length at tau > 0 from the next step on (the CFL step is
 * still recorded but not used; the hydrograph volume follows the clock);
 * tau = 0 returns to CFL steps. */
int    swe_hold_dt(swe_t* s, double tau);

/* Line taps (training data for the learned correction): with r > 0 every
 * later step adds tau * flux of the x faces whose column is a multiple of r,
 * per row, and of the y faces whose row is a multiple of r, per column, into
 * tapx [3][ny][nx/r + 1] and tapy [3][ny/r + 1][nx] (planes: mass, normal
 * momentum, tangential momentum; the wall faces at nx and ny stay 0).  nx
 * and ny must be multiples of r; default tile shape; r = 0 switches them
 * off.  swe_zero_line_taps clears them; swe_get_line_taps copies them to the
 * host (either may be NULL). */
int    swe_enable_line_taps(swe_t* s, int r);
int    swe_zero_line_taps(swe_t* s);
int    swe_get_line_taps(swe_t* s, double* tapx, double* tapy);

/* Set the current layer of coarse (both buffers) to the means of r x r
 * cells of fine's current layer, and its clock to fine's; the coarse grid is
 * r times smaller in each direction, same precision. */
int    swe_restrict(swe_t* fine, swe_t* coarse, int r);

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

/* ---- tile-shape autotuner -------------------------------------------------
 * The step kernels are compiled for several tile shapes per precision and
 * limiter (FP32: 32x32, 64x16, 16x16; FP64: 16x16, 32x16).  Every shape
 * rounds every cell identically, so the shape changes the speed and nothing
 * else.  The autotuner builds the grid (or the batch) once per compiled shape
 * of p's precision and limiter from the given inputs and initial state, runs
 * `warmup` steps (graph capture included), times the next `nsteps` with HIP
 * events on its stream, and frees it again.  On return the first
 * min(count, cap) entries of tile_x, tile_y and ms (ms may be NULL) hold the
 * shapes and their times [ms], fastest first; the return value is the count
 * of shapes timed (>= 1) or SWE_E*.  p's own tile_x/tile_y are ignored.
 * Allocates one grid or batch at a time; synchronises. */
int    swe_autotune(int nx, int ny, double dx, const double* b, const double* n_M,
                    const swe_params* p, int warmup, int nsteps, int cap,
                    int* tile_x, int* tile_y, double* ms);
int    swe_batch_autotune(int n, const int* nx, const int* ny, const double* dx,
                          const double* const* b, const double* const* n_M,
                          const swe_params* p, int warmup, int nsteps, int cap,
                          int* tile_x, int* tile_y, double* ms);

/* ------------------------------------------------------------------ nests
 * Hierarchical grids (Sec. 2.2: the small-scale flow of zoomed-in areas fed
 * back into the large-scale grid; Sec. 5: a 50 m grid with a 12.5 m local
 * grid): one coarse grid and patches refined by r over boxes of coarse
 * cells.  Per coarse step the coarse grid steps with tau_c, every patch takes
 * r substeps of tau_c / r inside a frame of SWE_NEST_FRAME fine cells filled
 * from the coarse layers n and n+1 (linear in time; fine depth
 * max(0, H_c + b_c - b_fine) where the coarse cell is wet, else dry, and
 * fine discharge the fine depth times the coarse velocity), and with
 * feedback the covered coarse cells take the mean of their fine cells while
 * the uncovered cells next to a box take the mismatch between the coarse and
 * the summed fine fluxes through their shared face (clamped as in the final
 * update; its momentum part weighted by the cell's depth after it, 0 up to
 * 5 cm, 1 from 10 cm, linear between).  tau_c = min(CFL step of the coarse layer as stepped and
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
 * 1 <= r <= 16 and 1 <= npatch <= 64 patches.  Every box keeps
 * ceil(SWE_NEST_FRAME / r) coarse cells from the domain edge, one uncovered
 * cell from every other box and from the inlet, and holds no closed gate
 * in it or its frame.  The coarse bed under a box should be the mean of the
 * fine bed (it is taken as given).  Patches skip dry tiles when the coarse
 * grid does (p->skip_dry), except the tiles holding their frame, which step
 * every substep.  NULL on error. */
swe_nest_t* swe_nest_create(int nx, int ny, double dx, const double* b, const double* n_M,
                            const swe_params* p, int r, int feedback, int npatch,
                            const swe_patch* patches);

/* Advance n coarse steps (each with its r substeps; hipGraph replay).
 * Synchronises; returns 0 or an SWE_E* code. */
int    swe_nest_run(swe_nest_t* n, long coarse_steps);

/* Hold the coarse step length at tau_c > 0 from the next coarse step on
 * (rounded to the stencil type; substeps tau_c / r; the CFL rule of
 * Sec. 2.3 is still evaluated but not used); tau_c = 0 returns to the CFL
 * rule, from the current layers.  Synchronises; SWE_EINVAL for a negative
 * or non-finite tau_c. */
int    swe_nest_hold_dt(swe_nest_t* n, double tau_c);

/* As swe_nest_run with a HIP event pair around every coarse step (all its
 * launches); the summed time goes to *kernel_ms. */
int    swe_nest_run_timed(swe_nest_t* n, long coarse_steps, double* kernel_ms);

/* Clock [s], volume of the nested solution (FP64 sum of the coarse depths,
 * covered cells holding the fine mean) [m^3], hydrograph volume [m^3], clamp
 * ledger (coarse grid plus feedback) [m^3], completed coarse steps, and the
 * time steps of the next coarse step and substeps [s].  Any may be NULL. */
int    swe_nest_query(swe_nest_t* n, double* t, double* volume, double* inflow, double* ledger,
                      long* steps, double* dt_coarse, double* dt_fine);

/* Processed cell-steps so far: the in-domain cells of the tiles each step
 * processed, of the coarse grid and of all patch substeps (extended patches:
 * listed tiles and the tiles holding the frame).  Either may be NULL. */
int    swe_nest_work(swe_nest_t* n, long long* coarse_cells, long long* fine_cells);

/* Host FP64 copy of the coarse state (nx*ny each) or of patch k's interior
 * ((r*ch) x (r*cw) each); any may be NULL. */
int    swe_nest_get_coarse(swe_nest_t* n, double* H, double* Qx, double* Qy);
int    swe_nest_get_patch(swe_nest_t* n, int k, double* H, double* Qx, double* Qy);

/* Free the nest and its device memory.  NULL-safe. */
void   swe_nest_destroy(swe_nest_t* n);

/* ------------------------------------------------------------------ learned correction
 * A convolutional network (four 3x3 valid convolutions, 6 -> 32 -> 32 -> 32
 * -> 6 channels, tanh after the first three; bf16 weights and activations,
 * FP32 accumulation on MFMA) that maps a crop of (S+9)^2 coarse cells to
 * flux corrections of its central (S+1)^2 cells (an S x S tile and the cell
 * row and column before it): (mass, x-momentum, y-momentum) through the
 * east face, then the north face of each cell.  The
 * corrections are added to the stage III fluxes (Sec. 2.3) of a coarse grid
 * before its final update.  The paper has no learned component; this is an
 * addition, trained on fine runs of this solver.
 *
 * Crops on the host are FP64 (n, S+9, S+9, 6) row-major, channels last:
 * H, Ux, Uy, b, n_M, wet (U = Q/H where H > eps, else 0; wet 0/1), each
 * divided by in_scale[k].  Network outputs (n, S+1, S+1, 6) are in units of
 * out_scale (the correction is output * out_scale[k]).  Parameters are
 * packed per layer as W[out][in][3][3] then b[out], layers in order, FP64 on
 * the host (FP32 on the device). */
typedef struct swe_lc_s swe_lc_t;

/* Number of packed parameters. */
int       swe_lc_nparams(void);

/* Network for tiles of S = tile cells, buffers for up to max_crops crops,
 * zero parameters; stream: hipStream_t or NULL for a private one.  NULL on
 * error. */
swe_lc_t* swe_lc_create(int tile, int max_crops, const double* in_scale, const double* out_scale,
                        void* stream);
void      swe_lc_destroy(swe_lc_t* c);

/* Set (resets the Adam moments) or read the packed parameters. */
int       swe_lc_set_params(swe_lc_t* c, const double* params);
int       swe_lc_get_params(swe_lc_t* c, double* params);

/* Network output of n host crops; out (n, S+1, S+1, 6) may be NULL. */
int       swe_lc_forward(swe_lc_t* c, int n, const double* x, double* out);

/* The same network output through the inference path that runs before each
 * step of a grid with an attached network: all four layers in one launch,
 * activations kept on chip (blocks of 11 x 11 outputs; S + 1 < 11 takes the
 * layer-by-layer path).  Keeps no activations: swe_lc_get_layer needs a
 * swe_lc_forward after it, as after steps of an attached grid.  out
 * (n, S+1, S+1, 6) is required. */
int       swe_lc_infer(swe_lc_t* c, int n, const double* x, double* out);

/* One training step on n host crops with labels y and mask (both
 * (n, S+1, S+1, 6)): loss 1/2 sum mask (out - y)^2 / max(sum mask, 1), its
 * gradient by back-propagation, then one Adam step (beta 0.9, 0.999, eps
 * 1e-8) with learning rate lr (lr = 0: gradient only).  *loss may be NULL. */
int       swe_lc_train_step(swe_lc_t* c, int n, const double* x, const double* y, const double* mask,
                            double lr, double* loss);

/* Packed gradient of the last training step. */
int       swe_lc_get_grads(swe_lc_t* c, double* grads);

/* Stored values of the last forward (test access): which = l in 0..3 gives
 * the bf16 input of layer l, (n, S+9-2l, S+9-2l, real input channels);
 * which = 4 + l the bf16 gradient dL/dz of layer l's output,
 * (n, S+7-2l, S+7-2l, real output channels). */
int       swe_lc_get_layer(swe_lc_t* c, int which, double* out);

/* Attach the network to grid s (same tile size S, max_crops at least the
 * grid's tile count, default tile shape): from then on every step of s first
 * evaluates the network on the crops of s's active tiles, on s's stream, and
 * uses the corrections of those tiles' cells and of the cell row and column
 * before each (so every face of an active tile carries a fresh correction;
 * other faces lie between dry cells and move no water).
 * c = NULL detaches.  The network must outlive the attachment and must not
 * be used on its own stream while s runs. */
int       swe_lc_attach(swe_lc_t* c, swe_t* s);

/* The crops the attached network would read before the next step of s: host
 * FP64 (n, S+9, S+9, 6) into x (room for every tile), their tile indices
 * (row-major tile order) into tiles (may be NULL).  Returns n, or a negative
 * SWE_E* code. */
int       swe_lc_gather(swe_lc_t* c, swe_t* s, double* x, int* tiles);

/* Training data from the solver's own fine runs.  swe_lc_data allocates a
 * device data set of `capacity` crops (emptying it).  swe_lc_collect takes
 * one coarse interval of the fine grid f (line taps r enabled) and the
 * coarse grid g (r times smaller, line taps 1 enabled, tiles of the
 * network's size): g's layer becomes the r x r means of f's, the interval is
 * tau_c = min(g's CFL step, m * f's CFL step); the crops of g's active tiles
 * are added with labels (mean fine flux through each coarse east and north
 * face over the m fine steps of tau_c / m, minus the coarse flux of one step
 * of tau_c from the same layer, divided by out_scale; mask 0 on wall faces
 * and cells outside the grid).  f advances by m steps and returns to CFL
 * steps; *tau_out (may be NULL) gets tau_c.  swe_lc_get_data copies crops
 * [first, first+n) back (any output may be NULL). */
int       swe_lc_data(swe_lc_t* c, int capacity);
int       swe_lc_data_count(swe_lc_t* c);
int       swe_lc_collect(swe_lc_t* c, swe_t* f, swe_t* g, int r, int m, double* tau_out);
int       swe_lc_get_data(swe_lc_t* c, int first, int n, double* x, double* y, double* mask, int* tiles);

/* iters Adam steps (learning rate lr) on minibatches of `batch` distinct
 * crops of the data set drawn with a seeded generator; losses (may be NULL)
 * gets the loss of each step. */
int       swe_lc_fit(swe_lc_t* c, int iters, int batch, double lr, unsigned long long seed, double* losses);

/* New output scales (6 values > 0); the labels already in the data set are
 * re-expressed in them. */
int       swe_lc_set_out_scale(swe_lc_t* c, const double* out_scale);

/* Message of the last error on this host thread ("" if none). */
const char* swe_last_error(void);

/* ------------------------------------------------------------------ step without allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step
 * of swe_step's arithmetic on a layer the caller owns, with no handle.  The
 * step's bookkeeping (control block, completion counters, per-tile volume
 * and clamp partials) lives in a fixed device array of about 300 KB that
 * each GPU the library runs on holds until the process ends; the call makes
 * no hipMalloc, hipFree or other allocation, and no memset (kernels clear
 * what must start at zero, so it can be captured in a graph).
 *
 *   nx, ny, dx   grid; at most SWE_NOALLOC_MAX_TILES tiles of the default
 *                tile shape of the precision (4096 x 4096 in FP32 with
 *                32 x 32 tiles, 2048 x 2048 in FP64 with 16 x 16 tiles);
 *                larger grids are SWE_EINVAL
 *   p            physics, precision, limiter, inlet and hydrograph, stream
 *                as for swe_create; solid, H0, Qx0, Qy0 and skip_dry are
 *                not used (every tile is stepped, so every output cell is
 *                written); tile_x, tile_y must be 0 or the default shape
 *   b, cf        device arrays of the stencil type (float for precision 32,
 *                double for 64), nx*ny row-major: bed (closed gates already
 *                raised above any level) and c_f = g n_M^2
 *   H, Qx, Qy    device layer n (depth >= 0; discharges 0 on dry cells)
 *   H1, Qx1, Qy1 device layer n+1, written; must not alias the inputs
 *   t            time of layer n [s] (the hydrograph's clock)
 *   out          optional device array of 5 doubles, written: t_{n+1}, the
 *                step length (the CFL step of layer n, Sec. 2.3), the
 *                hydrograph volume of the step, the clamped volume, and the
 *                device error code (0, SWE_ENONFINITE or SWE_EDTCOLLAPSE)
 *
 * Work is queued on p->stream and not waited for.  Every call on one GPU
 * shares that GPU's array and leaves the last call's contents in it: calls
 * that overlap on one GPU (other streams, other host threads) race and are
 * not allowed.  Returns 0 or SWE_EINVAL / SWE_EHIP (host-side checks). */
#define SWE_NOALLOC_MAX_TILES 16384
int    swe_step_noalloc(int nx, int ny, double dx, const swe_params* p, const void* b, const void* cf,
                        const void* H, const void* Qx, const void* Qy, void* H1, void* Qx1, void* Qy1,
                        double t, double* out);

#ifdef __cplusplus
}
#endif
#endif
