// swe_api.hip -- host side of libswe_hip.so: the C ABI declared in swe.h.
//
// The host validates arguments, owns the device buffers of a handle, and
// launches the step kernel (one launch per CSPH-TVD step, arXiv 1705.00614
// Sec. 2.3) on the caller's stream, replaying captured hipGraphs for long
// runs.  No arithmetic of the scheme runs on the host.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/swe.h"
#include "swe_step.hpp"

using swe::Args;
using swe::Ctrl;

namespace {

thread_local std::string g_err;

void set_err(const char* msg) { g_err = msg; }

void set_hip_err(const char* where, hipError_t e) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    g_err = buf;
}

#define HIPCHK(expr)                                                            \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            set_hip_err(#expr, e_);                                             \
            return SWE_EHIP;                                                    \
        }                                                                       \
    } while (0)

constexpr int GRAPH_STEPS = 32;   // steps per captured graph (even)

struct Launcher {
    int tx, ty, nt, precision, limiter;
    // step kernels; the optional events are stamped by the dispatch itself
    // (start and end of this kernel only)
    hipError_t (*step)(const void* args, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
    hipError_t (*step_tap)(const void* args, int grid, hipStream_t st, hipEvent_t e0,
                           hipEvent_t e1);   // nested grids; may be null
    hipError_t (*step_corr)(const void* args, int grid, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1);  // learned flux corrections; may be null
    hipError_t (*step_field)(const void* args, int grid, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1); // source rate field; may be null
    hipError_t (*step_disp)(const void* args, int grid, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1);  // displaced-particle corrector; may be null
    hipError_t (*step_per)(const void* args, int grid, hipStream_t st, hipEvent_t e0,
                           hipEvent_t e1);   // periodic domain; may be null
    hipError_t (*batch_step)(const void* bargs, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
    hipError_t (*batch_prepare_finish)(const void* bargs, hipStream_t st);
    hipError_t (*prepare)(const void* args, int grid, hipStream_t st);
    hipError_t (*prepare_finish)(const void* args, hipStream_t st);
    int (*occupancy)(int* blocks);
};

template <typename real, int TX, int TY, int NT, int LIM, int MODE>
hipError_t launch_step(const void* args, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const Args<real>& a = *static_cast<const Args<real>*>(args);
    hipExtLaunchKernelGGL((swe::k_step<real, TX, TY, NT, LIM, MODE>), dim3(grid), dim3(NT), 0, st, e0, e1, 0, a);
    return hipGetLastError();
}
template <typename real, int TX, int TY, int NT, int LIM>
hipError_t launch_batch_step(const void* bargs, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const swe::BatchArgs<real>& b = *static_cast<const swe::BatchArgs<real>*>(bargs);
    hipExtLaunchKernelGGL((swe::k_batch_step<real, TX, TY, NT, LIM>), dim3(grid), dim3(NT), 0, st, e0, e1, 0, b);
    return hipGetLastError();
}
template <typename real>
hipError_t launch_batch_prepare_finish(const void* bargs, hipStream_t st) {
    const swe::BatchArgs<real>& b = *static_cast<const swe::BatchArgs<real>*>(bargs);
    hipLaunchKernelGGL((swe::k_batch_prepare_finish<real>), dim3(1), dim3(256), 0, st, b);
    return hipGetLastError();
}
template <typename real, int TX, int TY, int NT>
hipError_t launch_prepare(const void* args, int grid, hipStream_t st) {
    const Args<real>& a = *static_cast<const Args<real>*>(args);
    hipLaunchKernelGGL((swe::k_prepare<real, TX, TY, NT>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
template <typename real>
hipError_t launch_prepare_finish(const void* args, hipStream_t st) {
    const Args<real>& a = *static_cast<const Args<real>*>(args);
    hipLaunchKernelGGL((swe::k_prepare_finish<real>), dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}
template <typename real, int TX, int TY, int NT, int LIM>
int occupancy(int* blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, swe::k_step<real, TX, TY, NT, LIM, swe::MODE_PLAIN>, NT, 0) ==
                   hipSuccess ? 0 : -1;
}

#define TAP_STEP(real, TX, TY, NT, LIM) launch_step<real, TX, TY, NT, LIM, swe::MODE_TAP>, \
                                        launch_step<real, TX, TY, NT, LIM, swe::MODE_CORR>, \
                                        launch_step<real, TX, TY, NT, LIM, swe::MODE_FIELD>, \
                                        launch_step<real, TX, TY, NT, LIM, swe::MODE_DISP>, \
                                        launch_step<real, TX, TY, NT, LIM, swe::MODE_PERIODIC>
#define NO_TAP_STEP(real, TX, TY, NT, LIM) nullptr, nullptr, nullptr, nullptr, nullptr
#define LAUNCHER(real, TX, TY, NT, P, LIM, TAPS)                                                 \
    Launcher{TX, TY, NT, P, LIM, launch_step<real, TX, TY, NT, LIM, swe::MODE_PLAIN>,             \
             TAPS(real, TX, TY, NT, LIM),                                                        \
             launch_batch_step<real, TX, TY, NT, LIM>, launch_batch_prepare_finish<real>,         \
             launch_prepare<real, TX, TY, NT>, launch_prepare_finish<real>,                      \
             occupancy<real, TX, TY, NT, LIM>}
#define LAUNCHERS(real, TX, TY, NT, P, TAPS)                                       \
    LAUNCHER(real, TX, TY, NT, P, 0, TAPS), LAUNCHER(real, TX, TY, NT, P, 1, TAPS), \
        LAUNCHER(real, TX, TY, NT, P, 2, TAPS)

// Tile shapes compiled in, each with the three limiters; the first shape of
// each precision is its default and the one nested grids use.
// 512 threads per 32 x 32 tile: two workgroups per CU (LDS-bound), four
// waves per SIMD within 128 VGPRs (short runs, no spills), and one pass of
// the workgroup per stage, which halves the latency of a tile; that latency
// sets the step time when few tiles are wet.
#ifndef SWE_F32_THREADS
#define SWE_F32_THREADS 512
#endif
const Launcher kLaunchers[] = {
    LAUNCHERS(float, 32, 32, SWE_F32_THREADS, 32, TAP_STEP),
    LAUNCHERS(float, 64, 16, 512, 32, NO_TAP_STEP),
    LAUNCHERS(float, 16, 16, 256, 32, NO_TAP_STEP),
    LAUNCHERS(double, 16, 16, 256, 64, TAP_STEP),
    LAUNCHERS(double, 32, 16, 256, 64, NO_TAP_STEP),
};

const Launcher* find_launcher(int precision, int tx, int ty, int limiter) {
    for (const Launcher& l : kLaunchers) {
        if (l.precision != precision || l.limiter != limiter) continue;
        if ((tx == 0 && ty == 0) || (l.tx == tx && l.ty == ty)) return &l;
    }
    return nullptr;
}

}  // namespace

struct swe_s {
    int nx = 0, ny = 0, precision = 32, rsize = 4;
    int ntx = 0, nty = 0, ntiles = 0, grid = 0, grid_max = 0;   // step launch grid, its default
    double h = 0.0;
    swe_params p{};
    const Launcher* L = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* Hb[2] = {nullptr, nullptr};
    void* Qxb[2] = {nullptr, nullptr};
    void* Qyb[2] = {nullptr, nullptr};
    void* bed = nullptr;
    void* cf = nullptr;
    Ctrl* ctrl = nullptr;
    int* hot = nullptr;         // completion and list counters (one per 256-byte line)
    int* lists = nullptr;       // [2 slots][NSEG segments][ntiles]
    int* stamp = nullptr;
    void* wg_speed = nullptr;   // per-workgroup maximum speed
    long long* wg_cells = nullptr;
    double* mass = nullptr;
    double* ledger = nullptr;
    double* scalar = nullptr;   // device scratch for reductions
    long long launched = 0;     // steps launched since creation
    int nin = 0;
    hipGraphExec_t graph = nullptr;
    std::vector<unsigned char> args[2];   // kernel arguments per parity
    std::vector<uint8_t> solid;           // closed gates (host copy)
    // member of a nest: the nest sets the time steps; flux taps
    int hold = 0, ntap = 0;
    const int* tap_rect = nullptr;
    void* tap = nullptr;
    // learned flux corrections (east and north faces, 3 planes each)
    void* corrE = nullptr;
    void* corrN = nullptr;
    int* claims = nullptr;      // unit claims of an attached network's pre-step, one per step parity
    bool corr = false;
    double corr_hmin = 0.0;
    // line taps (training labels): coarsening factor and buffers
    int tap_r = 0;
    void* tapx = nullptr;
    void* tapy = nullptr;
    // attached network: launched before every step to fill the corrections
    struct swe_lc_s* lc = nullptr;
    hipError_t (*pre_step)(swe_t* s, int par) = nullptr;
    // tiles stepped every step (patches of a nest), device array, and bounds
    const int* ring_tiles = nullptr;
    int nring = 0;
    int ring_b[4] = {-1, 1 << 30, -1, 1 << 30};
    // source rate field (stencil type), per-tile K1 source bits, per-tile
    // applied field volume (kept when the field is removed)
    void* sigma = nullptr;
    unsigned char* fmask = nullptr;
    double* fvol = nullptr;
    bool field = false;
};

namespace {

template <typename real>
void fill_args(swe_t* s, int parity, Args<real>* a) {
    std::memset(a, 0, sizeof *a);
    const swe_params& p = s->p;
    a->Hi = (const real*)s->Hb[parity];
    a->Qxi = (const real*)s->Qxb[parity];
    a->Qyi = (const real*)s->Qyb[parity];
    a->Ho = (real*)s->Hb[parity ^ 1];
    a->Qxo = (real*)s->Qxb[parity ^ 1];
    a->Qyo = (real*)s->Qyb[parity ^ 1];
    a->bed = (const real*)s->bed;
    a->cf = (const real*)s->cf;
    a->ctrl = s->ctrl;
    a->lctrl = s->ctrl;
    a->sid = 0;
    a->tile_base = 0;
    a->list_cap = s->ntiles;
    a->hot = s->hot;
    a->lists = s->lists;
    a->slot = parity;
    a->stamp = s->stamp;
    a->wg_speed = (real*)s->wg_speed;
    a->wg_cells = s->wg_cells;
    a->mass = s->mass;
    a->ledger = s->ledger;
    a->nx = s->nx; a->ny = s->ny; a->ntx = s->ntx; a->nty = s->nty; a->ntiles = s->ntiles;
    a->skip = p.skip_dry ? 1 : 0;
    a->limiter = p.limiter;
    a->periodic = p.periodic ? 1 : 0;
    if (s->nin > 0) {
        a->i0 = p.inlet_i0; a->j0 = p.inlet_j0; a->ni = p.inlet_ni; a->nj = p.inlet_nj;
    }
    a->h = (real)s->h;
    a->ih = (real)(1.0 / s->h);
    a->g = (real)p.g;
    a->eps = (real)p.eps;
    a->nuh2 = (real)(p.nu / (s->h * s->h));
    a->fcor = (real)p.f_coriolis;
    a->wx = (real)p.wind_x;
    a->wy = (real)p.wind_y;
    a->kw = (real)p.wind_kappa;
    a->hw = (real)p.h_wind;
    a->h_d = s->h; a->g_d = p.g; a->cfl = p.cfl; a->tau_max = p.dt_max; a->tau_min = p.dt_min;
    a->nu_d = p.nu;
    a->nin_h2 = s->nin > 0 ? (double)s->nin * s->h * s->h : 0.0;
    a->q_base = p.q_base; a->q_peak = p.q_peak; a->t_peak = p.t_peak; a->sigma_t = p.sigma_t;
    a->hold = s->hold;
    a->ntap = s->ntap;
    a->tap_rect = s->tap_rect;
    a->tap = (real*)s->tap;
    a->corrE = (const real*)s->corrE;
    a->corrN = (const real*)s->corrN;
    a->corr_hmin = (real)(s->corr_hmin > p.eps ? s->corr_hmin : p.eps);
    a->tap_r = s->tap_r;
    a->tapx = (real*)s->tapx;
    a->tapy = (real*)s->tapy;
    a->ring_tiles = s->ring_tiles;
    a->nring = s->nring;
    a->ring_x0 = s->ring_b[0]; a->ring_x1 = s->ring_b[1]; a->ring_y0 = s->ring_b[2]; a->ring_y1 = s->ring_b[3];
    if (s->field) {
        a->sigma = (const real*)s->sigma;
        a->fmask = s->fmask;
        a->fvol = s->fvol;
    }
}

// Step kernel of a grid: the tapping variant for members of a nest.
hipError_t launch_grid_step(swe_t* s, int par, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                            hipStream_t on = nullptr) {
    if (s->pre_step) {
        const hipError_t e = s->pre_step(s, par);
        if (e != hipSuccess) return e;
    }
    auto f = (s->ntap > 0 || s->tap_r > 0) ? s->L->step_tap
             : s->corr                       ? s->L->step_corr
             : s->field                      ? s->L->step_field
             : s->p.sph_displaced            ? s->L->step_disp
             : s->p.periodic                 ? s->L->step_per
                                             : s->L->step;
    return f(s->args[par].data(), s->grid, on ? on : s->stream, e0, e1);
}

void build_args(swe_t* s) {
    for (int par = 0; par < 2; ++par) {
        if (s->precision == 32) {
            s->args[par].resize(sizeof(Args<float>));
            fill_args<float>(s, par, (Args<float>*)s->args[par].data());
        } else {
            s->args[par].resize(sizeof(Args<double>));
            fill_args<double>(s, par, (Args<double>*)s->args[par].data());
        }
    }
}

int sync_ctrl(swe_t* s, Ctrl* out) {
    HIPCHK(hipMemcpyAsync(out, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return 0;
}

// Upload a host FP64 field as the stencil type.
int upload(swe_t* s, void* dst, const double* src, double fill) {
    const size_t n = (size_t)s->nx * s->ny;
    std::vector<unsigned char> buf(n * s->rsize);
    if (s->precision == 32) {
        float* f = (float*)buf.data();
        for (size_t i = 0; i < n; ++i) f[i] = (float)(src ? src[i] : fill);
    } else {
        double* d = (double*)buf.data();
        for (size_t i = 0; i < n; ++i) d[i] = src ? src[i] : fill;
    }
    HIPCHK(hipMemcpyAsync(dst, buf.data(), n * s->rsize, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return 0;
}

// Recompute the layer bookkeeping of the current buffer pair: wet tiles,
// next time step, volume partials.
int prepare(swe_t* s) {
    const int par = (int)(s->launched & 1);
    HIPCHK(hipMemsetAsync(s->stamp, 0, sizeof(int) * s->ntiles, s->stream));
    HIPCHK(hipMemsetAsync(s->hot, 0, sizeof(int) * swe::HOT_INTS, s->stream));
    char* cb = (char*)s->ctrl;
    HIPCHK(hipMemsetAsync(cb + offsetof(Ctrl, prep_speed), 0, sizeof(unsigned long long), s->stream));
    // k_prepare appends to the list slot `par` and reads the buffer pair `par`
    HIPCHK(s->L->prepare(s->args[par].data(), s->ntiles, s->stream));
    HIPCHK(s->L->prepare_finish(s->args[par].data(), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return 0;
}

int set_state_impl(swe_t* s, const double* H, const double* Qx, const double* Qy,
                   const uint8_t* solid) {
    const size_t n = (size_t)s->nx * s->ny;
    std::vector<double> h(n), qx(n), qy(n);
    for (size_t i = 0; i < n; ++i) {
        double hh = H ? H[i] : 0.0, a = Qx ? Qx[i] : 0.0, b = Qy ? Qy[i] : 0.0;
        if (!std::isfinite(hh) || !std::isfinite(a) || !std::isfinite(b) || hh < 0.0) {
            set_err("state: depth must be finite and >= 0, discharges finite");
            return SWE_EINVAL;
        }
        if (solid && solid[i]) hh = a = b = 0.0;
        if (!(hh > s->p.eps)) a = b = 0.0;   // dry cells are at rest
        h[i] = hh; qx[i] = a; qy[i] = b;
    }
    const int par = (int)(s->launched & 1);
    int rc;
    if ((rc = upload(s, s->Hb[par], h.data(), 0.0))) return rc;
    if ((rc = upload(s, s->Qxb[par], qx.data(), 0.0))) return rc;
    if ((rc = upload(s, s->Qyb[par], qy.data(), 0.0))) return rc;
    // the other buffer of the pair must hold the same layer for skipped tiles
    if ((rc = upload(s, s->Hb[par ^ 1], h.data(), 0.0))) return rc;
    if ((rc = upload(s, s->Qxb[par ^ 1], qx.data(), 0.0))) return rc;
    if ((rc = upload(s, s->Qyb[par ^ 1], qy.data(), 0.0))) return rc;
    return prepare(s);
}

void free_all(swe_t* s) {
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    void* ptrs[] = {s->Hb[0], s->Hb[1], s->Qxb[0], s->Qxb[1], s->Qyb[0], s->Qyb[1], s->bed, s->cf,
                    s->ctrl, s->hot, s->lists, s->stamp, s->wg_speed, s->wg_cells, s->mass, s->ledger,
                    s->scalar, s->corrE, s->corrN, s->claims, s->tapx, s->tapy, s->sigma, s->fmask, s->fvol};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

int launch_steps(swe_t* s, long n) {
    for (long k = 0; k < n; ++k) {
        const int par = (int)(s->launched & 1);
        HIPCHK(launch_grid_step(s, par));
        s->launched++;
    }
    return 0;
}

// The captured graph holds the kernel of the current mode; a mode change
// drops it.
void drop_graph(swe_t* s) {
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
}

int ensure_graph(swe_t* s) {
    if (s->graph) return 0;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_STEPS; ++k) {
        hipError_t e = launch_grid_step(s, k & 1);
        if (e != hipSuccess) {
            (void)hipStreamEndCapture(s->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            set_hip_err("graph capture", e);
            return SWE_EHIP;
        }
    }
    HIPCHK(hipStreamEndCapture(s->stream, &g));
    hipError_t e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph = nullptr;
        set_hip_err("graph instantiation", e);
        return SWE_EHIP;
    }
    return 0;
}

// Launch n steps, each given an event pair to stamp (launch_one(e0, e1));
// *ms gets the summed durations.  Up to POOL pairs are recorded before the stream is drained, so a
// run of that many steps has no host synchronisation inside it.
template <typename F>
int timed_launches(hipStream_t st, long n, double* ms, F&& launch_one) {
    constexpr long POOL = 16384;
    const long m = n < POOL ? n : POOL;
    std::vector<hipEvent_t> ev(2 * (size_t)m);
    int rc = 0;
    size_t made = 0;
    for (; made < ev.size(); ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) { set_err("timed run: hipEventCreate failed"); rc = SWE_EHIP; break; }
    double total = 0.0;
    long left = n;
    while (rc == 0 && left > 0) {
        const long c = left < m ? left : m;
        for (long k = 0; k < c && rc == 0; ++k) {
            const hipError_t e = launch_one(ev[2 * k], ev[2 * k + 1]);
            if (e != hipSuccess) { set_hip_err("timed run", e); rc = SWE_EHIP; }
        }
        if (rc == 0 && hipStreamSynchronize(st) != hipSuccess) { set_err("timed run: sync failed"); rc = SWE_EHIP; }
        for (long k = 0; k < c && rc == 0; ++k) {
            float f = 0.f;
            if (hipEventElapsedTime(&f, ev[2 * k], ev[2 * k + 1]) != hipSuccess) {
                set_err("timed run: event timing failed"); rc = SWE_EHIP;
            }
            total += f;
        }
        left -= c;
    }
    for (size_t k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
    *ms = total;
    return rc;
}

template <typename real>
hipError_t fill_dev(void* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(swe::k_fill<real>, dim3(1024), dim3(256), 0, st, (real*)p, (long)n, real(0));
    return hipGetLastError();
}

// Next step's length (tau <= 0: the layer's CFL step) and hydrograph
// scalars, on the device; the tile list is kept.
int set_dt_now(swe_t* s, double tau) {
    const int par = (int)(s->launched & 1);
    if (s->precision == 32)
        hipLaunchKernelGGL(swe::k_set_dt<float>, dim3(1), dim3(64), 0, s->stream, *(const Args<float>*)s->args[par].data(),
                           tau);
    else
        hipLaunchKernelGGL(swe::k_set_dt<double>, dim3(1), dim3(64), 0, s->stream,
                           *(const Args<double>*)s->args[par].data(), tau);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return 0;
}

int grid_for_cells(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

int finish(swe_t* s) {
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    if (c.err_gate || c.err) {
        const int e = c.err_gate ? c.err_gate : c.err;
        set_err(e == SWE_ENONFINITE ? "state became non-finite" : "time step collapsed below dt_min");
        return e;
    }
    return 0;
}

// Settings of a grid that is a member of a nest.
struct GridExtra {
    int hold, ntap;
    const int* tap_rect;
    void* tap;
    // tiles stepped every step (device array) and their bounds
    const int* ring_tiles;
    int nring, ring_x0, ring_x1, ring_y0, ring_y1;
};

}  // namespace

extern "C" {

const char* swe_last_error(void) { return g_err.c_str(); }

static swe_t* create_grid(int nx, int ny, double dx, const double* b, const double* n_M, const swe_params* p,
                          const GridExtra* ex) {
    g_err.clear();
    if (!p || !b) { set_err("swe_create: b and params are required"); return nullptr; }
    if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 31) - 1) {
        set_err("swe_create: grid must have 1 <= nx*ny < 2^31 cells"); return nullptr;
    }
    if (!(dx > 0.0) || !std::isfinite(dx)) { set_err("swe_create: dx must be > 0"); return nullptr; }
    if (p->precision != 32 && p->precision != 64) { set_err("swe_create: precision must be 32 or 64"); return nullptr; }
    if (!(p->g > 0.0) || !(p->cfl > 0.0) || !(p->cfl < 1.0) || !(p->eps > 0.0) || p->nu < 0.0 ||
        p->limiter < 0 || p->limiter > 2 || !(p->h_wind > 0.0) || !std::isfinite(p->dt_min) ||
        !std::isfinite(p->dt_max)) {
        set_err("swe_create: invalid physical or numerical parameter"); return nullptr;
    }
    const Launcher* L = find_launcher(p->precision, p->tile_x, p->tile_y, p->limiter);
    if (!L) { set_err("swe_create: tile shape not available for this precision"); return nullptr; }
    if (p->sph_displaced && (!L->step_disp || ex)) {
        set_err("swe_create: the displaced-particle corrector needs a single grid with the default tile shape");
        return nullptr;
    }
    if (p->periodic && (!L->step_per || ex || p->sph_displaced || p->solid || nx % L->tx || ny % L->ty)) {
        set_err("swe_create: a periodic domain needs a single grid with the default tile shape, nx and ny "
                "multiples of it, no solid cells and the lattice corrector");
        return nullptr;
    }
    // a tile-list entry holds the tile index in TILE_BITS bits
    if ((long long)((nx + L->tx - 1) / L->tx) * ((ny + L->ty - 1) / L->ty) >= (1LL << swe::TILE_BITS)) {
        set_err("swe_create: grid has too many tiles for the tile list (at most 2^20 - 1)"); return nullptr;
    }
    const size_t n = (size_t)nx * ny;
    for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(b[i]) || (n_M && (!std::isfinite(n_M[i]) || n_M[i] < 0.0))) {
            set_err("swe_create: bed must be finite and Manning n finite and >= 0"); return nullptr;
        }
    }
    int nin = 0;
    if (p->inlet_ni > 0 && p->inlet_nj > 0) {
        if (p->inlet_i0 < 0 || p->inlet_j0 < 0 || p->inlet_i0 + p->inlet_ni > nx || p->inlet_j0 + p->inlet_nj > ny) {
            set_err("swe_create: inlet rectangle outside the grid"); return nullptr;
        }
        for (int j = p->inlet_j0; j < p->inlet_j0 + p->inlet_nj; ++j)
            for (int i = p->inlet_i0; i < p->inlet_i0 + p->inlet_ni; ++i)
                if (p->solid && p->solid[(size_t)j * nx + i]) {
                    set_err("swe_create: the inlet contains a closed gate"); return nullptr;
                }
        nin = p->inlet_ni * p->inlet_nj;
    }

    swe_t* s = new (std::nothrow) swe_s();
    if (!s) { set_err("swe_create: out of host memory"); return nullptr; }
    s->nx = nx; s->ny = ny; s->h = dx; s->p = *p; s->L = L;
    s->precision = p->precision; s->rsize = p->precision == 32 ? 4 : 8;
    s->p.solid = nullptr; s->p.H0 = s->p.Qx0 = s->p.Qy0 = nullptr;
    s->nin = nin;
    if (ex) {
        s->hold = ex->hold;
        s->ntap = ex->ntap;
        s->tap_rect = ex->tap_rect;
        s->tap = ex->tap;
        s->ring_tiles = ex->ring_tiles;
        s->nring = ex->nring;
        s->ring_b[0] = ex->ring_x0; s->ring_b[1] = ex->ring_x1; s->ring_b[2] = ex->ring_y0; s->ring_b[3] = ex->ring_y1;
        if (s->ntap > 0 && !L->step_tap) {
            set_err("nest: the tile shape has no tapping step kernel"); delete s; return nullptr;
        }
        if (s->nring > 0 && s->ntap <= 0) {   // only the tapping step kernel steps ring tiles
            set_err("nest: a grid with ring tiles must tap its faces"); delete s; return nullptr;
        }
    }
    if (p->solid) s->solid.assign(p->solid, p->solid + (size_t)nx * ny);
    s->ntx = (nx + L->tx - 1) / L->tx;
    s->nty = (ny + L->ty - 1) / L->ty;
    s->ntiles = s->ntx * s->nty;

#define CK(expr)                                                                   \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_hip_err("swe_create", e_);                                         \
            free_all(s); delete s; return nullptr;                                 \
        }                                                                          \
    } while (0)

    if (p->stream) {
        s->stream = (hipStream_t)p->stream;
    } else {
        CK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    const size_t bytes = n * s->rsize;
    for (int k = 0; k < 2; ++k) {
        CK(hipMalloc(&s->Hb[k], bytes));
        CK(hipMalloc(&s->Qxb[k], bytes));
        CK(hipMalloc(&s->Qyb[k], bytes));
    }
    CK(hipMalloc((void**)&s->lists, sizeof(int) * 2 * swe::NSEG * (size_t)s->ntiles));
    CK(hipMalloc((void**)&s->hot, sizeof(int) * swe::HOT_INTS));
    CK(hipMalloc(&s->bed, bytes));
    CK(hipMalloc(&s->cf, bytes));
    CK(hipMalloc((void**)&s->ctrl, sizeof(Ctrl)));
    CK(hipMalloc((void**)&s->stamp, sizeof(int) * s->ntiles));
    CK(hipMalloc((void**)&s->mass, sizeof(double) * s->ntiles));
    CK(hipMalloc((void**)&s->ledger, sizeof(double) * s->ntiles));
    CK(hipMalloc((void**)&s->scalar, sizeof(double) * 4));
    CK(hipMemsetAsync(s->ctrl, 0, sizeof(Ctrl), s->stream));
    CK(hipMemsetAsync(s->ledger, 0, sizeof(double) * s->ntiles, s->stream));

    // static fields: bed (closed gates raised far above any level), c_f = g n_M^2
    {
        std::vector<double> bb(b, b + n), cf(n, 0.0);
        for (size_t i = 0; i < n; ++i) {
            if (p->solid && p->solid[i]) bb[i] = swe::GATE_BED;
            else if (n_M) cf[i] = p->g * n_M[i] * n_M[i];
        }
        if (upload(s, s->bed, bb.data(), 0.0) || upload(s, s->cf, cf.data(), 0.0)) {
            free_all(s); delete s; return nullptr;
        }
    }

    // grid of the step kernel: enough resident workgroups to fill the chip
    int dev = 0, cus = 0, occ = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (L->occupancy(&occ) != 0 || occ < 1) occ = 1;
    s->grid = cus * occ;
    if (s->grid < 8) s->grid = 8;
    if (!p->skip_dry && s->grid > s->ntiles) s->grid = s->ntiles;
    s->grid_max = s->grid;
    CK(hipMalloc(&s->wg_speed, sizeof(double) * s->grid));
    CK(hipMalloc((void**)&s->wg_cells, sizeof(long long) * s->grid));

    build_args(s);
    if (set_state_impl(s, p->H0, p->Qx0, p->Qy0, p->solid) != 0) {
        free_all(s); delete s; return nullptr;
    }
    return s;
#undef CK
}

swe_t* swe_create(int nx, int ny, double dx, const double* b, const double* n_M, const swe_params* p) {
    return create_grid(nx, ny, dx, b, n_M, p, nullptr);
}

void swe_destroy(swe_t* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
}

int swe_step(swe_t* s) {
    if (!s) { set_err("swe_step: NULL handle"); return SWE_EINVAL; }
    int rc = launch_steps(s, 1);
    if (rc) return rc;
    return finish(s);
}

// Queue nsteps steps (graph replays of GRAPH_STEPS steps, single launches
// for the rest) without waiting for them.
static int enqueue_steps(swe_t* s, long nsteps) {
    long left = nsteps;
    int rc;
    if (left > 0 && (s->launched & 1)) {
        if ((rc = launch_steps(s, 1))) return rc;
        --left;
    }
    if (left >= GRAPH_STEPS) {
        if ((rc = ensure_graph(s))) return rc;
        while (left >= GRAPH_STEPS) {
            HIPCHK(hipGraphLaunch(s->graph, s->stream));
            s->launched += GRAPH_STEPS;
            left -= GRAPH_STEPS;
        }
    }
    return launch_steps(s, left);
}

int swe_run(swe_t* s, long nsteps) {
    if (!s || nsteps < 0) { set_err("swe_run: invalid arguments"); return SWE_EINVAL; }
    const int rc = enqueue_steps(s, nsteps);
    return rc ? rc : finish(s);
}

int swe_enqueue(swe_t* s, long nsteps) {
    if (!s || nsteps < 0) { set_err("swe_enqueue: invalid arguments"); return SWE_EINVAL; }
    return enqueue_steps(s, nsteps);
}

int swe_run_timed(swe_t* s, long nsteps, double* kernel_ms) {
    if (!s || nsteps < 0 || !kernel_ms) { set_err("swe_run_timed: invalid arguments"); return SWE_EINVAL; }
    int rc = timed_launches(s->stream, nsteps, kernel_ms, [&](hipEvent_t e0, hipEvent_t e1) {
        const int par = (int)(s->launched & 1);
        const hipError_t e = launch_grid_step(s, par, e0, e1);
        s->launched++;
        return e;
    });
    if (rc) return rc;
    return finish(s);
}

int swe_get_state(swe_t* s, double* H, double* Qx, double* Qy) {
    if (!s) { set_err("swe_get_state: NULL handle"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    // step k reads buffer k&1 and writes buffer (k+1)&1, so after c.step
    // completed steps the current layer is in buffer c.step&1
    const int par = (int)(c.step & 1);
    const size_t n = (size_t)s->nx * s->ny;
    std::vector<unsigned char> buf(n * s->rsize);
    double* outs[3] = {H, Qx, Qy};
    void* srcs[3] = {s->Hb[par], s->Qxb[par], s->Qyb[par]};
    for (int k = 0; k < 3; ++k) {
        if (!outs[k]) continue;
        HIPCHK(hipMemcpyAsync(buf.data(), srcs[k], n * s->rsize, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (s->precision == 32) {
            const float* f = (const float*)buf.data();
            for (size_t i = 0; i < n; ++i) outs[k][i] = f[i];
        } else {
            std::memcpy(outs[k], buf.data(), n * sizeof(double));
        }
    }
    return 0;
}

int swe_set_state(swe_t* s, const double* H, const double* Qx, const double* Qy) {
    if (!s || !H) { set_err("swe_set_state: NULL argument"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    // continue from the device's completed-step parity
    s->launched = c.step;
    // closed gates keep their raised bed; their depth must be zero
    return set_state_impl(s, H, Qx, Qy, s->solid.empty() ? nullptr : s->solid.data());
}

int swe_set_time(swe_t* s, double t) {
    if (!s || !std::isfinite(t)) { set_err("swe_set_time: invalid arguments"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    char* cb = (char*)s->ctrl;
    HIPCHK(hipMemcpyAsync(cb + offsetof(Ctrl, t), &t, sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    // the next source volume depends on the clock; the step length and the
    // tile lists stay
    s->launched = c.step;
    return set_dt_now(s, s->hold ? c.tau : 0.0);
}

double swe_mass(swe_t* s) {
    if (!s) return NAN;
    hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, s->stream, s->mass, s->ntiles, s->scalar);
    double v = NAN;
    if (hipMemcpyAsync(&v, s->scalar, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return NAN;
    return v * s->h * s->h;
}

static double ctrl_field(swe_t* s, int which) {
    if (!s) return NAN;
    Ctrl c;
    if (sync_ctrl(s, &c)) return NAN;
    switch (which) {
        case 0: return c.t;
        case 1: return c.last_tau;
        case 2: return c.tau;
        case 3: return c.inflow;
        default: return NAN;
    }
}

double swe_time(swe_t* s) { return ctrl_field(s, 0); }
double swe_last_dt(swe_t* s) { return ctrl_field(s, 1); }
double swe_next_dt(swe_t* s) { return ctrl_field(s, 2); }
double swe_inflow(swe_t* s) { return ctrl_field(s, 3); }

double swe_ledger(swe_t* s) {
    if (!s) return NAN;
    hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, s->stream, s->ledger, s->ntiles, s->scalar);
    double v = NAN;
    if (hipMemcpyAsync(&v, s->scalar, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return NAN;
    return v;
}

long swe_steps(swe_t* s) {
    if (!s) return -1;
    Ctrl c;
    if (sync_ctrl(s, &c)) return -1;
    return (long)c.step;
}

int swe_work(swe_t* s, long long* tile_steps, long long* cell_steps, int* ntiles, int* tile_x, int* tile_y) {
    if (!s) { set_err("swe_work: NULL handle"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    if (tile_steps) *tile_steps = c.tiles;
    if (cell_steps) *cell_steps = c.cells;
    if (ntiles) *ntiles = s->ntiles;
    if (tile_x) *tile_x = s->L->tx;
    if (tile_y) *tile_y = s->L->ty;
    return 0;
}

int swe_set_source_field(swe_t* s, const double* sigma) {
    if (!s) { set_err("swe_set_source_field: NULL handle"); return SWE_EINVAL; }
    if (s->ntap > 0) { set_err("swe_set_source_field: not for grids of a nest"); return SWE_EINVAL; }
    if (sigma && !s->L->step_field) {
        set_err("swe_set_source_field: the tile shape has no field step kernel (default shapes only)");
        return SWE_EINVAL;
    }
    if (sigma && (s->corr || s->lc || s->tap_r > 0 || s->p.sph_displaced || s->p.periodic)) {
        set_err("swe_set_source_field: not with flux corrections, an attached network, line taps, the "
                "displaced-particle corrector or a periodic domain");
        return SWE_EINVAL;
    }
    const size_t n = (size_t)s->nx * s->ny;
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    s->launched = c.step;
    if (!sigma) {
        s->field = false;
    } else {
        std::vector<double> sg(sigma, sigma + n);
        for (size_t i = 0; i < n; ++i) {
            if (!std::isfinite(sg[i])) { set_err("swe_set_source_field: rates must be finite"); return SWE_EINVAL; }
            if (!s->solid.empty() && s->solid[i]) sg[i] = 0.0;   // a closed gate holds no water
        }
        // K1 source bits per tile: own cells, edge cells, outer face neighbours
        std::vector<unsigned char> fm(s->ntiles, 0);
        const int tx = s->L->tx, ty = s->L->ty;
        for (int t = 0; t < s->ntiles; ++t) {
            const int x0 = (t % s->ntx) * tx, y0 = (t / s->ntx) * ty;
            const int x1 = std::min(x0 + tx, s->nx), y1 = std::min(y0 + ty, s->ny);
            unsigned char m = 0;
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x)
                    if (sg[(size_t)y * s->nx + x] > 0.0) {
                        m |= 1;
                        if (x == x0) m |= 2;
                        if (x == x1 - 1) m |= 4;
                        if (y == y0) m |= 8;
                        if (y == y1 - 1) m |= 16;
                    }
            auto rain = [&](int x, int y) {
                return x >= 0 && x < s->nx && y >= 0 && y < s->ny && sg[(size_t)y * s->nx + x] > 0.0;
            };
            for (int x = x0; x < x1; ++x) if (rain(x, y0 - 1) || rain(x, y1)) m |= 32;
            for (int y = y0; y < y1; ++y) if (rain(x0 - 1, y) || rain(x1, y)) m |= 32;
            fm[t] = m;
        }
        if (!s->sigma) {
            HIPCHK(hipMalloc(&s->sigma, n * s->rsize));
            HIPCHK(hipMalloc((void**)&s->fmask, s->ntiles));
        }
        if (!s->fvol) {
            HIPCHK(hipMalloc((void**)&s->fvol, sizeof(double) * s->ntiles));
            HIPCHK(hipMemsetAsync(s->fvol, 0, sizeof(double) * s->ntiles, s->stream));
        }
        if ((rc = upload(s, s->sigma, sg.data(), 0.0))) return rc;
        HIPCHK(hipMemcpyAsync(s->fmask, fm.data(), s->ntiles, hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        s->field = true;
    }
    build_args(s);
    drop_graph(s);
    return prepare(s);
}

double swe_field_volume(swe_t* s) {
    if (!s) return NAN;
    if (!s->fvol) return 0.0;
    hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, s->stream, s->fvol, s->ntiles, s->scalar);
    double v = NAN;
    if (hipMemcpyAsync(&v, s->scalar, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return NAN;
    return v;
}

int swe_launch_grid(swe_t* s) {
    if (!s) { set_err("swe_launch_grid: NULL handle"); return SWE_EINVAL; }
    return s->grid;
}

int swe_set_launch_grid(swe_t* s, int grid) {
    if (!s || grid < 8 || grid > s->grid_max) {
        set_err("swe_set_launch_grid: the grid must be a handle's, from 8 to its default launch grid");
        return SWE_EINVAL;
    }
    if (s->ntap > 0) { set_err("swe_set_launch_grid: the nest launches its grids"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);   // queued launches keep the grid they were queued with
    if (rc) return rc;
    drop_graph(s);
    s->grid = grid;
    return 0;
}

int swe_active_tiles(swe_t* s, int* out, int cap) {
    if (!s || (!out && cap > 0) || cap < 0) { set_err("swe_active_tiles: invalid arguments"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    const int par = (int)(c.step & 1);
    if (!s->p.skip_dry) {
        const int m = s->ntiles < cap ? s->ntiles : cap;
        for (int i = 0; i < m; ++i) out[i] = i;
        return s->ntiles;
    }
    int got = 0;
    for (int g = 0; g < swe::NSEG && got < cap; ++g) {
        int n = c.seg_off[par][g + 1] - c.seg_off[par][g];
        if (n > cap - got) n = cap - got;
        if (n <= 0) continue;
        HIPCHK(hipMemcpyAsync(out + got, s->lists + ((size_t)par * swe::NSEG + g) * s->ntiles,
                              sizeof(int) * n, hipMemcpyDeviceToHost, s->stream));
        got += n;
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return c.seg_off[par][swe::NSEG];
}

static size_t line_tap_sizes(const swe_t* s, size_t* nyx) {
    const size_t ax = 3 * (size_t)s->ny * (s->nx / s->tap_r + 1);
    *nyx = 3 * (size_t)(s->ny / s->tap_r + 1) * s->nx;
    return ax;
}

int swe_enable_line_taps(swe_t* s, int r) {
    if (!s || r < 0) { set_err("swe_enable_line_taps: invalid arguments"); return SWE_EINVAL; }
    if (r > 0 && (s->field || s->p.sph_displaced || s->p.periodic)) {
        set_err("swe_enable_line_taps: not for a grid with a source rate field, the displaced-particle corrector "
                "or a periodic domain");
        return SWE_EINVAL;
    }
    if (r == 0) {
        if (s->tapx) (void)hipFree(s->tapx);
        if (s->tapy) (void)hipFree(s->tapy);
        s->tapx = s->tapy = nullptr;
        s->tap_r = 0;
        build_args(s);
        drop_graph(s);
        return 0;
    }
    if (s->nx % r || s->ny % r) { set_err("swe_enable_line_taps: grid size not a multiple of r"); return SWE_EINVAL; }
    if (!s->L->step_tap || s->ntap > 0 || s->corr) {
        set_err("swe_enable_line_taps: needs the default tile shape, not a nest member or corrected grid");
        return SWE_EINVAL;
    }
    if (s->tapx) { (void)hipFree(s->tapx); (void)hipFree(s->tapy); s->tapx = s->tapy = nullptr; }
    s->tap_r = r;
    size_t ny_ = 0, nx_ = line_tap_sizes(s, &ny_);
    HIPCHK(hipMalloc(&s->tapx, nx_ * s->rsize));
    HIPCHK(hipMalloc(&s->tapy, ny_ * s->rsize));
    build_args(s);
    drop_graph(s);
    return swe_zero_line_taps(s);
}

int swe_zero_line_taps(swe_t* s) {
    if (!s || !s->tap_r) { set_err("swe_zero_line_taps: no line taps"); return SWE_EINVAL; }
    size_t ny_ = 0, nx_ = line_tap_sizes(s, &ny_);
    if (s->precision == 32) {
        HIPCHK(fill_dev<float>(s->tapx, nx_, s->stream));
        HIPCHK(fill_dev<float>(s->tapy, ny_, s->stream));
    } else {
        HIPCHK(fill_dev<double>(s->tapx, nx_, s->stream));
        HIPCHK(fill_dev<double>(s->tapy, ny_, s->stream));
    }
    return 0;
}

int swe_get_line_taps(swe_t* s, double* tx, double* ty) {
    if (!s || !s->tap_r) { set_err("swe_get_line_taps: no line taps"); return SWE_EINVAL; }
    size_t ny_ = 0, nx_ = line_tap_sizes(s, &ny_);
    double* outs[2] = {tx, ty};
    void* srcs[2] = {s->tapx, s->tapy};
    size_t ns[2] = {nx_, ny_};
    for (int q = 0; q < 2; ++q) {
        if (!outs[q]) continue;
        std::vector<unsigned char> buf(ns[q] * s->rsize);
        HIPCHK(hipMemcpyAsync(buf.data(), srcs[q], buf.size(), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < ns[q]; ++i)
            outs[q][i] = s->precision == 32 ? (double)((float*)buf.data())[i] : ((double*)buf.data())[i];
    }
    return 0;
}

int swe_hold_dt(swe_t* s, double tau) {
    if (!s || !(tau >= 0.0) || !std::isfinite(tau)) { set_err("swe_hold_dt: invalid arguments"); return SWE_EINVAL; }
    if (s->ntap > 0) { set_err("swe_hold_dt: the nest sets the steps of its grids"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    s->launched = c.step;
    s->hold = tau > 0.0 ? 1 : 0;
    build_args(s);
    drop_graph(s);
    return set_dt_now(s, tau);
}

int swe_restrict(swe_t* fine, swe_t* coarse, int r) {
    if (!fine || !coarse || r < 1 || fine->nx != r * coarse->nx || fine->ny != r * coarse->ny ||
        fine->precision != coarse->precision) {
        set_err("swe_restrict: the fine grid must be r times the coarse grid, same precision");
        return SWE_EINVAL;
    }
    Ctrl cf, cc;
    int rc = sync_ctrl(fine, &cf);
    if (rc) return rc;
    if ((rc = sync_ctrl(coarse, &cc))) return rc;
    coarse->launched = cc.step;
    const int pf = (int)(cf.step & 1);
    const int nc = coarse->nx * coarse->ny;
    if (fine->precision == 32)
        hipLaunchKernelGGL(swe::k_restrict<float>, dim3(grid_for_cells(nc)), dim3(256), 0, fine->stream,
                           (const float*)fine->Hb[pf], (const float*)fine->Qxb[pf], (const float*)fine->Qyb[pf], fine->nx, r,
                           (float*)coarse->Hb[0], (float*)coarse->Qxb[0], (float*)coarse->Qyb[0], (float*)coarse->Hb[1],
                           (float*)coarse->Qxb[1], (float*)coarse->Qyb[1], coarse->nx, coarse->ny);
    else
        hipLaunchKernelGGL(swe::k_restrict<double>, dim3(grid_for_cells(nc)), dim3(256), 0, fine->stream,
                           (const double*)fine->Hb[pf], (const double*)fine->Qxb[pf], (const double*)fine->Qyb[pf],
                           fine->nx, r, (double*)coarse->Hb[0], (double*)coarse->Qxb[0], (double*)coarse->Qyb[0],
                           (double*)coarse->Hb[1], (double*)coarse->Qxb[1], (double*)coarse->Qyb[1], coarse->nx,
                           coarse->ny);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(fine->stream));
    // the coarse clock follows the fine one
    char* cb = (char*)coarse->ctrl;
    HIPCHK(hipMemcpyAsync(cb + offsetof(Ctrl, t), &cf.t, sizeof(double), hipMemcpyHostToDevice, coarse->stream));
    return prepare(coarse);
}

static int ensure_corr_buffers(swe_t* s) {
    if (s->corrE) return 0;
    const size_t n = 3 * (size_t)s->nx * s->ny;
    HIPCHK(hipMalloc(&s->corrE, n * s->rsize));
    HIPCHK(hipMalloc(&s->corrN, n * s->rsize));
    HIPCHK(hipMalloc((void**)&s->claims, 2 * sizeof(int)));
    HIPCHK(hipMemsetAsync(s->corrE, 0, n * s->rsize, s->stream));
    HIPCHK(hipMemsetAsync(s->corrN, 0, n * s->rsize, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    build_args(s);
    drop_graph(s);
    return 0;
}

int swe_set_correction_depth(swe_t* s, double hmin) {
    if (!s || !(hmin >= 0.0) || !std::isfinite(hmin)) { set_err("swe_set_correction_depth: invalid arguments"); return SWE_EINVAL; }
    s->corr_hmin = hmin;
    build_args(s);
    drop_graph(s);
    return 0;
}

int swe_set_correction(swe_t* s, const double* dE, const double* dN) {
    if (!s) { set_err("swe_set_correction: NULL handle"); return SWE_EINVAL; }
    if (!dE && !dN) {
        if (s->lc) { set_err("swe_set_correction: a network is attached"); return SWE_EINVAL; }
        if (s->corr) drop_graph(s);
        s->corr = false;
        return 0;
    }
    if (!s->L->step_corr) { set_err("swe_set_correction: the tile shape has no correcting step kernel"); return SWE_EINVAL; }
    if (s->field || s->p.sph_displaced || s->p.periodic) {
        set_err("swe_set_correction: not with a source rate field, the displaced-particle corrector or a "
                "periodic domain");
        return SWE_EINVAL;
    }
    if (s->ntap > 0) { set_err("swe_set_correction: not for grids of a nest"); return SWE_EINVAL; }
    const size_t n = 3 * (size_t)s->nx * s->ny;
    if (s->lc) { set_err("swe_set_correction: a network is attached (swe_lc_attach(NULL, grid) first)"); return SWE_EINVAL; }
    int rc = ensure_corr_buffers(s);
    if (rc) return rc;
    std::vector<unsigned char> buf(n * s->rsize);
    const double* src[2] = {dE, dN};
    void* dst[2] = {s->corrE, s->corrN};
    for (int q = 0; q < 2; ++q) {
        for (size_t i = 0; i < n; ++i) {
            const double v = src[q] ? src[q][i] : 0.0;
            if (!std::isfinite(v)) { set_err("swe_set_correction: non-finite correction"); return SWE_EINVAL; }
            if (s->precision == 32) ((float*)buf.data())[i] = (float)v;
            else ((double*)buf.data())[i] = v;
        }
        HIPCHK(hipMemcpyAsync(dst[q], buf.data(), buf.size(), hipMemcpyHostToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    if (!s->corr) drop_graph(s);
    s->corr = true;
    return 0;
}

}  // extern "C"


// ====================================================================== batched ensemble

namespace {

struct BScen {
    int nx = 0, ny = 0, ntx = 0, nty = 0, ntiles = 0, tile_base = 0, nin = 0;
    double h = 0.0;
    swe_params p{};
    void* Hb[2] = {nullptr, nullptr};
    void* Qxb[2] = {nullptr, nullptr};
    void* Qyb[2] = {nullptr, nullptr};
    void* bed = nullptr;
    void* cf = nullptr;
    double* mass = nullptr;
    double* ledger = nullptr;
};

}  // namespace

struct swe_batch_s {
    int n = 0, precision = 32, rsize = 4, grid = 0, total_tiles = 0;
    const Launcher* L = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<BScen> sc;
    Ctrl* lctrl = nullptr;
    Ctrl* ctrls = nullptr;
    int* hot = nullptr;
    int* lists = nullptr;
    int* stamp = nullptr;
    long long* wg_cells = nullptr;
    double* scalar = nullptr;
    void* dargs[2] = {nullptr, nullptr};
    std::vector<unsigned char> hargs[2];   // Args<real>[n] per parity (host copies)
    std::vector<unsigned char> bargs[2];   // BatchArgs<real> per parity
    long long launched = 0;
    hipGraphExec_t graph = nullptr;
};

namespace {

template <typename real>
void fill_batch_args(swe_batch_t* b, int par) {
    b->hargs[par].resize(sizeof(Args<real>) * b->n);
    Args<real>* A = (Args<real>*)b->hargs[par].data();
    for (int k = 0; k < b->n; ++k) {
        BScen& c = b->sc[k];
        Args<real>* a = &A[k];
        std::memset(a, 0, sizeof *a);
        const swe_params& p = c.p;
        a->Hi = (const real*)c.Hb[par]; a->Qxi = (const real*)c.Qxb[par]; a->Qyi = (const real*)c.Qyb[par];
        a->Ho = (real*)c.Hb[par ^ 1]; a->Qxo = (real*)c.Qxb[par ^ 1]; a->Qyo = (real*)c.Qyb[par ^ 1];
        a->bed = (const real*)c.bed; a->cf = (const real*)c.cf;
        a->ctrl = b->ctrls + k; a->lctrl = b->lctrl;
        a->sid = k; a->tile_base = c.tile_base;
        a->hot = b->hot; a->lists = b->lists; a->slot = par; a->stamp = b->stamp;
        a->wg_speed = nullptr; a->wg_cells = b->wg_cells;
        a->mass = c.mass; a->ledger = c.ledger;
        a->nx = c.nx; a->ny = c.ny; a->ntx = c.ntx; a->nty = c.nty; a->ntiles = c.ntiles;
        a->skip = 1; a->limiter = p.limiter; a->list_cap = b->total_tiles;
        if (c.nin > 0) { a->i0 = p.inlet_i0; a->j0 = p.inlet_j0; a->ni = p.inlet_ni; a->nj = p.inlet_nj; }
        a->h = (real)c.h; a->ih = (real)(1.0 / c.h); a->g = (real)p.g; a->eps = (real)p.eps;
        a->nuh2 = (real)(p.nu / (c.h * c.h)); a->fcor = (real)p.f_coriolis;
        a->wx = (real)p.wind_x; a->wy = (real)p.wind_y; a->kw = (real)p.wind_kappa; a->hw = (real)p.h_wind;
        a->h_d = c.h; a->g_d = p.g; a->cfl = p.cfl; a->tau_max = p.dt_max; a->tau_min = p.dt_min; a->nu_d = p.nu;
        a->nin_h2 = c.nin > 0 ? (double)c.nin * c.h * c.h : 0.0;
        a->q_base = p.q_base; a->q_peak = p.q_peak; a->t_peak = p.t_peak; a->sigma_t = p.sigma_t;
    }
    b->bargs[par].resize(sizeof(swe::BatchArgs<real>));
    swe::BatchArgs<real>* ba = (swe::BatchArgs<real>*)b->bargs[par].data();
    ba->scen = (const Args<real>*)b->dargs[par];
    ba->n = b->n; ba->lctrl = b->lctrl; ba->hot = b->hot; ba->lists = b->lists;
    ba->list_cap = b->total_tiles; ba->slot = par; ba->wg_cells = b->wg_cells;
}

void free_batch(swe_batch_t* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (BScen& c : b->sc) {
        void* ptrs[] = {c.Hb[0], c.Hb[1], c.Qxb[0], c.Qxb[1], c.Qyb[0], c.Qyb[1], c.bed, c.cf, c.mass, c.ledger};
        for (void* q : ptrs) if (q) (void)hipFree(q);
    }
    void* ptrs[] = {b->lctrl, b->ctrls, b->hot, b->lists, b->stamp, b->wg_cells, b->scalar, b->dargs[0], b->dargs[1]};
    for (void* q : ptrs) if (q) (void)hipFree(q);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

int batch_sync_ctrls(swe_batch_t* b, std::vector<Ctrl>& c, Ctrl* lc) {
    c.resize(b->n);
    HIPCHK(hipMemcpyAsync(c.data(), b->ctrls, sizeof(Ctrl) * b->n, hipMemcpyDeviceToHost, b->stream));
    if (lc) HIPCHK(hipMemcpyAsync(lc, b->lctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return 0;
}

int batch_finish(swe_batch_t* b) {
    std::vector<Ctrl> c;
    int rc = batch_sync_ctrls(b, c, nullptr);
    if (rc) return rc;
    for (int k = 0; k < b->n; ++k) {
        const int e = c[k].err_gate ? c[k].err_gate : c[k].err;
        if (e) {
            char buf[128];
            std::snprintf(buf, sizeof buf, "scenario %d: %s", k,
                          e == SWE_ENONFINITE ? "state became non-finite" : "time step collapsed below dt_min");
            g_err = buf;
            return e;
        }
    }
    return 0;
}

int batch_launch(swe_batch_t* b, long n) {
    for (long k = 0; k < n; ++k) {
        const int par = (int)(b->launched & 1);
        HIPCHK(b->L->batch_step(b->bargs[par].data(), b->grid, b->stream, nullptr, nullptr));
        b->launched++;
    }
    return 0;
}

}  // namespace

extern "C" {

swe_batch_t* swe_batch_create(int n, const int* nx, const int* ny, const double* dx, const double* const* b,
                              const double* const* n_M, const swe_params* p) {
    g_err.clear();
    if (n < 1 || n > (1 << (31 - swe::TILE_BITS)) || !nx || !ny || !dx || !b || !p) {
        set_err("swe_batch_create: invalid arguments"); return nullptr;
    }
    const swe_params& p0 = p[0];
    if (!p0.skip_dry) { set_err("swe_batch_create: a batch runs with dry-tile skipping"); return nullptr; }
    for (int k = 0; k < n; ++k) {
        if (p[k].sph_displaced) { set_err("swe_batch_create: no displaced-particle corrector in a batch"); return nullptr; }
        if (p[k].periodic) { set_err("swe_batch_create: no periodic domain in a batch"); return nullptr; }
    }
    const Launcher* L = find_launcher(p0.precision, p0.tile_x, p0.tile_y, p0.limiter);
    if (!L) { set_err("swe_batch_create: tile shape not available for this precision/limiter"); return nullptr; }
    long long total = 0;
    for (int k = 0; k < n; ++k) {
        if (p[k].precision != p0.precision || p[k].limiter != p0.limiter || !p[k].skip_dry) {
            set_err("swe_batch_create: precision, limiter and skipping must agree across the batch"); return nullptr;
        }
        if (nx[k] < 1 || ny[k] < 1 || (long long)nx[k] * ny[k] > (1LL << 31) - 1 || !b[k]) {
            set_err("swe_batch_create: invalid grid"); return nullptr;
        }
        const long long nt = (long long)((nx[k] + L->tx - 1) / L->tx) * ((ny[k] + L->ty - 1) / L->ty);
        if (nt >= (1LL << swe::TILE_BITS)) { set_err("swe_batch_create: grid has too many tiles"); return nullptr; }
        total += nt;
    }
    if (total > (1LL << 28)) { set_err("swe_batch_create: batch too large"); return nullptr; }

    swe_batch_t* B = new (std::nothrow) swe_batch_s();
    if (!B) { set_err("swe_batch_create: out of host memory"); return nullptr; }
#define BK(expr)                                                                 \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) { set_hip_err("swe_batch_create", e_); free_batch(B); delete B; return nullptr; } \
    } while (0)
    B->n = n; B->L = L; B->precision = p0.precision; B->rsize = p0.precision == 32 ? 4 : 8;
    B->total_tiles = (int)total;
    if (p0.stream) B->stream = (hipStream_t)p0.stream;
    else { BK(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking)); B->own_stream = true; }
    B->sc.resize(n);
    // validate and upload each scenario through a temporary single-grid handle's rules
    int base = 0;
    for (int k = 0; k < n; ++k) {
        BScen& c = B->sc[k];
        c.nx = nx[k]; c.ny = ny[k]; c.h = dx[k]; c.p = p[k];
        c.p.solid = nullptr; c.p.H0 = c.p.Qx0 = c.p.Qy0 = nullptr; c.p.stream = nullptr;
        c.ntx = (c.nx + L->tx - 1) / L->tx; c.nty = (c.ny + L->ty - 1) / L->ty; c.ntiles = c.ntx * c.nty;
        c.tile_base = base; base += c.ntiles;
        const swe_params& q = p[k];
        const size_t ncell = (size_t)c.nx * c.ny;
        if (!(c.h > 0.0) || !std::isfinite(c.h) || !(q.g > 0.0) || !(q.cfl > 0.0) || !(q.cfl < 1.0) ||
            !(q.eps > 0.0) || q.nu < 0.0 || !(q.h_wind > 0.0) || !std::isfinite(q.dt_min) || !std::isfinite(q.dt_max)) {
            set_err("swe_batch_create: invalid parameters"); free_batch(B); delete B; return nullptr;
        }
        if (q.inlet_ni > 0 && q.inlet_nj > 0) {
            if (q.inlet_i0 < 0 || q.inlet_j0 < 0 || q.inlet_i0 + q.inlet_ni > c.nx || q.inlet_j0 + q.inlet_nj > c.ny) {
                set_err("swe_batch_create: inlet outside the grid"); free_batch(B); delete B; return nullptr;
            }
            for (int j = q.inlet_j0; j < q.inlet_j0 + q.inlet_nj; ++j)
                for (int i = q.inlet_i0; i < q.inlet_i0 + q.inlet_ni; ++i)
                    if (q.solid && q.solid[(size_t)j * c.nx + i]) {
                        set_err("swe_batch_create: an inlet contains a closed gate"); free_batch(B); delete B; return nullptr;
                    }
            c.nin = q.inlet_ni * q.inlet_nj;
        }
        const size_t bytes = ncell * B->rsize;
        for (int t = 0; t < 2; ++t) {
            BK(hipMalloc(&c.Hb[t], bytes)); BK(hipMalloc(&c.Qxb[t], bytes)); BK(hipMalloc(&c.Qyb[t], bytes));
        }
        BK(hipMalloc(&c.bed, bytes)); BK(hipMalloc(&c.cf, bytes));
        BK(hipMalloc((void**)&c.mass, sizeof(double) * c.ntiles));
        BK(hipMalloc((void**)&c.ledger, sizeof(double) * c.ntiles));
        BK(hipMemsetAsync(c.ledger, 0, sizeof(double) * c.ntiles, B->stream));
        // static fields and the initial state (dry cells at rest, closed gates dry and raised)
        std::vector<unsigned char> buf(bytes);
        auto put = [&](void* dst, auto fn) -> hipError_t {
            if (B->precision == 32) { float* f = (float*)buf.data(); for (size_t i = 0; i < ncell; ++i) f[i] = (float)fn(i); }
            else { double* d = (double*)buf.data(); for (size_t i = 0; i < ncell; ++i) d[i] = fn(i); }
            hipError_t e = hipMemcpyAsync(dst, buf.data(), bytes, hipMemcpyHostToDevice, B->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
            return e;
        };
        const double* bk = b[k];
        const double* nm = n_M ? n_M[k] : nullptr;
        bool okv = true;
        for (size_t i = 0; i < ncell && okv; ++i) {
            okv = std::isfinite(bk[i]) && (!nm || (std::isfinite(nm[i]) && nm[i] >= 0.0));
            const double hh = q.H0 ? q.H0[i] : 0.0, a = q.Qx0 ? q.Qx0[i] : 0.0, bb = q.Qy0 ? q.Qy0[i] : 0.0;
            okv = okv && std::isfinite(hh) && hh >= 0.0 && std::isfinite(a) && std::isfinite(bb);
        }
        if (!okv) { set_err("swe_batch_create: non-finite or negative input"); free_batch(B); delete B; return nullptr; }
        const uint8_t* so = q.solid;
        const double eps = q.eps, g = q.g;
        BK(put(c.bed, [&](size_t i) { return so && so[i] ? swe::GATE_BED : bk[i]; }));
        BK(put(c.cf, [&](size_t i) { return (so && so[i]) || !nm ? 0.0 : g * nm[i] * nm[i]; }));
        auto Hf = [&](size_t i) { return so && so[i] ? 0.0 : (q.H0 ? q.H0[i] : 0.0); };
        auto Qf = [&](const double* Q, size_t i) { const double hh = Hf(i); return !(hh > eps) || !Q ? 0.0 : Q[i]; };
        for (int t = 0; t < 2; ++t) {
            BK(put(c.Hb[t], Hf));
            BK(put(c.Qxb[t], [&](size_t i) { return Qf(q.Qx0, i); }));
            BK(put(c.Qyb[t], [&](size_t i) { return Qf(q.Qy0, i); }));
        }
    }
    BK(hipMalloc((void**)&B->lctrl, sizeof(Ctrl)));
    BK(hipMalloc((void**)&B->ctrls, sizeof(Ctrl) * n));
    BK(hipMalloc((void**)&B->hot, sizeof(int) * swe::HOT_INTS));
    BK(hipMalloc((void**)&B->lists, sizeof(int) * 2 * swe::NSEG * (size_t)total));
    BK(hipMalloc((void**)&B->stamp, sizeof(int) * (size_t)total));
    BK(hipMalloc((void**)&B->scalar, sizeof(double) * n));
    BK(hipMemsetAsync(B->lctrl, 0, sizeof(Ctrl), B->stream));
    BK(hipMemsetAsync(B->ctrls, 0, sizeof(Ctrl) * n, B->stream));
    BK(hipMemsetAsync(B->hot, 0, sizeof(int) * swe::HOT_INTS, B->stream));
    BK(hipMemsetAsync(B->stamp, 0, sizeof(int) * (size_t)total, B->stream));
    int dev = 0, cus = 0, occ = 0;
    BK(hipGetDevice(&dev));
    BK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (L->occupancy(&occ) != 0 || occ < 1) occ = 1;
    B->grid = cus * occ;
    if (B->grid < 8) B->grid = 8;
    BK(hipMalloc((void**)&B->wg_cells, sizeof(long long) * B->grid));
    const size_t asz = B->precision == 32 ? sizeof(Args<float>) : sizeof(Args<double>);
    for (int t = 0; t < 2; ++t) {
        BK(hipMalloc(&B->dargs[t], asz * n));
        if (B->precision == 32) fill_batch_args<float>(B, t); else fill_batch_args<double>(B, t);
        BK(hipMemcpyAsync(B->dargs[t], B->hargs[t].data(), asz * n, hipMemcpyHostToDevice, B->stream));
    }
    // layer-0 bookkeeping of every scenario into list slot 0, then the first time steps
    for (int k = 0; k < n; ++k)
        BK(L->prepare(B->hargs[0].data() + asz * k, B->sc[k].ntiles, B->stream));
    BK(L->batch_prepare_finish(B->bargs[0].data(), B->stream));
    BK(hipStreamSynchronize(B->stream));
#undef BK
    return B;
}

void swe_batch_destroy(swe_batch_t* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
}

int swe_batch_run(swe_batch_t* b, long nsteps) {
    if (!b || nsteps < 0) { set_err("swe_batch_run: invalid arguments"); return SWE_EINVAL; }
    long left = nsteps;
    int rc;
    if (left > 0 && (b->launched & 1)) { if ((rc = batch_launch(b, 1))) return rc; --left; }
    if (left >= GRAPH_STEPS) {
        if (!b->graph) {
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < GRAPH_STEPS; ++k) {
                hipError_t e = b->L->batch_step(b->bargs[k & 1].data(), b->grid, b->stream, nullptr, nullptr);
                if (e != hipSuccess) {
                    (void)hipStreamEndCapture(b->stream, &g);
                    if (g) (void)hipGraphDestroy(g);
                    set_hip_err("batch graph capture", e);
                    return SWE_EHIP;
                }
            }
            HIPCHK(hipStreamEndCapture(b->stream, &g));
            hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) { b->graph = nullptr; set_hip_err("batch graph instantiation", e); return SWE_EHIP; }
        }
        while (left >= GRAPH_STEPS) {
            HIPCHK(hipGraphLaunch(b->graph, b->stream));
            b->launched += GRAPH_STEPS;
            left -= GRAPH_STEPS;
        }
    }
    if ((rc = batch_launch(b, left))) return rc;
    return batch_finish(b);
}

int swe_batch_run_timed(swe_batch_t* b, long nsteps, double* kernel_ms) {
    if (!b || nsteps < 0 || !kernel_ms) { set_err("swe_batch_run_timed: invalid arguments"); return SWE_EINVAL; }
    int rc = timed_launches(b->stream, nsteps, kernel_ms, [&](hipEvent_t e0, hipEvent_t e1) {
        const int par = (int)(b->launched & 1);
        const hipError_t e = b->L->batch_step(b->bargs[par].data(), b->grid, b->stream, e0, e1);
        b->launched++;
        return e;
    });
    if (rc) return rc;
    return batch_finish(b);
}

int swe_batch_query(swe_batch_t* b, double* t, double* mass, double* inflow, double* ledger, long* steps) {
    if (!b) { set_err("swe_batch_query: NULL handle"); return SWE_EINVAL; }
    std::vector<Ctrl> c;
    int rc = batch_sync_ctrls(b, c, nullptr);
    if (rc) return rc;
    for (int k = 0; k < b->n; ++k) {
        if (t) t[k] = c[k].t;
        if (inflow) inflow[k] = c[k].inflow;
        if (steps) steps[k] = (long)c[k].step;
    }
    double* outs[2] = {mass, ledger};
    for (int w = 0; w < 2; ++w) {
        if (!outs[w]) continue;
        for (int k = 0; k < b->n; ++k)
            hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, b->stream,
                               w == 0 ? b->sc[k].mass : b->sc[k].ledger, b->sc[k].ntiles, b->scalar + k);
        HIPCHK(hipGetLastError());
        std::vector<double> v(b->n);
        HIPCHK(hipMemcpyAsync(v.data(), b->scalar, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        for (int k = 0; k < b->n; ++k) outs[w][k] = w == 0 ? v[k] * b->sc[k].h * b->sc[k].h : v[k];
    }
    return 0;
}

int swe_batch_get_state(swe_batch_t* b, int k, double* H, double* Qx, double* Qy) {
    if (!b || k < 0 || k >= b->n) { set_err("swe_batch_get_state: invalid arguments"); return SWE_EINVAL; }
    std::vector<Ctrl> c;
    int rc = batch_sync_ctrls(b, c, nullptr);
    if (rc) return rc;
    const BScen& s = b->sc[k];
    const int par = (int)(c[k].step & 1);
    const size_t n = (size_t)s.nx * s.ny;
    std::vector<unsigned char> buf(n * b->rsize);
    double* outs[3] = {H, Qx, Qy};
    void* srcs[3] = {s.Hb[par], s.Qxb[par], s.Qyb[par]};
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        HIPCHK(hipMemcpyAsync(buf.data(), srcs[q], n * b->rsize, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        if (b->precision == 32) { const float* f = (const float*)buf.data(); for (size_t i = 0; i < n; ++i) outs[q][i] = f[i]; }
        else std::memcpy(outs[q], buf.data(), n * sizeof(double));
    }
    return 0;
}

int swe_batch_work(swe_batch_t* b, long long* tile_steps, long long* cell_steps, int* total_tiles) {
    if (!b) { set_err("swe_batch_work: NULL handle"); return SWE_EINVAL; }
    Ctrl lc;
    HIPCHK(hipMemcpyAsync(&lc, b->lctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (tile_steps) *tile_steps = lc.tiles;
    if (cell_steps) *cell_steps = lc.cells;
    if (total_tiles) *total_tiles = b->total_tiles;
    return 0;
}

}  // extern "C"

// Fixed-order FP64 reduction: thread t sums partials t, t+1024, ... in index
// order, then a fixed binary tree over the 1024 thread sums.
__global__ void swe::k_sum_tiles(const double* part, int n, double* out) {
    __shared__ double buf[1024];
    const int t = threadIdx.x;
    double v = 0.0;
    for (int i = t; i < n; i += 1024) v += part[i];
    buf[t] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) buf[t] += buf[t + o];
        __syncthreads();
    }
    if (t == 0) *out = buf[0];
}

// ====================================================================== nested grids

#include "swe_nest.hpp"

namespace {

constexpr int NEST_GRAPH_STEPS = 8;   // coarse steps per captured graph (even)

}  // namespace

struct swe_nest_s {
    int r = 1, np = 0, feedback = 1, precision = 32, rsize = 4;
    swe_t* c = nullptr;
    std::vector<swe_t*> p;
    std::vector<swe_patch> box;      // host copy of the layout (pointers not kept)
    hipStream_t stream = nullptr;
    void* tap = nullptr;             // device taps: coarse boxes, then patches
    int ntap = 0;
    int* ints = nullptr;             // device ints: rects, ring CSR, forced tiles, regions
    void* desc = nullptr;            // device NestPatch<real>[np]
    double* ring_ledger = nullptr;
    double* part = nullptr;          // volume partials
    int npart = 0, chunk = 0;
    double* scalar = nullptr;
    int nforce = 0, nregion = 0, nregion_cells = 0, nring = 0;
    const int* force_tiles = nullptr;
    const int* region = nullptr;
    long long launched = 0;          // coarse steps launched
    hipGraphExec_t graph = nullptr;
    std::vector<unsigned char> nargs;   // NestArgs<real>
    // one side stream per patch (default priority): the first substep of
    // every patch runs beside the coarse step, later substeps of patches 1..
    // beside patch 0; forked from and joined back into the nest's stream
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    hipEvent_t frame0 = nullptr;     // the first substep's frame is written
    std::vector<hipEvent_t> join;
};

namespace {

void free_nest(swe_nest_t* n) {
    if (n->graph) (void)hipGraphExecDestroy(n->graph);
    for (hipStream_t q : n->side) if (q) { (void)hipStreamSynchronize(q); (void)hipStreamDestroy(q); }
    if (n->fork) (void)hipEventDestroy(n->fork);
    if (n->frame0) (void)hipEventDestroy(n->frame0);
    for (hipEvent_t e : n->join) if (e) (void)hipEventDestroy(e);
    for (swe_t* q : n->p) if (q) swe_destroy(q);
    if (n->c) swe_destroy(n->c);
    void* ptrs[] = {n->tap, n->ints, n->desc, n->ring_ledger, n->part, n->scalar};
    for (void* q : ptrs) if (q) (void)hipFree(q);
}

template <typename real>
void fill_nest_args(swe_nest_t* n, int nframe, int ncov, int nring, const int* ring_cell, const int* ring_off,
                    const int* ring_face) {
    n->nargs.assign(sizeof(swe::NestArgs<real>), 0);
    swe::NestArgs<real>* a = (swe::NestArgs<real>*)n->nargs.data();
    a->P = (const swe::NestPatch<real>*)n->desc;
    a->np = n->np; a->r = n->r; a->nx = n->c->nx; a->ny = n->c->ny;
    a->nframe = nframe; a->ncov = ncov; a->nring = nring;
    for (int k = 0; k < 2; ++k) {
        a->Hc[k] = (real*)n->c->Hb[k]; a->Qxc[k] = (real*)n->c->Qxb[k]; a->Qyc[k] = (real*)n->c->Qyb[k];
    }
    a->bc = (const real*)n->c->bed;
    a->tap = (real*)n->tap;
    a->ring_cell = ring_cell; a->ring_off = ring_off; a->ring_face = ring_face;
    a->ring_ledger = n->ring_ledger;
    a->eps = (real)n->c->p.eps;
    a->ih = (real)(1.0 / n->c->h);
    a->h2 = n->c->h * n->c->h;
}

template <typename real>
int upload_desc(swe_nest_t* n, const std::vector<int>& frame_base, const std::vector<int>& cov_base,
                const std::vector<int>& ftap, const std::vector<int>& ctap) {
    std::vector<swe::NestPatch<real>> d(n->np);
    for (int k = 0; k < n->np; ++k) {
        const swe_patch& b = n->box[k];
        swe::NestPatch<real>& e = d[k];
        e.ci0 = b.ci0; e.cj0 = b.cj0; e.cw = b.cw; e.ch = b.ch;
        e.nxe = n->p[k]->nx; e.nye = n->p[k]->ny;
        e.frame_base = frame_base[k]; e.cov_base = cov_base[k];
        e.ftap = ftap[k]; e.ctap = ctap[k];
        for (int q = 0; q < 2; ++q) {
            e.Hf[q] = (real*)n->p[k]->Hb[q]; e.Qxf[q] = (real*)n->p[k]->Qxb[q]; e.Qyf[q] = (real*)n->p[k]->Qyb[q];
        }
        e.bf = (const real*)n->p[k]->bed;
        e.ctrl = n->p[k]->ctrl;
        e.mass = n->p[k]->mass;
        e.ntx = n->p[k]->ntx; e.tx = n->p[k]->L->tx; e.ty = n->p[k]->L->ty;
    }
    HIPCHK(hipMemcpyAsync(n->desc, d.data(), sizeof(swe::NestPatch<real>) * n->np, hipMemcpyHostToDevice,
                          n->stream));
    HIPCHK(hipStreamSynchronize(n->stream));
    return 0;
}

int blocks_for(long long work, int bs) { return (int)((work + bs - 1) / bs); }

// One coarse step with its substeps and the feedback, all launches on the
// nest's stream.
template <typename real>
hipError_t nest_step_t(swe_nest_t* n) {
    const swe::NestArgs<real>& na = *(const swe::NestArgs<real>*)n->nargs.data();
    swe_t* c = n->c;
    const int pc = (int)(c->launched & 1);
    hipError_t e;
    // The previous close cleared the taps (creation did for the first step).
    // Substep 0 takes its frame from layer n alone, so it runs beside the
    // coarse step: its frame and every patch's first step on side streams
    // forked before the coarse step and joined back before the next frame.
    // Later substeps need layer n+1: frame on the nest's stream, patch 0
    // there too, the others on side streams between a fork and a join.
    const int np = (int)n->p.size();
    if ((e = hipEventRecord(n->fork, n->stream)) != hipSuccess) return e;
    for (int k = 0; k < np; ++k)
        if ((e = hipStreamWaitEvent(n->side[k], n->fork, 0)) != hipSuccess) return e;
    if ((e = launch_grid_step(c, pc)) != hipSuccess) return e;
    c->launched++;
    for (int s = 0; s < n->r; ++s) {
        const int pf = (int)(n->p[0]->launched & 1);
        const bool first = s == 0;
        hipLaunchKernelGGL(swe::k_frame<real>, dim3(blocks_for(na.nframe, 256)), dim3(256), 0,
                           first ? n->side[0] : n->stream, na, pf, pc, (real)((double)s / (double)n->r));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (first) {   // the other patches' first step waits for the frame
            if ((e = hipEventRecord(n->frame0, n->side[0])) != hipSuccess) return e;
            for (int k = 1; k < np; ++k)
                if ((e = hipStreamWaitEvent(n->side[k], n->frame0, 0)) != hipSuccess) return e;
        } else if (np > 1) {
            if ((e = hipEventRecord(n->fork, n->stream)) != hipSuccess) return e;
            for (int k = 1; k < np; ++k)
                if ((e = hipStreamWaitEvent(n->side[k], n->fork, 0)) != hipSuccess) return e;
        }
        for (int k = 0; k < np; ++k) {
            swe_t* q = n->p[k];
            hipStream_t st = first || k ? n->side[k] : nullptr;   // nullptr: the nest's stream
            if ((e = launch_grid_step(q, pf, nullptr, nullptr, st)) != hipSuccess) return e;
            q->launched++;
        }
        for (int k = first ? 0 : 1; k < np; ++k) {
            if ((e = hipEventRecord(n->join[k], n->side[k])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(n->stream, n->join[k], 0)) != hipSuccess) return e;
        }
    }
    const Args<real>& an = *(const Args<real>*)c->args[pc ^ 1].data();
    if (n->feedback) {
        const int pf = (int)(n->p[0]->launched & 1);
        hipLaunchKernelGGL(swe::k_feedback<real>, dim3(blocks_for(na.ncov + na.nring, 256)), dim3(256), 0,
                           n->stream, na, pf, pc ^ 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nforce = c->p.skip_dry ? n->nforce : 0;
        const int blocks = std::max(blocks_for(n->nregion_cells, 256 * swe::NEST_CLOSE_CELLS),
                                    std::max(blocks_for(n->ntap, 256), blocks_for(nforce, 256)));
        const int grid = std::max(1, std::min(blocks, swe::NEST_CLOSE_GRID));
        hipLaunchKernelGGL(swe::k_nest_close<real>, dim3(grid), dim3(256), 0, n->stream, an, na, n->region,
                           n->nregion, n->nregion_cells, n->force_tiles, nforce, n->ntap, pc ^ 1);
        return hipGetLastError();
    }
    const int tb = blocks_for(n->ntap, 256);
    hipLaunchKernelGGL(swe::k_nest_tau<real>, dim3(tb < 1 ? 1 : tb > 1024 ? 1024 : tb), dim3(256), 0, n->stream, an,
                       na, pc ^ 1, n->ntap);
    return hipGetLastError();
}

hipError_t nest_step(swe_nest_t* n) {
    return n->precision == 32 ? nest_step_t<float>(n) : nest_step_t<double>(n);
}

// Time steps of the first coarse step: frames from the initial coarse layer,
// CFL steps of every grid, then the nest's rule.
template <typename real>
int nest_init_tau(swe_nest_t* n) {
    const swe::NestArgs<real>& na = *(const swe::NestArgs<real>*)n->nargs.data();
    const int pc = (int)(n->c->launched & 1), pf = (int)(n->p[0]->launched & 1);
    hipLaunchKernelGGL(swe::k_frame<real>, dim3(blocks_for(na.nframe, 256)), dim3(256), 0, n->stream, na, pf, pc,
                       (real)0);
    HIPCHK(hipGetLastError());
    for (swe_t* q : n->p) {
        int rc = prepare(q);
        if (rc) return rc;
    }
    const Args<real>& a = *(const Args<real>*)n->c->args[pc].data();
    hipLaunchKernelGGL(swe::k_nest_tau<real>, dim3(1), dim3(64), 0, n->stream, a, na, pc, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(n->stream));
    return 0;
}

int nest_finish(swe_nest_t* n) {
    HIPCHK(hipStreamSynchronize(n->stream));
    return finish(n->c);
}

int nest_launch(swe_nest_t* n, long k) {
    for (long i = 0; i < k; ++i) {
        hipError_t e = nest_step(n);
        if (e != hipSuccess) { set_hip_err("nest step", e); return SWE_EHIP; }
        n->launched++;
    }
    return 0;
}

int nest_graph(swe_nest_t* n) {
    if (n->graph) return 0;
    // capture starts and ends on even parities of every grid
    const long long c0 = n->c->launched;
    std::vector<long long> p0;
    for (swe_t* q : n->p) p0.push_back(q->launched);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(n->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < NEST_GRAPH_STEPS && e == hipSuccess; ++k) e = nest_step(n);
    hipError_t e2 = hipStreamEndCapture(n->stream, &g);
    // capture launched nothing: restore the host counters
    n->c->launched = c0;
    for (int k = 0; k < n->np; ++k) n->p[k]->launched = p0[k];
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_hip_err("nest graph capture", e != hipSuccess ? e : e2);
        return SWE_EHIP;
    }
    e = hipGraphInstantiate(&n->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { n->graph = nullptr; set_hip_err("nest graph instantiation", e); return SWE_EHIP; }
    return 0;
}

}  // namespace

extern "C" {

swe_nest_t* swe_nest_create(int nx, int ny, double dx, const double* b, const double* n_M, const swe_params* p,
                            int r, int feedback, int npatch, const swe_patch* patches) {
    g_err.clear();
    if (!p || !b || !patches || npatch < 1 || npatch > swe::NEST_MAX_PATCHES || r < 1 || r > 16) {
        set_err("swe_nest_create: need params, bed, 1 <= r <= 16 and 1 to 64 patches"); return nullptr;
    }
    if (p->tile_x != 0 || p->tile_y != 0) { set_err("swe_nest_create: nests use the default tile shape"); return nullptr; }
    const int G = swe::NEST_FRAME, m = (G + r - 1) / r;
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        if (!q.b || q.cw < 1 || q.ch < 1 || q.ci0 < m || q.cj0 < m || q.ci0 + q.cw + m > nx ||
            q.cj0 + q.ch + m > ny) {
            set_err("swe_nest_create: a patch box or its frame leaves the coarse grid"); return nullptr;
        }
        if ((long long)(r * q.cw + 2 * G) * (r * q.ch + 2 * G) > (1LL << 30)) {
            set_err("swe_nest_create: patch too large"); return nullptr;
        }
        if (p->inlet_ni > 0 && p->inlet_nj > 0 &&
            !(p->inlet_i0 + p->inlet_ni <= q.ci0 - 1 || p->inlet_i0 >= q.ci0 + q.cw + 1 ||
              p->inlet_j0 + p->inlet_nj <= q.cj0 - 1 || p->inlet_j0 >= q.cj0 + q.ch + 1)) {
            set_err("swe_nest_create: a patch covers or touches the inlet"); return nullptr;
        }
        if (p->solid)
            for (int j = q.cj0 - m; j < q.cj0 + q.ch + m; ++j)
                for (int i = q.ci0 - m; i < q.ci0 + q.cw + m; ++i)
                    if (p->solid[(size_t)j * nx + i]) {
                        set_err("swe_nest_create: a closed gate lies under a patch or its frame"); return nullptr;
                    }
        for (int l = k + 1; l < npatch; ++l) {
            const swe_patch& o = patches[l];
            if (!(q.ci0 + q.cw + 1 <= o.ci0 || o.ci0 + o.cw + 1 <= q.ci0 || q.cj0 + q.ch + 1 <= o.cj0 ||
                  o.cj0 + o.ch + 1 <= q.cj0)) {
                set_err("swe_nest_create: patches must keep one uncovered cell between them"); return nullptr;
            }
        }
    }
    swe_nest_t* n = new (std::nothrow) swe_nest_s();
    if (!n) { set_err("swe_nest_create: out of host memory"); return nullptr; }
    n->r = r; n->np = npatch; n->feedback = feedback ? 1 : 0;
    n->precision = p->precision; n->rsize = p->precision == 32 ? 4 : 8;
    n->box.assign(patches, patches + npatch);

#define NK(expr)                                                         \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) {                                          \
            set_hip_err("swe_nest_create", e_);                          \
            free_nest(n); delete n; return nullptr;                      \
        }                                                                \
    } while (0)

    // ---- host layout: taps, rects, ring CSR, forced tiles, speed regions
    std::vector<int> ctap(npatch), ftap(npatch), frame_base(npatch), cov_base(npatch);
    int ntap = 0, nframe = 0, ncov = 0;
    for (int k = 0; k < npatch; ++k) { ctap[k] = ntap; ntap += 3 * 2 * (patches[k].cw + patches[k].ch); }
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        ftap[k] = ntap; ntap += 3 * 2 * r * (q.cw + q.ch);
        frame_base[k] = nframe;
        nframe += (r * q.cw + 2 * G) * (r * q.ch + 2 * G) - r * q.cw * r * q.ch;
        cov_base[k] = ncov; ncov += q.cw * q.ch;
    }
    n->ntap = ntap;
    std::vector<int> ints;
    const size_t o_crect = ints.size();
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        int v[5] = {q.ci0, q.cj0, q.ci0 + q.cw, q.cj0 + q.ch, ctap[k]};
        ints.insert(ints.end(), v, v + 5);
    }
    const size_t o_frect = ints.size();
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        int v[5] = {G, G, G + r * q.cw, G + r * q.ch, ftap[k]};
        ints.insert(ints.end(), v, v + 5);
    }
    // ring cells: uncovered cells sharing a face with a box, with the faces
    std::map<int, std::vector<int>> faces_of;
    std::vector<int> ring_order;
    auto add_face = [&](int i, int j, int k, int side, int idx) {
        const int c = j * nx + i;
        std::vector<int>& f = faces_of[c];
        if (f.empty()) ring_order.push_back(c);
        f.push_back(k); f.push_back(side); f.push_back(idx);
    };
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        for (int j = 0; j < q.ch; ++j) add_face(q.ci0 - 1, q.cj0 + j, k, 0, j);
        for (int j = 0; j < q.ch; ++j) add_face(q.ci0 + q.cw, q.cj0 + j, k, 1, j);
        for (int i = 0; i < q.cw; ++i) add_face(q.ci0 + i, q.cj0 - 1, k, 2, i);
        for (int i = 0; i < q.cw; ++i) add_face(q.ci0 + i, q.cj0 + q.ch, k, 3, i);
    }
    const int nring = (int)ring_order.size();
    n->nring = nring;
    const size_t o_rcell = ints.size();
    ints.insert(ints.end(), ring_order.begin(), ring_order.end());
    const size_t o_roff = ints.size();
    {
        int off = 0;
        ints.push_back(0);
        for (int c : ring_order) { off += (int)faces_of[c].size() / 3; ints.push_back(off); }
    }
    const size_t o_rface = ints.size();
    for (int c : ring_order) ints.insert(ints.end(), faces_of[c].begin(), faces_of[c].end());
    faces_of.clear();

    const Launcher* L = find_launcher(p->precision, 0, 0, p->limiter);
    if (!L) { set_err("swe_nest_create: no kernel for this precision and limiter"); delete n; return nullptr; }
    const int ntx = (nx + L->tx - 1) / L->tx, nty = (ny + L->ty - 1) / L->ty;
    std::vector<char> forced((size_t)ntx * nty, 0);
    const size_t o_region = ints.size();
    int ncells = 0;
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        const int x0 = std::max(q.ci0 - 2, 0), y0 = std::max(q.cj0 - 2, 0);
        const int x1 = std::min(q.ci0 + q.cw + 2, nx), y1 = std::min(q.cj0 + q.ch + 2, ny);
        int v[5] = {x0, y0, x1, y1, ncells};
        ints.insert(ints.end(), v, v + 5);
        ncells += (x1 - x0) * (y1 - y0);
        for (int tj = y0 / L->ty; tj <= (y1 - 1) / L->ty; ++tj)
            for (int ti = x0 / L->tx; ti <= (x1 - 1) / L->tx; ++ti) forced[(size_t)tj * ntx + ti] = 1;
    }
    n->nregion = npatch;
    n->nregion_cells = ncells;
    const size_t o_force = ints.size();
    for (size_t t = 0; t < forced.size(); ++t)
        if (forced[t]) ints.push_back((int)t);
    n->nforce = (int)(ints.size() - o_force);
    // tiles of each patch holding frame cells: stepped every substep (the
    // frame is rewritten from the coarse grid between substeps), never listed
    std::vector<size_t> o_ring(npatch);
    std::vector<int> n_ring(npatch), ring_bounds(4 * (size_t)npatch);
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        const int nxe = r * q.cw + 2 * G, nye = r * q.ch + 2 * G;
        const int ptx = (nxe + L->tx - 1) / L->tx, pty = (nye + L->ty - 1) / L->ty;
        const int bx0 = (G - 1) / L->tx, bx1 = (nxe - G) / L->tx, by0 = (G - 1) / L->ty, by1 = (nye - G) / L->ty;
        o_ring[k] = ints.size();
        for (int tj = 0; tj < pty; ++tj)
            for (int ti = 0; ti < ptx; ++ti)
                if (ti <= bx0 || ti >= bx1 || tj <= by0 || tj >= by1) ints.push_back(tj * ptx + ti);
        n_ring[k] = (int)(ints.size() - o_ring[k]);
        ring_bounds[4 * k] = bx0; ring_bounds[4 * k + 1] = bx1; ring_bounds[4 * k + 2] = by0; ring_bounds[4 * k + 3] = by1;
    }

    // ---- device buffers
    hipStream_t st = (hipStream_t)p->stream;
    NK(hipMalloc(&n->tap, (size_t)ntap * n->rsize));
    NK(hipMalloc((void**)&n->ints, sizeof(int) * ints.size()));
    NK(hipMalloc(&n->ring_ledger, sizeof(double) * std::max(nring, 1)));
    NK(hipMalloc(&n->desc, (n->precision == 32 ? sizeof(swe::NestPatch<float>) : sizeof(swe::NestPatch<double>)) *
                               npatch));
    n->chunk = 1 << 16;
    n->npart = (int)(((long long)nx * ny + n->chunk - 1) / n->chunk);
    NK(hipMalloc((void**)&n->part, sizeof(double) * n->npart));
    NK(hipMalloc((void**)&n->scalar, sizeof(double)));
    NK(hipMemcpy(n->ints, ints.data(), sizeof(int) * ints.size(), hipMemcpyHostToDevice));
    NK(hipMemset(n->ring_ledger, 0, sizeof(double) * std::max(nring, 1)));
    NK(hipMemset(n->tap, 0, (size_t)ntap * n->rsize));
    n->force_tiles = n->ints + o_force;
    n->region = n->ints + o_region;

    // ---- grids: the coarse grid, then the patches on its stream
    GridExtra cx{1, npatch, n->ints + o_crect, n->tap};
    n->c = create_grid(nx, ny, dx, b, n_M, p, &cx);
    if (!n->c) { std::string m_ = g_err; free_nest(n); delete n; g_err = m_; return nullptr; }
    n->stream = n->c->stream;
    swe_params pp = *p;
    pp.inlet_i0 = pp.inlet_j0 = pp.inlet_ni = pp.inlet_nj = 0;
    pp.q_base = pp.q_peak = 0.0;
    pp.solid = nullptr;
    pp.stream = (void*)n->stream;
    for (int k = 0; k < npatch; ++k) {
        const swe_patch& q = patches[k];
        const int nxe = r * q.cw + 2 * G, nye = r * q.ch + 2 * G, nxf = r * q.cw;
        std::vector<double> H((size_t)nxe * nye, 0.0), Qx(H.size(), 0.0), Qy(H.size(), 0.0);
        for (int j = 0; j < r * q.ch; ++j)
            for (int i = 0; i < nxf; ++i) {
                const size_t src = (size_t)j * nxf + i, dst = (size_t)(j + G) * nxe + i + G;
                if (q.H0) H[dst] = q.H0[src];
                if (q.Qx0) Qx[dst] = q.Qx0[src];
                if (q.Qy0) Qy[dst] = q.Qy0[src];
            }
        pp.H0 = H.data(); pp.Qx0 = Qx.data(); pp.Qy0 = Qy.data();
        GridExtra fx{1, 1, n->ints + o_frect + 5 * k, n->tap, n->ints + o_ring[k], n_ring[k], ring_bounds[4 * k],
                     ring_bounds[4 * k + 1], ring_bounds[4 * k + 2], ring_bounds[4 * k + 3]};
        swe_t* g = create_grid(nxe, nye, dx / r, q.b, q.n_M, &pp, &fx);
        if (!g) { std::string m_ = g_err; free_nest(n); delete n; g_err = m_; return nullptr; }
        n->p.push_back(g);
    }
    n->side.assign(npatch, nullptr);
    n->join.assign(npatch, nullptr);
    NK(hipEventCreateWithFlags(&n->fork, hipEventDisableTiming));
    NK(hipEventCreateWithFlags(&n->frame0, hipEventDisableTiming));
    for (int k = 0; k < npatch; ++k) {
        NK(hipStreamCreateWithFlags(&n->side[k], hipStreamNonBlocking));
        NK(hipEventCreateWithFlags(&n->join[k], hipEventDisableTiming));
    }
    int rc = 0;
    if (n->precision == 32) {
        fill_nest_args<float>(n, nframe, ncov, nring, n->ints + o_rcell, n->ints + o_roff, n->ints + o_rface);
        rc = upload_desc<float>(n, frame_base, cov_base, ftap, ctap);
        if (!rc) rc = nest_init_tau<float>(n);
    } else {
        fill_nest_args<double>(n, nframe, ncov, nring, n->ints + o_rcell, n->ints + o_roff, n->ints + o_rface);
        rc = upload_desc<double>(n, frame_base, cov_base, ftap, ctap);
        if (!rc) rc = nest_init_tau<double>(n);
    }
    if (!rc) rc = nest_finish(n);
    if (rc) { std::string m_ = g_err; free_nest(n); delete n; g_err = m_; return nullptr; }
    (void)st;
    return n;
#undef NK
}

void swe_nest_destroy(swe_nest_t* n) {
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    free_nest(n);
    delete n;
}

int swe_nest_run(swe_nest_t* n, long steps) {
    if (!n || steps < 0) { set_err("swe_nest_run: invalid arguments"); return SWE_EINVAL; }
    long left = steps;
    int rc;
    if (left > 0 && (n->c->launched & 1)) {
        if ((rc = nest_launch(n, 1))) return rc;
        --left;
    }
    if (left >= NEST_GRAPH_STEPS) {
        if ((rc = nest_graph(n))) return rc;
        while (left >= NEST_GRAPH_STEPS) {
            HIPCHK(hipGraphLaunch(n->graph, n->stream));
            n->launched += NEST_GRAPH_STEPS;
            n->c->launched += NEST_GRAPH_STEPS;
            for (swe_t* q : n->p) q->launched += (long long)NEST_GRAPH_STEPS * n->r;
            left -= NEST_GRAPH_STEPS;
        }
    }
    if ((rc = nest_launch(n, left))) return rc;
    return nest_finish(n);
}

int swe_nest_hold_dt(swe_nest_t* n, double tau_c) {
    if (!n || !(tau_c >= 0.0) || !std::isfinite(tau_c)) { set_err("swe_nest_hold_dt: invalid arguments"); return SWE_EINVAL; }
    int rc = nest_finish(n);
    if (rc) return rc;
    if (n->graph) { (void)hipGraphExecDestroy(n->graph); n->graph = nullptr; }
    const int pc = (int)(n->c->launched & 1);
    if (n->precision == 32) {
        swe::NestArgs<float>& na = *(swe::NestArgs<float>*)n->nargs.data();
        na.hold = tau_c;
        hipLaunchKernelGGL(swe::k_nest_set_dt<float>, dim3(1), dim3(64), 0, n->stream,
                           *(const Args<float>*)n->c->args[pc].data(), na, tau_c);
    } else {
        swe::NestArgs<double>& na = *(swe::NestArgs<double>*)n->nargs.data();
        na.hold = tau_c;
        hipLaunchKernelGGL(swe::k_nest_set_dt<double>, dim3(1), dim3(64), 0, n->stream,
                           *(const Args<double>*)n->c->args[pc].data(), na, tau_c);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(n->stream));
    return 0;
}

int swe_nest_run_timed(swe_nest_t* n, long steps, double* kernel_ms) {
    if (!n || steps < 0 || !kernel_ms) { set_err("swe_nest_run_timed: invalid arguments"); return SWE_EINVAL; }
    int rc = timed_launches(n->stream, steps, kernel_ms, [&](hipEvent_t e0, hipEvent_t e1) {
        hipError_t e = hipEventRecord(e0, n->stream);
        if (e == hipSuccess) e = nest_step(n);
        if (e == hipSuccess) e = hipEventRecord(e1, n->stream);
        n->launched++;
        return e;
    });
    if (rc) return rc;
    return nest_finish(n);
}

int swe_nest_query(swe_nest_t* n, double* t, double* volume, double* inflow, double* ledger, long* steps,
                   double* dt_coarse, double* dt_fine) {
    if (!n) { set_err("swe_nest_query: NULL handle"); return SWE_EINVAL; }
    Ctrl c, f;
    int rc = sync_ctrl(n->c, &c);
    if (rc) return rc;
    if ((rc = sync_ctrl(n->p[0], &f))) return rc;
    if (t) *t = c.t;
    if (inflow) *inflow = c.inflow;
    if (steps) *steps = (long)c.step;
    if (dt_coarse) *dt_coarse = c.tau;
    if (dt_fine) *dt_fine = f.tau;
    const int par = (int)(c.step & 1);
    if (volume) {
        const int cells = n->c->nx * n->c->ny;
        if (n->precision == 32)
            hipLaunchKernelGGL(swe::k_field_partials<float>, dim3(n->npart), dim3(256), 0, n->stream,
                               (const float*)n->c->Hb[par], cells, n->chunk, n->part);
        else
            hipLaunchKernelGGL(swe::k_field_partials<double>, dim3(n->npart), dim3(256), 0, n->stream,
                               (const double*)n->c->Hb[par], cells, n->chunk, n->part);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, n->stream, n->part, n->npart, n->scalar);
        HIPCHK(hipGetLastError());
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, n->scalar, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        HIPCHK(hipStreamSynchronize(n->stream));
        *volume = v * n->c->h * n->c->h;
    }
    if (ledger) {
        hipLaunchKernelGGL(swe::k_sum_tiles, dim3(1), dim3(1024), 0, n->stream, n->ring_ledger, n->nring,
                           n->scalar);
        HIPCHK(hipGetLastError());
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, n->scalar, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        HIPCHK(hipStreamSynchronize(n->stream));
        *ledger = v + swe_ledger(n->c);
    }
    return 0;
}

int swe_nest_work(swe_nest_t* n, long long* coarse_cells, long long* fine_cells) {
    if (!n) { set_err("swe_nest_work: NULL handle"); return SWE_EINVAL; }
    Ctrl c;
    int rc = sync_ctrl(n->c, &c);
    if (rc) return rc;
    long long fine = 0;
    for (swe_t* q : n->p) {
        Ctrl f;
        if ((rc = sync_ctrl(q, &f))) return rc;
        fine += f.cells;
    }
    if (coarse_cells) *coarse_cells = c.cells;
    if (fine_cells) *fine_cells = fine;
    return 0;
}

int swe_nest_get_coarse(swe_nest_t* n, double* H, double* Qx, double* Qy) {
    if (!n) { set_err("swe_nest_get_coarse: NULL handle"); return SWE_EINVAL; }
    return swe_get_state(n->c, H, Qx, Qy);
}

int swe_nest_get_patch(swe_nest_t* n, int k, double* H, double* Qx, double* Qy) {
    if (!n || k < 0 || k >= n->np) { set_err("swe_nest_get_patch: invalid arguments"); return SWE_EINVAL; }
    swe_t* g = n->p[k];
    const int G = swe::NEST_FRAME, nxe = g->nx, nxf = nxe - 2 * G, nyf = g->ny - 2 * G;
    std::vector<double> a((size_t)nxe * g->ny), b(a.size()), c(a.size());
    int rc = swe_get_state(g, a.data(), b.data(), c.data());
    if (rc) return rc;
    double* outs[3] = {H, Qx, Qy};
    const std::vector<double>* srcs[3] = {&a, &b, &c};
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        for (int j = 0; j < nyf; ++j)
            std::memcpy(outs[q] + (size_t)j * nxf, srcs[q]->data() + (size_t)(j + G) * nxe + G, sizeof(double) * nxf);
    }
    return 0;
}

}  // extern "C"

// ====================================================================== learned coarse correction

#include "swe_lc.hpp"

struct swe_lc_s {
    int S = 32, So = 33, max_crops = 0;   // grid tile side; network output side S + 1
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float in_scale[6], out_scale[6];
    float* dscale = nullptr;           // device copies: input scales then output scales
    float* params = nullptr;           // packed FP32 master weights and biases
    float* grads = nullptr;
    float* m1 = nullptr;               // Adam moments
    float* m2 = nullptr;
    long long adam_t = 0;
    unsigned short* wf = nullptr;      // bf16 weights [tap][out][in]
    unsigned short* wb = nullptr;      // bf16 weights [tap][in][out]
    unsigned short* act[swe::lc::NL] = {};   // layer inputs (bf16)
    float* out = nullptr;              // last layer output (FP32, 16 channels)
    unsigned short* g[swe::lc::NL] = {};     // dL/dz of each layer (bf16)
    float* y = nullptr;                // labels and mask of a training batch
    float* mask = nullptr;
    float* part = nullptr;             // weight-gradient partials
    int part_blocks = 0;
    double* loss_part = nullptr;
    int loss_blocks = 0;
    int last_n = 0;                    // crops of the last forward
    int fwd_blocks[swe::lc::NL] = {};  // resident workgroups of each forward kernel
    int net_blocks = 0;                // resident workgroups of the fused inference kernel
    // training data set on the device: crops, labels, masks, tile indices
    int cap = 0, count = 0;
    unsigned short* dX = nullptr;
    float* dY = nullptr;
    float* dM = nullptr;
    int* dT = nullptr;
    int* dmc = nullptr;                // mask ones per crop (collection scratch)
    int* idx = nullptr;                // minibatch indices
    std::vector<int> mcount;           // mask ones per data-set crop (host)
};

namespace {

namespace L_ = swe::lc;

int lc_in(const swe_lc_t* c, int l) { return c->So + 2 * L_::HALO - 2 * l; }   // input side of layer l
constexpr int NET_T = 11;     // output block side of the fused inference kernel (a 33-wide crop is 3 x 3 blocks)
constexpr int NET_NTH = 512;  // its threads per workgroup

void free_lc(swe_lc_t* c) {
    void* ptrs[] = {c->params, c->grads, c->m1, c->m2, c->wf, c->wb, c->out, c->y, c->mask, c->part, c->loss_part,
                    c->dscale, c->dX, c->dY, c->dM, c->dT, c->dmc, c->idx};
    for (void* q : ptrs) if (q) (void)hipFree(q);
    for (int l = 0; l < L_::NL; ++l) {
        if (c->act[l]) (void)hipFree(c->act[l]);
        if (c->g[l]) (void)hipFree(c->g[l]);
    }
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

hipError_t lc_pack(swe_lc_t* c) {
    hipLaunchKernelGGL(L_::k_pack_weights, dim3(64), dim3(256), 0, c->stream, c->params, c->wf, c->wb);
    return hipGetLastError();
}

int grid_for(long long items, int per_block) {
    long long b = (items + per_block - 1) / per_block;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// Forward over n crops already in act[0]; the count may come from the device.
// The forward kernels loop over their items with the weights held in
// registers: at most as many workgroups as fit on the chip at once.
hipError_t lc_forward(swe_lc_t* c, int n, const int* cnt_dev, hipStream_t st) {
    const int S = c->S;
    // worst-case items for the grid size: n crops x 16-pixel blocks
    auto items = [&](int l) {
        const int so = lc_in(c, l) - 2;
        const long long it = (long long)n * ((so * so + 15) / 16);
        return it < 4LL * c->fwd_blocks[l] ? it : 4LL * c->fwd_blocks[l];
    };
    hipLaunchKernelGGL((L_::k_conv_fwd<16, 32, false>), dim3(grid_for(items(0), 4)), dim3(256), 0, st,
                       c->act[0], (void*)c->act[1], c->wf + L_::wb_off(0), c->params + L_::p_off(0) + L_::w_count(0),
                       32, lc_in(c, 0), cnt_dev, n);
    hipLaunchKernelGGL((L_::k_conv_fwd<32, 32, false>), dim3(grid_for(items(1), 4)), dim3(256), 0, st,
                       c->act[1], (void*)c->act[2], c->wf + L_::wb_off(1), c->params + L_::p_off(1) + L_::w_count(1),
                       32, lc_in(c, 1), cnt_dev, n);
    hipLaunchKernelGGL((L_::k_conv_fwd<32, 32, false>), dim3(grid_for(items(2), 4)), dim3(256), 0, st,
                       c->act[2], (void*)c->act[3], c->wf + L_::wb_off(2), c->params + L_::p_off(2) + L_::w_count(2),
                       32, lc_in(c, 2), cnt_dev, n);
    hipLaunchKernelGGL((L_::k_conv_fwd<32, 16, true>), dim3(grid_for(items(3), 4)), dim3(256), 0, st,
                       c->act[3], (void*)c->out, c->wf + L_::wb_off(3), c->params + L_::p_off(3) + L_::w_count(3),
                       6, lc_in(c, 3), cnt_dev, n);
    (void)S;
    return hipGetLastError();
}

// Inference only (no activations kept for a backward pass): all four layers
// in one launch when the output side allows blocks of NET_T, else the
// layer-by-layer forward.
hipError_t lc_infer(swe_lc_t* c, int n, const int* cnt_dev, hipStream_t st) {
    if (c->So < NET_T) return lc_forward(c, n, cnt_dev, st);
    const int ns = (c->So + NET_T - 1) / NET_T;
    const long long units = (long long)n * ns * ns;
    const int grid = (int)(units < c->net_blocks ? units : c->net_blocks);
    hipLaunchKernelGGL((L_::k_net_fwd<NET_T, NET_NTH>), dim3(grid > 0 ? grid : 1), dim3(NET_NTH), 0, st, c->act[0], c->out, c->wf,
                       c->params, c->So, cnt_dev, n);
    return hipGetLastError();
}

// Backward of the last forward (n crops) from g[3] (dL/dz of the last layer),
// into the packed FP32 gradient.
hipError_t lc_backward(swe_lc_t* c, int n) {
    hipError_t e;
    auto wgrad = [&](int l) -> hipError_t {
        const int so = lc_in(c, l) - 2;
        const long long total = (long long)n * so * so;
        int chunk = (int)((total + c->part_blocks - 1) / c->part_blocks);
        chunk = (chunk + 15) / 16 * 16;
        const int nblk = (int)((total + chunk - 1) / chunk);
        float* gl = c->grads + L_::p_off(l);
        if (l == 0) {
            hipLaunchKernelGGL((L_::k_conv_bwd_w<16, 32>), dim3(nblk), dim3(256), 0, c->stream, c->g[0], c->act[0],
                               c->part, lc_in(c, 0), n, chunk);
            hipLaunchKernelGGL((L_::k_reduce_w<16, 32>), dim3(32), dim3(256), 0, c->stream, c->part, nblk, gl, 6, 32);
        } else if (l < 3) {
            hipLaunchKernelGGL((L_::k_conv_bwd_w<32, 32>), dim3(nblk), dim3(256), 0, c->stream, c->g[l], c->act[l],
                               c->part, lc_in(c, l), n, chunk);
            hipLaunchKernelGGL((L_::k_reduce_w<32, 32>), dim3(32), dim3(256), 0, c->stream, c->part, nblk, gl, 32, 32);
        } else {
            hipLaunchKernelGGL((L_::k_conv_bwd_w<32, 16>), dim3(nblk), dim3(256), 0, c->stream, c->g[3], c->act[3],
                               c->part, lc_in(c, 3), n, chunk);
            hipLaunchKernelGGL((L_::k_reduce_w<32, 16>), dim3(32), dim3(256), 0, c->stream, c->part, nblk, gl, 32, 6);
        }
        return hipGetLastError();
    };
    auto bdata = [&](int l) -> hipError_t {   // g[l-1] from g[l]
        const int si = lc_in(c, l);
        const long long items = (long long)n * ((si * si + 15) / 16);
        if (l == 3)
            hipLaunchKernelGGL((L_::k_conv_bwd_data<32, 16>), dim3(grid_for(items, 4)), dim3(256), 0, c->stream,
                               c->g[3], c->act[3], c->g[2], c->wb + L_::wb_off(3), si, n);
        else
            hipLaunchKernelGGL((L_::k_conv_bwd_data<32, 32>), dim3(grid_for(items, 4)), dim3(256), 0, c->stream,
                               c->g[l], c->act[l], c->g[l - 1], c->wb + L_::wb_off(l), si, n);
        return hipGetLastError();
    };
    for (int l = 3; l >= 0; --l) {
        if ((e = wgrad(l)) != hipSuccess) return e;
        if (l > 0 && (e = bdata(l)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Host FP64 crops (n, Sin, Sin, 6) -> bf16 act[0] with 16 channels.
int lc_upload_crops(swe_lc_t* c, int n, const double* x) {
    const int si = lc_in(c, 0);
    const size_t npx = (size_t)n * si * si;
    std::vector<unsigned short> h(npx * 16, 0);
    for (size_t p = 0; p < npx; ++p)
        for (int k = 0; k < 6; ++k) {
            const float f = (float)x[p * 6 + k];
            unsigned u;
            std::memcpy(&u, &f, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);
            h[p * 16 + k] = (unsigned short)(u >> 16);
        }
    HIPCHK(hipMemcpyAsync(c->act[0], h.data(), h.size() * 2, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

}  // namespace

extern "C" {

int swe_lc_nparams(void) { return L_::NPARAM; }

swe_lc_t* swe_lc_create(int tile, int max_crops, const double* in_scale, const double* out_scale, void* stream) {
    g_err.clear();
    if (tile < 1 || tile > 64 || max_crops < 1 || max_crops > (1 << 20) || !in_scale || !out_scale) {
        set_err("swe_lc_create: need 1 <= tile <= 64, 1 <= max_crops <= 2^20 and both scale vectors");
        return nullptr;
    }
    for (int k = 0; k < 6; ++k)
        if (!(in_scale[k] > 0.0) || !(out_scale[k] > 0.0) || !std::isfinite(in_scale[k]) ||
            !std::isfinite(out_scale[k])) {
            set_err("swe_lc_create: scales must be finite and > 0"); return nullptr;
        }
    swe_lc_t* c = new (std::nothrow) swe_lc_s();
    if (!c) { set_err("swe_lc_create: out of host memory"); return nullptr; }
    c->S = tile; c->So = tile + 1; c->max_crops = max_crops;
    for (int k = 0; k < 6; ++k) { c->in_scale[k] = (float)in_scale[k]; c->out_scale[k] = (float)out_scale[k]; }
#define LK(expr)                                                               \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) { set_hip_err("swe_lc_create", e_); free_lc(c); delete c; return nullptr; } \
    } while (0)
    if (stream) c->stream = (hipStream_t)stream;
    else { LK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)); c->own_stream = true; }
    {
        int dev = 0, cus = 0;
        LK(hipGetDevice(&dev));
        LK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        int occ[L_::NL] = {};
        LK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], L_::k_conv_fwd<16, 32, false>, 256, 0));
        LK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], L_::k_conv_fwd<32, 32, false>, 256, 0));
        occ[2] = occ[1];
        LK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[3], L_::k_conv_fwd<32, 16, true>, 256, 0));
        for (int l = 0; l < L_::NL; ++l) c->fwd_blocks[l] = cus * (occ[l] > 0 ? occ[l] : 1);
        int on = 0;
        LK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&on, L_::k_net_fwd<NET_T, NET_NTH>, NET_NTH, 0));
        c->net_blocks = cus * (on > 0 ? on : 1);
    }
    LK(hipMalloc((void**)&c->dscale, sizeof(float) * 12));
    {
        float sc[12];
        for (int k = 0; k < 6; ++k) { sc[k] = c->in_scale[k]; sc[6 + k] = c->out_scale[k]; }
        LK(hipMemcpyAsync(c->dscale, sc, sizeof sc, hipMemcpyHostToDevice, c->stream));
        LK(hipStreamSynchronize(c->stream));
    }
    LK(hipMalloc((void**)&c->params, sizeof(float) * L_::NPARAM));
    LK(hipMalloc((void**)&c->grads, sizeof(float) * L_::NPARAM));
    LK(hipMalloc((void**)&c->m1, sizeof(float) * L_::NPARAM));
    LK(hipMalloc((void**)&c->m2, sizeof(float) * L_::NPARAM));
    LK(hipMalloc((void**)&c->wf, 2 * L_::NWB));
    LK(hipMalloc((void**)&c->wb, 2 * L_::NWB));
    for (int l = 0; l < L_::NL; ++l) {
        const size_t si = lc_in(c, l), so = si - 2;
        LK(hipMalloc((void**)&c->act[l], 2 * (size_t)max_crops * si * si * L_::CIN[l]));
        LK(hipMalloc((void**)&c->g[l], 2 * (size_t)max_crops * so * so * L_::COUT[l]));
    }
    LK(hipMalloc((void**)&c->out, sizeof(float) * (size_t)max_crops * c->So * c->So * 16));
    LK(hipMalloc((void**)&c->y, sizeof(float) * (size_t)max_crops * c->So * c->So * 6));
    LK(hipMalloc((void**)&c->mask, sizeof(float) * (size_t)max_crops * c->So * c->So * 6));
    c->part_blocks = 512;
    LK(hipMalloc((void**)&c->part, sizeof(float) * (size_t)c->part_blocks * (9 * 32 * 32 + 32)));
    c->loss_blocks = 256;
    LK(hipMalloc((void**)&c->loss_part, sizeof(double) * c->loss_blocks));
    LK(hipMemsetAsync(c->params, 0, sizeof(float) * L_::NPARAM, c->stream));
    LK(hipMemsetAsync(c->m1, 0, sizeof(float) * L_::NPARAM, c->stream));
    LK(hipMemsetAsync(c->m2, 0, sizeof(float) * L_::NPARAM, c->stream));
    LK(hipMemsetAsync(c->act[0], 0, 2 * (size_t)max_crops * lc_in(c, 0) * lc_in(c, 0) * 16, c->stream));
    LK(lc_pack(c));
    LK(hipStreamSynchronize(c->stream));
#undef LK
    return c;
}

void swe_lc_destroy(swe_lc_t* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_lc(c);
    delete c;
}

int swe_lc_set_params(swe_lc_t* c, const double* params) {
    if (!c || !params) { set_err("swe_lc_set_params: NULL argument"); return SWE_EINVAL; }
    std::vector<float> h(L_::NPARAM);
    for (int k = 0; k < L_::NPARAM; ++k) {
        if (!std::isfinite(params[k])) { set_err("swe_lc_set_params: non-finite parameter"); return SWE_EINVAL; }
        h[k] = (float)params[k];
    }
    HIPCHK(hipMemcpyAsync(c->params, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemsetAsync(c->m1, 0, sizeof(float) * L_::NPARAM, c->stream));
    HIPCHK(hipMemsetAsync(c->m2, 0, sizeof(float) * L_::NPARAM, c->stream));
    c->adam_t = 0;
    HIPCHK(lc_pack(c));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

static int lc_read_floats(swe_lc_t* c, const float* src, double* dst, size_t n) {
    std::vector<float> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < n; ++k) dst[k] = h[k];
    return 0;
}

int swe_lc_get_params(swe_lc_t* c, double* params) {
    if (!c || !params) { set_err("swe_lc_get_params: NULL argument"); return SWE_EINVAL; }
    return lc_read_floats(c, c->params, params, L_::NPARAM);
}

int swe_lc_get_grads(swe_lc_t* c, double* grads) {
    if (!c || !grads) { set_err("swe_lc_get_grads: NULL argument"); return SWE_EINVAL; }
    return lc_read_floats(c, c->grads, grads, L_::NPARAM);
}

int swe_lc_forward(swe_lc_t* c, int n, const double* x, double* out) {
    if (!c || !x || n < 1 || n > c->max_crops) { set_err("swe_lc_forward: invalid arguments"); return SWE_EINVAL; }
    int rc = lc_upload_crops(c, n, x);
    if (rc) return rc;
    HIPCHK(lc_forward(c, n, nullptr, c->stream));
    c->last_n = n;
    if (out) {
        const size_t np = (size_t)n * c->So * c->So;
        std::vector<float> h(np * 16);
        HIPCHK(hipMemcpyAsync(h.data(), c->out, sizeof(float) * h.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (size_t p = 0; p < np; ++p)
            for (int k = 0; k < 6; ++k) out[p * 6 + k] = h[p * 16 + k];
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int swe_lc_infer(swe_lc_t* c, int n, const double* x, double* out) {
    if (!c || !x || !out || n < 1 || n > c->max_crops) { set_err("swe_lc_infer: invalid arguments"); return SWE_EINVAL; }
    int rc = lc_upload_crops(c, n, x);
    if (rc) return rc;
    HIPCHK(lc_infer(c, n, nullptr, c->stream));
    c->last_n = 0;   // the stored activations no longer belong to one forward
    const size_t np = (size_t)n * c->So * c->So;
    std::vector<float> h(np * 16);
    HIPCHK(hipMemcpyAsync(h.data(), c->out, sizeof(float) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t p = 0; p < np; ++p)
        for (int k = 0; k < 6; ++k) out[p * 6 + k] = h[p * 16 + k];
    return 0;
}

int swe_lc_get_layer(swe_lc_t* c, int which, double* out) {
    if (!c || !out || which < 0 || which >= 2 * L_::NL || c->last_n < 1) {
        set_err("swe_lc_get_layer: invalid arguments or no forward yet"); return SWE_EINVAL;
    }
    const int l = which % L_::NL;
    const bool grad = which >= L_::NL;
    const int side = grad ? lc_in(c, l) - 2 : lc_in(c, l);
    const int C = grad ? L_::COUT[l] : L_::CIN[l];
    const int Creal = grad ? L_::COUT_REAL[l] : L_::CIN_REAL[l];
    const size_t np = (size_t)c->last_n * side * side;
    std::vector<unsigned short> h(np * C);
    HIPCHK(hipMemcpyAsync(h.data(), grad ? c->g[l] : c->act[l], 2 * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t p = 0; p < np; ++p)
        for (int k = 0; k < Creal; ++k) {
            const unsigned u = (unsigned)h[p * C + k] << 16;
            float f;
            std::memcpy(&f, &u, 4);
            out[p * Creal + k] = f;
        }
    return 0;
}

int swe_lc_train_step(swe_lc_t* c, int n, const double* x, const double* y, const double* mask, double lr,
                      double* loss) {
    if (!c || !x || !y || !mask || n < 1 || n > c->max_crops || !(lr >= 0.0)) {
        set_err("swe_lc_train_step: invalid arguments"); return SWE_EINVAL;
    }
    int rc = lc_upload_crops(c, n, x);
    if (rc) return rc;
    const size_t np = (size_t)n * c->So * c->So;
    std::vector<float> hy(np * 6), hm(np * 6);
    double cnt = 0.0;
    for (size_t k = 0; k < np * 6; ++k) { hy[k] = (float)y[k]; hm[k] = (float)mask[k]; cnt += mask[k]; }
    HIPCHK(hipMemcpyAsync(c->y, hy.data(), sizeof(float) * hy.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->mask, hm.data(), sizeof(float) * hm.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(lc_forward(c, n, nullptr, c->stream));
    c->last_n = n;
    const float inv = (float)(1.0 / (cnt > 1.0 ? cnt : 1.0));
    hipLaunchKernelGGL(L_::k_loss, dim3(c->loss_blocks), dim3(256), 0, c->stream, c->out, c->y, c->mask, c->g[3],
                       (int)np, inv, c->loss_part);
    HIPCHK(hipGetLastError());
    HIPCHK(lc_backward(c, n));
    if (lr > 0.0) {
        c->adam_t++;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(b1, (double)c->adam_t));
        const float c2 = (float)(1.0 - std::pow(b2, (double)c->adam_t));
        hipLaunchKernelGGL(L_::k_adam, dim3(64), dim3(256), 0, c->stream, c->params, c->grads, c->m1, c->m2,
                           L_::NPARAM, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
        HIPCHK(hipGetLastError());
        HIPCHK(lc_pack(c));
    }
    if (loss) {
        std::vector<double> lp(c->loss_blocks);
        HIPCHK(hipMemcpyAsync(lp.data(), c->loss_part, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double s = 0.0;
        for (double v : lp) s += v;
        *loss = s;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

}  // extern "C"

namespace {

// Before each step of a grid with an attached network: crops of the active
// tiles from the current layer, the network, the corrections of those tiles.
template <typename real>
hipError_t lc_pre_step_t(swe_t* s, int par) {
    swe_lc_t* c = s->lc;
    const Args<real>& a = *(const Args<real>*)s->args[par].data();
    const int S = c->S, So = c->So, Sin = So + 2 * L_::HALO;
    const int slot = par;
    const int nmax = s->ntiles;
    c->last_n = 0;   // the stored activations are not those of one forward
    if (So >= NET_T) {   // gather, network and scatter in one launch
        const int ns = (So + NET_T - 1) / NET_T;
        const long long units = (long long)nmax * ns * ns;
        const int grid = (int)(units < c->net_blocks ? units : c->net_blocks);
        hipLaunchKernelGGL((L_::k_net_grid<NET_T, NET_NTH, real>), dim3(grid > 0 ? grid : 1), dim3(NET_NTH), 0,
                           s->stream, a, slot, S, c->dscale, c->dscale + 6, (real*)s->corrE, (real*)s->corrN, c->wf,
                           c->params, s->claims);
        return hipGetLastError();
    }
    const int* cnt = s->p.skip_dry ? &s->ctrl->seg_off[slot][swe::NSEG] : nullptr;
    hipLaunchKernelGGL(L_::k_gather<real>, dim3(grid_for((long long)nmax * Sin * Sin, 256)), dim3(256), 0, s->stream,
                       a, slot, S, c->dscale, c->act[0], (int*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = lc_forward(c, nmax, cnt, s->stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(L_::k_scatter<real>, dim3(grid_for((long long)nmax * So * So, 256)), dim3(256), 0, s->stream, a,
                       slot, S, c->dscale + 6, c->out, (real*)s->corrE, (real*)s->corrN);
    return hipGetLastError();
}

hipError_t lc_pre_step(swe_t* s, int par) {
    return s->precision == 32 ? lc_pre_step_t<float>(s, par) : lc_pre_step_t<double>(s, par);
}

}  // namespace

extern "C" {

int swe_lc_attach(swe_lc_t* c, swe_t* s) {
    if (!s) { set_err("swe_lc_attach: NULL grid"); return SWE_EINVAL; }
    if (!c) {
        if (s->lc) drop_graph(s);
        s->lc = nullptr;
        s->pre_step = nullptr;
        s->corr = false;
        return 0;
    }
    if (s->field || s->p.sph_displaced || s->p.periodic) {
        set_err("swe_lc_attach: not for a grid with a source rate field, the displaced-particle corrector or a "
                "periodic domain");
        return SWE_EINVAL;
    }
    if (s->L->tx != c->S || s->L->ty != c->S) { set_err("swe_lc_attach: the network's tile differs from the grid's"); return SWE_EINVAL; }
    if (c->max_crops < s->ntiles) { set_err("swe_lc_attach: the network has fewer crop buffers than the grid has tiles"); return SWE_EINVAL; }
    if (!s->L->step_corr || s->ntap > 0) { set_err("swe_lc_attach: grid cannot take corrections"); return SWE_EINVAL; }
    // the network's kernels for this grid run on the grid's stream
    HIPCHK(hipStreamSynchronize(c->stream));
    int rc = ensure_corr_buffers(s);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(s->claims, 0, 2 * sizeof(int), s->stream));   // outside any captured graph
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->lc = c;
    s->pre_step = lc_pre_step;
    s->corr = true;
    return 0;
}

int swe_lc_gather(swe_lc_t* c, swe_t* s, double* x, int* tiles) {
    if (!c || !s || !x) { set_err("swe_lc_gather: NULL argument"); return SWE_EINVAL; }
    if (s->L->tx != c->S || s->L->ty != c->S || c->max_crops < s->ntiles) {
        set_err("swe_lc_gather: network and grid do not fit together"); return SWE_EINVAL;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    Ctrl ct;
    int rc = sync_ctrl(s, &ct);
    if (rc) return rc;
    const int par = (int)(s->launched & 1);
    const int n = s->p.skip_dry ? ct.seg_off[par][swe::NSEG] : s->ntiles;
    const int Sin = c->So + 2 * L_::HALO;
    if (s->precision == 32)
        hipLaunchKernelGGL(L_::k_gather<float>, dim3(grid_for((long long)s->ntiles * Sin * Sin, 256)), dim3(256), 0,
                           s->stream, *(const Args<float>*)s->args[par].data(), par, c->S, c->dscale, c->act[0],
                           (int*)nullptr);
    else
        hipLaunchKernelGGL(L_::k_gather<double>, dim3(grid_for((long long)s->ntiles * Sin * Sin, 256)), dim3(256), 0,
                           s->stream, *(const Args<double>*)s->args[par].data(), par, c->S, c->dscale, c->act[0],
                           (int*)nullptr);
    HIPCHK(hipGetLastError());
    const size_t np = (size_t)n * Sin * Sin;
    std::vector<unsigned short> h(np * 16);
    HIPCHK(hipMemcpyAsync(h.data(), c->act[0], 2 * h.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t p = 0; p < np; ++p)
        for (int k = 0; k < 6; ++k) {
            const unsigned u = (unsigned)h[p * 16 + k] << 16;
            float f;
            std::memcpy(&f, &u, 4);
            x[p * 6 + k] = f;
        }
    if (tiles) {
        if (!s->p.skip_dry) {
            for (int k = 0; k < n; ++k) tiles[k] = k;
        } else {
            int got = 0;
            for (int g = 0; g < swe::NSEG; ++g) {
                const int m = ct.seg_off[par][g + 1] - ct.seg_off[par][g];
                if (m <= 0) continue;
                HIPCHK(hipMemcpyAsync(tiles + got, s->lists + ((size_t)par * swe::NSEG + g) * s->ntiles,
                                      sizeof(int) * m, hipMemcpyDeviceToHost, s->stream));
                got += m;
            }
            HIPCHK(hipStreamSynchronize(s->stream));
            for (int k = 0; k < n; ++k) tiles[k] = swe::entry_tile(tiles[k]);
        }
    }
    return n;
}

}  // extern "C"

namespace {

// One optimisation step on the crops already in act[0], y and mask.
int lc_opt_step(swe_lc_t* c, int n, double cnt, double lr, double* loss) {
    HIPCHK(lc_forward(c, n, nullptr, c->stream));
    c->last_n = n;
    const size_t np = (size_t)n * c->So * c->So;
    const float inv = (float)(1.0 / (cnt > 1.0 ? cnt : 1.0));
    hipLaunchKernelGGL(L_::k_loss, dim3(c->loss_blocks), dim3(256), 0, c->stream, c->out, c->y, c->mask, c->g[3],
                       (int)np, inv, c->loss_part);
    HIPCHK(hipGetLastError());
    HIPCHK(lc_backward(c, n));
    if (lr > 0.0) {
        c->adam_t++;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(b1, (double)c->adam_t));
        const float c2 = (float)(1.0 - std::pow(b2, (double)c->adam_t));
        hipLaunchKernelGGL(L_::k_adam, dim3(64), dim3(256), 0, c->stream, c->params, c->grads, c->m1, c->m2,
                           L_::NPARAM, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
        HIPCHK(hipGetLastError());
        HIPCHK(lc_pack(c));
    }
    if (loss) {
        std::vector<double> lp(c->loss_blocks);
        HIPCHK(hipMemcpyAsync(lp.data(), c->loss_part, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double sum = 0.0;
        for (double v : lp) sum += v;
        *loss = sum;
    }
    return 0;
}

template <typename real>
int lc_collect_t(swe_lc_t* c, swe_t* f, swe_t* g, int r, double tau_c, int n) {
    const int S = c->S, So = c->So;
    const double inv = 1.0 / tau_c;
    hipLaunchKernelGGL(L_::k_labels<real>, dim3(grid_for_cells((long long)n * So * So)), dim3(256), 0, c->stream,
                       c->dT + c->count, n, S, g->ntx, g->nx, g->ny, r, (const real*)f->tapx, (const real*)f->tapy,
                       (const real*)g->tapx, (const real*)g->tapy, inv, c->dscale + 6,
                       c->dY + (size_t)c->count * So * So * 6, c->dM + (size_t)c->count * So * So * 6, c->dmc);
    HIPCHK(hipGetLastError());
    return 0;
}

}  // namespace

extern "C" {

int swe_lc_data(swe_lc_t* c, int capacity) {
    if (!c || capacity < 1) { set_err("swe_lc_data: invalid arguments"); return SWE_EINVAL; }
    void* old[] = {c->dX, c->dY, c->dM, c->dT, c->dmc, c->idx};
    for (void* q : old) if (q) (void)hipFree(q);
    const int So = c->So, Sin = So + 2 * L_::HALO;
    c->cap = capacity;
    c->count = 0;
    c->mcount.clear();
    HIPCHK(hipMalloc((void**)&c->dX, 2 * (size_t)capacity * Sin * Sin * 16));
    HIPCHK(hipMalloc((void**)&c->dY, sizeof(float) * (size_t)capacity * So * So * 6));
    HIPCHK(hipMalloc((void**)&c->dM, sizeof(float) * (size_t)capacity * So * So * 6));
    HIPCHK(hipMalloc((void**)&c->dT, sizeof(int) * (size_t)capacity));
    HIPCHK(hipMalloc((void**)&c->dmc, sizeof(int) * (size_t)capacity));
    HIPCHK(hipMalloc((void**)&c->idx, sizeof(int) * (size_t)c->max_crops));
    HIPCHK(hipMemsetAsync(c->dX, 0, 2 * (size_t)capacity * Sin * Sin * 16, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int swe_lc_data_count(swe_lc_t* c) { return c ? c->count : -1; }

// Put the tile list of a grid's current layer in ascending order as one
// segment.  The set of tiles, and so every result of a step, is unchanged
// (tiles are independent); what becomes reproducible is the order in which
// a gather of the list's crops fills the training set (device appends land
// in the order of their atomics).
static int sort_tile_list(swe_t* s) {
    if (!s->p.skip_dry) return 0;
    Ctrl c;
    int rc = sync_ctrl(s, &c);
    if (rc) return rc;
    const int par = (int)(c.step & 1), n = c.seg_off[par][swe::NSEG];
    if (n <= 1) return 0;
    std::vector<int> t(n);
    rc = swe_active_tiles(s, t.data(), n);
    if (rc < 0) return rc;
    std::sort(t.begin(), t.end());
    int off[swe::NSEG + 1];
    off[0] = 0;
    for (int g = 1; g <= swe::NSEG; ++g) off[g] = n;
    HIPCHK(hipMemcpyAsync(s->lists + (size_t)par * swe::NSEG * s->ntiles, t.data(), sizeof(int) * n,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync((char*)s->ctrl + offsetof(Ctrl, seg_off) + sizeof(int) * (swe::NSEG + 1) * par, off,
                          sizeof off, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return 0;
}

int swe_lc_collect(swe_lc_t* c, swe_t* f, swe_t* g, int r, int m, double* tau_out) {
    if (!c || !f || !g || r < 1 || m < 1 || !c->dX) { set_err("swe_lc_collect: invalid arguments or no data set"); return SWE_EINVAL; }
    if (f->tap_r != r || g->tap_r != 1 || f->precision != g->precision || g->L->tx != c->S || g->L->ty != c->S ||
        c->max_crops < g->ntiles) {
        set_err("swe_lc_collect: fine grid needs line taps r, coarse grid line taps 1, tiles of the network's size");
        return SWE_EINVAL;
    }
    int rc = swe_restrict(f, g, r);   // coarse layer = restricted fine layer, CFL step recorded
    if (rc) return rc;
    if ((rc = sort_tile_list(g))) return rc;   // crops in tile order: a reproducible data set
    Ctrl cf, cg;
    if ((rc = sync_ctrl(f, &cf)) || (rc = sync_ctrl(g, &cg))) return rc;
    double tau_c = std::fmin(cg.tau_cfl, (double)m * cf.tau_cfl);
    if (!(tau_c > 0.0) || !std::isfinite(tau_c)) { set_err("swe_lc_collect: no finite time step"); return SWE_EDTCOLLAPSE; }
    const double tau_f = g->precision == 32 ? (double)(float)(tau_c / m) : tau_c / m;
    tau_c = tau_f * m;
    // crops of the restricted layer
    const int parg = (int)(g->launched & 1);
    const int n = g->p.skip_dry ? cg.seg_off[parg][swe::NSEG] : g->ntiles;
    if (n == 0) { if (tau_out) *tau_out = 0.0; return 0; }
    if (c->count + n > c->cap) { set_err("swe_lc_collect: data set full"); return SWE_ENOMEM; }
    const int S = c->S, Sin = c->So + 2 * L_::HALO;
    unsigned short* xo = c->dX + (size_t)c->count * Sin * Sin * 16;
    if (g->precision == 32)
        hipLaunchKernelGGL(L_::k_gather<float>, dim3(grid_for_cells((long long)n * Sin * Sin)), dim3(256), 0, g->stream,
                           *(const Args<float>*)g->args[parg].data(), parg, S, c->dscale, xo, c->dT + c->count);
    else
        hipLaunchKernelGGL(L_::k_gather<double>, dim3(grid_for_cells((long long)n * Sin * Sin)), dim3(256), 0,
                           g->stream, *(const Args<double>*)g->args[parg].data(), parg, S, c->dscale, xo,
                           c->dT + c->count);
    HIPCHK(hipGetLastError());
    // one coarse step and m fine steps of the same interval, line taps on
    if ((rc = swe_hold_dt(g, tau_c)) || (rc = swe_zero_line_taps(g)) || (rc = launch_steps(g, 1)) ||
        (rc = finish(g)))
        return rc;
    if ((rc = swe_hold_dt(f, tau_f)) || (rc = swe_zero_line_taps(f)) || (rc = launch_steps(f, m)) ||
        (rc = finish(f)) || (rc = swe_hold_dt(f, 0.0)))
        return rc;
    HIPCHK(hipMemsetAsync(c->dmc, 0, sizeof(int) * n, c->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    rc = g->precision == 32 ? lc_collect_t<float>(c, f, g, r, tau_c, n) : lc_collect_t<double>(c, f, g, r, tau_c, n);
    if (rc) return rc;
    std::vector<int> mc(n);
    HIPCHK(hipMemcpyAsync(mc.data(), c->dmc, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->mcount.insert(c->mcount.end(), mc.begin(), mc.end());
    c->count += n;
    if (tau_out) *tau_out = tau_c;
    return 0;
}

int swe_lc_get_data(swe_lc_t* c, int first, int n, double* x, double* y, double* mask, int* tiles) {
    if (!c || first < 0 || n < 0 || first + n > c->count) { set_err("swe_lc_get_data: invalid range"); return SWE_EINVAL; }
    const int So = c->So, Sin = So + 2 * L_::HALO;
    if (x) {
        std::vector<unsigned short> h((size_t)n * Sin * Sin * 16);
        HIPCHK(hipMemcpyAsync(h.data(), c->dX + (size_t)first * Sin * Sin * 16, 2 * h.size(), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (size_t p = 0; p < (size_t)n * Sin * Sin; ++p)
            for (int k = 0; k < 6; ++k) {
                const unsigned u = (unsigned)h[p * 16 + k] << 16;
                float fl;
                std::memcpy(&fl, &u, 4);
                x[p * 6 + k] = fl;
            }
    }
    float* srcs[2] = {c->dY, c->dM};
    double* outs[2] = {y, mask};
    for (int q = 0; q < 2; ++q) {
        if (!outs[q]) continue;
        int rc = lc_read_floats(c, srcs[q] + (size_t)first * So * So * 6, outs[q], (size_t)n * So * So * 6);
        if (rc) return rc;
    }
    if (tiles) {
        HIPCHK(hipMemcpyAsync(tiles, c->dT + first, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return 0;
}

int swe_lc_fit(swe_lc_t* c, int iters, int batch, double lr, unsigned long long seed, double* losses) {
    if (!c || iters < 0 || batch < 1 || batch > c->max_crops || !(lr > 0.0) || c->count < 1) {
        set_err("swe_lc_fit: invalid arguments or empty data set"); return SWE_EINVAL;
    }
    const int So = c->So;
    const int nb = batch < c->count ? batch : c->count;
    std::vector<int> perm(c->count), pick(nb);
    for (int k = 0; k < c->count; ++k) perm[k] = k;
    unsigned long long st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto next = [&]() {   // 64-bit LCG (Knuth's MMIX constants), upper bits
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return (unsigned)(st >> 33);
    };
    for (int it = 0; it < iters; ++it) {
        // partial Fisher-Yates: nb distinct crops
        double cnt = 0.0;
        for (int b = 0; b < nb; ++b) {
            const int j = b + (int)(next() % (unsigned)(c->count - b));
            std::swap(perm[b], perm[j]);
            pick[b] = perm[b];
            cnt += c->mcount[perm[b]];
        }
        HIPCHK(hipMemcpyAsync(c->idx, pick.data(), sizeof(int) * nb, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(L_::k_batch_copy, dim3(2048), dim3(256), 0, c->stream, c->idx, nb, So, c->dX, c->dY, c->dM,
                           c->act[0], c->y, c->mask);
        HIPCHK(hipGetLastError());
        int rc = lc_opt_step(c, nb, cnt, lr, losses ? &losses[it] : nullptr);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int swe_lc_set_out_scale(swe_lc_t* c, const double* out_scale) {
    if (!c || !out_scale) { set_err("swe_lc_set_out_scale: NULL argument"); return SWE_EINVAL; }
    float ratio[6];
    for (int k = 0; k < 6; ++k) {
        if (!(out_scale[k] > 0.0) || !std::isfinite(out_scale[k])) { set_err("swe_lc_set_out_scale: scales must be > 0"); return SWE_EINVAL; }
        ratio[k] = (float)(c->out_scale[k] / out_scale[k]);
        c->out_scale[k] = (float)out_scale[k];
    }
    HIPCHK(hipMemcpyAsync(c->dscale + 6, c->out_scale, sizeof(float) * 6, hipMemcpyHostToDevice, c->stream));
    if (c->count > 0) {
        float* dr = c->out + 0;   // scratch: the output buffer holds at least 6 floats
        HIPCHK(hipMemcpyAsync(dr, ratio, sizeof ratio, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(L_::k_rescale, dim3(2048), dim3(256), 0, c->stream, c->dY,
                           (size_t)c->count * c->So * c->So * 6, (const float*)dr);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------- tile-shape autotuner

namespace {

// Time `nsteps` steps of a freshly built grid or batch after `warmup` steps
// (graph capture happens in the warm-up), with HIP events on its stream.
template <class Run>
int time_steps(hipStream_t st, Run run, int warmup, int nsteps, double* ms) {
    int rc = run(warmup);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e != hipSuccess) { (void)hipEventDestroy(e0); if (e1) (void)hipEventDestroy(e1); set_hip_err("autotune", e); return SWE_EHIP; }
    rc = run(nsteps);
    float f = 0.f;
    if (!rc) {
        e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        if (e != hipSuccess) { set_hip_err("autotune", e); rc = SWE_EHIP; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return rc;
}

// Shapes compiled for a precision and limiter, in table order.
int shapes_of(int precision, int limiter, const Launcher** out, int cap) {
    int n = 0;
    for (const Launcher& l : kLaunchers)
        if (l.precision == precision && l.limiter == limiter && n < cap) out[n++] = &l;
    return n;
}

// Sort the trials by time (best first) into the caller's arrays.
int report_shapes(const Launcher* const* sh, const double* t, int n, int cap, int* tx, int* ty, double* ms) {
    int idx[16];
    for (int k = 0; k < n; ++k) idx[k] = k;
    std::sort(idx, idx + n, [&](int a, int b) { return t[a] < t[b]; });
    for (int k = 0; k < n && k < cap; ++k) {
        tx[k] = sh[idx[k]]->tx;
        ty[k] = sh[idx[k]]->ty;
        if (ms) ms[k] = t[idx[k]];
    }
    return n;
}

}  // namespace

int swe_autotune(int nx, int ny, double dx, const double* b, const double* n_M, const swe_params* p, int warmup,
                 int nsteps, int cap, int* tile_x, int* tile_y, double* ms) {
    g_err.clear();
    if (!p || !b || warmup < 0 || nsteps < 1 || cap < 1 || !tile_x || !tile_y) {
        set_err("swe_autotune: invalid arguments"); return SWE_EINVAL;
    }
    if (p->periodic) { set_err("swe_autotune: a periodic domain runs the default tile shape only"); return SWE_EINVAL; }
    const Launcher* sh[16];
    const int n = shapes_of(p->precision, p->limiter, sh, 16);
    if (n == 0) { set_err("swe_autotune: no tile shape for this precision and limiter"); return SWE_EINVAL; }
    double t[16];
    for (int k = 0; k < n; ++k) {
        swe_params q = *p;
        q.tile_x = sh[k]->tx;
        q.tile_y = sh[k]->ty;
        swe_t* s = swe_create(nx, ny, dx, b, n_M, &q);
        if (!s) return SWE_EINVAL;
        const int rc = time_steps(s->stream, [&](int m) { return m > 0 ? swe_run(s, m) : 0; }, warmup, nsteps, &t[k]);
        swe_destroy(s);
        if (rc) return rc;
    }
    return report_shapes(sh, t, n, cap, tile_x, tile_y, ms);
}

int swe_batch_autotune(int nb, const int* nx, const int* ny, const double* dx, const double* const* b,
                       const double* const* n_M, const swe_params* p, int warmup, int nsteps, int cap, int* tile_x,
                       int* tile_y, double* ms) {
    g_err.clear();
    if (nb < 1 || !p || !nx || !ny || !dx || !b || warmup < 0 || nsteps < 1 || cap < 1 || !tile_x || !tile_y) {
        set_err("swe_batch_autotune: invalid arguments"); return SWE_EINVAL;
    }
    const Launcher* sh[16];
    const int n = shapes_of(p[0].precision, p[0].limiter, sh, 16);
    if (n == 0) { set_err("swe_batch_autotune: no tile shape for this precision and limiter"); return SWE_EINVAL; }
    std::vector<swe_params> q(p, p + nb);
    double t[16];
    for (int k = 0; k < n; ++k) {
        for (swe_params& e : q) { e.tile_x = sh[k]->tx; e.tile_y = sh[k]->ty; }
        swe_batch_t* B = swe_batch_create(nb, nx, ny, dx, b, n_M, q.data());
        if (!B) return SWE_EINVAL;
        const int rc = time_steps(B->stream, [&](int m) { return m > 0 ? swe_batch_run(B, m) : 0; }, warmup, nsteps,
                                  &t[k]);
        swe_batch_destroy(B);
        if (rc) return rc;
    }
    return report_shapes(sh, t, n, cap, tile_x, tile_y, ms);
}

// ---------------------------------------------------------------- step without allocation
//
// One step of a caller-owned layer for callers that cannot allocate (code
// under HIP graph capture, tight serving loops).  The step's bookkeeping --
// control block, completion counters, per-workgroup maxima and cell counts,
// per-tile volume and clamp partials -- lives in `scratch`, a fixed device
// array that every GPU holds for the life of the process.  In host code the
// array's name stands for no device address: its address on each device is
// taken once with hipGetSymbolAddress and only that pointer is passed on.

namespace {

constexpr int NOALLOC_MAX_GRID = 4096;   // workgroups of one step launch
constexpr size_t NOALLOC_CTRL = 0;
constexpr size_t NOALLOC_HOT = 256;
constexpr size_t NOALLOC_MASS = NOALLOC_HOT + sizeof(int) * swe::HOT_INTS;
constexpr size_t NOALLOC_LEDGER = NOALLOC_MASS + sizeof(double) * SWE_NOALLOC_MAX_TILES;
constexpr size_t NOALLOC_BYTES = NOALLOC_LEDGER + sizeof(double) * SWE_NOALLOC_MAX_TILES;
static_assert(sizeof(Ctrl) <= NOALLOC_HOT, "control block must fit its slot");
static_assert(NOALLOC_HOT % 256 == 0 && NOALLOC_MASS % 256 == 0, "counters on 256-byte lines");

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};   // device address of `scratch` per device
int g_noalloc_cus[NOALLOC_MAX_DEV] = {};

// Clear the bookkeeping of one step and set the clock: a kernel, not a
// memset, so the call can be captured in a graph.
__global__ void k_noalloc_init(unsigned char* sc, int ntiles, double t) {
    Ctrl* c = reinterpret_cast<Ctrl*>(sc + NOALLOC_CTRL);
    int* hot = reinterpret_cast<int*>(sc + NOALLOC_HOT);
    double* ledger = reinterpret_cast<double*>(sc + NOALLOC_LEDGER);
    for (int i = threadIdx.x; i < swe::HOT_INTS; i += blockDim.x) hot[i] = 0;
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) ledger[i] = 0.0;
    if (threadIdx.x == 0) {
        Ctrl z{};
        z.t = t;
        *c = z;
    }
}

// Scalars of the step for the caller: t_{n+1}, the step length, the
// hydrograph volume and the clamped volume (fixed-order sum of the partials).
__global__ void k_noalloc_out(const unsigned char* sc, int ntiles, double* out) {
    __shared__ double red[256];
    const double* ledger = reinterpret_cast<const double*>(sc + NOALLOC_LEDGER);
    double s = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) s += ledger[i];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int q = 0; q < (int)blockDim.x; ++q) v += red[q];
        const Ctrl* c = reinterpret_cast<const Ctrl*>(sc + NOALLOC_CTRL);
        out[0] = c->t;
        out[1] = c->last_tau;
        out[2] = c->inflow;
        out[3] = v;
        out[4] = (double)c->err;
    }
}

template <typename real>
void fill_args_noalloc(Args<real>* a, const swe_params& p, int nx, int ny, double dx, int ntx, int nty,
                       const void* b, const void* cf, const void* H, const void* Qx, const void* Qy, void* H1,
                       void* Qx1, void* Qy1, unsigned char* sc) {
    std::memset(a, 0, sizeof *a);
    a->Hi = (const real*)H; a->Qxi = (const real*)Qx; a->Qyi = (const real*)Qy;
    a->Ho = (real*)H1; a->Qxo = (real*)Qx1; a->Qyo = (real*)Qy1;
    a->bed = (const real*)b; a->cf = (const real*)cf;
    a->ctrl = a->lctrl = reinterpret_cast<Ctrl*>(sc + NOALLOC_CTRL);
    a->hot = reinterpret_cast<int*>(sc + NOALLOC_HOT);
    a->mass = reinterpret_cast<double*>(sc + NOALLOC_MASS);
    a->ledger = reinterpret_cast<double*>(sc + NOALLOC_LEDGER);
    a->nx = nx; a->ny = ny; a->ntx = ntx; a->nty = nty; a->ntiles = ntx * nty;
    a->list_cap = ntx * nty;
    a->skip = 0;   // every tile is stepped, so every output cell is written
    a->limiter = p.limiter;
    a->periodic = 0;
    const int nin = p.inlet_ni > 0 && p.inlet_nj > 0 ? p.inlet_ni * p.inlet_nj : 0;
    if (nin > 0) { a->i0 = p.inlet_i0; a->j0 = p.inlet_j0; a->ni = p.inlet_ni; a->nj = p.inlet_nj; }
    a->h = (real)dx; a->ih = (real)(1.0 / dx); a->g = (real)p.g; a->eps = (real)p.eps;
    a->nuh2 = (real)(p.nu / (dx * dx)); a->fcor = (real)p.f_coriolis;
    a->wx = (real)p.wind_x; a->wy = (real)p.wind_y; a->kw = (real)p.wind_kappa; a->hw = (real)p.h_wind;
    a->h_d = dx; a->g_d = p.g; a->cfl = p.cfl; a->tau_max = p.dt_max; a->tau_min = p.dt_min; a->nu_d = p.nu;
    a->nin_h2 = nin > 0 ? (double)nin * dx * dx : 0.0;
    a->q_base = p.q_base; a->q_peak = p.q_peak; a->t_peak = p.t_peak; a->sigma_t = p.sigma_t;
    a->corr_hmin = (real)p.eps;
    a->ring_x0 = -1; a->ring_x1 = 1 << 30; a->ring_y0 = -1; a->ring_y1 = 1 << 30;
}

}  // namespace

extern "C" {

int swe_step_noalloc(int nx, int ny, double dx, const swe_params* p, const void* b, const void* cf,
                     const void* H, const void* Qx, const void* Qy, void* H1, void* Qx1, void* Qy1, double t,
                     double* out) {
    if (nx < 1 || ny < 1 || !(dx > 0.0) || !std::isfinite(dx) || !p || !b || !cf || !H || !Qx || !Qy || !H1 ||
        !Qx1 || !Qy1 || !std::isfinite(t)) {
        set_err("swe_step_noalloc: invalid arguments");
        return SWE_EINVAL;
    }
    if (H1 == H || H1 == Qx || H1 == Qy || Qx1 == H || Qx1 == Qx || Qx1 == Qy || Qy1 == H || Qy1 == Qx ||
        Qy1 == Qy) {
        set_err("swe_step_noalloc: outputs must not alias the inputs");
        return SWE_EINVAL;
    }
    if ((p->precision != 32 && p->precision != 64) || !(p->cfl > 0.0 && p->cfl < 1.0) || !(p->eps > 0.0) ||
        p->limiter < 0 || p->limiter > 2 || p->periodic) {
        set_err("swe_step_noalloc: invalid parameters (walls only)");
        return SWE_EINVAL;
    }
    const Launcher* L = find_launcher(p->precision, 0, 0, p->limiter);
    if (!L || ((p->tile_x || p->tile_y) && (p->tile_x != L->tx || p->tile_y != L->ty))) {
        set_err("swe_step_noalloc: default tile shape only");
        return SWE_EINVAL;
    }
    const int ntx = (nx + L->tx - 1) / L->tx, nty = (ny + L->ty - 1) / L->ty;
    if ((long long)ntx * nty > SWE_NOALLOC_MAX_TILES) {
        set_err("swe_step_noalloc: the grid has more tiles than the fixed scratch holds (SWE_NOALLOC_MAX_TILES)");
        return SWE_EINVAL;
    }
    if (p->inlet_ni > 0 && p->inlet_nj > 0 &&
        (p->inlet_i0 < 0 || p->inlet_j0 < 0 || p->inlet_i0 + p->inlet_ni > nx || p->inlet_j0 + p->inlet_nj > ny)) {
        set_err("swe_step_noalloc: inlet outside the grid");
        return SWE_EINVAL;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) { set_err("swe_step_noalloc: device index out of range"); return SWE_EINVAL; }
    unsigned char* sc;
    int cus;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void* ptr = nullptr;
            HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            int c = 0;
            HIPCHK(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
            g_noalloc_cus[dev] = c;
            g_noalloc_ptr[dev] = (unsigned char*)ptr;
        }
        sc = g_noalloc_ptr[dev];
        cus = g_noalloc_cus[dev];
    }
    int occ = 0;
    if (L->occupancy(&occ) != 0 || occ < 1) occ = 1;
    int grid = cus * occ;
    if (grid < 8) grid = 8;
    if (grid > ntx * nty) grid = ntx * nty;
    if (grid > NOALLOC_MAX_GRID) grid = NOALLOC_MAX_GRID;
    hipStream_t st = (hipStream_t)p->stream;
    constexpr size_t ARGS_BYTES = std::max(sizeof(Args<double>), sizeof(Args<float>));
    alignas(16) unsigned char args[ARGS_BYTES];
    if (p->precision == 32)
        fill_args_noalloc<float>((Args<float>*)args, *p, nx, ny, dx, ntx, nty, b, cf, H, Qx, Qy, H1, Qx1, Qy1, sc);
    else
        fill_args_noalloc<double>((Args<double>*)args, *p, nx, ny, dx, ntx, nty, b, cf, H, Qx, Qy, H1, Qx1, Qy1,
                                  sc);
    hipLaunchKernelGGL(k_noalloc_init, dim3(1), dim3(256), 0, st, sc, ntx * nty, t);
    HIPCHK(hipGetLastError());
    HIPCHK(L->prepare(args, ntx * nty, st));          // CFL step of the layer, volume partials
    HIPCHK(L->prepare_finish(args, st));              // tau, hydrograph volume of the step
    HIPCHK((p->sph_displaced ? L->step_disp : L->step)(args, grid, st, nullptr, nullptr));
    if (out) {
        hipLaunchKernelGGL(k_noalloc_out, dim3(1), dim3(256), 0, st, (const unsigned char*)sc, ntx * nty, out);
        HIPCHK(hipGetLastError());
    }
    return 0;
}

}  // extern "C"
