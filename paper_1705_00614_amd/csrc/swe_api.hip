// swe_api.hip -- host side of libswe_hip.so: the C ABI declared in swe.h.
//
// The host validates arguments, owns the device buffers of a handle, and
// launches the step kernel (one launch per CSPH-TVD step, arXiv 1705.00614
// Sec. 2.3) on the caller's stream, replaying captured hipGraphs for long
// runs.  No arithmetic of the scheme runs on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
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
    hipError_t (*step)(const void* args, int grid, hipStream_t st);
    hipError_t (*batch_step)(const void* bargs, int grid, hipStream_t st);
    hipError_t (*batch_prepare_finish)(const void* bargs, hipStream_t st);
    hipError_t (*prepare)(const void* args, int grid, hipStream_t st);
    hipError_t (*prepare_finish)(const void* args, hipStream_t st);
    int (*occupancy)(int* blocks);
};

template <typename real, int TX, int TY, int NT, int LIM>
hipError_t launch_step(const void* args, int grid, hipStream_t st) {
    const Args<real>& a = *static_cast<const Args<real>*>(args);
    hipLaunchKernelGGL((swe::k_step<real, TX, TY, NT, LIM>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}
template <typename real, int TX, int TY, int NT, int LIM>
hipError_t launch_batch_step(const void* bargs, int grid, hipStream_t st) {
    const swe::BatchArgs<real>& b = *static_cast<const swe::BatchArgs<real>*>(bargs);
    hipLaunchKernelGGL((swe::k_batch_step<real, TX, TY, NT, LIM>), dim3(grid), dim3(NT), 0, st, b);
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
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, swe::k_step<real, TX, TY, NT, LIM>, NT, 0) ==
                   hipSuccess ? 0 : -1;
}

#define LAUNCHER(real, TX, TY, NT, P, LIM)                                                       \
    Launcher{TX, TY, NT, P, LIM, launch_step<real, TX, TY, NT, LIM>,                              \
             launch_batch_step<real, TX, TY, NT, LIM>, launch_batch_prepare_finish<real>,         \
             launch_prepare<real, TX, TY, NT>, launch_prepare_finish<real>,                      \
             occupancy<real, TX, TY, NT, LIM>}
#define LAUNCHERS(real, TX, TY, NT, P) \
    LAUNCHER(real, TX, TY, NT, P, 0), LAUNCHER(real, TX, TY, NT, P, 1), LAUNCHER(real, TX, TY, NT, P, 2)

// Tile shapes compiled in, each with the three limiters; the first shape of
// each precision is its default.
const Launcher kLaunchers[] = {
    LAUNCHERS(float, 32, 32, 512, 32),
    LAUNCHERS(float, 64, 16, 512, 32),
    LAUNCHERS(float, 16, 16, 256, 32),
    LAUNCHERS(double, 16, 16, 256, 64),
    LAUNCHERS(double, 32, 16, 256, 64),
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
    int ntx = 0, nty = 0, ntiles = 0, grid = 0;
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
    if (s->graph) hipGraphExecDestroy(s->graph);
    void* ptrs[] = {s->Hb[0], s->Hb[1], s->Qxb[0], s->Qxb[1], s->Qyb[0], s->Qyb[1], s->bed, s->cf,
                    s->ctrl, s->hot, s->lists, s->stamp, s->wg_speed, s->wg_cells, s->mass, s->ledger,
                    s->scalar};
    for (void* q : ptrs)
        if (q) hipFree(q);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
}

int launch_steps(swe_t* s, long n) {
    for (long k = 0; k < n; ++k) {
        const int par = (int)(s->launched & 1);
        HIPCHK(s->L->step(s->args[par].data(), s->grid, s->stream));
        s->launched++;
    }
    return 0;
}

int ensure_graph(swe_t* s) {
    if (s->graph) return 0;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_STEPS; ++k) {
        hipError_t e = s->L->step(s->args[k & 1].data(), s->grid, s->stream);
        if (e != hipSuccess) {
            hipStreamEndCapture(s->stream, &g);
            if (g) hipGraphDestroy(g);
            set_hip_err("graph capture", e);
            return SWE_EHIP;
        }
    }
    HIPCHK(hipStreamEndCapture(s->stream, &g));
    hipError_t e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph = nullptr;
        set_hip_err("graph instantiation", e);
        return SWE_EHIP;
    }
    return 0;
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

}  // namespace

extern "C" {

const char* swe_last_error(void) { return g_err.c_str(); }

swe_t* swe_create(int nx, int ny, double dx, const double* b, const double* n_M, const swe_params* p) {
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
    CK(hipMalloc(&s->wg_speed, sizeof(double) * s->grid));
    CK(hipMalloc((void**)&s->wg_cells, sizeof(long long) * s->grid));

    build_args(s);
    if (set_state_impl(s, p->H0, p->Qx0, p->Qy0, p->solid) != 0) {
        free_all(s); delete s; return nullptr;
    }
    return s;
#undef CK
}

void swe_destroy(swe_t* s) {
    if (!s) return;
    hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
}

int swe_step(swe_t* s) {
    if (!s) { set_err("swe_step: NULL handle"); return SWE_EINVAL; }
    int rc = launch_steps(s, 1);
    if (rc) return rc;
    return finish(s);
}

int swe_run(swe_t* s, long nsteps) {
    if (!s || nsteps < 0) { set_err("swe_run: invalid arguments"); return SWE_EINVAL; }
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
    if ((rc = launch_steps(s, left))) return rc;
    return finish(s);
}

int swe_run_timed(swe_t* s, long nsteps, double* kernel_ms) {
    if (!s || nsteps < 0 || !kernel_ms) { set_err("swe_run_timed: invalid arguments"); return SWE_EINVAL; }
    const long chunk = 256;
    std::vector<hipEvent_t> ev(2 * chunk);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    double total = 0.0;
    long left = nsteps;
    int rc = 0;
    while (left > 0 && rc == 0) {
        const long m = left < chunk ? left : chunk;
        for (long k = 0; k < m; ++k) {
            const int par = (int)(s->launched & 1);
            HIPCHK(hipEventRecord(ev[2 * k], s->stream));
            HIPCHK(s->L->step(s->args[par].data(), s->grid, s->stream));
            HIPCHK(hipEventRecord(ev[2 * k + 1], s->stream));
            s->launched++;
        }
        HIPCHK(hipStreamSynchronize(s->stream));
        for (long k = 0; k < m; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
            total += ms;
        }
        left -= m;
    }
    for (auto& e : ev) hipEventDestroy(e);
    *kernel_ms = total;
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
    // the next source volume depends on the clock: recompute the layer scalars
    s->launched = c.step;
    return prepare(s);
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
        HIPCHK(b->L->batch_step(b->bargs[par].data(), b->grid, b->stream));
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
                hipError_t e = b->L->batch_step(b->bargs[k & 1].data(), b->grid, b->stream);
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
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double total = 0.0;
    for (long k = 0; k < nsteps; ++k) {
        const int par = (int)(b->launched & 1);
        HIPCHK(hipEventRecord(e0, b->stream));
        HIPCHK(b->L->batch_step(b->bargs[par].data(), b->grid, b->stream));
        HIPCHK(hipEventRecord(e1, b->stream));
        b->launched++;
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *kernel_ms = total;
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
