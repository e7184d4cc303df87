// pond_api.hip -- C ABI of libpond (see include/pond.h): handle lifetime, device
// memory, step scheduling with HIP graphs, error state, readback and timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "pond.h"
#include "pond_eos.h"
#include "pond_handle.h"
#include "pond_internal.h"

using namespace pond;

#define HIP_TRY(h, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return handle_fail((h), POND_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

namespace pond {

int handle_fail(pond_handle *h, int code, const char *fmt, ...)
{
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->msg, sizeof h->msg, fmt, ap);
        va_end(ap);
    }
    return code;
}

// rebuild the step descriptors of a lattice (after allocation or a tile change)
int handle_update_desc(pond_handle *h)
{
    int stx, stc, fcx, fcc;
    tile_counts(h->lc, &stx, &stc, &fcx, &fcc);
    h->st_tiles = stc;
    h->fc_tiles = fcc;
    const int R = h->states();
    for (int p = 0; p < R; ++p) {
        SlotDesc &d = h->desc_h[p];
        std::memset(&d, 0, sizeof d);
        d.P = h->ds.params;
        d.flags = h->ds.flags;
        d.st_tiles_x = stx;
        d.st_begin = 0;
        d.st_count = stc;
        d.fc_tiles_x = fcx;
        d.fc_begin = 0;
        d.fc_count = fcc;
        d.parity = p;
        d.dmom = h->ds.dmom;
        d.kor = h->ds.kor;
        d.aux = h->ds.aux;
        if (h->lc.fused) {
            // the step reads slot p and writes slot p + 1; the collision kernel (check and
            // read-back) reads slot p and writes the read-back state
            d.smom_src = h->ds.ring[p];
            d.smom_dst = h->ds.ring[(p + 1) % R];
            d.mom = (double *)h->ds.ring[p];
            d.pop_dst = h->ds.pop[0];
            d.side_dst = h->ds.side[0];
        } else {
            d.pop_src = h->ds.pop[p];
            d.side_src = h->ds.side[p];
            d.pop_dst = h->ds.pop[1 - p];
            d.side_dst = h->ds.side[1 - p];
            d.mom = h->ds.mom;
        }
    }
    // synchronous: the descriptors are read by work already queued on the stream
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->desc_d, h->desc_h, sizeof(SlotDesc) * R, hipMemcpyHostToDevice));
    return POND_OK;
}

int err_code(int bits)
{
    if (bits & kErrNonfinite) return POND_E_NONFINITE;
    if (bits & kErrPressure) return POND_E_PRESSURE;
    if (bits & kErrHalo) return POND_E_HALO;
    return POND_E_DEVICE;
}

const char *err_name(int bits)
{
    if (bits & kErrNonfinite) return "non-finite state";
    if (bits & kErrPressure) return "state outside the EoS domain (p <= 0, rho <= 0 or 1 - b rho <= 0)";
    if (bits & kErrHalo) return "departure stencil outside the +-2 window (|v| dt >= 1)";
    return "unknown";
}

// Completed steps of a run of nsteps steps that started on state buffer or ring slot `cur`
// of `states`, given its flags.  The launch that raised the first error (launch k reads
// the state of slot (cur + k) mod states) is known from the slot it recorded and from the
// launch counter, which is k or k + 1 (whether that launch's first tile started before
// the error was raised).  Two-kernel steps: the state k launches on is the last good one.
// Fused steps: launch k first recomputes the collision of the state it reads (an error
// there, kErrCollideStage, makes that state bad and the one before it the last good one),
// and the run ends with a check of its last state's closure, counted as launch nsteps.
int completed_steps(const int *fl, int cur, int states, int nsteps)
{
    if (!fl[kFlagErr]) return nsteps;
    const int count = fl[kFlagSteps];
    const int slot = fl[kFlagErrParity] - 1;
    if (slot < 0) return count > 0 ? count - 1 : 0; // not raised by a step kernel
    const int want = ((slot - cur) % states + states) % states;
    const int k = ((count - want) % states + states) % states == 0 ? count : count - 1;
    if (states == kFusedRing && (fl[kFlagErr] & kErrCollideStage)) return k - 1;
    return k;
}

int run_length(const pond_handle *h, int kind)
{
    if (h->lc.fused) return kind ? kFusedRun : kFusedRing;
    return kind ? 2 * kRunPairs : 2;
}

// move the handle to the last completed state of a run of nsteps steps, given its flags
int handle_finish_batch(pond_handle *h, const int *fl, int nsteps)
{
    const int done = completed_steps(fl, h->cur, h->states(), nsteps);
    h->cur = (h->cur + done) % h->states();
    h->steps += done;
    if (fl[kFlagErr]) {
        h->failed = true;
        return handle_fail(h, err_code(fl[kFlagErr]), "step %lld: %s", h->steps + 1, err_name(fl[kFlagErr]));
    }
    return POND_OK;
}

} // namespace pond

namespace {

const double kW1h[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};

// pressure of the configured equation of state (the device helpers' definitions)
double host_p(const pond_config &c, double rho, double T)
{
    if (c.eos == POND_EOS_DIETERICI) return rho * c.R * T / (1.0 - c.b * rho) * std::exp(-c.a * rho / (c.R * T));
    if (c.eos == POND_EOS_DOUBLE_WELL) {
        const double dl = rho - c.eos_c[1], dv = rho - c.eos_c[2];
        return c.eos_c[3] + c.eos_c[0] * dl * dv * (2.0 * rho * (dl + dv) - dl * dv);
    }
    return rho * c.R * T / (1.0 - c.b * rho) - c.a * rho * rho;
}

// equilibrium populations of (rho, u, T) with F = 0 in their own gauge (eqs. 7-8);
// isothermal runs take T0
bool make_ghost(const pond_config &c, const double st[5], GhostFace &G)
{
    const double rho = st[0], T = c.isothermal ? c.T0 : st[4];
    const double u[2] = {st[1], c.dim == 2 ? st[2] : 0.0};
    const double p = host_p(c, rho, T);
    const bool domain = c.eos == POND_EOS_DOUBLE_WELL || 1.0 - c.b * rho > 0.0;
    if (!(rho > 0.0) || !(p > 0.0) || !domain || !std::isfinite(p)) return false;
    const double Cv = c.R / c.delta;
    const double e = c.eos == POND_EOS_DIETERICI ? diet_energy(c.a, c.b, c.R, Cv, rho, T, nullptr)
                                                 : Cv * T - (c.eos == POND_EOS_VDW ? c.a * rho : 0.0);
    const double theta = p / (rho * (1.0 / 3.0));
    const double s = std::sqrt(theta);
    const int Q = c.dim == 2 ? 9 : 3;
    std::memset(&G, 0, sizeof G);
    for (int q = 0; q < Q; ++q) {
        const int cx = c.dim == 2 ? q / 3 - 1 : q - 1;
        const int cy = c.dim == 2 ? q % 3 - 1 : 0;
        const double w = c.dim == 2 ? kW1h[q / 3] * kW1h[q % 3] : kW1h[q];
        const double vx = u[0] + s * cx, vy = u[1] + s * cy;
        G.f[q] = rho * w;
        G.g[q] = rho * w * (2.0 * e - c.dim * p / rho + vx * vx + vy * vy);
    }
    G.ux = u[0];
    G.uy = u[1];
    G.theta = theta;
    G.rho = rho;
    G.T = T;
    G.h = e + p / rho;
    G.mu = (1.0 / c.omega - 0.5) * p * c.dt;
    G.kc = c.k_scale * G.mu * c.R * (1.0 + c.delta) / c.delta;
    return true;
}

// bytes of one population buffer: 2Q planes, plus (FP32 storage) the two sum planes
size_t pop_bytes(int dim, long long N, int fp32)
{
    const int Q = dim == 3 ? 27 : dim == 2 ? 9 : 3;
    return fp32 ? (size_t)N * (2 * Q * sizeof(float) + 2 * sizeof(double)) : (size_t)N * 2 * Q * sizeof(double);
}

// 3D donor-moment scratch: 54 planes, float when the donors are streamed in FP32
size_t dmom_bytes(int dim, long long N, int fp32)
{
    return dim == 3 ? (size_t)N * 54 * (fp32 == 1 ? sizeof(float) : sizeof(double)) : 0;
}

// bytes of one streamed state of the fused step: the moment planes, FP64 or mixed
size_t ring_bytes(int dim, long long N, int fp32)
{
    const int planes = mom_planes(dim), dbl = fp32 ? dim + 2 : planes;
    return (size_t)N * (dbl * sizeof(double) + (planes - dbl) * sizeof(float));
}

// the fused step serves D1Q3 and D2Q9 lattices that do not ask for two kernels
bool fused_step(const pond_config &c) { return c.dim != 3 && !c.two_kernel; }

// device bytes of one lattice of the given shape (all buffers of pond_create)
size_t footprint(int dim, long long N, int fp32, bool fused)
{
    const size_t mon = sizeof(double) * 8 * ((N + 255) / 256) + sizeof(double) * 8;
    const size_t common = (size_t)N * sizeof(double) * (kor_planes(dim) + aux_planes(dim)) + sizeof(int) * kFlagWords +
                          sizeof(DevParams) + kFusedRing * sizeof(SlotDesc) + mon;
    if (fused) // the ring, and one population buffer with its side planes for read-back
        return kFusedRing * ring_bytes(dim, N, fp32) + pop_bytes(dim, N, fp32) +
               (size_t)N * sizeof(double) * side_planes(dim) + common;
    return 2 * pop_bytes(dim, N, fp32) + (size_t)N * sizeof(double) * (2 * side_planes(dim) + mom_planes(dim)) +
           dmom_bytes(dim, N, fp32) + common;
}

int validate(const pond_config *cfg)
{
    if (!cfg) return POND_E_INVALID;
    const pond_config &c = *cfg;
    if (c.dim < 1 || c.dim > 3) return POND_E_INVALID;
    const int nx = c.n[0], ny = c.dim >= 2 ? c.n[1] : 1, nz = c.dim == 3 ? c.n[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz > (1LL << 30)) return POND_E_INVALID;
    // D3Q27: the plane staging of the streaming kernel addresses a field plane with
    // 32-bit byte offsets (N * 8 < 2^32)
    if (c.dim == 3 && (long long)nx * ny * nz > (1LL << 29)) return POND_E_INVALID;
    if (c.dim == 3) // D3Q27: periodic box only
        for (int a = 0; a < 3; ++a)
            for (int s = 0; s < 2; ++s)
                if (c.bc[a][s] != POND_BC_PERIODIC) return POND_E_INVALID;
    if (!(c.delta > 0.0 && c.delta <= 2.0 / 3.0)) return POND_E_INVALID;
    if (!(c.omega > 0.0 && c.omega < 2.0)) return POND_E_INVALID;
    if (c.n_pass < 1 || c.n_pass > 64 || !(c.dt > 0.0) || !(c.R > 0.0)) return POND_E_INVALID;
    if (c.precision != POND_FP64 && c.precision != POND_FP32_STORE && c.precision != POND_FP32_STORE_FP64_MATH)
        return POND_E_INVALID;
    // equation of state: the double-well pressure only isothermally
    if (c.eos < POND_EOS_VDW || c.eos > POND_EOS_DOUBLE_WELL) return POND_E_INVALID;
    if (c.eos == POND_EOS_DOUBLE_WELL && !c.isothermal) return POND_E_INVALID;
    if (c.isothermal && !(c.T0 > 0.0 && std::isfinite(c.T0))) return POND_E_INVALID;
    if (c.eos == POND_EOS_DOUBLE_WELL &&
        !(c.eos_c[0] > 0.0 && c.eos_c[1] > c.eos_c[2] && c.eos_c[2] > 0.0 && c.eos_c[3] > 0.0))
        return POND_E_INVALID;
    if (c.tile < -1 || c.tile >= stream_variants(c.dim)) return POND_E_INVALID;
    if (c.two_kernel != 0 && c.two_kernel != 1) return POND_E_INVALID;
    for (int a = 0; a < c.dim && a < 2; ++a)
        for (int s = 0; s < 2; ++s)
            if (c.bc[a][s] < 0 || c.bc[a][s] > 2) return POND_E_INVALID;
    return POND_OK;
}

// one step from state buffer or ring slot `from`
int enqueue_step(pond_handle *h, hipStream_t st, int from)
{
    LaunchCtx c = h->lc;
    c.st = st;
    if (h->lc.fused) {
        HIP_TRY(h, launch_step_fused(c, h->desc_d + from, 1, h->st_tiles));
        return POND_OK;
    }
    HIP_TRY(h, launch_stream(c, h->desc_d + from, 1, h->st_tiles));
    HIP_TRY(h, launch_force_collide(c, h->desc_d + from, 1, h->fc_tiles));
    return POND_OK;
}

// fused step: the closure check of the state in ring slot `slot` (ends every run of steps)
int enqueue_check(pond_handle *h, int slot)
{
    HIP_TRY(h, launch_collide_check(h->lc, h->desc_d + slot, 1, h->fc_tiles));
    return POND_OK;
}

// record a run of run_length(h, kind) steps starting from state buffer or ring slot
// `from` into an executable graph; the run ends on the slot it starts from
int build_step_graph(pond_handle *h, int kind, int from)
{
    hipGraphExec_t &exec = h->step_exec[kind][from];
    if (exec) return POND_OK;
    // the capture stream is created with the first graph
    if (!h->capture_stream)
        HIP_TRY(h, hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = POND_OK;
    const int R = h->states();
    for (int k = 0; k < run_length(h, kind) && rc == POND_OK; ++k) rc = enqueue_step(h, h->capture_stream, (from + k) % R);
    hipError_t e = hipStreamEndCapture(h->capture_stream, &g);
    if (rc != POND_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return handle_fail(h, POND_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        exec = nullptr;
        return handle_fail(h, POND_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    return POND_OK;
}

// Record every step graph pond_step can use (both run lengths, both buffer parities)
// now, so that no capture or instantiation happens inside a caller's stepping.  A
// failure leaves the handle on direct launches, as a failed capture in pond_step does.
void build_all_graphs(pond_handle *h)
{
    for (int kind = 1; kind >= 0 && h->graphs_ok; --kind)
        for (int from = 0; from < h->states() && h->graphs_ok; ++from)
            if (build_step_graph(h, kind, from) != POND_OK) h->graphs_ok = false;
}

// copy the flags into pinned host memory (a plain DMA, no staging through a bounce
// buffer: this read-back ends every pond_step) and wait for it
int read_flags(pond_handle *h, int out[kFlagWords])
{
    HIP_TRY(h, hipMemcpyAsync(h->flags_host, h->ds.flags, sizeof(int) * kFlagWords, hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::memcpy(out, h->flags_host, sizeof(int) * kFlagWords);
    return POND_OK;
}

int finish_batch(pond_handle *h, int nsteps)
{
    int fl[kFlagWords];
    int rc = read_flags(h, fl);
    if (rc != POND_OK) return rc;
    return handle_finish_batch(h, fl, nsteps);
}

void drop_graphs(pond_handle *h)
{
    for (auto &kind : h->step_exec)
        for (auto &g : kind)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

void free_all(pond_handle *h)
{
    drop_graphs(h);
    for (int i = 0; i < 2; ++i) {
        if (h->ds.pop[i]) (void)hipFree(h->ds.pop[i]);
        if (h->ds.side[i]) (void)hipFree(h->ds.side[i]);
    }
    if (h->ds.mom) (void)hipFree(h->ds.mom);
    if (h->ds.kor) (void)hipFree(h->ds.kor);
    if (h->ds.aux) (void)hipFree(h->ds.aux);
    if (h->ds.dmom) (void)hipFree(h->ds.dmom);
    for (void *r : h->ds.ring)
        if (r) (void)hipFree(r);
    if (h->ds.flags) (void)hipFree(h->ds.flags);
    if (h->ds.params) (void)hipFree(h->ds.params);
    if (h->desc_d) (void)hipFree(h->desc_d);
    if (h->mon_partials) (void)hipFree(h->mon_partials);
    if (h->mon_out) (void)hipFree(h->mon_out);
    if (h->flags_host) (void)hipHostFree(h->flags_host);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

// the kernel whose tile shape is tuned, on the current state: the fused step, or the
// streaming kernel of the two-kernel step; neither changes the current state
hipError_t launch_streaming(const pond_handle *h, const LaunchCtx &c)
{
    return h->lc.fused ? launch_step_fused(c, h->desc_d + h->cur, 1, h->st_tiles)
                       : launch_stream(c, h->desc_d + h->cur, 1, h->st_tiles);
}

// Time every compiled tile shape of the streaming (or fused step) kernel on the current
// state (one warm-up launch, then `reps` launches between HIP events) and keep the fastest.
int tune_stream_tile(pond_handle *h, int reps)
{
    const int nv = stream_variants(h->lc.dim);
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    int best = 0;
    float best_ms = 1e30f;
    int rc = POND_OK;
    for (int v = 0; v < nv && rc == POND_OK; ++v) {
        h->lc.stream_tile = v;
        rc = handle_update_desc(h);
        if (rc != POND_OK) break;
        HIP_TRY(h, launch_streaming(h, h->lc));
        HIP_TRY(h, hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) HIP_TRY(h, launch_streaming(h, h->lc));
        HIP_TRY(h, hipEventRecord(e1, h->stream));
        HIP_TRY(h, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != POND_OK) return rc;
    drop_graphs(h);
    h->lc.stream_tile = best;
    h->tuned = true;
    return handle_update_desc(h);
}

} // namespace

namespace pond {

int config_valid(const pond_config *cfg) { return validate(cfg); }

size_t state_pop_bytes(int dim, long long N, int fp32) { return pop_bytes(dim, N, fp32); }

// device parameter block of a validated configuration; POND_E_INVALID when an inflow
// face's state is outside the EoS domain
int make_params(const pond_config &c, DevParams &P)
{
    const int nx = c.n[0], ny = c.dim >= 2 ? c.n[1] : 1, nz = c.dim == 3 ? c.n[2] : 1;
    std::memset(&P, 0, sizeof P);
    P.dim = c.dim;
    P.nx = nx;
    P.ny = ny;
    P.N = nx * ny * nz;
    for (int a = 0; a < 2; ++a)
        for (int s = 0; s < 2; ++s) P.bc[a][s] = a < c.dim ? c.bc[a][s] : kPeriodic;
    P.n_pass = c.n_pass;
    P.nz = nz;
    P.a = c.a;
    P.b = c.b;
    P.R = c.R;
    P.delta = c.delta;
    P.omega = c.omega;
    P.kappa = c.kappa;
    P.k_scale = c.k_scale;
    P.dt = c.dt;
    P.Cv = c.R / c.delta;
    P.inv_Cv = c.delta / c.R;
    P.Cp_ig = c.R * (1.0 + c.delta) / c.delta;
    P.eos = c.eos;
    P.isothermal = c.isothermal ? 1 : 0;
    P.T0 = c.T0;
    for (int i = 0; i < 4; ++i) P.eos_c[i] = c.eos_c[i];
    for (int a = 0; a < c.dim; ++a)
        for (int s = 0; s < 2; ++s)
            if (c.bc[a][s] == kInflow && !make_ghost(c, c.inflow[a][s], P.ghost[2 * a + s])) return POND_E_INVALID;
    return POND_OK;
}

} // namespace pond

extern "C" {

int pond_footprint(const pond_config *cfg, unsigned long long *bytes)
{
    if (!bytes) return POND_E_INVALID;
    const int rc = validate(cfg);
    if (rc != POND_OK) return rc;
    const long long N = (long long)cfg->n[0] * (cfg->dim >= 2 ? cfg->n[1] : 1) * (cfg->dim == 3 ? cfg->n[2] : 1);
    const int fp32 = cfg->precision == POND_FP64 ? 0 : (cfg->precision == POND_FP32_STORE ? 1 : 2);
    *bytes = footprint(cfg->dim, N, fp32, fused_step(*cfg));
    return POND_OK;
}

int pond_create(const pond_config *cfg, pond_handle **out)
{
    if (!out) return POND_E_INVALID;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != POND_OK) return rc;
    const pond_config &c = *cfg;
    const int nx = c.n[0], ny = c.dim >= 2 ? c.n[1] : 1, nz = c.dim == 3 ? c.n[2] : 1;

    pond_handle *h = new (std::nothrow) pond_handle();
    if (!h) return POND_E_NOMEM;
    h->cfg = c;
    if (c.dim == 1) h->cfg.n[1] = 1;
    if (c.dim < 3) h->cfg.n[2] = 1;
    const int N = nx * ny * nz;
    h->lc = LaunchCtx{c.dim, nx, ny, N, c.precision == POND_FP64 ? 0 : (c.precision == POND_FP32_STORE ? 1 : 2), nullptr,
                      c.tile < 0 ? 0 : c.tile};
    h->lc.nz = nz;
    h->lc.gen_eos = c.eos != POND_EOS_VDW || c.isothermal;
    h->lc.fused = fused_step(c);
    h->tuned = c.tile >= 0 || c.dim == 3;

    DevParams P;
    if (make_params(c, P) != POND_OK) {
        delete h;
        return POND_E_INVALID;
    }

    const size_t popb = pop_bytes(c.dim, N, h->lc.fp32);
    auto alloc = [&](void **p, size_t bytes) {
        if (rc != POND_OK) return;
        if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            rc = handle_fail(h, POND_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
    };
    if (h->lc.fused) {
        // the ring of streamed states, and one collided state for read-back
        for (int i = 0; i < kFusedRing; ++i) alloc(&h->ds.ring[i], ring_bytes(c.dim, N, h->lc.fp32));
        alloc(&h->ds.pop[0], popb);
        alloc((void **)&h->ds.side[0], sizeof(double) * side_planes(c.dim) * N);
    } else {
        for (int i = 0; i < 2; ++i) {
            alloc(&h->ds.pop[i], popb);
            alloc((void **)&h->ds.side[i], sizeof(double) * side_planes(c.dim) * N);
        }
        alloc((void **)&h->ds.mom, sizeof(double) * mom_planes(c.dim) * N);
    }
    alloc((void **)&h->ds.kor, sizeof(double) * kor_planes(c.dim) * N);
    alloc((void **)&h->ds.aux, sizeof(double) * aux_planes(c.dim) * N);
    if (c.dim == 3) alloc(&h->ds.dmom, dmom_bytes(3, N, h->lc.fp32));
    alloc((void **)&h->ds.flags, sizeof(int) * kFlagWords);
    alloc((void **)&h->ds.params, sizeof(DevParams));
    alloc((void **)&h->desc_d, kFusedRing * sizeof(SlotDesc));
    h->mon_blocks = monitor_blocks(h->lc);
    alloc((void **)&h->mon_partials, sizeof(double) * 8 * h->mon_blocks);
    alloc((void **)&h->mon_out, sizeof(double) * 8);
    if (rc == POND_OK && hipHostMalloc((void **)&h->flags_host, sizeof(int) * kFlagWords, hipHostMallocDefault) != hipSuccess) {
        h->flags_host = nullptr;
        rc = handle_fail(h, POND_E_NOMEM, "hipHostMalloc of the flag read-back buffer failed");
    }
    if (rc == POND_OK) {
        if (c.stream) {
            h->stream = (hipStream_t)c.stream;
        } else if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) == hipSuccess) {
            h->own_stream = true;
        } else {
            rc = POND_E_DEVICE;
        }
    }
    if (rc == POND_OK) {
        h->lc.st = h->stream;
        if (hipMemcpy(h->ds.params, &P, sizeof P, hipMemcpyHostToDevice) != hipSuccess) rc = POND_E_DEVICE;
    }
    if (rc == POND_OK && launch_reset_flags(h->lc, h->ds.flags) != hipSuccess) rc = POND_E_DEVICE;
    if (rc == POND_OK) rc = handle_update_desc(h);
    if (rc != POND_OK) {
        free_all(h);
        delete h;
        return rc;
    }
    *out = h;
    return POND_OK;
}

int pond_init_fields(pond_handle *h, const double *rho, const double *u, const double *T)
{
    if (!h) return POND_E_INVALID;
    if (!rho || !u || !T) return handle_fail(h, POND_E_INVALID, "NULL field");
    if (h->batch) return handle_fail(h, POND_E_STATE, "handle is a member of a batch");
    const int N = h->lc.N, dim = h->lc.dim;
    h->initialised = false;
    h->failed = false;
    // stage the inputs in the aux planes: rho | u (dim planes) | T
    double *d_rho = h->ds.aux, *d_u = h->ds.aux + N, *d_T = h->ds.aux + (size_t)(1 + dim) * N;
    HIP_TRY(h, hipMemcpyAsync(d_rho, rho, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(d_u, u, sizeof(double) * N * dim, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(d_T, T, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    if (dim == 3) {
        // the initial state's streamed-state planes, from the staged fields
        HIP_TRY(h, launch_init3(h->lc, h->ds, h->desc_d + 1));
    } else {
        if (h->cfg.kappa != 0.0) HIP_TRY(h, launch_korteweg(h->lc, h->ds, d_rho));
        HIP_TRY(h, launch_init_equilibrium(h->lc, h->ds, d_rho, d_u, d_T, h->lc.fused ? h->ds.ring[0] : h->ds.mom));
    }
    if (h->lc.fused) {
        // the state is ring slot 0; its closure must be admissible
        int rc = enqueue_check(h, 0);
        if (rc != POND_OK) return rc;
    } else {
        // the descriptor of parity 1 writes state 0
        HIP_TRY(h, launch_force_collide(h->lc, h->desc_d + 1, 1, h->fc_tiles));
    }
    int fl[kFlagWords];
    int rc = read_flags(h, fl);
    if (rc != POND_OK) return rc;
    if (fl[kFlagErr]) return handle_fail(h, err_code(fl[kFlagErr]), "init: %s", err_name(fl[kFlagErr]));
    h->cur = 0;
    h->steps = 0;
    if (!h->tuned) {
        rc = tune_stream_tile(h, 10);
        if (rc != POND_OK) return rc;
    }
    // the tuning launches count as started steps: clear the counters again
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    build_all_graphs(h);
    h->initialised = true;
    std::snprintf(h->msg, sizeof h->msg, "ok");
    return POND_OK;
}

int pond_step(pond_handle *h, int nsteps)
{
    if (!h || nsteps < 0) return POND_E_INVALID;
    if (!h->initialised || h->failed)
        return handle_fail(h, POND_E_STATE, h->failed ? "handle in error state" : "not initialised");
    if (h->batch) return handle_fail(h, POND_E_STATE, "handle is a member of a batch");
    if (nsteps == 0) return POND_OK;
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    int slot = h->cur;
    int left = nsteps;
    // long runs, then short runs; each returns to the slot it starts from
    for (int kind = 1; kind >= 0 && h->graphs_ok; --kind) {
        const int len = run_length(h, kind);
        if (left < len) continue;
        if (build_step_graph(h, kind, slot) != POND_OK) {
            h->graphs_ok = false;
            break;
        }
        for (; left >= len; left -= len) HIP_TRY(h, hipGraphLaunch(h->step_exec[kind][slot], h->stream));
    }
    for (; left > 0; --left) {
        int rc = enqueue_step(h, h->stream, slot);
        if (rc != POND_OK) return rc;
        slot = (slot + 1) % h->states();
    }
    if (h->lc.fused) {
        // the last state's closure runs in the next step: check it now
        int rc = enqueue_check(h, slot);
        if (rc != POND_OK) return rc;
    }
    return finish_batch(h, nsteps);
}

// the state buffer holding the collided current state: a fused-step lattice recomputes
// the collision of its ring slot into buffer 0 first
static int readback_state(pond_handle *h, int *buf)
{
    *buf = h->cur;
    if (!h->lc.fused) return POND_OK;
    // flags of an earlier failure would make the collision kernel leave the state alone
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    HIP_TRY(h, launch_force_collide(h->lc, h->desc_d + h->cur, 1, h->fc_tiles));
    *buf = 0;
    return POND_OK;
}

int pond_moments(pond_handle *h, double *rho, double *u, double *T, double *p, double *E)
{
    if (!h) return POND_E_INVALID;
    if (!h->initialised) return handle_fail(h, POND_E_STATE, "not initialised");
    const size_t N = h->lc.N;
    const int dim = h->lc.dim;
    int buf = 0;
    int rc = readback_state(h, &buf);
    if (rc != POND_OK) return rc;
    HIP_TRY(h, launch_macro(h->lc, h->ds, buf, h->ds.aux));
    const double *base = h->ds.aux;
    struct {
        double *dst;
        size_t off, count;
    } parts[] = {{rho, 0, N}, {u, N, N * dim}, {T, (1 + dim) * N, N}, {p, (2 + dim) * N, N},
                 {E, (3 + dim) * N, N}};
    for (auto &pt : parts)
        if (pt.dst)
            HIP_TRY(h, hipMemcpyAsync(pt.dst, base + pt.off, sizeof(double) * pt.count,
                                      hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return POND_OK;
}

int pond_monitors(pond_handle *h, double *out)
{
    if (!h || !out) return POND_E_INVALID;
    if (!h->initialised) return handle_fail(h, POND_E_STATE, "not initialised");
    int buf = 0;
    int rc = readback_state(h, &buf);
    if (rc != POND_OK) return rc;
    HIP_TRY(h, launch_monitors(h->lc, h->ds, buf, h->mon_partials, h->mon_blocks, h->mon_out));
    double tmp[8];
    HIP_TRY(h, hipMemcpyAsync(tmp, h->mon_out, sizeof tmp, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::memcpy(out, tmp, sizeof(double) * (h->lc.dim + 5));
    return POND_OK;
}

int pond_steps_done(const pond_handle *h, long long *out)
{
    if (!h || !out) return POND_E_INVALID;
    *out = h->steps;
    return POND_OK;
}

const char *pond_last_error(const pond_handle *h) { return h ? h->msg : "NULL handle"; }

int pond_tile_info(const pond_handle *h, int *out)
{
    if (!h || !out) return POND_E_INVALID;
    out[0] = h->lc.stream_tile;
    if (h->lc.dim == 3)
        stream3_tile(h->lc.fp32, &out[1], &out[2]);
    else
        stream_tile_shape(h->lc.dim, h->lc.stream_tile, &out[1], &out[2]);
    out[3] = stream_variants(h->lc.dim);
    return POND_OK;
}

int pond_destroy(pond_handle *h)
{
    if (!h) return POND_OK;
    if (h->batch) pond_batch_remove(h->batch, h);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return POND_OK;
}

namespace {
// checkpoint layout: header, then the state: the population buffer and the side planes
// (two-kernel step, D3Q27), or the streamed-state moment planes of the current ring slot
// (fused step; side_bytes is then 0)
struct CheckpointHeader {
    char magic[8];          // "PONDCKP3"
    int dim, n[3], precision, tile, n_pass, eos;
    int bc[3][2];
    long long steps;
    double a, b, R, delta, omega, kappa, k_scale, dt;
    int isothermal, fused;
    double T0, eos_c[4];
    double inflow[3][2][5];
    unsigned long long pop_bytes, side_bytes;
};

CheckpointHeader make_header(const pond_handle *h)
{
    CheckpointHeader H;
    std::memset(&H, 0, sizeof H);
    std::memcpy(H.magic, "PONDCKP3", 8);
    const pond_config &c = h->cfg;
    H.dim = c.dim;
    for (int a = 0; a < 3; ++a) H.n[a] = c.n[a];
    H.precision = c.precision;
    H.tile = h->lc.stream_tile;
    H.n_pass = c.n_pass;
    std::memcpy(H.bc, c.bc, sizeof H.bc);
    H.steps = h->steps;
    H.a = c.a;
    H.b = c.b;
    H.R = c.R;
    H.delta = c.delta;
    H.omega = c.omega;
    H.kappa = c.kappa;
    H.k_scale = c.k_scale;
    H.dt = c.dt;
    H.eos = c.eos;
    H.isothermal = c.isothermal ? 1 : 0;
    H.T0 = c.T0;
    for (int i = 0; i < 4; ++i) H.eos_c[i] = c.eos_c[i];
    std::memcpy(H.inflow, c.inflow, sizeof H.inflow);
    H.fused = h->lc.fused ? 1 : 0;
    H.pop_bytes = h->lc.fused ? ring_bytes(c.dim, h->lc.N, h->lc.fp32) : pop_bytes(c.dim, h->lc.N, h->lc.fp32);
    H.side_bytes = h->lc.fused ? 0 : sizeof(double) * side_planes(h->lc.dim) * (size_t)h->lc.N;
    return H;
}

// same lattice and parameters (tile shape and step count may differ)
bool same_config(const CheckpointHeader &x, const CheckpointHeader &y)
{
    return std::memcmp(x.magic, y.magic, 8) == 0 && x.dim == y.dim && std::memcmp(x.n, y.n, sizeof x.n) == 0 &&
           x.precision == y.precision && x.n_pass == y.n_pass && std::memcmp(x.bc, y.bc, sizeof x.bc) == 0 &&
           x.a == y.a && x.b == y.b && x.R == y.R && x.delta == y.delta && x.omega == y.omega &&
           x.kappa == y.kappa && x.k_scale == y.k_scale && x.dt == y.dt && x.eos == y.eos &&
           x.isothermal == y.isothermal && x.fused == y.fused && x.T0 == y.T0 &&
           std::memcmp(x.eos_c, y.eos_c, sizeof x.eos_c) == 0 &&
           std::memcmp(x.inflow, y.inflow, sizeof x.inflow) == 0 && x.pop_bytes == y.pop_bytes &&
           x.side_bytes == y.side_bytes;
}
} // namespace

int pond_checkpoint_size(const pond_handle *h, unsigned long long *bytes)
{
    if (!h || !bytes) return POND_E_INVALID;
    const CheckpointHeader H = make_header(h);
    *bytes = sizeof H + H.pop_bytes + H.side_bytes;
    return POND_OK;
}

int pond_save(pond_handle *h, void *buf, unsigned long long bytes)
{
    if (!h) return POND_E_INVALID;
    if (!buf) return handle_fail(h, POND_E_INVALID, "NULL buffer");
    if (!h->initialised) return handle_fail(h, POND_E_STATE, "not initialised");
    const CheckpointHeader H = make_header(h);
    if (bytes < sizeof H + H.pop_bytes + H.side_bytes)
        return handle_fail(h, POND_E_INVALID, "checkpoint buffer of %llu bytes, %llu needed", bytes,
                           (unsigned long long)(sizeof H + H.pop_bytes + H.side_bytes));
    char *p = (char *)buf;
    std::memcpy(p, &H, sizeof H);
    const void *state = h->lc.fused ? h->ds.ring[h->cur] : h->ds.pop[h->cur];
    HIP_TRY(h, hipMemcpyAsync(p + sizeof H, state, H.pop_bytes, hipMemcpyDeviceToHost, h->stream));
    if (H.side_bytes)
        HIP_TRY(h, hipMemcpyAsync(p + sizeof H + H.pop_bytes, h->ds.side[h->cur], H.side_bytes, hipMemcpyDeviceToHost,
                                  h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return POND_OK;
}

int pond_load(pond_handle *h, const void *buf, unsigned long long bytes)
{
    if (!h) return POND_E_INVALID;
    if (!buf) return handle_fail(h, POND_E_INVALID, "NULL buffer");
    if (h->batch) return handle_fail(h, POND_E_STATE, "handle is a member of a batch");
    CheckpointHeader S;
    if (bytes < sizeof S) return handle_fail(h, POND_E_INVALID, "buffer shorter than a checkpoint header");
    std::memcpy(&S, buf, sizeof S);
    const CheckpointHeader H = make_header(h);
    if (!same_config(S, H)) return handle_fail(h, POND_E_INVALID, "not a checkpoint of this configuration");
    if (bytes < sizeof S + S.pop_bytes + S.side_bytes)
        return handle_fail(h, POND_E_INVALID, "checkpoint truncated");
    if (S.tile < 0 || S.tile >= stream_variants(h->lc.dim))
        return handle_fail(h, POND_E_INVALID, "checkpoint tile shape out of range");
    const char *p = (const char *)buf;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->lc.fused ? h->ds.ring[0] : h->ds.pop[0], p + sizeof S, S.pop_bytes, hipMemcpyHostToDevice));
    if (S.side_bytes)
        HIP_TRY(h, hipMemcpy(h->ds.side[0], p + sizeof S + S.pop_bytes, S.side_bytes, hipMemcpyHostToDevice));
    if (S.tile != h->lc.stream_tile) {
        drop_graphs(h);
        h->lc.stream_tile = S.tile;
        const int rc = handle_update_desc(h);
        if (rc != POND_OK) return rc;
    }
    h->tuned = true;
    h->cur = 0;
    h->steps = S.steps;
    h->failed = false;
    h->initialised = true;
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    // D3Q27: the donor moments of the loaded state (the descriptor of parity 0 reads it)
    if (h->lc.dim == 3) HIP_TRY(h, launch_donor_moments3(h->lc, h->desc_d));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    build_all_graphs(h);
    std::snprintf(h->msg, sizeof h->msg, "ok");
    return POND_OK;
}

int pond_time_kernel(pond_handle *h, int which, int reps, double *avg_us)
{
    if (!h || !avg_us || reps < 1 || which < 0 || which > 1) return POND_E_INVALID;
    if (!h->initialised || h->failed) return handle_fail(h, POND_E_STATE, "not initialised");
    if (h->batch) return handle_fail(h, POND_E_STATE, "handle is a member of a batch");
    const LaunchCtx &c = h->lc;
    const SlotDesc *d = h->desc_d + h->cur;
    HIP_TRY(h, launch_reset_flags(c, h->ds.flags));
    // two-kernel step: bring the scratch planes to the current step's values first
    if (!c.fused) HIP_TRY(h, launch_stream(c, d, 1, h->st_tiles));
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    HIP_TRY(h, hipEventRecord(e0, h->stream));
    for (int r = 0; r < reps; ++r) {
        hipError_t e = which == 0 ? launch_streaming(h, c)
                                  : (c.fused ? launch_collide_check(c, d, 1, h->fc_tiles)
                                             : launch_force_collide(c, d, 1, h->fc_tiles));
        if (e != hipSuccess) return handle_fail(h, POND_E_DEVICE, "timing launch: %s", hipGetErrorString(e));
    }
    HIP_TRY(h, hipEventRecord(e1, h->stream));
    // D3Q27: the timed collisions overwrote the donor moments; those of the current state
    // again
    if (c.dim == 3 && which == 1) HIP_TRY(h, launch_donor_moments3(c, d));
    HIP_TRY(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_us = 1000.0 * (double)ms / reps;
    int fl[kFlagWords];
    int rc = read_flags(h, fl);
    if (rc != POND_OK) return rc;
    if (fl[kFlagErr]) return handle_fail(h, err_code(fl[kFlagErr]), "timing: %s", err_name(fl[kFlagErr]));
    return POND_OK;
}

int pond_step_timed(pond_handle *h, int nsteps, double *kernel_us)
{
    if (!h || !kernel_us || nsteps < 1) return POND_E_INVALID;
    if (!h->initialised || h->failed)
        return handle_fail(h, POND_E_STATE, h->failed ? "handle in error state" : "not initialised");
    if (h->batch) return handle_fail(h, POND_E_STATE, "handle is a member of a batch");
    HIP_TRY(h, launch_reset_flags(h->lc, h->ds.flags));
    hipEvent_t *ev = (hipEvent_t *)std::calloc((size_t)4 * nsteps, sizeof(hipEvent_t));
    if (!ev) return handle_fail(h, POND_E_NOMEM, "event array");
    int rc = POND_OK;
    int created = 0;
    for (; created < 4 * nsteps; ++created)
        if (hipEventCreate(&ev[created]) != hipSuccess) {
            rc = handle_fail(h, POND_E_DEVICE, "hipEventCreate");
            break;
        }
    int slot = h->cur;
    const bool fused = h->lc.fused;
    for (int i = 0; rc == POND_OK && i < nsteps; ++i) {
        hipEvent_t *e = ev + 4 * i;
        LaunchCtx c1 = h->lc, c2 = h->lc;
        c1.ev_start = e[0];
        c1.ev_stop = e[1];
        c2.ev_start = e[2];
        c2.ev_stop = e[3];
        const hipError_t err = fused ? launch_step_fused(c1, h->desc_d + slot, 1, h->st_tiles)
                                     : (launch_stream(c1, h->desc_d + slot, 1, h->st_tiles) != hipSuccess
                                            ? hipErrorUnknown
                                            : launch_force_collide(c2, h->desc_d + slot, 1, h->fc_tiles));
        if (err != hipSuccess) rc = handle_fail(h, POND_E_DEVICE, "timed step launch");
        slot = (slot + 1) % h->states();
    }
    if (rc == POND_OK && fused) rc = enqueue_check(h, slot);
    if (rc == POND_OK && hipStreamSynchronize(h->stream) != hipSuccess) rc = handle_fail(h, POND_E_DEVICE, "sync");
    double acc[2] = {0.0, 0.0};
    for (int i = 0; rc == POND_OK && i < nsteps; ++i) {
        float a = 0.0f, b = 0.0f;
        if (hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]) != hipSuccess ||
            (!fused && hipEventElapsedTime(&b, ev[4 * i + 2], ev[4 * i + 3]) != hipSuccess))
            rc = handle_fail(h, POND_E_DEVICE, "hipEventElapsedTime");
        acc[0] += a;
        acc[1] += b;
    }
    for (int i = 0; i < created; ++i) (void)hipEventDestroy(ev[i]);
    std::free(ev);
    if (rc != POND_OK) return rc;
    kernel_us[0] = 1000.0 * acc[0] / nsteps;
    kernel_us[1] = 1000.0 * acc[1] / nsteps;
    return finish_batch(h, nsteps);
}

} // extern "C"
