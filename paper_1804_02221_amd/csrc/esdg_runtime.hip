// Host runtime of the C ABI declared in include/esdg.h: argument checks,
// device buffers, the per-step launch sequence and error reporting.  Every
// numerical step runs in the kernels of esdg_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "esdg.h"
#include "esdg_kernels.hpp"
#include "esdg_launch.hpp"
#include "esdg_tables.hpp"

namespace esdg {

// Kernel classes timed by esdg_profile (index of esdg_profile_read_kernels).
constexpr int kProfStage = 0, kProfIndicator = 1, kProfAvFaces = 2, kProfAvDiv = 3, kProfDt = 4,
              kProfAdjoint = 5, kProfClasses = 6;

// Reduce the dt slots: dt[0] = step, dt[1..3] = CFL, viscous, Lemma 2
// bounds; fixed > 0 overrides the step.  Adds the step to *tacc when
// advance.  Resets the slots to +inf.
__global__ void dt_finalize_kernel(unsigned long long *slots_all, double *dt_all, double fixed, int use_pos,
                                   int advance, int *flags)
{
    // workgroup k: instance k (slots [3][kDtSlots], scalars dt[8k..8k+7], time at dt[8k+4])
    unsigned long long *slots = slots_all + (int64_t)blockIdx.x * 3 * kDtSlots;
    double *dt = dt_all + 8 * (int64_t)blockIdx.x;
    double *tacc = dt + 4;
    __shared__ double s[3][kDtSlots];
    const int t = threadIdx.x;
    const unsigned long long inf = 0x7FF0000000000000ull;
    for (int c = 0; c < 3; ++c) {
        s[c][t] = __longlong_as_double((long long)slots[c * kDtSlots + t]);
        slots[c * kDtSlots + t] = inf;
    }
    __syncthreads();
    for (int st = kDtSlots / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < 3; ++c) s[c][t] = fmin(s[c][t], s[c][t + st]);
        __syncthreads();
    }
    if (t == 0) {
        double step = fixed;
        if (!(fixed > 0.0)) {
            step = fmin(s[0][0], s[1][0]);
            if (use_pos) step = fmin(step, s[2][0]);
            if (!(step > 0.0) || !(step < __builtin_huge_val())) {
                atomicOr(&flags[kFlagDtPos], 1);
                step = 0.0;
            }
        }
        dt[0] = step;
        dt[1] = s[0][0];
        dt[2] = s[1][0];
        dt[3] = s[2][0];
        if (advance) tacc[0] += step;
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void fill_int_kernel(int *p, int v, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// The viscous-element list of a state from its element viscosities (count
// zeroed beforehand; the list order does not matter to the viscous passes).
template <typename R>
__global__ void relist_kernel(const R *eps, int32_t *list, int *count, int64_t K)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < K && eps[e] > R(0)) list[atomicAdd(count, 1)] = (int32_t)e;
}

// Step status flags: [0] negative element mean, [1] limited elements,
// [2] no admissible step, [3] J <= 0 at mesh upload (kept), [4] non-finite
// stage output, [5] step above twice the bounds of its result.  Clears all
// but [3].
__global__ void reset_flags_kernel(int *flags)
{
    const int t = threadIdx.x;
    if (t < kNumFlags && t != kFlagBadJ) flags[t] = 0;
}

// A-posteriori check of a step (reading of the remark that the step is
// adjusted when a smaller one is found to be needed, section 6): the dt pass
// has just reduced the CFL and viscous bounds of the state the step produced
// into the slots; a step above kStepBoundFactor times the smaller of the two
// (the factors cfl and cfl_visc are inside the bounds) raises
// kFlagStepBound.  Like dt_finalize_kernel it resets the slots; the step in
// dt[0] is left as it was (a retry halves it).
// One workgroup per instance (slots [instance][3][kDtSlots], step at
// dt[8k]); with iflags (ensembles) the instance's flag gets bit 2.
constexpr double kStepBoundFactor = 2.0;
__global__ void step_check_kernel(unsigned long long *slots_all, double *dt_all, int *flags, int *iflags)
{
    __shared__ double s[2][kDtSlots];
    unsigned long long *slots = slots_all + (int64_t)blockIdx.x * 3 * kDtSlots;
    const double *dt = dt_all + 8 * (int64_t)blockIdx.x;
    const int t = threadIdx.x;
    const unsigned long long inf = 0x7FF0000000000000ull;
    for (int c = 0; c < 2; ++c) s[c][t] = __longlong_as_double((long long)slots[c * kDtSlots + t]);
    for (int c = 0; c < 3; ++c) slots[c * kDtSlots + t] = inf;
    __syncthreads();
    for (int st = kDtSlots / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < 2; ++c) s[c][t] = fmin(s[c][t], s[c][t + st]);
        __syncthreads();
    }
    if (t == 0 && dt[0] > kStepBoundFactor * fmin(s[0][0], s[1][0])) {
        atomicOr(&flags[kFlagStepBound], 1);
        if (iflags) atomicOr(&iflags[blockIdx.x], 2);
    }
}

// Ensemble retry support: step <- f * step for the instances k with mask[k],
// their time corrected by the removed part.
__global__ void scale_steps_masked_kernel(double *dt_all, const int *mask, double f, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && mask[k]) {
        double *dt = dt_all + 8 * (int64_t)k;
        const double old = dt[0];
        dt[0] = old * f;
        dt[4] -= old * (1.0 - f);
    }
}

// Retry support: step <- f * step, time corrected by the removed part.
__global__ void scale_step_kernel(double *dt, double f, double *tacc)
{
    if (threadIdx.x == 0) {
        const double old = dt[0];
        dt[0] = old * f;
        tacc[0] -= old * (1.0 - f);
    }
}

// p[8k] = v for the n instances k (times live at dscal[8k + 4]).
__global__ void set_scalar_kernel(double *p, double v, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[8 * k] = v;
}

// Element permutation between the caller's order and the internal
// locality order: internal element e holds the caller's element perm[e].
template <typename A, typename B>
__global__ void gather_kernel(const A *__restrict__ src, B *__restrict__ dst, const int32_t *__restrict__ perm,
                              int64_t K, int np)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * np) return;
    const int64_t e = q / np;
    dst[q] = (B)src[(int64_t)perm[e] * np + (q - e * np)];
}

template <typename A, typename B>
__global__ void scatter_kernel(const A *__restrict__ src, B *__restrict__ dst, const int32_t *__restrict__ perm,
                               int64_t K, int np)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * np) return;
    const int64_t e = q / np;
    dst[(int64_t)perm[e] * np + (q - e * np)] = (B)src[q];
}

// Metric terms in the ABI's layout and order: x_xi, x_eta, y_xi, y_eta, J (float64).
template <typename R>
__global__ void geometry_out_kernel(const R *Ax, const R *Cx, const R *Ae, const R *Ce, const R *mref, double *out,
                                    const int32_t *perm, int64_t K, int np)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = K * np;
    if (q >= n) return;
    const int64_t e = q / np;
    const int64_t o = (int64_t)perm[e] * np + (q - e * np);
    // (single precision: the stored terms less the element's reference)
    R rax = Ax[q], rcx = Cx[q], rae = Ae[q], rce = Ce[q];
    if (mref) { rax += mref[4 * e]; rcx += mref[4 * e + 1]; rae += mref[4 * e + 2]; rce += mref[4 * e + 3]; }
    const double ax = rax, cx = rcx, ae = rae, ce = rce;
    out[o] = ce;             // x_xi
    out[n + o] = -cx;        // x_eta
    out[2 * n + o] = -ae;    // y_xi
    out[3 * n + o] = ax;     // y_eta
    out[4 * n + o] = ce * ax - cx * ae;
}

// Diagnostics without allocation (esdg_diagnostics_noalloc): the
// per-workgroup partial rows of diag_kernel go to a fixed array of the
// library, `scratch`, one copy per GPU, instead of the context's buffer;
// row kScratchRows receives the final sums.  Host code never passes the
// array's name to a kernel or copy: it uses the device address that
// hipGetSymbolAddress returns for the current GPU (scratch_ptr below).
constexpr int64_t kScratchRows = 65536;   // 65536 x 8 doubles = 4 MiB
static __device__ __align__(256) double scratch[(kScratchRows + 1) * 8];

// Sums the nb partial rows in row order, as the host loop of
// esdg_diagnostics does (the same operations in the same order, so the
// results are bitwise those of that loop): columns 0-4 and 7 are sums,
// 5 a minimum, 6 a maximum.  One lane per column.
__global__ void diag_reduce_kernel(const double *__restrict__ part, int64_t nb, double *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= 8) return;
    double acc = c == 5 ? __builtin_huge_val() : (c == 6 ? -__builtin_huge_val() : 0.0);
#pragma unroll 8
    for (int64_t b = 0; b < nb; ++b) {
        const double v = part[b * 8 + c];
        acc = c == 5 ? fmin(acc, v) : (c == 6 ? fmax(acc, v) : acc + v);
    }
    out[c] = acc;
}

}  // namespace esdg

using namespace esdg;

namespace {

// Device address of `scratch` on each GPU, looked up once per device (with
// that device current) by esdg_create.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t lookup_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
    return hipSuccess;
}

double *scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

struct esdg_ctx {
    int device = 0;
    int prec = 64;
    hipStream_t stream = nullptr;
    esdg_params P{};
    Bufs B;
    int N = 0;
    int64_t K = 0;
    bool have_mesh = false, have_b = false, have_state = false;
    int cur = 0;
    bool eps_valid[3] = {false, false, false};   // viscosity/list of state buffer b are current
    int dtb_buf = -1;   // state buffer whose per-element dt bounds are in dtc/dtv (-1: none)
    int stage_variant = 0;   // compiled stage-kernel variant (esdg_autotune)
    bool masked_attempt = false;  // stage launches cover only the instances set in B.imask
    // Executable graphs of one time step (esdg_step), one per start buffer:
    // the kernel sequence of a step is fixed once the viscosity of the start
    // state and (adaptive step) its dt bounds are current.  A graph is valid
    // for its start buffer, fixed step (0: adaptive), variant and generation;
    // the generation changes with anything captured by value (parameters,
    // tables, variant) or by address (buffers).
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        double dt = 0.0;
        int variant = -1;
        uint64_t gen = 0;
    } graphs[3];
    uint64_t graph_gen = 1;
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;   // private stream the graphs are captured on
    hipEvent_t tune_ev[2] = {nullptr, nullptr};   // the autotuner's own timing events
    int64_t last_limited = 0;   // limited element-stages of the last esdg_step call
    // instances (ensembles): element ranges [inst_off[k], inst_off[k+1]) in
    // the caller's order and, since the locality order permutes inside each
    // range, in the internal order too
    std::vector<int64_t> inst_off{0, 0};
    HostTables ht{};
    Tab<double> td{};
    Tab<float> tf{};
    double *stage_d = nullptr;   // float64 staging [5][n] (conversions, geometry output)
    int32_t *perm = nullptr;     // [K] caller's element of each internal element
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    // timed launches per kernel class (kProf*) and their drained totals
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_log[kProfClasses];
    size_t ev_next = 0;
    double acc_ms[kProfClasses] = {};
    int64_t acc_n[kProfClasses] = {};
    std::string err = "no error";
    std::vector<int32_t> inv_h;   // caller's element -> internal element
    uint64_t b_version = 0;       // bumped by every esdg_set_bathymetry
    // discrete adjoint (gauges, checkpoints, cotangent fields)
    struct Adjoint {
        int ng = 0;
        int32_t *gel = nullptr;    // [ng] internal element of each gauge
        double *gw = nullptr;      // [ng][np] Lagrange weights of each gauge point
        int nu = 0;                // elements holding gauges
        int32_t *ug = nullptr;     // [nu] those elements, [nu + 1] offsets, [ng] gauges sorted by element
        double *gH = nullptr;      // [ng] scratch for esdg_gauge_values
        double *lam = nullptr;     // [4][3][n]: dL/dW (two buffers), dL/d(register) (two buffers)
        double *gbf = nullptr;     // [4][n]: cotangents of b_x, b_y, face b; assembled dL/db
        double *ckpt = nullptr;    // [ckpt_cap][3][n] states at the checkpoints
        int64_t ckpt_cap = 0;
        double *store = nullptr;   // [store_cap][3][n] stage inputs of one segment
        int64_t store_cap = 0;
        double *Hg = nullptr, *Tg = nullptr;   // [nsteps][ng] gauge values and target
        int64_t h_cap = 0;
        double *loss = nullptr;    // [1]
        int nsteps = 0, every = 0;
        double dt = 0.0;
        bool ready = false;        // a forward sweep is recorded
        uint64_t b_version = 0;
        esdg_params P{};           // the parameters of the recorded sweep
    } adj;
};

namespace {

// SSPRK(3,3) in the Shu-Osher form of eq. RKSSP:
// W_k = alpha_k W^n + beta_k (W_{k-1} + dt R(W_{k-1}))
constexpr double kSspAlpha[3] = {0.0, 0.75, 1.0 / 3.0};
constexpr double kSspBeta[3] = {1.0, 0.25, 2.0 / 3.0};

int fail(esdg_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define CK(expr)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, ESDG_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                   \
    } while (0)

#define TRY(expr)               \
    do {                        \
        int st_ = (expr);       \
        if (st_) return st_;    \
    } while (0)

int64_t nodes(const esdg_ctx *c) { return c->K * (int64_t)(c->N + 1) * (c->N + 1); }
int n_inst(const esdg_ctx *c) { return (int)c->inst_off.size() - 1; }
size_t rsz(const esdg_ctx *c) { return c->prec == 64 ? sizeof(double) : sizeof(float); }

template <typename R>
Phys<R> phys(const esdg_ctx *c)
{
    Phys<R> p;
    p.g = (R)c->P.g;
    p.h_tol = (R)c->P.h_tol;
    p.eps0 = (R)c->P.eps0;
    p.sigma_min = (R)c->P.sigma_min;
    p.sigma_max = (R)c->P.sigma_max;
    p.cfl = (R)c->P.cfl;
    p.cfl_visc = (R)c->P.cfl_visc;
    p.i2g = (R)(0.5 / c->P.g);
    p.ratio_min = (R)std::pow(10.0, c->P.sigma_min);
    p.ratio_max = (R)std::pow(10.0, c->P.sigma_max);
    p.visc_c = (R)(c->P.cfl_visc * 4.0 * kLsrkRealLimit);
    p.br1 = (c->N >= 2 && c->N <= 8) ? (R)kBR1Radius[c->N] : R(1);
    p.ec = c->P.surface_flux == 1;
    p.limiter_on = c->P.limiter_on != 0;
    return p;
}

template <typename R>
const Tab<R> &tab(const esdg_ctx *c);
template <>
const Tab<double> &tab<double>(const esdg_ctx *c) { return c->td; }
template <>
const Tab<float> &tab<float>(const esdg_ctx *c) { return c->tf; }

// Call f(Launch<N,R>{}, R{}) for the context's degree and precision.
template <typename F>
hipError_t dispatch(const esdg_ctx *c, F &&f)
{
#define ESDG_CASE(n)                                                        \
    case n:                                                                 \
        return c->prec == 64 ? f(Launch<n, double>{}, double{}) : f(Launch<n, float>{}, float{});
    switch (c->N) {
        ESDG_CASE(2)
        ESDG_CASE(3)
        ESDG_CASE(4)
        ESDG_CASE(5)
        ESDG_CASE(6)
        ESDG_CASE(7)
        ESDG_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
#undef ESDG_CASE
}

void free_bufs(esdg_ctx *c)
{
    // the step graphs hold the buffers' addresses
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = esdg_ctx::StepGraph{};
    }
    ++c->graph_gen;
    Bufs &B = c->B;
    void *ps[] = {B.x, B.y, B.xr, B.yr, B.mref, B.Ax, B.Cx, B.Ae, B.Ce, B.bx, B.by, B.bface, B.b, B.nbr, B.code, B.count,
                  B.vtr, B.gmax, B.dtc, B.dtv, B.fgeo, B.frec, B.tabg, B.lv[0], B.lv[1], B.dscal, B.slots, B.flags, B.part, c->stage_d,
                  B.eps[0], B.eps[1], B.eps[2], B.list[0], B.list[1], B.list[2], B.inst, B.cstart, B.cinst,
                  B.iflags, B.imask};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    for (auto &w : B.W)
        for (void *p : w)
            if (p) (void)hipFree(p);
    for (void *p : B.dU)
        if (p) (void)hipFree(p);
    for (void *p : B.Rb)
        if (p) (void)hipFree(p);
    B = Bufs{};
    {
        auto &A = c->adj;
        void *qs[] = {A.gel, A.gw, A.ug, A.gH, A.lam, A.gbf, A.ckpt, A.store, A.Hg, A.Tg, A.loss};
        for (void *p : qs)
            if (p) (void)hipFree(p);
        A = esdg_ctx::Adjoint{};
    }
    if (c->perm) (void)hipFree(c->perm);
    c->perm = nullptr;
    c->stage_d = nullptr;
    c->have_mesh = c->have_b = c->have_state = false;
    c->inst_off = {0, 0};
}

hipEvent_t next_event(esdg_ctx *c)
{
    if (c->ev_next == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_next++];
}

// Launch with optional timing: the events are recorded by the kernel
// dispatch itself (no marker packets between kernels).
template <typename F>
int timed(esdg_ctx *ctx, int cls, F &&launch)
{
    auto &log = ctx->ev_log[cls];
    Ev ev;
    if (ctx->prof) {
        ev.a = next_event(ctx);
        ev.b = next_event(ctx);
        if (!ev.a || !ev.b) return fail(ctx, ESDG_EHIP, "hipEventCreate failed");
    }
    CK(launch(ev));
    if (ctx->prof) log.emplace_back(ev.a, ev.b);
    return ESDG_OK;
}

// Derived per-state data (viscosity, viscous list, dt bounds) is stale.
void invalidate_eps(esdg_ctx *ctx)
{
    for (bool &v : ctx->eps_valid) v = false;
    ctx->dtb_buf = -1;
}

// Element viscosity and viscous-element list of state buffer buf, when stale
// (the stage kernel keeps them current for the states it writes).
int ensure_eps(esdg_ctx *ctx, int buf)
{
    if (ctx->eps_valid[buf]) return ESDG_OK;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.count + buf, 0, 1);
    CK(hipGetLastError());
    TRY(timed(ctx, kProfIndicator, [&](Ev ev) {
        return dispatch(ctx, [&](auto L, auto r) {
            using R = decltype(r);
            return decltype(L)::indicator(ctx->B, buf, phys<R>(ctx), tab<R>(ctx), ctx->stream, ev);
        });
    }));
    ctx->eps_valid[buf] = true;
    return ESDG_OK;
}

// Viscous terms of the listed elements of state buffer buf (both passes);
// reset >= 0 zeroes that buffer's list counter for the stage about to run.
int launch_viscous(esdg_ctx *ctx, int buf, int reset)
{
    TRY(ensure_eps(ctx, buf));
    TRY(timed(ctx, kProfAvFaces, [&](Ev ev) {
        return dispatch(ctx, [&](auto L, auto r) {
            using R = decltype(r);
            return decltype(L)::av_faces(ctx->B, buf, phys<R>(ctx), tab<R>(ctx), ctx->stream, ev);
        });
    }));
    return timed(ctx, kProfAvDiv, [&](Ev ev) {
        return dispatch(ctx, [&](auto L, auto r) {
            using R = decltype(r);
            return decltype(L)::av_div(ctx->B, buf, reset, phys<R>(ctx), tab<R>(ctx), ctx->stream, ev);
        });
    });
}

int launch_stage(esdg_ctx *ctx, StageCall sc)
{
    sc.variant = ctx->stage_variant;
    sc.masked = ctx->masked_attempt;
    return timed(ctx, kProfStage, [&](Ev ev) {
        return dispatch(ctx, [&](auto L, auto r) {
            using R = decltype(r);
            return decltype(L)::stage(ctx->B, sc, phys<R>(ctx), tab<R>(ctx), ctx->stream, ev);
        });
    });
}

// Time step of state buffer buf (fixed > 0: that step) for every instance;
// the bounds the last stage left for buf are used when current.
int launch_dt(esdg_ctx *ctx, int buf, double fixed, int advance)
{
    const bool av = ctx->P.av_on != 0;
    if (!(fixed > 0.0)) {
        const bool fused = ctx->dtb_buf == buf;
        if (av && !fused) TRY(ensure_eps(ctx, buf));
        TRY(timed(ctx, kProfDt, [&](Ev ev) {
            return dispatch(ctx, [&](auto L, auto r) {
                using R = decltype(r);
                return decltype(L)::dt(ctx->B, buf, av, fused, phys<R>(ctx), ctx->stream, ev);
            });
        }));
    }
    hipLaunchKernelGGL(dt_finalize_kernel, dim3(n_inst(ctx)), dim3(kDtSlots), 0, ctx->stream, ctx->B.slots,
                       ctx->B.dscal, fixed, ctx->P.limiter_on ? 1 : 0, advance, ctx->B.flags);
    CK(hipGetLastError());
    return ESDG_OK;
}

int reset_flags(esdg_ctx *ctx)
{
    hipLaunchKernelGGL(reset_flags_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.flags);
    CK(hipGetLastError());
    return ESDG_OK;
}

int read_flags(esdg_ctx *ctx, int flags[kNumFlags])
{
    CK(hipMemcpyAsync(flags, ctx->B.flags, kNumFlags * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

// Copy a float64 host/device array in the caller's element order into a
// context array (compute precision, internal order); per = values per element.
int upload_field(esdg_ctx *ctx, void *dst, const double *src, int64_t per, int mem)
{
    const int64_t n = ctx->K * per;
    const double *s = src;
    if (!mem) {
        CK(hipMemcpyAsync(ctx->stage_d, src, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        s = ctx->stage_d;
    }
    const unsigned g = (unsigned)((n + 255) / 256);
    if (ctx->prec == 64)
        hipLaunchKernelGGL((gather_kernel<double, double>), dim3(g), dim3(256), 0, ctx->stream, s,
                           (double *)dst, ctx->perm, ctx->K, (int)per);
    else
        hipLaunchKernelGGL((gather_kernel<double, float>), dim3(g), dim3(256), 0, ctx->stream, s,
                           (float *)dst, ctx->perm, ctx->K, (int)per);
    CK(hipGetLastError());
    if (!mem) CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

// Copy a context array out into a float64 host/device array in the caller's order.
int download_field(esdg_ctx *ctx, double *dst, const void *src, int64_t per, int mem)
{
    const int64_t n = ctx->K * per;
    double *d = mem ? dst : ctx->stage_d;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (ctx->prec == 64)
        hipLaunchKernelGGL((scatter_kernel<double, double>), dim3(g), dim3(256), 0, ctx->stream,
                           (const double *)src, d, ctx->perm, ctx->K, (int)per);
    else
        hipLaunchKernelGGL((scatter_kernel<float, double>), dim3(g), dim3(256), 0, ctx->stream,
                           (const float *)src, d, ctx->perm, ctx->K, (int)per);
    CK(hipGetLastError());
    if (!mem) {
        CK(hipMemcpyAsync(dst, ctx->stage_d, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    return ESDG_OK;
}

// Locality order of the elements: recursive coordinate bisection of the
// element centroids (split the longer extent at the median).  Consecutive
// elements, hence the elements of one workgroup and of neighbouring
// workgroups, are close in space, so neighbour traces are mostly read from
// LDS or the XCD's L2.
void rcb_order(int32_t *idx, int64_t n, const std::vector<double> &cx, const std::vector<double> &cy)
{
    if (n <= 2) return;
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t k = 0; k < n; ++k) {
        x0 = std::fmin(x0, cx[idx[k]]); x1 = std::fmax(x1, cx[idx[k]]);
        y0 = std::fmin(y0, cy[idx[k]]); y1 = std::fmax(y1, cy[idx[k]]);
    }
    const bool byx = (x1 - x0) >= (y1 - y0);
    const int64_t mid = n / 2;
    std::nth_element(idx, idx + mid, idx + n, [&](int32_t a, int32_t b) {
        const double va = byx ? cx[a] : cy[a], vb = byx ? cx[b] : cy[b];
        return va < vb || (va == vb && a < b);
    });
    rcb_order(idx, mid, cx, cy);
    rcb_order(idx + mid, n - mid, cx, cy);
}

template <typename T>
int alloc(esdg_ctx *ctx, T **p, size_t bytes)
{
    hipError_t e = hipMalloc((void **)p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, ESDG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return ESDG_OK;
}

bool check_ctx(esdg_ctx *ctx, bool need_state)
{
    if (!ctx) return false;
    if (!ctx->have_mesh || !ctx->have_b || (need_state && !ctx->have_state)) {
        fail(ctx, ESDG_EINVAL, "call order: upload_mesh, set_bathymetry and set_state first");
        return false;
    }
    return hipSetDevice(ctx->device) == hipSuccess;
}

// One time step launched on the context stream, no host synchronisation and
// no retry: the dt pass (dt > 0: that step for every instance; skipped when
// !with_dt, the step already in place) and the stages.
int launch_one_step(esdg_ctx *ctx, double dt, bool with_dt = true)
{
    const bool av = ctx->P.av_on != 0;
    const bool ssp = ctx->P.integrator == 1;
    const int nst = ssp ? 3 : 5;
    // W^n stays untouched in its buffer for the whole step: the stages
    // alternate between the other two (the last one ends in o1), so a retry
    // restarts from it without a copy
    const int base = ctx->cur;
    const int o1 = (base + 1) % 3, o2 = (base + 2) % 3;
    if (with_dt) TRY(launch_dt(ctx, base, dt > 0.0 ? dt : 0.0, 1));
    int in = base;
    for (int k = 0; k < nst; ++k) {
        const int out = (k % 2 == 0) ? o1 : o2;
        if (av) TRY(launch_viscous(ctx, in, out));
        const bool last = k == nst - 1;
        StageCall sc = ssp ? StageCall{kModeSsp, av, in, out, base, false, kSspAlpha[k], kSspBeta[k], last}
                           : StageCall{kModeLsrk, av, in, out, base, false, kLsrkA[k], kLsrkB[k], last, !last};
        TRY(launch_stage(ctx, sc));
        ctx->eps_valid[out] = av;   // written by the stage epilogue
        in = out;
    }
    ctx->cur = o1;
    ctx->dtb_buf = o1;   // the last stage left its dt bounds
    return ESDG_OK;
}

void destroy_graphs(esdg_ctx *ctx)
{
    for (auto &g : ctx->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = esdg_ctx::StepGraph{};
    }
    ++ctx->graph_gen;
}

// The host-side bookkeeping of launch_one_step(ctx, dt) without launching.
void advance_step_bookkeeping(esdg_ctx *ctx)
{
    const bool av = ctx->P.av_on != 0;
    const int nst = ctx->P.integrator == 1 ? 3 : 5;
    const int base = ctx->cur, o1 = (base + 1) % 3, o2 = (base + 2) % 3;
    for (int k = 0; k < nst; ++k) ctx->eps_valid[(k % 2 == 0) ? o1 : o2] = av;
    ctx->cur = o1;
    ctx->dtb_buf = o1;
}

// A step can replay a captured graph when nothing of its launch sequence
// depends on host-side state other than the graph's key: no kernel timing,
// and the start state's viscosity (AV) and dt bounds (adaptive step)
// already on the device.
bool graph_ready(const esdg_ctx *ctx, double dt)
{
    if (!ctx->use_graphs || ctx->prof) return false;
    if (ctx->P.av_on && !ctx->eps_valid[ctx->cur]) return false;
    if (!(dt > 0.0) && ctx->dtb_buf != ctx->cur) return false;
    return true;
}

// One time step by graph replay: capture it first if the cached graph of
// this start buffer does not match (capture records the launches on a
// private stream without running them), then launch it on the context
// stream.  If capture is unavailable the step runs eagerly and graphs stay
// off for the context.
int graph_step(esdg_ctx *ctx, double dt)
{
    const double key_dt = dt > 0.0 ? dt : 0.0;
    auto &g = ctx->graphs[ctx->cur];
    if (!(g.exec && g.dt == key_dt && g.variant == ctx->stage_variant && g.gen == ctx->graph_gen)) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = esdg_ctx::StepGraph{};
        if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            ctx->cap_stream = nullptr;
            ctx->use_graphs = false;
            return launch_one_step(ctx, dt);
        }
        // capture the launches of one step; the bookkeeping they change is
        // restored afterwards and applied again after the replay
        const int cur = ctx->cur, dtb = ctx->dtb_buf;
        bool ev[3];
        std::copy(ctx->eps_valid, ctx->eps_valid + 3, ev);
        hipStream_t run = ctx->stream;
        ctx->stream = ctx->cap_stream;
        hipGraph_t graph = nullptr;
        int st = ESDG_OK;
        if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            st = ESDG_EHIP;
        } else {
            st = launch_one_step(ctx, dt);
            const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
            if (e != hipSuccess) st = ESDG_EHIP;
        }
        ctx->stream = run;
        ctx->cur = cur;
        ctx->dtb_buf = dtb;
        std::copy(ev, ev + 3, ctx->eps_valid);
        hipGraphExec_t exec = nullptr;
        if (st == ESDG_OK && graph && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
            exec = nullptr;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();   // a failed capture leaves its error behind
        if (!exec) {
            ctx->use_graphs = false;
            return launch_one_step(ctx, dt);
        }
        g.exec = exec;
        g.dt = key_dt;
        g.variant = ctx->stage_variant;
        g.gen = ctx->graph_gen;
    }
    CK(hipGraphLaunch(g.exec, ctx->stream));
    advance_step_bookkeeping(ctx);
    return ESDG_OK;
}

int run_rhs(esdg_ctx *ctx, int buf)
{
    if (ctx->P.av_on) TRY(launch_viscous(ctx, buf, -1));
    StageCall sc{kModeRhs, ctx->P.av_on != 0, buf, buf, buf, true, 0.0, 0.0, false};
    return launch_stage(ctx, sc);
}

}  // namespace

extern "C" {

static_assert(kStageVariants == ESDG_STAGE_VARIANTS, "header and kernels disagree on the variant count");

int esdg_abi_version(void) { return 103; }

void esdg_default_params(esdg_params *p, int N)
{
    if (!p) return;
    const double s0 = -4.0 * std::log10((double)(N > 0 ? N : 1));
    p->g = 9.81;
    p->h_tol = 1e-4;
    p->eps0 = 0.0;
    p->sigma_min = s0 - 1.0;
    p->sigma_max = s0 + 1.0;
    p->cfl = 0.5;
    p->cfl_visc = 0.5;
    p->surface_flux = 0;
    p->av_on = 0;
    p->limiter_on = 0;
    p->integrator = 0;
    p->max_dt_retries = 0;
}

const char *esdg_last_error(const esdg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int esdg_create(esdg_ctx **out, int device, int precision)
{
    if (!out) return ESDG_EINVAL;
    *out = nullptr;
    if (precision != 64 && precision != 32) return ESDG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ESDG_EHIP;
    if (hipSetDevice(device) != hipSuccess) return ESDG_EHIP;
    // device address of the fixed diagnostics scratch on this GPU (once per device)
    if (lookup_scratch(device) != hipSuccess) return ESDG_EHIP;
    esdg_ctx *c = new (std::nothrow) esdg_ctx;
    if (!c) return ESDG_ENOMEM;
    c->device = device;
    c->prec = precision;
    esdg_default_params(&c->P, 3);
    *out = c;
    return ESDG_OK;
}

int esdg_destroy(esdg_ctx *ctx)
{
    if (!ctx) return ESDG_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_bufs(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->tune_ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return ESDG_OK;
}

int esdg_set_stream(esdg_ctx *ctx, void *s)
{
    if (!ctx) return ESDG_EINVAL;
    ctx->stream = (hipStream_t)s;
    return ESDG_OK;
}

int esdg_set_params(esdg_ctx *ctx, const esdg_params *p)
{
    if (!ctx || !p) return ESDG_EINVAL;
    if (!(p->g > 0) || !(p->cfl > 0) || !(p->cfl_visc > 0) || !(p->eps0 >= 0) ||
        !(p->sigma_max > p->sigma_min) || p->surface_flux < 0 || p->surface_flux > 1 || p->integrator < 0 ||
        p->integrator > 1 || p->max_dt_retries < 0 || !std::isfinite(p->h_tol))
        return fail(ctx, ESDG_EINVAL, "invalid parameter value");
    ctx->P = *p;
    invalidate_eps(ctx);
    destroy_graphs(ctx);
    return ESDG_OK;
}

int esdg_get_params(const esdg_ctx *ctx, esdg_params *p)
{
    if (!ctx || !p) return ESDG_EINVAL;
    *p = ctx->P;
    return ESDG_OK;
}

}  // extern "C"

namespace {

// Mesh upload for one or several instances: off = element ranges of the
// instances (caller's order; the face map must not cross them).
int upload_mesh_impl(esdg_ctx *ctx, int N, int64_t K, const double *x, const double *y, const int32_t *nbr_elem,
                     const int8_t *nbr_side, const int8_t *flip, int mem, const std::vector<int64_t> &off)
{
    if (!ctx) return ESDG_EINVAL;
    if (N < 2 || N > kMaxN) return fail(ctx, ESDG_EINVAL, "N=%d outside [2, %d]", N, kMaxN);
    if (K < 1 || K > (int64_t)INT32_MAX) return fail(ctx, ESDG_EINVAL, "K=%lld out of range", (long long)K);
    if (!x || !y || !nbr_elem || !nbr_side || !flip) return fail(ctx, ESDG_EINVAL, "null pointer");
    CK(hipSetDevice(ctx->device));
    // face map to the host for validation
    std::vector<int32_t> ne(4 * K);
    std::vector<int8_t> ns(4 * K), fl(4 * K);
    if (mem) {
        CK(hipMemcpyAsync(ne.data(), nbr_elem, 4 * K * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(ns.data(), nbr_side, 4 * K, hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(fl.data(), flip, 4 * K, hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    } else {
        std::memcpy(ne.data(), nbr_elem, 4 * K * sizeof(int32_t));
        std::memcpy(ns.data(), nbr_side, 4 * K);
        std::memcpy(fl.data(), flip, 4 * K);
    }
    std::vector<int8_t> code(4 * K);
    for (int64_t e = 0; e < K; ++e)
        for (int s = 0; s < 4; ++s) {
            const int64_t f = e * 4 + s;
            const int32_t en = ne[f];
            if (en == -1) {
                // solid wall: internally the side names itself, flagged
                code[f] = (int8_t)(s | (1 << 3));
                continue;
            }
            const int sn = ns[f], fv = fl[f];
            if (en < 0 || en >= K || sn < 0 || sn > 3 || (fv != 0 && fv != 1))
                return fail(ctx, ESDG_EMESH, "face map entry (%lld,%d) out of range", (long long)e, s);
            const int64_t g = (int64_t)en * 4 + sn;
            if (ne[g] != e || ns[g] != s || fl[g] != fv)
                return fail(ctx, ESDG_EMESH, "face map not symmetric at element %lld side %d", (long long)e, s);
            code[f] = (int8_t)(sn | (fv << 2));
        }
    // locality order of the elements (internal), from the element centroids
    const int64_t npn = (int64_t)(N + 1) * (N + 1);
    std::vector<double> hx, hy;
    const double *xs = x, *ys = y;
    if (mem) {
        hx.resize(K * npn);
        hy.resize(K * npn);
        CK(hipMemcpyAsync(hx.data(), x, K * npn * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(hy.data(), y, K * npn * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        xs = hx.data();
        ys = hy.data();
    }
    std::vector<double> cxv(K), cyv(K);
    for (int64_t e = 0; e < K; ++e) {
        double sx = 0, sy = 0;
        for (int64_t p = 0; p < npn; ++p) { sx += xs[e * npn + p]; sy += ys[e * npn + p]; }
        cxv[e] = sx / npn;
        cyv[e] = sy / npn;
    }
    const int ni = (int)off.size() - 1;
    if (ni < 1 || off[0] != 0 || off[ni] != K) return fail(ctx, ESDG_EINVAL, "bad instance ranges");
    std::vector<int32_t> inst_of(K);
    for (int k = 0; k < ni; ++k) {
        if (off[k + 1] <= off[k]) return fail(ctx, ESDG_EINVAL, "empty instance %d", k);
        for (int64_t e = off[k]; e < off[k + 1]; ++e) inst_of[e] = k;
    }
    for (int64_t f = 0; f < 4 * K; ++f)
        if (ne[f] >= 0 && inst_of[ne[f]] != inst_of[f / 4])
            return fail(ctx, ESDG_EMESH, "face map connects two instances at element %lld", (long long)(f / 4));
    // locality order inside each instance (instances stay contiguous)
    std::vector<int32_t> perm(K), inv(K);
    for (int64_t e = 0; e < K; ++e) perm[e] = (int32_t)e;
    for (int k = 0; k < ni; ++k) rcb_order(perm.data() + off[k], off[k + 1] - off[k], cxv, cyv);
    for (int64_t e = 0; e < K; ++e) inv[perm[e]] = (int32_t)e;
    std::vector<int32_t> ne2(4 * K);
    std::vector<int8_t> code2(4 * K);
    for (int64_t e = 0; e < K; ++e)
        for (int s = 0; s < 4; ++s) {
            const int32_t en = ne[(int64_t)perm[e] * 4 + s];
            ne2[e * 4 + s] = en >= 0 ? inv[en] : (int32_t)e;
            code2[e * 4 + s] = code[(int64_t)perm[e] * 4 + s];
        }
    bool walls = false;
    for (int64_t f = 0; f < 4 * K; ++f) walls = walls || ne[f] < 0;
    free_bufs(ctx);
    ctx->inv_h = inv;
    ctx->B.walls = walls ? 1 : 0;
    ctx->N = N;
    ctx->K = K;
    build_tables(N, ctx->ht);
    std::memset(&ctx->td, 0, sizeof(ctx->td));
    std::memset(&ctx->tf, 0, sizeof(ctx->tf));
    ctx->td.iw0 = (double)(1.0L / ctx->ht.w[0]);
    ctx->tf.iw0 = (float)(1.0L / ctx->ht.w[0]);
    for (int i = 0; i <= N; ++i) {
        ctx->td.w[i] = (double)ctx->ht.w[i];
        ctx->tf.w[i] = (float)ctx->ht.w[i];
        for (int j = 0; j <= N; ++j) {
            ctx->td.D[i * kMaxNF + j] = (double)ctx->ht.D[i][j];
            ctx->tf.D[i * kMaxNF + j] = (float)ctx->ht.D[i][j];
            ctx->td.Dz[i * kMaxNF + j] = i == j ? 0.0 : (double)ctx->ht.D[i][j];
            ctx->tf.Dz[i * kMaxNF + j] = i == j ? 0.0f : (float)ctx->ht.D[i][j];
            ctx->td.Vinv[i * kMaxNF + j] = (double)ctx->ht.Vinv[i][j];
            ctx->tf.Vinv[i * kMaxNF + j] = (float)ctx->ht.Vinv[i][j];
        }
    }
    Bufs &B = ctx->B;
    B.N = N;
    B.K = K;
    const int64_t n = nodes(ctx);
    const int nf = N + 1;
    const size_t r = rsz(ctx);
    TRY(alloc(ctx, &B.x, n * sizeof(double)));
    TRY(alloc(ctx, &B.y, n * sizeof(double)));
    if (ctx->prec == 64) {
        TRY(alloc(ctx, &B.xr, n * sizeof(double)));
        TRY(alloc(ctx, &B.yr, n * sizeof(double)));
    } else {
        TRY(alloc(ctx, &B.mref, K * 4 * sizeof(float)));
    }
    void **rn[] = {&B.Ax, &B.Cx, &B.Ae, &B.Ce, &B.bx, &B.by, &B.b, &B.dU[0], &B.dU[1], &B.dU[2],
                   &B.Rb[0], &B.Rb[1], &B.Rb[2]};
    for (void **p : rn) TRY(alloc(ctx, p, n * r));
    for (auto &w : B.W)
        for (void *&p : w) TRY(alloc(ctx, &p, n * r));
    TRY(alloc(ctx, &B.bface, K * 4 * nf * r));
    TRY(alloc(ctx, &B.nbr, K * 4 * sizeof(int32_t)));
    TRY(alloc(ctx, &B.code, K * 4));
    for (void *&p : B.eps) TRY(alloc(ctx, &p, K * r));
    TRY(alloc(ctx, &B.gmax, K * r));
    TRY(alloc(ctx, &B.dtc, K * r));
    TRY(alloc(ctx, &B.dtv, K * r));
    TRY(alloc(ctx, &B.fgeo, K * 4 * nf * 3 * r));
    TRY(alloc(ctx, &B.frec, K * 4 * nf * 3 * r));
    TRY(alloc(ctx, &B.tabg, ctx->prec == 64 ? sizeof(Tab<double>) : sizeof(Tab<float>)));
    if (ctx->prec == 64)
        CK(hipMemcpyAsync(B.tabg, &ctx->td, sizeof(Tab<double>), hipMemcpyHostToDevice, ctx->stream));
    else
        CK(hipMemcpyAsync(B.tabg, &ctx->tf, sizeof(Tab<float>), hipMemcpyHostToDevice, ctx->stream));
    for (int32_t *&p : B.list) TRY(alloc(ctx, &p, K * sizeof(int32_t)));
    TRY(alloc(ctx, &B.count, 4 * sizeof(int)));
    TRY(alloc(ctx, &B.lv[0], n * r));
    TRY(alloc(ctx, &B.lv[1], n * r));
    TRY(alloc(ctx, &B.vtr, K * 4 * nf * 4 * r));
    TRY(alloc(ctx, &B.dscal, 8 * ni * sizeof(double)));
    TRY(alloc(ctx, &B.slots, (size_t)3 * kDtSlots * ni * sizeof(unsigned long long)));
    B.n_inst = ni;
    if (ni > 1) {
        // instance of every (internal) element and chunks of the time-step pass
        std::vector<int64_t> cst;
        std::vector<int32_t> cin;
        for (int k = 0; k < ni; ++k)
            for (int64_t e = off[k]; e < off[k + 1]; e += kDtChunk) {
                cst.push_back(e);
                cin.push_back(k);
            }
        cst.push_back(K);
        B.nchunks = (int64_t)cin.size();
        TRY(alloc(ctx, &B.inst, K * sizeof(int32_t)));
        TRY(alloc(ctx, &B.iflags, ni * sizeof(int)));
        TRY(alloc(ctx, &B.imask, ni * sizeof(int)));
        CK(hipMemsetAsync(B.iflags, 0, ni * sizeof(int), ctx->stream));
        TRY(alloc(ctx, &B.cstart, cst.size() * sizeof(int64_t)));
        TRY(alloc(ctx, &B.cinst, cin.size() * sizeof(int32_t)));
        CK(hipMemcpyAsync(B.inst, inst_of.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        CK(hipMemcpyAsync(B.cstart, cst.data(), cst.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        CK(hipMemcpyAsync(B.cinst, cin.data(), cin.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    TRY(alloc(ctx, &B.flags, kNumFlags * sizeof(int)));
    int64_t T = 0;
    (void)dispatch(ctx, [&](auto L, auto) {
        T = decltype(L)::threads();
        return hipSuccess;
    });
    B.part_cap = (n + T - 1) / T;
    TRY(alloc(ctx, &B.part, B.part_cap * 8 * sizeof(double)));
    TRY(alloc(ctx, &ctx->stage_d, 5 * n * sizeof(double)));
    // zero-filled registers and traces
    for (void *p : B.dU) CK(hipMemsetAsync(p, 0, n * r, ctx->stream));
    CK(hipMemsetAsync(B.vtr, 0, K * 4 * nf * 4 * r, ctx->stream));
    for (void *p : B.eps) CK(hipMemsetAsync(p, 0, K * r, ctx->stream));
    CK(hipMemsetAsync(B.count, 0, 4 * sizeof(int), ctx->stream));
    invalidate_eps(ctx);
    CK(hipMemsetAsync(B.dscal, 0, 8 * ni * sizeof(double), ctx->stream));
    CK(hipMemsetAsync(B.flags, 0, kNumFlags * sizeof(int), ctx->stream));
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)ni), dim3(3 * kDtSlots), 0, ctx->stream, B.slots,
                       0x7FF0000000000000ull, 3 * kDtSlots * ni);
    CK(hipGetLastError());
    TRY(alloc(ctx, &ctx->perm, K * sizeof(int32_t)));
    CK(hipMemcpyAsync(ctx->perm, perm.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    CK(hipMemcpyAsync(B.nbr, ne2.data(), 4 * K * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    CK(hipMemcpyAsync(B.code, code2.data(), 4 * K, hipMemcpyHostToDevice, ctx->stream));
    {
        const double *sx = x, *sy = y;
        if (!mem) {
            CK(hipMemcpyAsync(ctx->stage_d, x, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            CK(hipMemcpyAsync(ctx->stage_d + n, y, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            sx = ctx->stage_d;
            sy = ctx->stage_d + n;
        }
        const unsigned g = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL((gather_kernel<double, double>), dim3(g), dim3(256), 0, ctx->stream, sx, B.x,
                           ctx->perm, K, (int)npn);
        hipLaunchKernelGGL((gather_kernel<double, double>), dim3(g), dim3(256), 0, ctx->stream, sy, B.y,
                           ctx->perm, K, (int)npn);
        CK(hipGetLastError());
    }
    CK(dispatch(ctx, [&](auto L, auto) { return decltype(L)::geometry(ctx->B, ctx->td, ctx->stream); }));
    int flags[kNumFlags];
    TRY(read_flags(ctx, flags));
    if (flags[kFlagBadJ]) {
        free_bufs(ctx);
        return fail(ctx, ESDG_EMESH, "Jacobian not positive at some node");
    }
    ctx->inst_off = off;
    ctx->have_mesh = true;
    ctx->cur = 0;
    return ESDG_OK;
}

}  // namespace

extern "C" {

int esdg_upload_mesh(esdg_ctx *ctx, int N, int64_t K, const double *x, const double *y,
                     const int32_t *nbr_elem, const int8_t *nbr_side, const int8_t *flip, int mem)
{
    return upload_mesh_impl(ctx, N, K, x, y, nbr_elem, nbr_side, flip, mem, std::vector<int64_t>{0, K});
}

int esdg_set_bathymetry(esdg_ctx *ctx, const double *b, int mem)
{
    if (!ctx || !b) return ESDG_EINVAL;
    if (!ctx->have_mesh) return fail(ctx, ESDG_EINVAL, "upload_mesh first");
    CK(hipSetDevice(ctx->device));
    const int64_t n = nodes(ctx);
    const double *src = b;
    if (!mem) {
        CK(hipMemcpyAsync(ctx->stage_d, b, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        src = ctx->stage_d;
    }
    double *db = ctx->stage_d + n;   // internal order
    hipLaunchKernelGGL((gather_kernel<double, double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       ctx->stream, src, db, ctx->perm, ctx->K, (ctx->N + 1) * (ctx->N + 1));
    CK(hipGetLastError());
    CK(dispatch(ctx, [&](auto L, auto) { return decltype(L)::bathymetry(ctx->B, db, ctx->td, ctx->stream); }));
    CK(hipStreamSynchronize(ctx->stream));
    ctx->have_b = true;
    ++ctx->b_version;
    return ESDG_OK;
}

int esdg_set_state(esdg_ctx *ctx, const double *h, const double *hu, const double *hv, int mem)
{
    if (!ctx || !h || !hu || !hv) return ESDG_EINVAL;
    if (!ctx->have_mesh) return fail(ctx, ESDG_EINVAL, "upload_mesh first");
    CK(hipSetDevice(ctx->device));
    const int64_t n = nodes(ctx);
    ctx->cur = 0;
    const int64_t per = n / ctx->K;
    TRY(upload_field(ctx, ctx->B.W[0][0], h, per, mem));
    TRY(upload_field(ctx, ctx->B.W[0][1], hu, per, mem));
    TRY(upload_field(ctx, ctx->B.W[0][2], hv, per, mem));
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.dscal + 4, 0.0,
                       n_inst(ctx));
    CK(hipGetLastError());
    invalidate_eps(ctx);
    ctx->have_state = true;
    return ESDG_OK;
}

int esdg_get_state(esdg_ctx *ctx, double *h, double *hu, double *hv, int mem)
{
    if (!ctx || !h || !hu || !hv) return ESDG_EINVAL;
    if (!ctx->have_state) return fail(ctx, ESDG_EINVAL, "no state");
    CK(hipSetDevice(ctx->device));
    const int64_t n = nodes(ctx);
    const int64_t per = n / ctx->K;
    TRY(download_field(ctx, h, ctx->B.W[ctx->cur][0], per, mem));
    TRY(download_field(ctx, hu, ctx->B.W[ctx->cur][1], per, mem));
    TRY(download_field(ctx, hv, ctx->B.W[ctx->cur][2], per, mem));
    return ESDG_OK;
}

int esdg_rhs(esdg_ctx *ctx, double *rh, double *rhu, double *rhv, int mem)
{
    if (!rh || !rhu || !rhv) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ctx ? ESDG_EINVAL : ESDG_EINVAL;
    TRY(run_rhs(ctx, ctx->cur));
    const int64_t n = nodes(ctx);
    const int64_t per = n / ctx->K;
    TRY(download_field(ctx, rh, ctx->B.Rb[0], per, mem));
    TRY(download_field(ctx, rhu, ctx->B.Rb[1], per, mem));
    TRY(download_field(ctx, rhv, ctx->B.Rb[2], per, mem));
    return ESDG_OK;
}

int esdg_limit(esdg_ctx *ctx, int64_t *n_limited)
{
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    TRY(reset_flags(ctx));
    CK(dispatch(ctx, [&](auto L, auto r) {
        using R = decltype(r);
        return decltype(L)::limit(ctx->B, ctx->cur, phys<R>(ctx), tab<R>(ctx), ctx->stream);
    }));
    ctx->eps_valid[ctx->cur] = false;
    if (ctx->dtb_buf == ctx->cur) ctx->dtb_buf = -1;
    int flags[kNumFlags];
    TRY(read_flags(ctx, flags));
    if (n_limited) *n_limited = flags[kFlagLimited];
    if (flags[kFlagNegMean]) return fail(ctx, ESDG_ENEGMEAN, "negative element mean in the limiter");
    return ESDG_OK;
}

int esdg_compute_dt(esdg_ctx *ctx, double out[4])
{
    if (!out) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    TRY(reset_flags(ctx));
    TRY(launch_dt(ctx, ctx->cur, 0.0, 0));
    CK(hipMemcpyAsync(out, ctx->B.dscal, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_step(esdg_ctx *ctx, int nsteps, double dt, double *t_out)
{
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    if (nsteps < 0) return fail(ctx, ESDG_EINVAL, "nsteps < 0");
    const int retries = ctx->P.max_dt_retries;
    if (retries > 0 && n_inst(ctx) > 1) return fail(ctx, ESDG_EINVAL, "dt retries need a single instance");
    TRY(reset_flags(ctx));
    int status = ESDG_OK;
    for (int it = 0; it < nsteps; ++it) {
        if (retries <= 0) {
            if (graph_ready(ctx, dt)) TRY(graph_step(ctx, dt));
            else TRY(launch_one_step(ctx, dt));
            continue;
        }
        const int base = ctx->cur;
        TRY(reset_flags(ctx));
        for (int attempt = 0;; ++attempt) {
            if (attempt == 0) {
                TRY(launch_one_step(ctx, dt));
            } else {
                // the halved step is already in place: replay the stages with it
                ctx->cur = base;
                TRY(launch_one_step(ctx, dt, false));
            }
            {
                // check the step against the bounds of the state it produced (the
                // last stage left them; the next step's dt pass recomputes them)
                TRY(dispatch(ctx, [&](auto L, auto r) {
                    using R = decltype(r);
                    return decltype(L)::dt(ctx->B, ctx->cur, ctx->P.av_on != 0, true, phys<R>(ctx), ctx->stream,
                                           Ev{});
                }));
                hipLaunchKernelGGL(step_check_kernel, dim3(1), dim3(kDtSlots), 0, ctx->stream, ctx->B.slots,
                                   ctx->B.dscal, ctx->B.flags, (int *)nullptr);
                CK(hipGetLastError());
            }
            int flags[kNumFlags];
            TRY(read_flags(ctx, flags));
            if (flags[kFlagNonFinite]) break;   // reported below; halving the step cannot help
            if (!(flags[kFlagNegMean] || flags[kFlagStepBound]) || attempt >= retries) {
                // out of retries a step above the bounds of its result is kept
                if (flags[kFlagNegMean]) status = ESDG_ENEGMEAN;
                break;
            }
            // negative mean, or a step above the bounds of its result: restart
            // from W^n (untouched) with half the step
            ctx->cur = base;
            hipLaunchKernelGGL(scale_step_kernel, dim3(1), dim3(1), 0, ctx->stream, ctx->B.dscal, 0.5,
                               ctx->B.dscal + 4);
            CK(hipGetLastError());
            TRY(reset_flags(ctx));
        }
    }
    int flags[kNumFlags];
    TRY(read_flags(ctx, flags));
    if (t_out) {
        CK(hipMemcpyAsync(t_out, ctx->B.dscal + 4, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    ctx->last_limited = flags[kFlagLimited];
    if (flags[kFlagNonFinite]) return fail(ctx, ESDG_ENONFINITE, "non-finite value in a stage output");
    if (flags[kFlagDtPos]) return fail(ctx, ESDG_EDTPOS, "no admissible time step");
    if (status == ESDG_OK && flags[kFlagNegMean] && retries <= 0) status = ESDG_ENEGMEAN;
    if (status == ESDG_ENEGMEAN) return fail(ctx, ESDG_ENEGMEAN, "negative element mean in the limiter");
    return ESDG_OK;
}

int esdg_get_time(esdg_ctx *ctx, double *t)
{
    if (!ctx || !t || !ctx->have_mesh) return ESDG_EINVAL;
    CK(hipSetDevice(ctx->device));
    CK(hipMemcpyAsync(t, ctx->B.dscal + 4, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_set_time(esdg_ctx *ctx, double t)
{
    if (!ctx || !ctx->have_mesh) return ESDG_EINVAL;
    CK(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.dscal + 4, t, n_inst(ctx));
    CK(hipGetLastError());
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_diagnostics(esdg_ctx *ctx, double out[8])
{
    if (!out) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    TRY(run_rhs(ctx, ctx->cur));
    int64_t nb = 0;
    CK(dispatch(ctx, [&](auto L, auto r) {
        using R = decltype(r);
        return decltype(L)::diag(ctx->B, ctx->cur, phys<R>(ctx), tab<R>(ctx), &nb, ctx->stream);
    }));
    std::vector<double> part(nb * 8);
    CK(hipMemcpyAsync(part.data(), ctx->B.part, nb * 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    double acc[8] = {0, 0, 0, 0, 0, INFINITY, -INFINITY, 0};
    for (int64_t b = 0; b < nb; ++b) {
        for (int c = 0; c < 5; ++c) acc[c] += part[b * 8 + c];
        acc[5] = std::fmin(acc[5], part[b * 8 + 5]);
        acc[6] = std::fmax(acc[6], part[b * 8 + 6]);
        acc[7] += part[b * 8 + 7];
    }
    std::memcpy(out, acc, sizeof acc);
    return ESDG_OK;
}

int esdg_diagnostics_noalloc(esdg_ctx *ctx, double out[8])
{
    if (!out) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    double *sc = scratch_ptr(ctx->device);
    if (!sc) return fail(ctx, ESDG_EHIP, "no scratch address for device %d", ctx->device);
    int64_t T = 0;
    (void)dispatch(ctx, [&](auto L, auto) {
        T = decltype(L)::threads();
        return hipSuccess;
    });
    const int64_t nb = (ctx->K * (int64_t)(ctx->N + 1) * (ctx->N + 1) + T - 1) / T;
    if (nb > kScratchRows)
        return fail(ctx, ESDG_EINVAL,
                    "mesh too large for esdg_diagnostics_noalloc: %lld partial rows of %lld threads, "
                    "the fixed scratch holds %lld (at most %lld nodes at this degree)",
                    (long long)nb, (long long)T, (long long)kScratchRows, (long long)(kScratchRows * T));
    TRY(run_rhs(ctx, ctx->cur));
    Bufs B = ctx->B;
    B.part = sc;
    B.part_cap = kScratchRows;
    int64_t nb2 = 0;
    CK(dispatch(ctx, [&](auto L, auto r) {
        using R = decltype(r);
        return decltype(L)::diag(B, ctx->cur, phys<R>(ctx), tab<R>(ctx), &nb2, ctx->stream);
    }));
    double *fin = sc + kScratchRows * 8;
    hipLaunchKernelGGL(diag_reduce_kernel, dim3(1), dim3(64), 0, ctx->stream, sc, nb2, fin);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(out, fin, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_get_eps(esdg_ctx *ctx, double *eps, int mem)
{
    if (!eps) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    if (ctx->P.av_on) {
        TRY(ensure_eps(ctx, ctx->cur));
    } else {
        CK(hipMemsetAsync(ctx->B.eps[ctx->cur], 0, ctx->K * rsz(ctx), ctx->stream));
        ctx->eps_valid[ctx->cur] = false;
    }
    return download_field(ctx, eps, ctx->B.eps[ctx->cur], 1, mem);
}

int esdg_get_geometry(esdg_ctx *ctx, double *xxi, double *xeta, double *yxi, double *yeta, double *J,
                      int mem)
{
    if (!ctx || !ctx->have_mesh || !xxi || !xeta || !yxi || !yeta || !J) return ESDG_EINVAL;
    CK(hipSetDevice(ctx->device));
    const int64_t n = nodes(ctx);
    const unsigned g = (unsigned)((n + 255) / 256);
    const int npn = (ctx->N + 1) * (ctx->N + 1);
    if (ctx->prec == 64)
        hipLaunchKernelGGL((geometry_out_kernel<double>), dim3(g), dim3(256), 0, ctx->stream,
                           (const double *)ctx->B.Ax, (const double *)ctx->B.Cx, (const double *)ctx->B.Ae,
                           (const double *)ctx->B.Ce, (const double *)nullptr, ctx->stage_d, ctx->perm, ctx->K,
                           npn);
    else
        hipLaunchKernelGGL((geometry_out_kernel<float>), dim3(g), dim3(256), 0, ctx->stream,
                           (const float *)ctx->B.Ax, (const float *)ctx->B.Cx, (const float *)ctx->B.Ae,
                           (const float *)ctx->B.Ce, (const float *)ctx->B.mref, ctx->stage_d, ctx->perm, ctx->K,
                           npn);
    CK(hipGetLastError());
    double *outs[5] = {xxi, xeta, yxi, yeta, J};
    const hipMemcpyKind k = mem ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int c = 0; c < 5; ++c)
        CK(hipMemcpyAsync(outs[c], ctx->stage_d + c * n, n * sizeof(double), k, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_autotune(esdg_ctx *ctx, int reps, int *choice, double ms[ESDG_STAGE_VARIANTS])
{
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    if (reps < 1 || reps > 1000) return fail(ctx, ESDG_EINVAL, "reps outside [1, 1000]");
    const bool av = ctx->P.av_on != 0;
    const int base = ctx->cur, o1 = (base + 1) % 3;
    TRY(reset_flags(ctx));
    if (av) TRY(launch_viscous(ctx, base, -1));
    // trial stages in the integrator's own form, W^n -> o1, each variant timed
    // over reps launches, twice, alternating: for LSRK(5,4) an interior stage
    // that reads the register dU (as stages 2-5 do) but does not write it --
    // repeated in place, d <- a_3 d + dt R with |a_3| > 1 would grow without
    // bound -- for SSPRK(3,3) an SSP stage (W^n untouched)
    const bool ssp = ctx->P.integrator == 1;
    if (!ctx->tune_ev[0]) {
        CK(hipEventCreate(&ctx->tune_ev[0]));
        CK(hipEventCreate(&ctx->tune_ev[1]));
    }
    hipEvent_t e0 = ctx->tune_ev[0], e1 = ctx->tune_ev[1];
    double best[kStageVariants];
    for (double &b : best) b = 1e300;
    const int keep = ctx->stage_variant;
    const bool prof = ctx->prof;
    ctx->prof = false;   // trial launches stay out of the kernel timings
    for (int round = 0; round < 2; ++round)
        for (int v = 0; v < kStageVariants; ++v) {
            ctx->stage_variant = v;
            CK(hipEventRecord(e0, ctx->stream));
            for (int r = 0; r < reps; ++r) {
                // the epilogue appends to o1's viscous-element list: empty it first
                hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.count + o1, 0, 1);
                StageCall sc = ssp ? StageCall{kModeSsp, av, base, o1, base, false, 0.0, 1.0, false, false, v}
                                   : StageCall{kModeLsrk, av, base, o1, base, false, kLsrkA[2], kLsrkB[2], false,
                                               false, v};
                const int st = launch_stage(ctx, sc);
                if (st) {
                    ctx->stage_variant = keep;
                    ctx->prof = prof;
                    return st;
                }
            }
            CK(hipEventRecord(e1, ctx->stream));
            CK(hipEventSynchronize(e1));
            float t = 0;
            CK(hipEventElapsedTime(&t, e0, e1));
            best[v] = std::min(best[v], (double)t / reps);
        }
    ctx->prof = prof;
    int pick = 0;
    for (int v = 1; v < kStageVariants; ++v)
        if (best[v] < best[pick]) pick = v;
    ctx->stage_variant = pick;
    ctx->eps_valid[o1] = false;
    if (ctx->dtb_buf == o1) ctx->dtb_buf = -1;
    TRY(reset_flags(ctx));
    if (choice) *choice = pick;
    if (ms)
        for (int v = 0; v < kStageVariants; ++v) ms[v] = best[v];
    return ESDG_OK;
}

int esdg_set_stage_variant(esdg_ctx *ctx, int variant)
{
    if (!ctx || variant < 0 || variant >= kStageVariants)
        return ctx ? fail(ctx, ESDG_EINVAL, "variant outside [0, %d)", kStageVariants) : ESDG_EINVAL;
    ctx->stage_variant = variant;
    return ESDG_OK;
}

int esdg_set_graphs(esdg_ctx *ctx, int enable)
{
    if (!ctx) return ESDG_EINVAL;
    ctx->use_graphs = enable != 0;
    if (!ctx->use_graphs) {
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        destroy_graphs(ctx);
    }
    return ESDG_OK;
}

int esdg_step_stats(esdg_ctx *ctx, int64_t *limited, int64_t *viscous)
{
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    if (limited) *limited = ctx->last_limited;
    if (viscous) {
        *viscous = 0;
        if (ctx->P.av_on) {
            TRY(ensure_eps(ctx, ctx->cur));
            int cnt = 0;
            CK(hipMemcpyAsync(&cnt, ctx->B.count + ctx->cur, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            CK(hipStreamSynchronize(ctx->stream));
            *viscous = cnt;
        }
    }
    return ESDG_OK;
}

int esdg_profile(esdg_ctx *ctx, int enable)
{
    if (!ctx) return ESDG_EINVAL;
    ctx->prof = enable != 0;
    return ESDG_OK;
}

}  // extern "C"

namespace {

// Sum the recorded event pairs of every log into the accumulators; the
// events return to the pool.
int drain_events(esdg_ctx *ctx)
{
    CK(hipSetDevice(ctx->device));
    CK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < kProfClasses; ++k) {
        for (auto &pr : ctx->ev_log[k]) {
            float ms = 0;
            CK(hipEventElapsedTime(&ms, pr.first, pr.second));
            ctx->acc_ms[k] += ms;
        }
        ctx->acc_n[k] += (int64_t)ctx->ev_log[k].size();
        ctx->ev_log[k].clear();
    }
    ctx->ev_next = 0;
    return ESDG_OK;
}

}  // namespace

extern "C" {

int esdg_profile_read(esdg_ctx *ctx, double *stage_ms, int64_t *stage_n, double *av_ms, int64_t *av_n)
{
    if (!ctx) return ESDG_EINVAL;
    TRY(drain_events(ctx));
    if (stage_ms) *stage_ms = ctx->acc_ms[kProfStage];
    if (stage_n) *stage_n = ctx->acc_n[kProfStage];
    const int av[3] = {kProfIndicator, kProfAvFaces, kProfAvDiv};
    double ams = 0;
    int64_t an = 0;
    for (int k : av) {
        ams += ctx->acc_ms[k];
        an += ctx->acc_n[k];
    }
    if (av_ms) *av_ms = ams;
    if (av_n) *av_n = an;
    for (int k : {kProfStage, kProfIndicator, kProfAvFaces, kProfAvDiv, kProfDt}) {
        ctx->acc_ms[k] = 0;
        ctx->acc_n[k] = 0;
    }
    return ESDG_OK;
}

int esdg_profile_read_kernels(esdg_ctx *ctx, double ms[6], int64_t launches[6])
{
    if (!ctx || !ms || !launches) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    TRY(drain_events(ctx));
    for (int k = 0; k < kProfClasses; ++k) {
        ms[k] = ctx->acc_ms[k];
        launches[k] = ctx->acc_n[k];
        ctx->acc_ms[k] = 0;
        ctx->acc_n[k] = 0;
    }
    return ESDG_OK;
}

int esdg_profile_read_adjoint(esdg_ctx *ctx, double *ms, int64_t *n)
{
    if (!ctx) return ESDG_EINVAL;
    TRY(drain_events(ctx));
    if (ms) *ms = ctx->acc_ms[kProfAdjoint];
    if (n) *n = ctx->acc_n[kProfAdjoint];
    ctx->acc_ms[kProfAdjoint] = 0;
    ctx->acc_n[kProfAdjoint] = 0;
    return ESDG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Ensembles: instances of one degree share a context whose mesh is the
// disjoint union of their meshes (one launch per stage for all of them),
// with a time step and a time per instance.  Degrees run on their own
// streams.
// ------------------------------------------------------------------------
struct esdg_ensemble {
    struct Inst {
        esdg_params P{};
        int N = 0;
        int64_t K = 0;
        std::vector<double> x, y, b, h, hu, hv;
        std::vector<int32_t> ne;
        std::vector<int8_t> ns, fl;
        int group = -1, local = -1;
        int64_t off = 0;   // first element in the group's union
    };
    struct Group {
        int N = 0;
        esdg_ctx *ctx = nullptr;
        hipStream_t stream = nullptr;
        std::vector<int> members;
        double *scratch = nullptr;   // [3][nodes] device copy of the union state (get_state)
        int *hflags = nullptr;       // pinned host ints (step retries): step flags, instance flags, retry mask
    };
    int device = 0, prec = 64;
    std::vector<Inst> inst;
    std::vector<Group> groups;
    bool built = false;
    std::string err = "no error";
};

namespace {

int efail(esdg_ensemble *en, int code, const char *msg)
{
    if (en) en->err = msg;
    return code;
}

int efail_ctx(esdg_ensemble *en, esdg_ctx *c, int code)
{
    if (en) en->err = c ? c->err : std::string("context failure");
    return code;
}

bool same_params(const esdg_params &a, const esdg_params &b)
{
    return a.g == b.g && a.h_tol == b.h_tol && a.eps0 == b.eps0 && a.sigma_min == b.sigma_min &&
           a.sigma_max == b.sigma_max && a.cfl == b.cfl && a.cfl_visc == b.cfl_visc &&
           a.surface_flux == b.surface_flux && a.av_on == b.av_on && a.limiter_on == b.limiter_on &&
           a.integrator == b.integrator && a.max_dt_retries == b.max_dt_retries;
}

int ensemble_build(esdg_ensemble *en)
{
    if (en->built) return ESDG_OK;
    if (en->inst.empty()) return efail(en, ESDG_EINVAL, "no instances");
    if (hipSetDevice(en->device) != hipSuccess) return efail(en, ESDG_EHIP, "hipSetDevice failed");
    for (size_t k = 0; k < en->inst.size(); ++k) {
        auto &I = en->inst[k];
        int g = -1;
        for (size_t j = 0; j < en->groups.size(); ++j)
            if (en->groups[j].N == I.N) g = (int)j;
        if (g < 0) {
            en->groups.push_back({});
            g = (int)en->groups.size() - 1;
            en->groups[g].N = I.N;
        }
        auto &G = en->groups[g];
        if (!G.members.empty() && !same_params(en->inst[G.members[0]].P, I.P))
            return efail(en, ESDG_EINVAL, "instances of one degree must share their parameters");
        I.group = g;
        I.local = (int)G.members.size();
        G.members.push_back((int)k);
    }
    for (auto &G : en->groups) {
        const int N = G.N;
        const int64_t npn = (int64_t)(N + 1) * (N + 1);
        std::vector<int64_t> off{0};
        for (int m : G.members) {
            en->inst[m].off = off.back();
            off.push_back(off.back() + en->inst[m].K);
        }
        const int64_t K = off.back();
        std::vector<double> x(K * npn), y(K * npn), b(K * npn), h(K * npn), hu(K * npn), hv(K * npn);
        std::vector<int32_t> ne(4 * K);
        std::vector<int8_t> ns(4 * K), fl(4 * K);
        for (int m : G.members) {
            const auto &I = en->inst[m];
            const int64_t o = I.off;
            std::copy(I.x.begin(), I.x.end(), x.begin() + o * npn);
            std::copy(I.y.begin(), I.y.end(), y.begin() + o * npn);
            std::copy(I.b.begin(), I.b.end(), b.begin() + o * npn);
            std::copy(I.h.begin(), I.h.end(), h.begin() + o * npn);
            std::copy(I.hu.begin(), I.hu.end(), hu.begin() + o * npn);
            std::copy(I.hv.begin(), I.hv.end(), hv.begin() + o * npn);
            for (int64_t f = 0; f < 4 * I.K; ++f) {
                ne[4 * o + f] = I.ne[f] >= 0 ? (int32_t)(I.ne[f] + o) : -1;   // walls stay walls
                ns[4 * o + f] = I.ns[f];
                fl[4 * o + f] = I.fl[f];
            }
        }
        int st = esdg_create(&G.ctx, en->device, en->prec);
        if (st) return efail(en, st, "esdg_create failed");
        if (hipStreamCreate(&G.stream) != hipSuccess) return efail(en, ESDG_EHIP, "hipStreamCreate failed");
        esdg_ctx *c = G.ctx;
        if ((st = esdg_set_stream(c, G.stream))) return efail_ctx(en, c, st);
        if ((st = esdg_set_params(c, &en->inst[G.members[0]].P))) return efail_ctx(en, c, st);
        if ((st = upload_mesh_impl(c, N, K, x.data(), y.data(), ne.data(), ns.data(), fl.data(), 0, off)))
            return efail_ctx(en, c, st);
        if ((st = esdg_set_bathymetry(c, b.data(), 0))) return efail_ctx(en, c, st);
        if ((st = esdg_set_state(c, h.data(), hu.data(), hv.data(), 0))) return efail_ctx(en, c, st);
        if (hipMalloc((void **)&G.scratch, 3 * K * npn * sizeof(double)) != hipSuccess)
            return efail(en, ESDG_ENOMEM, "hipMalloc failed");
    }
    for (auto &I : en->inst) {   // the host copies are no longer needed
        std::vector<double>().swap(I.x); std::vector<double>().swap(I.y); std::vector<double>().swap(I.b);
        std::vector<double>().swap(I.h); std::vector<double>().swap(I.hu); std::vector<double>().swap(I.hv);
        std::vector<int32_t>().swap(I.ne); std::vector<int8_t>().swap(I.ns); std::vector<int8_t>().swap(I.fl);
    }
    en->built = true;
    return ESDG_OK;
}

}  // namespace

extern "C" {

int esdg_ensemble_create(esdg_ensemble **out, int device, int precision)
{
    if (!out || (precision != 64 && precision != 32)) return ESDG_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ESDG_EINVAL;
    auto *en = new esdg_ensemble;
    en->device = device;
    en->prec = precision;
    *out = en;
    return ESDG_OK;
}

int esdg_ensemble_destroy(esdg_ensemble *en)
{
    if (!en) return ESDG_EINVAL;
    (void)hipSetDevice(en->device);
    for (auto &G : en->groups) {
        if (G.stream) (void)hipStreamSynchronize(G.stream);
        if (G.ctx) esdg_destroy(G.ctx);
        if (G.scratch) (void)hipFree(G.scratch);
        if (G.hflags) (void)hipHostFree(G.hflags);
        if (G.stream) (void)hipStreamDestroy(G.stream);
    }
    delete en;
    return ESDG_OK;
}

int esdg_ensemble_add(esdg_ensemble *en, const esdg_params *p, int N, int64_t K, const double *x, const double *y,
                      const int32_t *nbr_elem, const int8_t *nbr_side, const int8_t *flip, const double *b,
                      const double *h, const double *hu, const double *hv, int *id)
{
    if (!en) return ESDG_EINVAL;
    if (en->built) return efail(en, ESDG_EINVAL, "instances must be added before the first step");
    if (!p || !x || !y || !nbr_elem || !nbr_side || !flip || !b || !h || !hu || !hv)
        return efail(en, ESDG_EINVAL, "null pointer");
    if (N < 2 || N > kMaxN || K < 1) return efail(en, ESDG_EINVAL, "N or K out of range");
    for (int64_t f = 0; f < 4 * K; ++f)
        if (nbr_elem[f] < -1 || nbr_elem[f] >= K) return efail(en, ESDG_EMESH, "face map entry out of range");
    esdg_ensemble::Inst I;
    I.P = *p;
    I.N = N;
    I.K = K;
    const int64_t n = K * (int64_t)(N + 1) * (N + 1);
    I.x.assign(x, x + n); I.y.assign(y, y + n); I.b.assign(b, b + n);
    I.h.assign(h, h + n); I.hu.assign(hu, hu + n); I.hv.assign(hv, hv + n);
    I.ne.assign(nbr_elem, nbr_elem + 4 * K);
    I.ns.assign(nbr_side, nbr_side + 4 * K);
    I.fl.assign(flip, flip + 4 * K);
    en->inst.push_back(std::move(I));
    if (id) *id = (int)en->inst.size() - 1;
    return ESDG_OK;
}

int esdg_ensemble_build(esdg_ensemble *en)
{
    if (!en) return ESDG_EINVAL;
    return ensemble_build(en);
}

}  // extern "C"

namespace {

// Ensemble steps with the after-the-fact check per instance (the section 6
// step adjustment, as esdg_step does for one instance): an instance whose
// step met a negative element mean or exceeds twice the CFL / viscous bound
// of its result redoes it with half its step, at most `retries` times.  W^n
// stays untouched in its buffer, so a degree group's step is relaunched from
// it and its instances that keep their step redo it bit for bit.  All groups
// launch their step and its check on their own streams before the host waits
// for any, so the degrees still overlap.

// Launch one attempt of a group's step (the first by graph replay when
// ready), its check, and the copies of the flags to the group's pinned
// host buffer: [kNumFlags] step flags, then [ni] instance flags.
int group_attempt(esdg_ctx *ctx, int base, bool first, int *hflags)
{
    const int ni = n_inst(ctx);
    if (first) {
        TRY(graph_ready(ctx, 0.0) ? graph_step(ctx, 0.0) : launch_one_step(ctx, 0.0));
    } else {
        // a redo covers only the instances in the mask: the stage kernels
        // leave the other instances' elements, whose outputs of the step
        // before are the same bit for bit, as they are.  Only the result's
        // viscous-element list is rebuilt for all of them (each stage
        // rebuilds its output's list from the elements it covers).
        ctx->cur = base;
        ctx->masked_attempt = ni > 1;
        const int st = launch_one_step(ctx, 0.0, false);
        ctx->masked_attempt = false;
        TRY(st);
        if (ni > 1 && ctx->P.av_on) {
            const int o = ctx->cur;
            hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.count + o, 0, 1);
            CK(hipGetLastError());
            const unsigned g = (unsigned)((ctx->K + 255) / 256);
            if (ctx->prec == 64)
                hipLaunchKernelGGL(relist_kernel<double>, dim3(g), dim3(256), 0, ctx->stream,
                                   (const double *)ctx->B.eps[o], ctx->B.list[o], ctx->B.count + o, ctx->K);
            else
                hipLaunchKernelGGL(relist_kernel<float>, dim3(g), dim3(256), 0, ctx->stream,
                                   (const float *)ctx->B.eps[o], ctx->B.list[o], ctx->B.count + o, ctx->K);
            CK(hipGetLastError());
        }
    }
    TRY(dispatch(ctx, [&](auto L, auto r) {
        using R = decltype(r);
        return decltype(L)::dt(ctx->B, ctx->cur, ctx->P.av_on != 0, true, phys<R>(ctx), ctx->stream, Ev{});
    }));
    hipLaunchKernelGGL(step_check_kernel, dim3((unsigned)ni), dim3(kDtSlots), 0, ctx->stream, ctx->B.slots,
                       ctx->B.dscal, ctx->B.flags, ctx->B.iflags);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(hflags, ctx->B.flags, kNumFlags * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipMemcpyAsync(hflags + kNumFlags, ctx->B.iflags, ni * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    return ESDG_OK;
}

int clear_step_flags(esdg_ctx *ctx)
{
    const int ni = n_inst(ctx);
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0, ctx->stream,
                       ctx->B.iflags, 0, ni);
    CK(hipGetLastError());
    return reset_flags(ctx);
}

}  // namespace

extern "C" {

int esdg_ensemble_step(esdg_ensemble *en, int nsteps)
{
    if (!en) return ESDG_EINVAL;
    if (nsteps < 0) return efail(en, ESDG_EINVAL, "nsteps < 0");
    TRY(ensemble_build(en));
    if (hipSetDevice(en->device) != hipSuccess) return efail(en, ESDG_EHIP, "hipSetDevice failed");
    for (auto &G : en->groups) {
        const int st = reset_flags(G.ctx);
        if (st) return efail_ctx(en, G.ctx, st);
    }
    // interleave the degrees step by step; each degree's launches are
    // ordered on its own stream.  Groups with step retries launch their step
    // and its check first; then the host waits for each and relaunches the
    // groups with instances to redo, until none is left.
    bool negmean = false;
    const size_t ng = en->groups.size();
    std::vector<int> base(ng);
    std::vector<std::vector<int>> tries(ng);
    for (size_t g = 0; g < ng; ++g) {
        auto &G = en->groups[g];
        if (G.ctx->P.max_dt_retries > 0 && !G.hflags) {
            const size_t nb = (kNumFlags + 2 * (size_t)n_inst(G.ctx)) * sizeof(int);
            if (hipHostMalloc((void **)&G.hflags, nb, hipHostMallocDefault) != hipSuccess)
                return efail(en, ESDG_ENOMEM, "hipHostMalloc failed");
        }
    }
    for (int it = 0; it < nsteps; ++it) {
        std::vector<size_t> pending;
        for (size_t g = 0; g < ng; ++g) {
            auto &G = en->groups[g];
            int st;
            if (G.ctx->P.max_dt_retries > 0) {
                base[g] = G.ctx->cur;
                tries[g].assign(n_inst(G.ctx), 0);
                st = clear_step_flags(G.ctx);
                if (!st) st = group_attempt(G.ctx, base[g], true, G.hflags);
                pending.push_back(g);
            } else {
                st = graph_ready(G.ctx, 0.0) ? graph_step(G.ctx, 0.0) : launch_one_step(G.ctx, 0.0);
            }
            if (st) return efail_ctx(en, G.ctx, st);
        }
        while (!pending.empty()) {
            std::vector<size_t> again;
            for (size_t g : pending) {
                auto &G = en->groups[g];
                esdg_ctx *c = G.ctx;
                if (hipStreamSynchronize(c->stream) != hipSuccess)
                    return efail(en, ESDG_EHIP, "hipStreamSynchronize failed");
                const int ni = n_inst(c);
                const int *fl = G.hflags, *ifl = G.hflags + kNumFlags;
                int *mask = G.hflags + kNumFlags + ni;
                if (fl[kFlagNonFinite]) return efail(en, ESDG_ENONFINITE, "non-finite value in a stage output");
                if (fl[kFlagDtPos]) return efail(en, ESDG_EDTPOS, "no admissible time step");
                bool any = false;
                for (int k = 0; k < ni; ++k) {
                    mask[k] = (ifl[k] != 0 && tries[g][k] < c->P.max_dt_retries) ? 1 : 0;
                    any = any || mask[k];
                    // an instance out of retries keeps its step (a redo of
                    // the others skips it, so its flags are taken here)
                    if (!mask[k] && (ifl[k] & 1)) negmean = true;
                }
                if (!any) continue;
                for (int k = 0; k < ni; ++k) tries[g][k] += mask[k];
                int st = ESDG_OK;
                if (hipMemcpyAsync(c->B.imask, mask, ni * sizeof(int), hipMemcpyHostToDevice, c->stream) !=
                    hipSuccess)
                    return efail(en, ESDG_EHIP, "hipMemcpyAsync failed");
                hipLaunchKernelGGL(scale_steps_masked_kernel, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0,
                                   c->stream, c->B.dscal, c->B.imask, 0.5, ni);
                st = clear_step_flags(c);
                if (!st) st = group_attempt(c, base[g], false, G.hflags);
                if (st) return efail_ctx(en, c, st);
                again.push_back(g);
            }
            pending.swap(again);
        }
    }
    int status = negmean ? ESDG_ENEGMEAN : ESDG_OK;
    for (auto &G : en->groups) {
        int flags[kNumFlags];
        const int st = read_flags(G.ctx, flags);
        if (st) return efail_ctx(en, G.ctx, st);
        if (flags[kFlagNonFinite]) return efail(en, ESDG_ENONFINITE, "non-finite value in a stage output");
        if (flags[kFlagDtPos]) return efail(en, ESDG_EDTPOS, "no admissible time step");
        if (flags[kFlagNegMean] && G.ctx->P.max_dt_retries <= 0) status = ESDG_ENEGMEAN;
    }
    if (status) return efail(en, status, "negative element mean in the limiter");
    return ESDG_OK;
}

int esdg_ensemble_set_graphs(esdg_ensemble *en, int enable)
{
    if (!en) return ESDG_EINVAL;
    TRY(ensemble_build(en));
    for (auto &G : en->groups) {
        const int st = esdg_set_graphs(G.ctx, enable);
        if (st) return efail_ctx(en, G.ctx, st);
    }
    return ESDG_OK;
}

int esdg_ensemble_size(const esdg_ensemble *en, int *n)
{
    if (!en || !n) return ESDG_EINVAL;
    *n = (int)en->inst.size();
    return ESDG_OK;
}

int esdg_ensemble_get_state(esdg_ensemble *en, int id, double *h, double *hu, double *hv, int mem)
{
    if (!en || !h || !hu || !hv) return ESDG_EINVAL;
    if (id < 0 || id >= (int)en->inst.size()) return efail(en, ESDG_EINVAL, "no such instance");
    TRY(ensemble_build(en));
    if (hipSetDevice(en->device) != hipSuccess) return efail(en, ESDG_EHIP, "hipSetDevice failed");
    const auto &I = en->inst[id];
    auto &G = en->groups[I.group];
    const int64_t npn = (int64_t)(G.N + 1) * (G.N + 1);
    const int64_t n = nodes(G.ctx);
    int st = esdg_get_state(G.ctx, G.scratch, G.scratch + n, G.scratch + 2 * n, 1);
    if (st) return efail_ctx(en, G.ctx, st);
    double *dst[3] = {h, hu, hv};
    for (int c = 0; c < 3; ++c)
        if (hipMemcpyAsync(dst[c], G.scratch + c * n + I.off * npn, I.K * npn * sizeof(double),
                           mem ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, G.stream) != hipSuccess)
            return efail(en, ESDG_EHIP, "hipMemcpyAsync failed");
    if (hipStreamSynchronize(G.stream) != hipSuccess) return efail(en, ESDG_EHIP, "hipStreamSynchronize failed");
    return ESDG_OK;
}

int esdg_ensemble_get_time(esdg_ensemble *en, int id, double *t)
{
    if (!en || !t) return ESDG_EINVAL;
    if (id < 0 || id >= (int)en->inst.size()) return efail(en, ESDG_EINVAL, "no such instance");
    TRY(ensemble_build(en));
    const auto &I = en->inst[id];
    auto &G = en->groups[I.group];
    if (hipSetDevice(en->device) != hipSuccess ||
        hipMemcpyAsync(t, G.ctx->B.dscal + 8 * I.local + 4, sizeof(double), hipMemcpyDeviceToHost, G.stream) !=
            hipSuccess ||
        hipStreamSynchronize(G.stream) != hipSuccess)
        return efail(en, ESDG_EHIP, "time download failed");
    return ESDG_OK;
}

int esdg_ensemble_autotune(esdg_ensemble *en, int reps, int *choices)
{
    if (!en) return ESDG_EINVAL;
    TRY(ensemble_build(en));
    for (size_t g = 0; g < en->groups.size(); ++g) {
        int c = 0;
        const int st = esdg_autotune(en->groups[g].ctx, reps, &c, nullptr);
        if (st) return efail_ctx(en, en->groups[g].ctx, st);
        if (choices) choices[g] = c;
    }
    return ESDG_OK;
}

int esdg_ensemble_degrees(const esdg_ensemble *en, int *n, int *N)
{
    if (!en || !n) return ESDG_EINVAL;
    *n = (int)en->groups.size();
    if (N)
        for (size_t g = 0; g < en->groups.size(); ++g) N[g] = en->groups[g].N;
    return ESDG_OK;
}

const char *esdg_ensemble_last_error(const esdg_ensemble *en)
{
    return en ? en->err.c_str() : "null ensemble";
}

}  // extern "C"

// ==========================================================================
// Discrete adjoint: gauges, gauge-misfit loss, checkpointed reverse sweep
// ==========================================================================
namespace {

__global__ void fill_double_kernel(double *p, double v, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

constexpr int kGaugeThreads = 128;   // >= (N+1)^2 for every degree

// Water surface H = h + b interpolated at every gauge point: workgroup g
// reduces the weighted nodal values of gauge g.
__global__ __launch_bounds__(kGaugeThreads) void gauge_kernel(const double *__restrict__ h,
                                                              const double *__restrict__ b,
                                                              const int32_t *__restrict__ gel,
                                                              const double *__restrict__ gw, int np,
                                                              double *__restrict__ out)
{
    __shared__ double s[kGaugeThreads];
    const int g = blockIdx.x, p = threadIdx.x;
    const int64_t o = (int64_t)gel[g] * np;
    s[p] = p < np ? gw[(int64_t)g * np + p] * (h[o + p] + b[o + p]) : 0.0;
    __syncthreads();
    for (int st = kGaugeThreads / 2; st > 0; st >>= 1) {
        if (p < st) s[p] += s[p + st];
        __syncthreads();
    }
    if (p == 0) out[g] = s[0];
}

// Cotangent of one step's gauge misfit, w (H_g - T_g) l_g, added to dL/dh and
// to dL/db at the nodes of the gauge's element.  Workgroup u takes the u-th
// element holding gauges (gauges sorted by element: uorder[ustart[u] ..
// ustart[u+1]) are its gauges, summed in that order), lane p its node p.
__global__ __launch_bounds__(kGaugeThreads) void gauge_adjoint_kernel(
    const double *__restrict__ H, const double *__restrict__ Tg, double w, const int32_t *__restrict__ uel,
    const int32_t *__restrict__ ustart, const int32_t *__restrict__ uorder, const double *__restrict__ gw, int np,
    double *ah, double *gbn)
{
    const int u = blockIdx.x, p = threadIdx.x;
    if (p >= np) return;
    double c = 0.0;
    for (int k = ustart[u]; k < ustart[u + 1]; ++k) {
        const int g = uorder[k];
        c += (H[g] - Tg[g]) * w * gw[(int64_t)g * np + p];
    }
    const int64_t q = (int64_t)uel[u] * np + p;
    ah[q] += c;
    gbn[q] += c;
}

// L = 1/2 dt sum (H - T)^2 over every step and gauge (one workgroup).
__global__ void misfit_loss_kernel(const double *__restrict__ H, const double *__restrict__ Tg, int64_t n,
                                   double dt, double *out)
{
    __shared__ double s[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t k = t; k < n; k += 256) {
        const double r = H[k] - Tg[k];
        acc += r * r;
    }
    s[t] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) s[t] += s[t + st];
        __syncthreads();
    }
    if (t == 0) out[0] = 0.5 * dt * s[0];
}

int fill(esdg_ctx *ctx, double *p, double v, int64_t n)
{
    const int64_t want = (n + 255) / 256;
    hipLaunchKernelGGL(fill_double_kernel, dim3((unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096)), dim3(256), 0,
                       ctx->stream, p, v, n);
    CK(hipGetLastError());
    return ESDG_OK;
}

bool check_adjoint_ctx(esdg_ctx *ctx)
{
    if (!check_ctx(ctx, true)) return false;
    if (ctx->prec != 64) return fail(ctx, ESDG_EINVAL, "the adjoint needs a float64 context"), false;
    if (ctx->P.av_on) return fail(ctx, ESDG_EINVAL, "the adjoint covers the inviscid operator (av_on = 0)"), false;
    if (n_inst(ctx) != 1) return fail(ctx, ESDG_EINVAL, "the adjoint runs on single-instance contexts"), false;
    return true;
}

// Cotangent fields (allocated once per mesh).
int adj_fields(esdg_ctx *ctx)
{
    auto &A = ctx->adj;
    const int64_t n = nodes(ctx);
    if (!A.lam) TRY(alloc(ctx, &A.lam, 12 * n * sizeof(double)));
    if (!A.gbf) TRY(alloc(ctx, &A.gbf, 4 * n * sizeof(double)));
    if (!A.loss) TRY(alloc(ctx, &A.loss, sizeof(double)));
    return ESDG_OK;
}

// Grow a [slots][3][n] state array.
int adj_slots(esdg_ctx *ctx, double **p, int64_t *cap, int64_t want)
{
    if (*cap >= want) return ESDG_OK;
    if (*p) CK(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    TRY(alloc(ctx, p, (size_t)want * 3 * nodes(ctx) * sizeof(double)));
    *cap = want;
    return ESDG_OK;
}

int copy_state(esdg_ctx *ctx, double *dst, void *const src[3])
{
    const int64_t n = nodes(ctx);
    for (int c = 0; c < 3; ++c)
        CK(hipMemcpyAsync(dst + c * n, src[c], n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    return ESDG_OK;
}

// One forward stage k from state `in` to `out` (the stage kernel of
// esdg_step, writing the given buffers): LSRK(5,4), or SSPRK(3,3) with the
// step's start state `base`.
int adj_forward_stage(esdg_ctx *ctx, double *in, double *out, double *base, int k)
{
    Bufs B2 = ctx->B;
    const int64_t n = nodes(ctx);
    for (int c = 0; c < 3; ++c) {
        B2.W[0][c] = in + c * n;
        B2.W[1][c] = out + c * n;
        B2.W[2][c] = base + c * n;
    }
    StageCall sc = ctx->P.integrator == 1
                       ? StageCall{kModeSsp, false, 0, 1, 2, false, kSspAlpha[k], kSspBeta[k], false, false}
                       : StageCall{kModeLsrk, false, 0, 1, 0, false, kLsrkA[k], kLsrkB[k], false, k < 4};
    sc.variant = ctx->stage_variant;
    CK(dispatch(ctx, [&](auto L, auto r) {
        using R = decltype(r);
        return decltype(L)::stage(B2, sc, phys<R>(ctx), tab<R>(ctx), ctx->stream, Ev{});
    }));
    return ESDG_OK;
}

int adj_stage(esdg_ctx *ctx, const AdjCall &c)
{
    return timed(ctx, kProfAdjoint, [&](Ev ev) {
        return dispatch(ctx, [&](auto L, auto r) {
            using R = decltype(r);
            return decltype(L)::adjoint_stage(ctx->B, c, phys<R>(ctx), tab<R>(ctx), ctx->stream, ev);
        });
    });
}

int adj_assemble_b(esdg_ctx *ctx)
{
    const int64_t n = nodes(ctx);
    double *g = ctx->adj.gbf;
    CK(dispatch(ctx, [&](auto L, auto) {
        return decltype(L)::bathymetry_adjoint(ctx->B, ctx->td, g, g + n, g + 2 * n, g + 3 * n, ctx->stream);
    }));
    return ESDG_OK;
}

int gauge_values_into(esdg_ctx *ctx, int buf_or_neg, const double *state_h, double *out)
{
    auto &A = ctx->adj;
    const int np = (ctx->N + 1) * (ctx->N + 1);
    const double *h = state_h ? state_h : (const double *)ctx->B.W[buf_or_neg][0];
    hipLaunchKernelGGL(gauge_kernel, dim3((unsigned)A.ng), dim3(kGaugeThreads), 0, ctx->stream, h,
                       (const double *)ctx->B.b, A.gel, A.gw, np, out);
    CK(hipGetLastError());
    return ESDG_OK;
}

}  // namespace

extern "C" {

int esdg_set_gauges(esdg_ctx *ctx, int ng, const int32_t *elem, const double *xi, const double *eta)
{
    if (!ctx) return ESDG_EINVAL;
    if (!ctx->have_mesh) return fail(ctx, ESDG_EINVAL, "upload_mesh first");
    if (ng < 1 || !elem || !xi || !eta) return fail(ctx, ESDG_EINVAL, "gauges: need ng >= 1 and three arrays");
    CK(hipSetDevice(ctx->device));
    const int N = ctx->N, nf = N + 1, np = nf * nf;
    std::vector<int32_t> gel(ng);
    std::vector<double> gw((size_t)ng * np);
    for (int g = 0; g < ng; ++g) {
        if (elem[g] < 0 || elem[g] >= ctx->K) return fail(ctx, ESDG_EINVAL, "gauge %d: element out of range", g);
        if (!(std::fabs(xi[g]) <= 1.0) || !(std::fabs(eta[g]) <= 1.0))
            return fail(ctx, ESDG_EINVAL, "gauge %d: reference point outside [-1, 1]^2", g);
        gel[g] = ctx->inv_h[elem[g]];
        // Lagrange basis of the LGL nodes at xi and eta
        long double lx[kMaxNF], le[kMaxNF];
        for (int k = 0; k < nf; ++k) {
            long double px = 1.0L, pe = 1.0L;
            for (int m = 0; m < nf; ++m)
                if (m != k) {
                    const long double d = ctx->ht.x[k] - ctx->ht.x[m];
                    px *= ((long double)xi[g] - ctx->ht.x[m]) / d;
                    pe *= ((long double)eta[g] - ctx->ht.x[m]) / d;
                }
            lx[k] = px;
            le[k] = pe;
        }
        for (int i = 0; i < nf; ++i)
            for (int j = 0; j < nf; ++j) gw[(size_t)g * np + i * nf + j] = (double)(lx[i] * le[j]);
    }
    // gauges grouped by element (stable: gauge order inside an element)
    std::vector<int32_t> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return gel[a] < gel[c]; });
    std::vector<int32_t> uel, ustart;
    for (int k = 0; k < ng; ++k)
        if (k == 0 || gel[order[k]] != gel[order[k - 1]]) {
            uel.push_back(gel[order[k]]);
            ustart.push_back(k);
        }
    ustart.push_back(ng);
    const int nu = (int)uel.size();
    std::vector<int32_t> ug(uel);
    ug.insert(ug.end(), ustart.begin(), ustart.end());
    ug.insert(ug.end(), order.begin(), order.end());
    auto &A = ctx->adj;
    for (void *p : {(void *)A.gel, (void *)A.gw, (void *)A.gH, (void *)A.ug})
        if (p) CK(hipFree(p));
    A.gel = nullptr; A.gw = nullptr; A.gH = nullptr; A.ug = nullptr; A.ng = 0; A.nu = 0; A.ready = false;
    TRY(alloc(ctx, &A.gel, ng * sizeof(int32_t)));
    TRY(alloc(ctx, &A.gw, gw.size() * sizeof(double)));
    TRY(alloc(ctx, &A.gH, ng * sizeof(double)));
    TRY(alloc(ctx, &A.ug, ug.size() * sizeof(int32_t)));
    CK(hipMemcpyAsync(A.gel, gel.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    CK(hipMemcpyAsync(A.gw, gw.data(), gw.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    CK(hipMemcpyAsync(A.ug, ug.data(), ug.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    A.ng = ng;
    A.nu = nu;
    return ESDG_OK;
}

int esdg_gauge_values(esdg_ctx *ctx, double *H, int mem)
{
    if (!H) return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_ctx(ctx, true)) return ESDG_EINVAL;
    if (ctx->prec != 64) return fail(ctx, ESDG_EINVAL, "gauges need a float64 context");
    if (ctx->adj.ng < 1) return fail(ctx, ESDG_EINVAL, "esdg_set_gauges first");
    TRY(gauge_values_into(ctx, ctx->cur, nullptr, ctx->adj.gH));
    CK(hipMemcpyAsync(H, ctx->adj.gH, ctx->adj.ng * sizeof(double),
                      mem ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_rhs_vjp(esdg_ctx *ctx, const double *lh, const double *lhu, const double *lhv, double *gh, double *ghu,
                 double *ghv, double *gb, int mem)
{
    if (!lh || !lhu || !lhv || !gh || !ghu || !ghv || !gb)
        return ctx ? fail(ctx, ESDG_EINVAL, "null pointer") : ESDG_EINVAL;
    if (!check_adjoint_ctx(ctx)) return ESDG_EINVAL;
    TRY(adj_fields(ctx));
    const int64_t n = nodes(ctx), per = n / ctx->K;
    double *L = ctx->adj.lam;   // [0..2] result, [6..8] input cotangent
    TRY(upload_field(ctx, L + 6 * n, lh, per, mem));
    TRY(upload_field(ctx, L + 7 * n, lhu, per, mem));
    TRY(upload_field(ctx, L + 8 * n, lhv, per, mem));
    TRY(fill(ctx, ctx->adj.gbf, 0.0, 3 * n));
    AdjCall c{};
    for (int k = 0; k < 3; ++k) {
        c.W[k] = ctx->B.W[ctx->cur][k];
        c.a[k] = nullptr;
        c.c[k] = L + (6 + k) * n;
        c.ao[k] = L + k * n;
        c.co[k] = nullptr;
    }
    c.gbx = ctx->adj.gbf;
    c.gby = ctx->adj.gbf + n;
    c.gbn = ctx->adj.gbf + 2 * n;
    c.ca = 0.0;
    c.cb = 0.0;
    c.dt = 1.0;
    TRY(adj_stage(ctx, c));
    TRY(adj_assemble_b(ctx));
    TRY(download_field(ctx, gh, L, per, mem));
    TRY(download_field(ctx, ghu, L + n, per, mem));
    TRY(download_field(ctx, ghv, L + 2 * n, per, mem));
    TRY(download_field(ctx, gb, ctx->adj.gbf + 3 * n, per, mem));
    if (mem) CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

int esdg_adjoint_forward(esdg_ctx *ctx, int nsteps, double dt, int every, const double *target, int mem,
                         double *loss, double *H)
{
    if (!target) return ctx ? fail(ctx, ESDG_EINVAL, "null target") : ESDG_EINVAL;
    if (!check_adjoint_ctx(ctx)) return ESDG_EINVAL;
    auto &A = ctx->adj;
    if (A.ng < 1) return fail(ctx, ESDG_EINVAL, "esdg_set_gauges first");
    if (nsteps < 1 || every < 1 || !(dt > 0.0) || !std::isfinite(dt))
        return fail(ctx, ESDG_EINVAL, "need nsteps >= 1, every >= 1 and a finite dt > 0");
    A.ready = false;
    TRY(adj_fields(ctx));
    const int64_t nseg = (nsteps + every - 1) / every;
    TRY(adj_slots(ctx, &A.ckpt, &A.ckpt_cap, nseg));
    const int64_t nh = (int64_t)nsteps * A.ng;
    if (A.h_cap < nh) {
        if (A.Hg) CK(hipFree(A.Hg));
        if (A.Tg) CK(hipFree(A.Tg));
        A.Hg = A.Tg = nullptr;
        A.h_cap = 0;
        TRY(alloc(ctx, &A.Hg, nh * sizeof(double)));
        TRY(alloc(ctx, &A.Tg, nh * sizeof(double)));
        A.h_cap = nh;
    }
    CK(hipMemcpyAsync(A.Tg, target, nh * sizeof(double), mem ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                      ctx->stream));
    const int64_t n = nodes(ctx);
    TRY(reset_flags(ctx));
    for (int it = 0; it < nsteps; ++it) {
        if (it % every == 0) TRY(copy_state(ctx, A.ckpt + (it / every) * 3 * n, ctx->B.W[ctx->cur]));
        TRY(launch_one_step(ctx, dt));
        TRY(gauge_values_into(ctx, ctx->cur, nullptr, A.Hg + (int64_t)it * A.ng));
    }
    hipLaunchKernelGGL(misfit_loss_kernel, dim3(1), dim3(256), 0, ctx->stream, A.Hg, A.Tg, nh, dt, A.loss);
    CK(hipGetLastError());
    int flags[kNumFlags];
    TRY(read_flags(ctx, flags));
    if (flags[kFlagNegMean] || flags[kFlagLimited])
        return fail(ctx, ESDG_EINVAL, "the limiter acted during the run: outside the adjoint's scope");
    if (loss) {
        CK(hipMemcpyAsync(loss, A.loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    if (H) {
        CK(hipMemcpyAsync(H, A.Hg, nh * sizeof(double), mem ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
    }
    A.nsteps = nsteps;
    A.every = every;
    A.dt = dt;
    A.b_version = ctx->b_version;
    A.P = ctx->P;
    A.ready = true;
    return ESDG_OK;
}

int esdg_adjoint_backward(esdg_ctx *ctx, double seed, double *gb, double *gh0, double *ghu0, double *ghv0, int mem)
{
    if (!gb) return ctx ? fail(ctx, ESDG_EINVAL, "null gb") : ESDG_EINVAL;
    if (!check_adjoint_ctx(ctx)) return ESDG_EINVAL;
    auto &A = ctx->adj;
    if (!A.ready) return fail(ctx, ESDG_EINVAL, "esdg_adjoint_forward first");
    if (A.b_version != ctx->b_version) return fail(ctx, ESDG_EINVAL, "the bathymetry changed since the forward sweep");
    if (!same_params(A.P, ctx->P)) return fail(ctx, ESDG_EINVAL, "the parameters changed since the forward sweep");
    if (!std::isfinite(seed)) return fail(ctx, ESDG_EINVAL, "seed must be finite");
    const int64_t n = nodes(ctx), per = n / ctx->K;
    const int np = (ctx->N + 1) * (ctx->N + 1);
    const bool ssp = ctx->P.integrator == 1;
    const int S = ssp ? 3 : 5;   // stages per step
    TRY(adj_slots(ctx, &A.store, &A.store_cap, (int64_t)std::min(A.every, A.nsteps) * S + 1));
    double *lamA[2] = {A.lam, A.lam + 3 * n}, *lamC[2] = {A.lam + 6 * n, A.lam + 9 * n};
    double *gbx = A.gbf, *gby = A.gbf + n, *gbn = A.gbf + 2 * n;
    TRY(fill(ctx, A.gbf, 0.0, 3 * n));
    TRY(fill(ctx, lamA[0], 0.0, 3 * n));
    // the recomputed stages read the step from the scalar block
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->B.dscal, A.dt, 1);
    CK(hipGetLastError());
    int pa = 0;
    const int nseg = (A.nsteps + A.every - 1) / A.every;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * A.every, s1 = std::min(A.nsteps, s0 + A.every);
        // recompute the segment from its checkpoint, keeping every stage input
        CK(hipMemcpyAsync(A.store, A.ckpt + (int64_t)seg * 3 * n, 3 * n * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
        for (int it = s0; it < s1; ++it)
            for (int k = 0; k < S; ++k) {
                const int64_t s = (int64_t)(it - s0) * S, sl = s + k;
                TRY(adj_forward_stage(ctx, A.store + sl * 3 * n, A.store + (sl + 1) * 3 * n, A.store + s * 3 * n,
                                      k));
            }
        // reverse the steps of the segment
        for (int it = s1 - 1; it >= s0; --it) {
            hipLaunchKernelGGL(gauge_adjoint_kernel, dim3((unsigned)A.nu), dim3(kGaugeThreads), 0, ctx->stream,
                               A.Hg + (int64_t)it * A.ng, A.Tg + (int64_t)it * A.ng, seed * A.dt, A.ug,
                               A.ug + A.nu, A.ug + 2 * A.nu + 1, A.gw, np, lamA[pa], gbn);
            CK(hipGetLastError());
            if (ssp) {
                // dL/dW_{k-1} = beta_k (a + dt (dR/dW)^T a); the alpha_k a
                // terms of dL/dW^n are summed in lamC[0] and added by stage 0
                double *z = lamC[0];
                for (int k = 2; k >= 0; --k) {
                    const int64_t sl = (int64_t)(it - s0) * 3 + k;
                    AdjCall c{};
                    for (int q = 0; q < 3; ++q) {
                        c.W[q] = A.store + (sl * 3 + q) * n;
                        c.a[q] = lamA[pa] + q * n;
                        c.c[q] = nullptr;
                        c.ao[q] = lamA[1 - pa] + q * n;
                        c.co[q] = k == 0 ? nullptr : z + q * n;
                        c.y[q] = k == 1 ? z + q * n : nullptr;
                        c.x[q] = k == 0 ? z + q * n : nullptr;
                    }
                    c.gbx = gbx;
                    c.gby = gby;
                    c.gbn = gbn;
                    c.ca = kSspAlpha[k] / kSspBeta[k];
                    c.cb = kSspBeta[k];
                    c.sa = kSspBeta[k];
                    c.dt = A.dt;
                    TRY(adj_stage(ctx, c));
                    pa = 1 - pa;
                }
                continue;
            }
            for (int k = 4; k >= 0; --k) {
                const int64_t sl = (int64_t)(it - s0) * 5 + k;
                AdjCall c{};
                for (int q = 0; q < 3; ++q) {
                    c.W[q] = A.store + (sl * 3 + q) * n;
                    c.a[q] = lamA[pa] + q * n;
                    c.c[q] = k == 4 ? nullptr : lamC[pa] + q * n;
                    c.ao[q] = lamA[1 - pa] + q * n;
                    c.co[q] = k == 0 ? nullptr : lamC[1 - pa] + q * n;
                }
                c.gbx = gbx;
                c.gby = gby;
                c.gbn = gbn;
                c.ca = kLsrkA[k];
                c.cb = kLsrkB[k];
                c.dt = A.dt;
                TRY(adj_stage(ctx, c));
                pa = 1 - pa;
            }
        }
    }
    TRY(adj_assemble_b(ctx));
    TRY(download_field(ctx, gb, A.gbf + 3 * n, per, mem));
    if (gh0) TRY(download_field(ctx, gh0, lamA[pa], per, mem));
    if (ghu0) TRY(download_field(ctx, ghu0, lamA[pa] + n, per, mem));
    if (ghv0) TRY(download_field(ctx, ghv0, lamA[pa] + 2 * n, per, mem));
    CK(hipStreamSynchronize(ctx->stream));
    return ESDG_OK;
}

}  // extern "C"

// ==========================================================================
// Empirical LDS roofline (the paper's shared-memory roofline): 16-byte LDS
// reads in the volume term's pattern, an 8 x 8 element per wave read along
// its lines (row reads are shared by the 8 lanes of a row, column reads are
// 8 different addresses), with one FMA per read so the ALUs stay idle.
// ==========================================================================
namespace {

constexpr int kLdsProbeThreads = 256;

__global__ __launch_bounds__(kLdsProbeThreads) void lds_probe_kernel(int iters, double *out)
{
    __shared__ double2 s[kLdsProbeThreads];
    const int t = threadIdx.x;
    s[t] = double2{(double)t, 1.0 + t};
    __syncthreads();
    const int base = t & ~63, row = (t & 63) >> 3, col = t & 7;
    double ax = 0.0, ay = 0.0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int mm = (m + it) & 7;   // the addresses change every iteration: nothing to hoist
            const double2 a = s[base + row * 8 + mm];
            const double2 b = s[base + mm * 8 + col];
            ax = fma(a.x, b.y, ax);
            ay = fma(a.y, b.x, ay);
        }
    }
    out[(int64_t)blockIdx.x * kLdsProbeThreads + t] = ax + ay;
}

}  // namespace

extern "C" {

int esdg_lds_bandwidth(int device, double *bytes_per_s)
{
    if (!bytes_per_s) return ESDG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ESDG_EHIP;
    const int blocks = 256 * 16, iters = 256;
    double *out = nullptr;
    if (hipMalloc((void **)&out, (size_t)blocks * kLdsProbeThreads * sizeof(double)) != hipSuccess)
        return ESDG_ENOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = ESDG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = ESDG_EHIP;
    float best = 0.0f;
    for (int rep = 0; rep < 4 && st == ESDG_OK; ++rep) {
        hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(kLdsProbeThreads), 0, nullptr, iters, out);
        hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess) { st = ESDG_EHIP; break; }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best == 0.0f || ms < best)) best = ms;   // the first launch warms up
    }
    if (st == ESDG_OK) {
        const double bytes = (double)blocks * kLdsProbeThreads * iters * 8 * 2 * 16;
        *bytes_per_s = bytes / (best * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}

}  // extern "C"
