// Instantiation of the kernels for one polynomial degree ESDG_N (set by the
// build, one object file per degree so the degrees compile in parallel).
#include <hip/hip_ext.h>

#include <type_traits>

#include "esdg_adjoint.hpp"
#include "esdg_kernels.hpp"
#include "esdg_launch.hpp"

#ifndef ESDG_N
#error "ESDG_N must be defined"
#endif

namespace esdg {

template <typename R>
static Mesh<R> mesh_view(const Bufs &B)
{
    Mesh<R> m;
    m.K = B.K;
    m.Ax = (const R *)B.Ax;
    m.Cx = (const R *)B.Cx;
    m.Ae = (const R *)B.Ae;
    m.Ce = (const R *)B.Ce;
    m.bx = (const R *)B.bx;
    m.by = (const R *)B.by;
    m.mref = (const R *)B.mref;
    m.xr = B.xr;
    m.yr = B.yr;
    m.bface = (const R *)B.bface;
    m.nbr = B.nbr;
    m.code = B.code;
    m.walls = B.walls;
    return m;
}

// Kernel launch with the optional timing events recorded by the dispatch
// itself; without events a plain launch (which stream capture records as a
// kernel node).
template <typename Kern, typename... Args>
static void launch_ev(Kern kernel, dim3 grid, dim3 block, hipStream_t s, Ev ev, Args... args)
{
    if (ev.a) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev.a, ev.b, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

template <int N>
static int64_t ntiles_of(int64_t K)
{
    return (K + Shape<N>::E - 1) / Shape<N>::E;
}

template <int N>
static dim3 tile_grid(int64_t K)
{
    const int64_t nt = ntiles_of<N>(K);
    return dim3((unsigned)(((nt + kXcds - 1) / kXcds) * kXcds));
}

template <int N, typename R>
int Launch<N, R>::threads() { return Shape<N>::T; }

template <int N, typename R>
int Launch<N, R>::elems_per_block() { return Shape<N>::E; }

template <int N, typename R>
hipError_t Launch<N, R>::geometry(const Bufs &B, const Tab<double> &td, hipStream_t s)
{
    constexpr int np = (N + 1) * (N + 1);
    const int64_t n = B.K * np;
    const int bs = 256;
    hipLaunchKernelGGL((geometry_kernel<N, R>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, B.K,
                       B.x, B.y, (R *)B.Ax, (R *)B.Cx, (R *)B.Ae, (R *)B.Ce, (R *)B.mref, B.xr, B.yr, B.flags + kFlagBadJ,
                       td);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gmax_kernel<N, R>), dim3((unsigned)((B.K + bs - 1) / bs)), dim3(bs), 0, s,
                       mesh_view<R>(B), (R *)B.gmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nfn = B.K * 4 * (N + 1);
    hipLaunchKernelGGL((face_geometry_kernel<N, R>), dim3((unsigned)((nfn + bs - 1) / bs)), dim3(bs), 0, s,
                       mesh_view<R>(B), (R)td.w[0], (R *)B.fgeo);
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::bathymetry(const Bufs &B, const double *b, const Tab<double> &td, hipStream_t s)
{
    constexpr int np = (N + 1) * (N + 1);
    const int64_t n = B.K * np;
    const int bs = 256;
    hipLaunchKernelGGL((bathymetry_kernel<N, R>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, B.K,
                       B.x, B.y, b, (R *)B.bx, (R *)B.by, (R *)B.bface, td);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((convert_kernel<double, R>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, b,
                       (R *)B.b, n);
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::indicator(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, hipStream_t s,
                                   Ev ev)
{
    IndicatorArgs<N, R> a;
    a.P = P;
    a.tab = t;
    a.tg = (const Tab<R> *)B.tabg;
    a.K = B.K;
    a.h = (const R *)B.W[buf][0];
    a.eps = (R *)B.eps[buf];
    a.list = B.list[buf];
    a.count = B.count + buf;
    a.ntiles = ntiles_of<N>(B.K);
    launch_ev(indicator_kernel<N, R>, tile_grid<N>(B.K), dim3(Shape<N>::T), s, ev, a);
    return hipGetLastError();
}

template <int N, typename R>
static ListArgs<N, R> list_args(const Bufs &B, int in, const Phys<R> &P, const Tab<R> &t)
{
    ListArgs<N, R> a;
    a.m = mesh_view<R>(B);
    a.P = P;
    a.tab = t;
    a.tg = (const Tab<R> *)B.tabg;
    a.h = (const R *)B.W[in][0];
    a.hu = (const R *)B.W[in][1];
    a.hv = (const R *)B.W[in][2];
    a.eps = (const R *)B.eps[in];
    a.list = B.list[in];
    a.count = B.count + in;
    a.vtr = (R *)B.vtr;
    a.lv2 = (R *)B.lv[0];
    a.lv3 = (R *)B.lv[1];
    a.count_reset = nullptr;
    return a;
}

// Fixed grid for the list passes: a few workgroups per CU, grid-stride over
// the list (its length is only known on the device).
constexpr unsigned kListBlocks = 1024;

template <int N, typename R>
hipError_t Launch<N, R>::av_faces(const Bufs &B, int in, const Phys<R> &P, const Tab<R> &t, hipStream_t s,
                                  Ev ev)
{
    launch_ev(av_faces_kernel<N, R>, dim3(kListBlocks), dim3(Shape<N>::T), s, ev, list_args<N, R>(B, in, P, t));
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::av_div(const Bufs &B, int in, int reset, const Phys<R> &P, const Tab<R> &t,
                                hipStream_t s, Ev ev)
{
    ListArgs<N, R> a = list_args<N, R>(B, in, P, t);
    a.count_reset = reset >= 0 ? B.count + reset : nullptr;
    launch_ev(av_div_kernel<N, R>, dim3(kListBlocks), dim3(Shape<N>::T), s, ev, a);
    return hipGetLastError();
}

template <int N, typename R, int MODE, int V>
static void launch_stage_variant(StageArgs<R> a, int64_t K, hipStream_t s, Ev ev)
{
    using S = TileShape<N, StageCfg<N, V>::T>;
    a.ntiles = (K + S::E - 1) / S::E;
    const dim3 grid((unsigned)(((a.ntiles + kXcds - 1) / kXcds) * kXcds));
    launch_ev(stage_kernel<N, R, MODE, V>, grid, dim3(S::T), s, ev, a);
}

template <int N, typename R, int MODE>
static void launch_stage(StageArgs<R> a, int64_t K, hipStream_t s, Ev ev)
{
    // the compiled variants of the stage kernel (the autotuner picks one)
    switch (a.variant) {
    case 1: launch_stage_variant<N, R, MODE, 1>(a, K, s, ev); break;
    case 2: launch_stage_variant<N, R, MODE, 2>(a, K, s, ev); break;
    case 3: launch_stage_variant<N, R, MODE, 3>(a, K, s, ev); break;
    case 4: launch_stage_variant<N, R, MODE, 4>(a, K, s, ev); break;
    default: launch_stage_variant<N, R, MODE, 0>(a, K, s, ev); break;
    }
}

template <int N, typename R>
hipError_t Launch<N, R>::stage(const Bufs &B, const StageCall &c, const Phys<R> &P, const Tab<R> &t,
                               hipStream_t s, Ev ev)
{
    StageArgs<R> a;
    a.m = mesh_view<R>(B);
    a.P = P;
    a.tab = t;
    a.tg = (const Tab<R> *)B.tabg;
    a.h = (const R *)B.W[c.in][0];
    a.hu = (const R *)B.W[c.in][1];
    a.hv = (const R *)B.W[c.in][2];
    a.h0 = (const R *)B.W[c.base][0];
    a.hu0 = (const R *)B.W[c.base][1];
    a.hv0 = (const R *)B.W[c.base][2];
    void *const *o = c.out_rhs ? B.Rb : B.W[c.out];
    a.oh = (R *)o[0];
    a.ohu = (R *)o[1];
    a.ohv = (R *)o[2];
    a.dh = (R *)B.dU[0];
    a.dhu = (R *)B.dU[1];
    a.dhv = (R *)B.dU[2];
    a.store_du = c.store_du ? 1 : 0;
    a.eps = c.av ? (const R *)B.eps[c.in] : nullptr;
    a.vtr = (const R *)B.vtr;
    a.lv2 = (const R *)B.lv[0];
    a.lv3 = (const R *)B.lv[1];
    a.eps_out = c.out_rhs ? nullptr : (R *)B.eps[c.out];
    a.list_out = c.out_rhs ? nullptr : B.list[c.out];
    a.count_out = c.out_rhs ? nullptr : B.count + c.out;
    a.dtc_out = c.dt_next && !c.out_rhs ? (R *)B.dtc : nullptr;
    a.dtv_out = c.dt_next && !c.out_rhs && c.av ? (R *)B.dtv : nullptr;
    a.frec_out = c.dt_next && !c.out_rhs && P.limiter_on ? (R *)B.frec : nullptr;
    a.gmax = (const R *)B.gmax;
    a.inst = B.n_inst > 1 ? B.inst : nullptr;
    a.dt = B.dscal;
    a.ca = (R)c.ca;
    a.cb = (R)c.cb;
    a.flags = B.flags;
    a.iflags = B.iflags;
    a.imask = (c.masked && a.inst) ? B.imask : nullptr;
    a.variant = c.variant;
    if (c.mode == kModeRhs) launch_stage<N, R, kModeRhs>(a, B.K, s, ev);
    else if (c.mode == kModeLsrk) launch_stage<N, R, kModeLsrk>(a, B.K, s, ev);
    else launch_stage<N, R, kModeSsp>(a, B.K, s, ev);
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::limit(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, hipStream_t s)
{
    hipLaunchKernelGGL((limit_kernel<N, R>), tile_grid<N>(B.K), dim3(Shape<N>::T), 0, s, mesh_view<R>(B), P,
                       t, (R *)B.W[buf][0], (R *)B.W[buf][1], (R *)B.W[buf][2], B.flags, ntiles_of<N>(B.K));
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::dt(const Bufs &B, int in, bool av, bool fused, const Phys<R> &P, hipStream_t s, Ev ev)
{
    DtArgs<R> a;
    a.m = mesh_view<R>(B);
    a.P = P;
    a.h = (const R *)B.W[in][0];
    a.hu = (const R *)B.W[in][1];
    a.hv = (const R *)B.W[in][2];
    a.eps = av && !fused ? (const R *)B.eps[in] : nullptr;
    a.dtc = fused ? (const R *)B.dtc : nullptr;
    a.dtv = fused && av ? (const R *)B.dtv : nullptr;
    a.gmax = (const R *)B.gmax;
    a.fgeo = (const R *)B.fgeo;
    a.frec = fused && P.limiter_on ? (const R *)B.frec : nullptr;
    a.slots = B.slots;
    a.cstart = B.cstart;
    a.cinst = B.cinst;
    a.nchunks = B.nchunks;
    if (B.n_inst > 1) {
        const unsigned grid = (unsigned)(B.nchunks < (int64_t)kDtMaxBlocks ? B.nchunks : (int64_t)kDtMaxBlocks);
        launch_ev(dt_batch_kernel<N, R>, dim3(grid), dim3(kDtThreads), s, ev, a);
        return hipGetLastError();
    }
    constexpr int64_t np = (N + 1) * (N + 1);
    const int64_t items = fused ? B.K * 4 * (N + 1) : B.K * np;
    const int64_t want = ((items + kDtThreads * kXcds - 1) / (kDtThreads * kXcds)) * kXcds;
    const unsigned grid = (unsigned)(want < (int64_t)kDtMaxBlocks ? want : (int64_t)kDtMaxBlocks);
    launch_ev(dt_kernel<N, R>, dim3(grid), dim3(kDtThreads), s, ev, a);
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::diag(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, int64_t *nblocks,
                              hipStream_t s)
{
    constexpr int np = (N + 1) * (N + 1), T = Shape<N>::T;
    const int64_t nb = (B.K * np + T - 1) / T;
    *nblocks = nb;
    if (nb > B.part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL((diag_kernel<N, R>), dim3((unsigned)nb), dim3(T), 0, s, mesh_view<R>(B), P, t,
                       (const R *)B.W[buf][0], (const R *)B.W[buf][1], (const R *)B.W[buf][2],
                       (const R *)B.b, (const R *)B.Rb[0], (const R *)B.Rb[1], (const R *)B.Rb[2], B.part);
    return hipGetLastError();
}

template <int N, typename R>
hipError_t Launch<N, R>::adjoint_stage(const Bufs &B, const AdjCall &c, const Phys<R> &P, const Tab<R> &t,
                                       hipStream_t s, Ev ev)
{
    if constexpr (std::is_same<R, double>::value) {
        AdjArgs a;
        a.m = mesh_view<double>(B);
        a.P = P;
        a.tab = t;
        a.tg = (const Tab<double> *)B.tabg;
        a.h = (const double *)c.W[0];
        a.hu = (const double *)c.W[1];
        a.hv = (const double *)c.W[2];
        for (int k = 0; k < 3; ++k) {
            a.a[k] = (const double *)c.a[k];
            a.c[k] = (const double *)c.c[k];
            a.ao[k] = (double *)c.ao[k];
            a.co[k] = (double *)c.co[k];
            a.x[k] = (const double *)c.x[k];
            a.y[k] = (const double *)c.y[k];
        }
        a.gbx = c.gbx;
        a.gby = c.gby;
        a.gbn = c.gbn;
        a.ca = c.ca;
        a.cb = c.cb;
        a.dt = c.dt;
        a.sa = c.sa;
        a.ntiles = ntiles_of<N>(B.K);
        launch_ev(adjoint_stage_kernel<N>, tile_grid<N>(B.K), dim3(Shape<N>::T), s, ev, a);
        return hipGetLastError();
    } else {
        (void)B; (void)c; (void)P; (void)t; (void)s; (void)ev;
        return hipErrorNotSupported;
    }
}

template <int N, typename R>
hipError_t Launch<N, R>::bathymetry_adjoint(const Bufs &B, const Tab<double> &td, const double *gbx,
                                            const double *gby, const double *gbn, double *gb, hipStream_t s)
{
    if constexpr (std::is_same<R, double>::value) {
        constexpr int np = (N + 1) * (N + 1);
        const int64_t n = B.K * np;
        const int bs = 256;
        hipLaunchKernelGGL((bathymetry_adjoint_kernel<N>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                           B.K, (const double *)B.Ax, (const double *)B.Cx, (const double *)B.Ae,
                           (const double *)B.Ce, gbx, gby, gbn, gb, td);
        return hipGetLastError();
    } else {
        (void)B; (void)td; (void)gbx; (void)gby; (void)gbn; (void)gb; (void)s;
        return hipErrorNotSupported;
    }
}

template struct Launch<ESDG_N, double>;
template struct Launch<ESDG_N, float>;

}  // namespace esdg
