// Device kernels of the entropy-stable DGSEM shallow-water solver for gfx950.
//
// Work decomposition: a workgroup holds E elements of (N+1)^2 nodes, one
// thread per node (E ~ 256 / (N+1)^2, so a workgroup is four 64-wide waves);
// nodal state and the contravariant metric directions are staged in LDS, the
// state arrays are read and written in the coalesced SoA order
// [K][(N+1)^2], and the face work of the E elements is spread over the same
// threads (one face node per thread and pass).  Workgroup -> element-tile
// mapping is XCD-aware so that each of the eight XCDs sweeps one contiguous
// block of tiles and neighbour traces mostly hit its own L2.
//
// Kernels (per RK stage): av_kernel (artificial viscosity: element
// viscosity from the modal indicator and the BR1 viscous fluxes on the
// element faces, only with AV on), stage_kernel (split-form volume term,
// interface flux, source, viscous divergence, stage update and positivity
// limiter, fused); per step: dt_kernel + dt_finalize_kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "esdg_tables.hpp"

namespace esdg {

// ------------------------------------------------------------------------
// Shapes
// ------------------------------------------------------------------------
// Workgroup shape per degree.  Where whole elements fill a 64-wide wave
// with (almost) no idle lanes (N = 2, 3, 7) a workgroup is one wave: its
// barriers are cheap and waves run independently.  Otherwise four waves
// hold E = floor(256/(N+1)^2) elements packed across the waves.
template <int N>
struct Shape {
    static constexpr int nf = N + 1;
    static constexpr int np = nf * nf;
    static constexpr bool one_wave = (np <= 64) && (64 - (64 / np) * np) * 16 <= 64;
    static constexpr int T = one_wave ? 64 : 256;                  // threads per workgroup
    static constexpr int E = (T / np) > 0 ? (T / np) : 1;          // elements per workgroup
    static constexpr int NFACE = E * 4 * nf;                       // face-node slots per workgroup
    static_assert(E * np <= T, "elements must fit the workgroup");
};

// The alternative workgroup size of the stage kernel: 256 threads where the
// default is one wave, else 128.
template <int N>
struct AltThreads {
    static constexpr int value = Shape<N>::T == 64 ? 256 : 128;
};

template <int N, int TT>
struct TileShape {
    static constexpr int nf = N + 1;
    static constexpr int np = nf * nf;
    static constexpr int T = TT;
    static constexpr int E = (T / np) > 0 ? (T / np) : 1;
    static constexpr int NFACE = E * 4 * nf;
    static_assert(E * np <= T, "elements must fit the workgroup");
};

// Compiled variants of the stage kernel, chosen at run time by the
// autotuner (esdg_autotune); every variant does the same arithmetic per
// element in the same order (results are bitwise the same):
//   0  the default tile of Shape, its register budget and partner unroll;
//   1  the alternative workgroup size (AltThreads), no register budget;
//   2  the default tile with one wave per SIMD less in its register budget
//      (more registers, no spills where the default spills);
//   3  the default tile with the other partner-loop unroll (full where the
//      default unrolls partly, by two where it unrolls fully);
//   4  the default tile with bank-conflict-free staging rows: padded by one
//      node (the paper's LDS padding, appendix C), or at N = 7 XOR-swizzled
//      columns (no more LDS; StageCfg::SWZ).
// Default register budget in the FP64 update modes: six waves per SIMD at
// N = 6, five otherwise (N = 7 reaches six by its partner-loop unroll); in
// the FP32 update modes eight (seven for variant 2, none for variant 1): left
// free, the compiler gave some FP32 variants 100-120 registers; no
// constraint in the right-hand-side mode.  Default unroll: fully,
// except at N = 7 with one-wave tiles (by two: 79 VGPRs and six waves per
// SIMD instead of five), N = 6 (by two) and N = 8 (by three: five waves).
constexpr int kStageVariants = 5;

template <int N, int V>
struct StageCfg {
    static_assert(V >= 0 && V < kStageVariants, "stage variant");
    static constexpr int T = V == 1 ? AltThreads<N>::value : Shape<N>::T;
    static constexpr int base_waves = V == 1 ? 1 : ((N == 6 || N == 7) ? 6 : 5);
    static constexpr int waves = V == 2 ? base_waves - 1 : base_waves;
    static constexpr int vu_default = (N == 7 && T == 64) ? 2 : (N == 8 ? 3 : (N == 6 ? 2 : N + 1));
    static constexpr int VU = V == 3 ? (vu_default == N + 1 ? 2 : N + 1) : vu_default;
    // Variant 4 avoids the LDS bank conflicts of the eta-direction partner
    // reads (a wave reads column mm of every row, rows 16(N+1) bytes apart in
    // FP64: at N = 7 eight rows on two bank groups).  At N = 7 the columns of
    // row i are XOR-swizzled (node (i, j) in column j ^ (i >> 1)), which puts
    // the eight rows' reads on distinct banks in both directions with no more
    // LDS; at the other degrees, whose N + 1 is no power of two, each row is
    // padded by one node.
    static constexpr bool SWZ = V == 4 && N == 7;
    static constexpr int PAD = (V == 4 && !SWZ) ? 1 : 0;
};

// Column of node (i, j) in its LDS staging row (see StageCfg::SWZ).
template <int N, int V>
__device__ __forceinline__ int stage_col(int i, int j)
{
    if constexpr (StageCfg<N, V>::SWZ) return j ^ (i >> 1);
    else return j;
}

template <int N, typename R, int MODE, int V>
struct StageWaves {
    static constexpr int value =
        MODE == 0 ? 1 : (sizeof(R) == 8 ? StageCfg<N, V>::waves : (V == 1 ? 1 : (V == 2 ? 7 : 8)));
};

// Workgroup barrier for exchanges through LDS only: orders LDS accesses
// without waiting for outstanding global loads and stores (which
// __syncthreads() would).  A one-wave workgroup needs no barrier.
template <int T>
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    if constexpr (T > 64) __builtin_amdgcn_s_barrier();
    else __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kXcds = 8;
constexpr int kDtSlots = 64;

// Device status flags of a context: negative element mean, limited
// elements, no admissible step, J <= 0 at mesh upload, non-finite output.
constexpr int kFlagNegMean = 0, kFlagLimited = 1, kFlagDtPos = 2, kFlagBadJ = 3, kFlagNonFinite = 4;
// a step that exceeded twice the CFL / viscous bound of the state it produced
constexpr int kFlagStepBound = 5;
constexpr int kNumFlags = 8;

// Tile of workgroup b when B = round_up(ntiles, 8) workgroups are launched:
// hardware places workgroup b on XCD b % 8, so XCD x gets tiles
// [x*per, (x+1)*per).  Tiles >= ntiles return -1.
__device__ inline int64_t xcd_tile(int64_t ntiles)
{
    const int64_t b = blockIdx.x;
    const int64_t per = (ntiles + kXcds - 1) / kXcds;
    const int64_t tile = (b % kXcds) * per + b / kXcds;
    return tile < ntiles ? tile : -1;
}

// Face node k of local side s -> local (i, j).
template <int N>
__device__ __forceinline__ void side_node(int s, int k, int &i, int &j)
{
    i = (s == 0 || s == 2) ? k : (s == 1 ? N : 0);
    j = (s == 1 || s == 3) ? k : (s == 2 ? N : 0);
}

// ------------------------------------------------------------------------
// Arguments
// ------------------------------------------------------------------------
template <typename R>
struct Tab {
    R D[kMaxNF * kMaxNF];     // derivative matrix, row-major
    R Dz[kMaxNF * kMaxNF];    // the same with a zero diagonal (flux differencing)
    R Vinv[kMaxNF * kMaxNF];  // Vandermonde inverse
    R w[kMaxNF];              // LGL weights
    R iw0;                    // 1 / w_0 (end weight)
};

template <typename R>
struct Mesh {
    int64_t K;
    const R *Ax, *Cx;   // J grad(xi)  = ( y_eta, -x_eta)  [K][np]
    const R *Ae, *Ce;   // J grad(eta) = (-y_xi,   x_xi)   [K][np]
    const R *bx, *by;   // split-form bathymetry derivatives (eq. SourceDisc)
    const double *xr, *yr;  // float64 coordinates less the element's first node [K][np] (float64 contexts)
    const R *mref;      // float32 contexts: [K][4] (Ax, Cx, Ae, Ce) of each element's middle node
    const R *bface;     // bathymetry on the faces [K][4][nf]
    const int32_t *nbr; // [K][4] neighbour element
    const int8_t *code; // [K][4] neighbour side | flip << 2 | wall << 3 (a wall names the element itself)
    int walls;          // some side is a wall (else the wall bit is never looked at)
};

// Single precision stores the metric terms of each node less those of its
// element's middle node (Mesh::mref): differences between an element's
// nodes, which the jump-form volume sums take, are then rounded at the size
// of the terms' variation across the element rather than of the terms.  On a
// fine mesh the terms vary little across an element, and their rounding at
// full size breaks the discrete metric identities by far more than the
// arithmetic's own rounding.  The terms themselves are the sums.
template <typename R>
constexpr bool kMetricRel = sizeof(R) == 4;

// Metric terms J grad(xi) = (Ax, Cx), J grad(eta) = (Ae, Ce) at node q of
// element e.
template <typename R>
__device__ __forceinline__ void metric_at(const Mesh<R> &m, int64_t q, int64_t e, R &Ax, R &Cx, R &Ae, R &Ce)
{
    Ax = m.Ax[q]; Cx = m.Cx[q]; Ae = m.Ae[q]; Ce = m.Ce[q];
    if constexpr (kMetricRel<R>) {
        const R *r = m.mref + 4 * e;
        Ax += r[0]; Cx += r[1]; Ae += r[2]; Ce += r[3];
    }
}

template <typename R>
struct Phys {
    R g, h_tol, eps0, sigma_min, sigma_max, cfl, cfl_visc;
    R i2g;                 // 1 / (2 g)
    R ratio_min, ratio_max; // 10^sigma_min, 10^sigma_max
    R visc_c, br1;          // viscous bound: visc_c / (br1 eps max|grad|^2)
    int ec, limiter_on;
};

// Neighbour node of face node (s, k) of element e.  At a solid wall the face
// map names the element's own side (the node itself): the interface flux then
// mirrors the velocity (is_wall), the viscous terms see no jump.
template <int N, typename R>
__device__ __forceinline__ int64_t nbr_node(const Mesh<R> &m, int64_t e, int s, int k,
                                           int64_t &en, int &ns, int &kk)
{
    constexpr int nf = N + 1, np = nf * nf;
    en = m.nbr[e * 4 + s];
    const int c = m.code[e * 4 + s];
    ns = c & 3;
    kk = ((c >> 2) & 1) ? N - k : k;
    int i, j;
    side_node<N>(ns, kk, i, j);
    return en * np + i * nf + j;
}

template <typename R>
__device__ __forceinline__ bool is_wall(const Mesh<R> &m, int64_t e, int s)
{
    return m.walls && ((m.code[e * 4 + s] >> 3) & 1);
}

// Reflecting-wall outside state: the velocity with its normal component
// reversed about the unit normal (nx, ny); height and bathymetry unchanged.
template <typename R>
__device__ __forceinline__ void wall_mirror(R nx, R ny, R &u, R &v)
{
    const R dn = u * nx + v * ny;
    u -= R(2) * dn * nx;
    v -= R(2) * dn * ny;
}

// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (quadratic convergence; normal positive x)
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <typename R>
__device__ __forceinline__ R rcp_wet(R h, R h_tol)
{
    return h > h_tol ? rcp_nr(h) : R(0);
}

// The single-precision stage kernel forms the volume and interface terms from
// jumps to the own node (interface_flux_delta and the volume loop): the
// two-point sums of flux-sized terms whose result is a derivative lose the
// flux-to-derivative ratio (about N^2 / element size) in relative accuracy,
// which double precision absorbs and single precision does not.
template <typename R>
constexpr bool kJumpForm = sizeof(R) == 4;

// At N <= 4 the double-precision stage kernel reads each node's two
// coordinates (relative to its element's first node) instead of its four
// metric terms and forms the metric terms itself, with the sums of
// geometry_kernel in the same order (so bit for bit the stored values): 16
// fewer bytes per node and stage for 4(N+1) multiply-adds and two more
// workgroup barriers.  Measured on the stage kernel: 3-7% faster at N = 2..4,
// 5-7% slower at N = 5..8, where the registers it holds across the face
// prefetch cost occupancy or spills.  In single precision the four metric
// terms take as many bytes as the two float64 coordinates.
template <int N, typename R>
constexpr bool kMetricInKernel = sizeof(R) == 8 && N <= 4;

// Rotated numerical interface flux along the unit normal (nx, ny), '-' =
// own trace, '+' = neighbour (appendix B): EC part plus, for the entropy
// stable flux, -1/2 R |Lambda| R^T [[q~]] expanded in closed form.
// Velocities are the primitive ones (zero at dry nodes).
template <typename R>
__device__ __forceinline__ void interface_flux(R hm, R um, R vm, R bm, R hp, R up, R vp, R bp, R nx, R ny,
                                               const Phys<R> &P, R &F0, R &F1, R &F2)
{
    const R g = P.g;
    const R utm = nx * um + ny * vm, vtm = nx * vm - ny * um;
    const R utp = nx * up + ny * vp, vtp = nx * vp - ny * up;
    const R cm = sqrt(g * fmax(hm, R(0)));
    const R cp = sqrt(g * fmax(hp, R(0)));
    const R ah = R(0.5) * (hm + hp), au = R(0.5) * (utm + utp), av = R(0.5) * (vtm + vtp);
    const R ah2 = R(0.5) * (hm * hm + hp * hp), ac = R(0.5) * (cm + cp);
    R f0 = ah * au;
    R f1 = ah * au * au + R(0.5) * g * ah2;
    R f2 = ah * au * av;
    if (!P.ec) {
        const R dq1 = g * ((hp + bp) - (hm + bm)) -
                      R(0.5) * ((utp * utp + vtp * vtp) - (utm * utm + vtm * vtm));
        const R dq2 = utp - utm, dq3 = vtp - vtm;
        const R lp = fabs(au + ac) * P.i2g, l2 = fabs(ah * au), lm = fabs(au - ac) * P.i2g;
        const R r1 = lp * (dq1 + (au + ac) * dq2 + av * dq3);
        const R r2 = l2 * dq3;
        const R r3 = lm * (dq1 + (au - ac) * dq2 + av * dq3);
        f0 -= R(0.5) * (r1 + r3);
        f1 -= R(0.5) * ((au + ac) * r1 + (au - ac) * r3);
        f2 -= R(0.5) * (av * (r1 + r3) + r2);
    }
    F0 = f0;
    F1 = nx * f1 - ny * f2;
    F2 = ny * f1 + nx * f2;
}

// The same interface flux less the own trace's physical flux along n,
// f*(-, +) - f(-).n, written in the jumps dh = h+ - h-, du, dv only (the
// single-precision stage kernel).  With a mean m = a- + d/2:
//   {h}{u_n} - h- u_n-           = (h- du_n + dh {u_n}) / 2
//   {h}{u_n}^2 - h- u_n-^2       = {u_n} df0 + du_n h- u_n- / 2
//   g/2 ({h^2} - h-^2)           = g dh {h} / 2
//   {h}{u_n}{v_t} - h- u_n- v_t- = {v_t} df0 + dv_t h- u_n- / 2
// and, in the dissipation, [[g(h+b) - |u|^2/2]] with |u+|^2 - |u-|^2 =
// du (u+ + u-) + dv (v+ + v-).  The own flux is the row-sum part of the
// volume term's two-point sums at a face node, where it cancels against this
// subtracted part; formed from the jumps, neither part is rounded at the
// size of the flux itself, only at the size of its variation.
template <typename R>
__device__ __forceinline__ void interface_flux_delta(R hm, R um, R vm, R bm, R hp, R up, R vp, R bp, R nx,
                                                     R ny, const Phys<R> &P, R &F0, R &F1, R &F2)
{
    const R g = P.g;
    const R dh = hp - hm, du = up - um, dv = vp - vm;
    const R utm = nx * um + ny * vm, vtm = nx * vm - ny * um;
    const R dut = nx * du + ny * dv, dvt = nx * dv - ny * du;
    const R ah = R(0.5) * (hm + hp), au = utm + R(0.5) * dut, av = vtm + R(0.5) * dvt;
    const R fo = hm * utm;
    R f0 = R(0.5) * (hm * dut + dh * au);
    R f1 = au * f0 + R(0.5) * (dut * fo + g * dh * ah);
    R f2 = av * f0 + R(0.5) * dvt * fo;
    if (!P.ec) {
        const R cm = sqrt(g * fmax(hm, R(0)));
        const R cp = sqrt(g * fmax(hp, R(0)));
        const R ac = R(0.5) * (cm + cp);
        const R dq1 = g * (dh + (bp - bm)) - R(0.5) * (du * (up + um) + dv * (vp + vm));
        const R dq2 = dut, dq3 = dvt;
        const R lp = fabs(au + ac) * P.i2g, l2 = fabs(ah * au), lm = fabs(au - ac) * P.i2g;
        const R r1 = lp * (dq1 + (au + ac) * dq2 + av * dq3);
        const R r2 = l2 * dq3;
        const R r3 = lm * (dq1 + (au - ac) * dq2 + av * dq3);
        f0 -= R(0.5) * (r1 + r3);
        f1 -= R(0.5) * ((au + ac) * r1 + (au - ac) * r3);
        f2 -= R(0.5) * (av * (r1 + r3) + r2);
    }
    F0 = f0;
    F1 = nx * f1 - ny * f2;
    F2 = ny * f1 + nx * f2;
}

// ------------------------------------------------------------------------
// Geometry: metric terms by the derivative matrix (eq. NablaRelation)
// ------------------------------------------------------------------------
template <int N, typename R>
__global__ void geometry_kernel(int64_t K, const double *__restrict__ x, const double *__restrict__ y,
                                R *Ax, R *Cx, R *Ae, R *Ce, R *mref, double *xr, double *yr, int *bad,
                                Tab<double> tab)
{
    constexpr int nf = N + 1, np = nf * nf;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * np) return;
    const int64_t e = q / np;
    const int p = (int)(q - e * np), i = p / nf, j = p - i * nf;
    const double *xe = x + e * np, *ye = y + e * np;
    // differentiate coordinates relative to the element's first node: the
    // metric terms are translation invariant and the sums stay at the
    // element's size (no cancellation against the absolute position)
    const double x0 = xe[0], y0 = ye[0];
    double xxi = 0, xeta = 0, yxi = 0, yeta = 0;
#pragma unroll
    for (int m = 0; m < nf; ++m) {
        xxi += tab.D[i * kMaxNF + m] * (xe[m * nf + j] - x0);
        yxi += tab.D[i * kMaxNF + m] * (ye[m * nf + j] - y0);
        xeta += tab.D[j * kMaxNF + m] * (xe[i * nf + m] - x0);
        yeta += tab.D[j * kMaxNF + m] * (ye[i * nf + m] - y0);
    }
    const double J = xxi * yeta - xeta * yxi;
    if (!(J > 0.0)) atomicOr(bad, 1);
    // the differenced coordinates themselves, for the float64 stage kernel,
    // which forms the same sums from them (the same values bit for bit)
    if (xr) {
        xr[q] = xe[p] - x0;
        yr[q] = ye[p] - y0;
    }
    if constexpr (kMetricRel<R>) {
        // the middle node's terms by the same sums, rounded, and each node's
        // terms less them (kMetricRel)
        constexpr int c = N / 2;
        double cxxi = 0, cxeta = 0, cyxi = 0, cyeta = 0;
#pragma unroll
        for (int m = 0; m < nf; ++m) {
            cxxi += tab.D[c * kMaxNF + m] * (xe[m * nf + c] - x0);
            cyxi += tab.D[c * kMaxNF + m] * (ye[m * nf + c] - y0);
            cxeta += tab.D[c * kMaxNF + m] * (xe[c * nf + m] - x0);
            cyeta += tab.D[c * kMaxNF + m] * (ye[c * nf + m] - y0);
        }
        const R r0 = (R)cyeta, r1 = (R)(-cxeta), r2 = (R)(-cyxi), r3 = (R)cxxi;
        if (p == 0) {
            mref[4 * e + 0] = r0;
            mref[4 * e + 1] = r1;
            mref[4 * e + 2] = r2;
            mref[4 * e + 3] = r3;
        }
        Ax[q] = (R)(yeta - (double)r0);
        Cx[q] = (R)(-xeta - (double)r1);
        Ae[q] = (R)(-yxi - (double)r2);
        Ce[q] = (R)(xxi - (double)r3);
    } else {
        Ax[q] = (R)yeta;
        Cx[q] = (R)(-xeta);
        Ae[q] = (R)(-yxi);
        Ce[q] = (R)xxi;
    }
}

// Split-form bathymetry derivatives (eq. SourceDisc, read with D) and face
// traces of b; metrics recomputed in float64 from the coordinates.
template <int N, typename R>
__global__ void bathymetry_kernel(int64_t K, const double *__restrict__ x, const double *__restrict__ y,
                                  const double *__restrict__ b, R *bx, R *by, R *bface,
                                  Tab<double> tab)
{
    constexpr int nf = N + 1, np = nf * nf;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * np) return;
    const int64_t e = q / np;
    const int p = (int)(q - e * np), i = p / nf, j = p - i * nf;
    const double *xe = x + e * np, *ye = y + e * np, *be = b + e * np;
    // metric terms at the line nodes are needed inside D(y_eta b) etc.
    const double x0 = xe[0], y0 = ye[0];
    auto met = [&](int a, int c, double &xxi, double &xeta, double &yxi, double &yeta) {
        xxi = xeta = yxi = yeta = 0.0;
        for (int m = 0; m < nf; ++m) {
            xxi += tab.D[a * kMaxNF + m] * (xe[m * nf + c] - x0);
            yxi += tab.D[a * kMaxNF + m] * (ye[m * nf + c] - y0);
            xeta += tab.D[c * kMaxNF + m] * (xe[a * nf + m] - x0);
            yeta += tab.D[c * kMaxNF + m] * (ye[a * nf + m] - y0);
        }
    };
    double Db_xi = 0, Dyb_xi = 0, Dxb_xi = 0, Db_eta = 0, Dyb_eta = 0, Dxb_eta = 0;
    for (int m = 0; m < nf; ++m) {
        double a0, a1, a2, a3;
        const double dxi = tab.D[i * kMaxNF + m], deta = tab.D[j * kMaxNF + m];
        met(m, j, a0, a1, a2, a3);   // node (m, j)
        const double bm = be[m * nf + j];
        Db_xi += dxi * bm;
        Dyb_xi += dxi * (a3 * bm);   // y_eta b
        Dxb_xi += dxi * (a1 * bm);   // x_eta b
        met(i, m, a0, a1, a2, a3);   // node (i, m)
        const double bn = be[i * nf + m];
        Db_eta += deta * bn;
        Dyb_eta += deta * (a2 * bn); // y_xi b
        Dxb_eta += deta * (a0 * bn); // x_xi b
    }
    double xxi, xeta, yxi, yeta;
    met(i, j, xxi, xeta, yxi, yeta);
    bx[q] = (R)(yeta * Db_xi + Dyb_xi - yxi * Db_eta - Dyb_eta);
    by[q] = (R)(-xeta * Db_xi - Dxb_xi + xxi * Db_eta + Dxb_eta);
    // face traces: thread of a face node writes every side the node is on
    if (j == 0) bface[(e * 4 + 0) * nf + i] = (R)be[p];
    if (i == N) bface[(e * 4 + 1) * nf + j] = (R)be[p];
    if (j == N) bface[(e * 4 + 2) * nf + i] = (R)be[p];
    if (i == 0) bface[(e * 4 + 3) * nf + j] = (R)be[p];
}

// ------------------------------------------------------------------------
// Cross-lane reductions inside one wave with DPP moves (GFX9 encodings:
// quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, row_mirror = 0x140,
// row_half_mirror = 0x141, row_bcast:15 = 0x142, row_bcast:31 = 0x143).
// Lanes of rows outside ROWMASK receive an unspecified value.  Called in
// uniform control flow with every lane of the wave active.
// ------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, ROWMASK, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

__device__ __forceinline__ double read_lane63(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float read_lane63(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <bool MIN, int CTRL, int ROWMASK, typename R>
__device__ __forceinline__ R dpp_step(R v)
{
    const R o = dpp_mov<CTRL, ROWMASK>(v);
    return MIN ? fmin(o, v) : v + o;
}

// Sum (MIN: minimum) over the 16 lanes of each row, in every lane of the row
// (the four patterns read valid lanes only).
template <bool MIN, typename R>
__device__ __forceinline__ R row16_reduce(R v)
{
    v = dpp_step<MIN, 0xB1, 0xF>(v);
    v = dpp_step<MIN, 0x4E, 0xF>(v);
    v = dpp_step<MIN, 0x141, 0xF>(v);
    return dpp_step<MIN, 0x140, 0xF>(v);
}

// Sum (MIN: minimum) over the 64 lanes of the wave, in every lane: the row
// totals are carried into lane 63 (rows 1, 3 add row 0, 2; rows 2, 3 add
// lane 31), whose value is broadcast; the other lanes' partials are not used.
template <bool MIN, typename R>
__device__ __forceinline__ R wave64_reduce(R v)
{
    v = row16_reduce<MIN>(v);
    v = dpp_step<MIN, 0x142, 0xA>(v);
    v = dpp_step<MIN, 0x143, 0xC>(v);
    return read_lane63(v);
}

// True in every thread if pred holds in some thread of the workgroup.
template <int T>
__device__ __forceinline__ bool block_any(bool pred)
{
    if constexpr (T == 64) return __ballot(pred) != 0ull;   // one wave
    else return __syncthreads_or(pred) != 0;
}

// ------------------------------------------------------------------------
// Workgroup-level per-element reductions over the nodes of each element.
// red: LDS scratch of T*NQ reals; returns the element total in every thread.
// ------------------------------------------------------------------------
template <int N, typename R, int NQ>
struct ElemReduce {
    static constexpr int nf = N + 1, np = nf * nf, E = Shape<N>::E, T = Shape<N>::T;
    // v[0..NQ-1] summed, except v[NQ-1] which is reduced by min when MINLAST
    template <bool MINLAST>
    __device__ __forceinline__ static void run(R (&v)[NQ], R *red, int t, int el, int p)
    {
#pragma unroll
        for (int c = 0; c < NQ; ++c) red[c * T + t] = v[c];
        lds_sync<T>();
        R part[NQ];
        const bool row = (t < E * np) && (p < nf);   // thread (el, p<nf) reduces column p
        if (row) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                R s = red[c * T + el * np + p];
#pragma unroll
                for (int r = 1; r < nf; ++r) {
                    const R val = red[c * T + el * np + r * nf + p];
                    if (MINLAST && c == NQ - 1) s = val < s ? val : s;
                    else s += val;
                }
                part[c] = s;
            }
        }
        lds_sync<T>();
        if (row) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) red[c * T + el * np + p] = part[c];
        }
        lds_sync<T>();
        if (t < E * np) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                R s = red[c * T + el * np];
#pragma unroll
                for (int r = 1; r < nf; ++r) {
                    const R val = red[c * T + el * np + r];
                    if (MINLAST && c == NQ - 1) s = val < s ? val : s;
                    else s += val;
                }
                v[c] = s;
            }
        }
        lds_sync<T>();
    }
};

// Element totals: NQ values per thread summed over the nodes of each element
// (the last reduced by min when MINLAST); only thread p == 0 of each element
// receives the totals.  Two barriers; red: NQ*T reals of LDS.  The caller
// synchronises before reusing red.
template <int N, typename R, int NQ, bool MINLAST, int T = Shape<N>::T>
__device__ __forceinline__ void elem_totals(R (&v)[NQ], R *red, int t, int el, int p, bool lane)
{
    constexpr int nf = N + 1, np = nf * nf;
#pragma unroll
    for (int c = 0; c < NQ; ++c) red[c * T + t] = v[c];
    lds_sync<T>();
    if (lane && p < nf) {
        // column p of element el; its total goes to the column's first slot,
        // which only this thread reads
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            R s = red[c * T + el * np + p];
#pragma unroll
            for (int r = 1; r < nf; ++r) {
                const R val = red[c * T + el * np + r * nf + p];
                if (MINLAST && c == NQ - 1) s = val < s ? val : s;
                else s += val;
            }
            red[c * T + el * np + p] = s;
        }
    }
    lds_sync<T>();
    if (lane && p == 0) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            R s = red[c * T + el * np];
#pragma unroll
            for (int r = 1; r < nf; ++r) {
                const R val = red[c * T + el * np + r];
                if (MINLAST && c == NQ - 1) s = val < s ? val : s;
                else s += val;
            }
            v[c] = s;
        }
    }
}

// Element totals as elem_totals (valid at least in thread p == 0): with lane
// exchanges where an element is one whole wave (np = 64) or one 16-lane row
// of a one-wave workgroup (np = 16), through LDS otherwise.
template <int N, typename R, int NQ, bool MINLAST, int T = Shape<N>::T>
__device__ __forceinline__ void elem_totals_any(R (&v)[NQ], R *red, int t, int el, int p, bool lane)
{
    constexpr int np = (N + 1) * (N + 1);
    if constexpr (np == 64 && T % 64 == 0) {
        // one element per wave
#pragma unroll
        for (int c = 0; c < NQ; ++c)
            v[c] = (MINLAST && c == NQ - 1) ? wave64_reduce<true>(v[c]) : wave64_reduce<false>(v[c]);
    } else if constexpr (np == 16 && T % 64 == 0) {
        // one element per 16-lane row
#pragma unroll
        for (int c = 0; c < NQ; ++c)
            v[c] = (MINLAST && c == NQ - 1) ? row16_reduce<true>(v[c]) : row16_reduce<false>(v[c]);
    } else {
        elem_totals<N, R, NQ, MINLAST, T>(v, red, t, el, p, lane);
    }
}

// ------------------------------------------------------------------------
// Artificial viscosity (appendix A, Theorem 1)
// ------------------------------------------------------------------------
// Viscosity from the indicator's element totals: modal energy of all modes,
// of the top shell, of the modes up to N-1 and of shell N-1; zero for a dry
// element (no node above h_tol).
template <typename R>
__device__ __forceinline__ R viscosity_from_totals(R all, R top, R allM, R topM, bool wet, const Phys<R> &P)
{
    if (!wet) return R(0);
    // smooth elements (both fractions clearly below 10^sigma_min) leave
    // before the divisions; the margin keeps the decision that of the
    // quotients below
    const R pre = R(0.999999) * P.ratio_min;
    if (!(top > pre * all) && !(topM > pre * allM)) return R(0);
    const R r1 = all > R(0) ? top / all : R(0);
    const R r2 = allM > R(0) ? topM / allM : R(0);
    const R rm = r1 > r2 ? r1 : r2;
    // sigma = log10(rm) against the thresholds, compared as rm against
    // 10^sigma (the ramp is continuous at both ends); log10 and sin only on
    // the ramp
    if (!(rm > P.ratio_min)) return R(0);
    if (rm >= P.ratio_max) return P.eps0;
    const R sg = log10(rm);
    const R smin = P.sigma_min, smax = P.sigma_max;
    if (sg >= smax) return P.eps0;
    if (!(sg > smin)) return R(0);
    return R(0.5) * P.eps0 *
           (R(1) + sin(R(3.14159265358979323846) * (sg - R(0.5) * (smax + smin)) / (smax - smin)));
}

// Element viscosity of the elements whose nodal water heights are staged in
// sh[el*np + p]: modal coefficients Q^ = V^{-1} h V^{-T}, the energy
// fractions of the top two mode shells, sigma = log10 of the larger, and the
// sine ramp between sigma_min and sigma_max; zero for dry elements.  The
// result is valid in thread p == 0 of each element.  red: 6*T reals of LDS
// (the last T hold the intermediate V^{-1} h); vinv: V^{-1} row-major with
// row stride N+1, staged in LDS by the caller (stage_vinv).  Three barriers.
template <int N, typename R, int T = Shape<N>::T>
__device__ R element_viscosity(const R *sh, R *red, const R *vinv, const Phys<R> &P, int t, int el, int p,
                               bool lane, R h)
{
    constexpr int nf = N + 1, np = nf * nf;
    const int i = p / nf, j = p - i * nf;
    // single precision transforms h - c (c the element's first nodal height):
    // the higher modes of a smooth element are small against h itself, and
    // in h their FP32 rounding would move the energy ratios, hence eps on
    // the ramp.  A constant has the one mode (0, 0), of coefficient 2c (the
    // orthonormal Legendre L_0 = 1/sqrt(2) in both directions), restored below.
    const R c0 = (kJumpForm<R> && lane) ? sh[el * np] : R(0);
    R Tq = 0;
    if (lane) {
#pragma unroll
        for (int r = 0; r < nf; ++r) Tq += vinv[i * nf + r] * (sh[el * np + r * nf + j] - c0);
    }
    red[5 * T + t] = Tq;
    lds_sync<T>();
    R Qh = 0;
    if (lane) {
#pragma unroll
        for (int c = 0; c < nf; ++c) Qh += red[5 * T + el * np + i * nf + c] * vinv[j * nf + c];
    }
    if constexpr (kJumpForm<R>)
        if (p == 0) Qh += R(2) * c0;
    const R q2 = Qh * Qh;
    const int mx = i > j ? i : j;
    // the energy of all modes is the top shell's plus that of the modes up to N-1
    if constexpr ((np == 64 || np == 16) && T % 64 == 0) {
        // the element's lanes lie in one wave: its wetness by a ballot
        // instead of a max reduction of h
        const uint64_t wm = __ballot(lane && h > P.h_tol);
        const uint64_t mine = np == 64 ? ~0ull : (0xFFFFull << ((t & 63) - p));
        R vals[3] = {mx == N ? q2 : R(0), mx <= N - 1 ? q2 : R(0), mx == N - 1 ? q2 : R(0)};
        elem_totals_any<N, R, 3, false, T>(vals, red, t, el, p, lane);
        return viscosity_from_totals<R>(vals[0] + vals[1], vals[0], vals[1], vals[2], (wm & mine) != 0ull, P);
    } else {
        R vals[4] = {mx == N ? q2 : R(0), mx <= N - 1 ? q2 : R(0), mx == N - 1 ? q2 : R(0),
                     lane ? -h : R(3.0e38)};
        elem_totals_any<N, R, 4, true, T>(vals, red, t, el, p, lane);
        return viscosity_from_totals<R>(vals[0] + vals[1], vals[0], vals[1], vals[2], -vals[3] > P.h_tol, P);
    }
}

// Copy V^{-1} (row stride N+1) into LDS; ordered by the caller's next barrier.
template <int N, typename R, int T>
__device__ __forceinline__ void stage_vinv(R *dst, const Tab<R> &tab, int t)
{
    constexpr int nf = N + 1;
    for (int q = t; q < nf * nf; q += T) dst[q] = tab.Vinv[(q / nf) * kMaxNF + (q - (q / nf) * nf)];
}

// Viscous physical fluxes at node (i,j) of the element whose u, v are in
// LDS (su, sv offset to the element), with U*, V* per face slot in us, vs
// (BR1 gradients of eq. BR1 with the lifted reference derivatives).
template <int N, typename R>
__device__ __forceinline__ void viscous_flux_at(int i, int j, const R *su, const R *sv, const R *us,
                                                const R *vs, R Ax, R Cx, R Ae, R Ce, R he,
                                                const Tab<R> &tab, R &Fv2, R &Fv3, R &Gv2, R &Gv3)
{
    constexpr int nf = N + 1;
    const R u0 = su[i * nf + j], v0 = sv[i * nf + j];
    R dxu = 0, dxv = 0, deu = 0, dev = 0;
    // single precision: the sums over the jumps from the node's own values
    // (D's rows sum to zero), so that neither the rounding of the table's
    // row sums nor that of products at the size of the values themselves
    // enters the derivatives (kJumpForm)
    const R ou = kJumpForm<R> ? u0 : R(0), ov = kJumpForm<R> ? v0 : R(0);
#pragma unroll
    for (int m = 0; m < nf; ++m) {
        const R di = tab.D[i * kMaxNF + m], dj = tab.D[j * kMaxNF + m];
        dxu += di * (su[m * nf + j] - ou);
        dxv += di * (sv[m * nf + j] - ov);
        deu += dj * (su[i * nf + m] - ou);
        dev += dj * (sv[i * nf + m] - ov);
    }
    const R iw = tab.iw0;
    // BR1 lift (U* - u)/w on the faces the node lies on
    if (i == N) { dxu += (us[1 * nf + j] - u0) * iw; dxv += (vs[1 * nf + j] - v0) * iw; }
    if (i == 0) { dxu -= (us[3 * nf + j] - u0) * iw; dxv -= (vs[3 * nf + j] - v0) * iw; }
    if (j == N) { deu += (us[2 * nf + i] - u0) * iw; dev += (vs[2 * nf + i] - v0) * iw; }
    if (j == 0) { deu -= (us[0 * nf + i] - u0) * iw; dev -= (vs[0 * nf + i] - v0) * iw; }
    // J grad = (y_eta d_xi - y_xi d_eta, -x_eta d_xi + x_xi d_eta) = (Ax dxi + Ae deta, Cx dxi + Ce deta)
    const R J = Ce * Ax - Cx * Ae;   // x_xi y_eta - x_eta y_xi
    const R s = he / J;
    Fv2 = s * (Ax * dxu + Ae * deu);
    Gv2 = s * (Cx * dxu + Ce * deu);
    Fv3 = s * (Ax * dxv + Ae * dev);
    Gv3 = s * (Cx * dxv + Ce * dev);
}

// Indicator sweep over all elements (initial data, or after the state was
// replaced): element viscosity, and the list of elements with eps > 0.
template <int N, typename R>
struct IndicatorArgs {
    Phys<R> P;
    Tab<R> tab;                  // uniform entries (read as scalars)
    const Tab<R> *tg;            // the same tables in device memory: per-lane entries
    int64_t K;
    const R *h;
    R *eps;             // [K]
    int32_t *list;      // [K] elements with eps > 0 (order unspecified)
    int *count;         // list length (zeroed beforehand)
    int64_t ntiles;
};

template <int N, typename R>
__global__ __launch_bounds__(Shape<N>::T) void indicator_kernel(IndicatorArgs<N, R> a)
{
    using S = Shape<N>;
    constexpr int np = S::np, E = S::E, T = S::T;
    __shared__ R s_h[T], s_red[6 * T], s_vinv[(N + 1) * (N + 1)];
    const int64_t tile = xcd_tile(a.ntiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    stage_vinv<N, R, T>(s_vinv, *a.tg, t);
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0;
    const int64_t e = tile * E + el;
    const bool act = lane && (e < a.K);
    const R h = act ? a.h[e * np + p] : R(0);
    s_h[t] = h;
    lds_sync<T>();
    const R eps = element_viscosity<N, R>(s_h, s_red, s_vinv, a.P, t, el, p, lane, h);
    if (act && p == 0) {
        a.eps[e] = eps;
        if (eps > R(0)) a.list[atomicAdd(a.count, 1)] = (int32_t)e;
    }
}

// Work over the viscous-element list: groups of E listed elements per
// iteration, grid-stride; an empty list exits at once.
template <int N, typename R>
struct ListArgs {
    Mesh<R> m;
    Phys<R> P;
    Tab<R> tab;                  // uniform entries (read as scalars)
    const Tab<R> *tg;            // the same tables in device memory: per-lane entries
    const R *h, *hu, *hv;     // stage input state
    const R *eps;             // [K] viscosity of this state
    const int32_t *list;      // elements with eps > 0
    const int *count;
    R *vtr;                   // [K][4][nf][4] face viscous fluxes (pass 1 writes, pass 2 reads)
    R *lv2, *lv3;             // [K][np] viscous terms (pass 2)
    int *count_reset;         // pass 2: list counter of the next state, zeroed here
};

// Stage the listed elements' velocities and the BR1 interface states
// U* = {u}, V* = {v} in LDS (shared by both passes).
template <int N, typename R>
__device__ __forceinline__ void load_viscous_element(const ListArgs<N, R> &a, int64_t g, int cnt, int t, int el,
                                                     int p, bool lane, int64_t *s_e, R *s_h, R *s_u, R *s_v,
                                                     R *s_us, R *s_vs, int64_t &e, R &h)
{
    using S = Shape<N>;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T, NF = S::NFACE;
    if (lane && p == 0) s_e[el] = (g * E + el < cnt) ? (int64_t)a.list[g * E + el] : int64_t(-1);
    lds_sync<T>();
    e = s_e[el];
    const bool act = lane && e >= 0;
    const int64_t q = e * np + p;
    h = 0;
    R u = 0, v = 0;
    if (act) {
        h = a.h[q];
        const R ih = rcp_wet(h, a.P.h_tol);
        u = a.hu[q] * ih;
        v = a.hv[q] * ih;
    }
    s_h[t] = h;
    s_u[t] = u;
    s_v[t] = v;
    lds_sync<T>();
    for (int f = t; f < NF; f += T) {
        const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
        const int64_t fe = s_e[fel];
        R us = 0, vs = 0;
        if (fe >= 0) {
            int fi, fj, ns, kk;
            int64_t en;
            side_node<N>(s, k, fi, fj);
            const int lp = fel * np + fi * nf + fj;
            const int64_t qn = nbr_node<N>(a.m, fe, s, k, en, ns, kk);
            const R in = rcp_wet(a.h[qn], a.P.h_tol);
            us = R(0.5) * (s_u[lp] + a.hu[qn] * in);
            vs = R(0.5) * (s_v[lp] + a.hv[qn] * in);
        }
        s_us[f] = us;
        s_vs[f] = vs;
    }
    lds_sync<T>();
}

// Pass 1: the physical viscous fluxes h eps (U1, V1), h eps (U2, V2) on the
// faces of the listed elements (their neighbours' divergence needs them).
template <int N, typename R>
__global__ __launch_bounds__(Shape<N>::T) void av_faces_kernel(ListArgs<N, R> a)
{
    using S = Shape<N>;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T, NF = S::NFACE;
    __shared__ R s_h[T], s_u[T], s_v[T], s_us[NF], s_vs[NF];
    __shared__ int64_t s_e[E];
    const int cnt = *a.count;
    const int t = threadIdx.x;
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0;
    for (int64_t g = blockIdx.x; g * E < cnt; g += gridDim.x) {
        int64_t e;
        R h;
        load_viscous_element<N, R>(a, g, cnt, t, el, p, lane, s_e, s_h, s_u, s_v, s_us, s_vs, e, h);
        for (int f = t; f < NF; f += T) {
            const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
            const int64_t fe = s_e[fel];
            if (fe < 0) continue;
            int fi, fj;
            side_node<N>(s, k, fi, fj);
            const int lp = fel * np + fi * nf + fj;
            const int64_t qo = fe * np + fi * nf + fj;
            R Fv2, Fv3, Gv2, Gv3, oAx, oCx, oAe, oCe;
            metric_at(a.m, qo, fe, oAx, oCx, oAe, oCe);
            viscous_flux_at<N, R>(fi, fj, s_u + fel * np, s_v + fel * np, s_us + fel * 4 * nf,
                                  s_vs + fel * 4 * nf, oAx, oCx, oAe, oCe, s_h[lp] * a.eps[fe], *a.tg, Fv2, Fv3,
                                  Gv2, Gv3);
            R *o = a.vtr + ((fe * 4 + s) * nf + k) * 4;
            o[0] = Fv2;
            o[1] = Fv3;
            o[2] = Gv2;
            o[3] = Gv3;
        }
        lds_sync<T>();
    }
}

// Pass 2: the BR1 viscous divergence (Theorem 1, eq. ViscTermsDisc) L^v on
// the momentum rows of the listed elements, interface fluxes averaged with
// the neighbours' pass-1 fluxes (zero for neighbours without viscosity).
// Elements without viscosity get their (face-only) viscous terms inside the
// stage kernel.
template <int N, typename R>
__global__ __launch_bounds__(Shape<N>::T) void av_div_kernel(ListArgs<N, R> a)
{
    using S = Shape<N>;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T, NF = S::NFACE;
    __shared__ R s_h[T], s_u[T], s_v[T], s_us[NF], s_vs[NF], s_Fv[4][T], s_vn[4][NF];
    __shared__ int64_t s_e[E];
    if (a.count_reset && blockIdx.x == 0 && threadIdx.x == 0) *a.count_reset = 0;
    const int cnt = *a.count;
    const int t = threadIdx.x;
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0, i = p / nf, j = p - i * nf;
    for (int64_t g = blockIdx.x; g * E < cnt; g += gridDim.x) {
        int64_t e;
        R h;
        load_viscous_element<N, R>(a, g, cnt, t, el, p, lane, s_e, s_h, s_u, s_v, s_us, s_vs, e, h);
        const bool act = lane && e >= 0;
        const int64_t q = e * np + p;
        // neighbours' face fluxes
        for (int f = t; f < NF; f += T) {
            const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
            const int64_t fe = s_e[fel];
            R n0 = 0, n1 = 0, n2 = 0, n3 = 0;
            if (fe >= 0) {
                int ns, kk;
                int64_t en;
                (void)nbr_node<N>(a.m, fe, s, k, en, ns, kk);
                if (a.eps[en] > R(0)) {
                    const R *vn = a.vtr + ((en * 4 + ns) * nf + kk) * 4;
                    n0 = vn[0]; n1 = vn[1]; n2 = vn[2]; n3 = vn[3];
                }
            }
            s_vn[0][f] = n0; s_vn[1][f] = n1; s_vn[2][f] = n2; s_vn[3][f] = n3;
        }
        R Ax = 0, Cx = 0, Ae = 0, Ce = 0, Fv2 = 0, Fv3 = 0, Gv2 = 0, Gv3 = 0;
        if (act) {
            metric_at(a.m, q, e, Ax, Cx, Ae, Ce);
            viscous_flux_at<N, R>(i, j, s_u + el * np, s_v + el * np, s_us + el * 4 * nf, s_vs + el * 4 * nf,
                                  Ax, Cx, Ae, Ce, h * a.eps[e], *a.tg, Fv2, Fv3, Gv2, Gv3);
        }
        // contravariant fluxes: F~v = J grad(xi) . (Fv, Gv), G~v = J grad(eta) . (Fv, Gv)
        s_Fv[0][t] = Ax * Fv2 + Cx * Gv2;
        s_Fv[1][t] = Ax * Fv3 + Cx * Gv3;
        s_Fv[2][t] = Ae * Fv2 + Ce * Gv2;
        s_Fv[3][t] = Ae * Fv3 + Ce * Gv3;
        lds_sync<T>();
        if (act) {
            R Lv2 = 0, Lv3 = 0;
            const int base = el * np;
            // (single precision: over the jumps from the own fluxes, as in
            // viscous_flux_at)
            const R o0 = kJumpForm<R> ? s_Fv[0][t] : R(0), o1 = kJumpForm<R> ? s_Fv[1][t] : R(0);
            const R o2 = kJumpForm<R> ? s_Fv[2][t] : R(0), o3 = kJumpForm<R> ? s_Fv[3][t] : R(0);
#pragma unroll
            for (int mm = 0; mm < nf; ++mm) {
                const R di = a.tg->D[i * kMaxNF + mm], dj = a.tg->D[j * kMaxNF + mm];
                Lv2 += di * (s_Fv[0][base + mm * nf + j] - o0) + dj * (s_Fv[2][base + i * nf + mm] - o2);
                Lv3 += di * (s_Fv[1][base + mm * nf + j] - o1) + dj * (s_Fv[3][base + i * nf + mm] - o3);
            }
            // faces: (1/(2 w_0)) n_s . (Fv_nbr - Fv_own), n_s outward scaled normal
            const R hw = R(0.5) * a.tab.iw0;
            const int fb = el * 4 * nf;
            auto face = [&](int s, int k, R snx, R sny) {
                const int f = fb + s * nf + k;
                Lv2 += hw * (snx * (s_vn[0][f] - Fv2) + sny * (s_vn[2][f] - Gv2));
                Lv3 += hw * (snx * (s_vn[1][f] - Fv3) + sny * (s_vn[3][f] - Gv3));
            };
            if (j == 0) face(0, i, -Ae, -Ce);
            if (i == N) face(1, j, Ax, Cx);
            if (j == N) face(2, i, Ae, Ce);
            if (i == 0) face(3, j, -Ax, -Cx);
            a.lv2[q] = Lv2;
            a.lv3[q] = Lv3;
        }
        lds_sync<T>();
    }
}

// ------------------------------------------------------------------------
// Stage kernel
// ------------------------------------------------------------------------
enum StageMode { kModeRhs = 0, kModeLsrk = 1, kModeSsp = 2 };

// CFL bound of one node: cfl (2/(N+1)) J / (|(A_xi . u)| + c |A_xi| + |(A_eta . u)| + c |A_eta|),
// with the contravariant directions A_xi = (Ax, Cx), A_eta = (Ae, Ce).
template <int N, typename R>
__device__ __forceinline__ R cfl_bound(R h, R hu, R hv, R Ax, R Cx, R Ae, R Ce, R J, const Phys<R> &P)
{
    const R ih = rcp_wet(h, P.h_tol);
    const R u = hu * ih, v = hv * ih;
    const R cs = sqrt(P.g * fmax(h, R(0)));
    const R lx = fabs(Ax * u + Cx * v) + cs * sqrt(Ax * Ax + Cx * Cx);
    const R le = fabs(Ae * u + Ce * v) + cs * sqrt(Ae * Ae + Ce * Ce);
    return lx + le > R(0) ? P.cfl * (R(2) / R(N + 1)) * J / (lx + le) : R(3.0e38);
}

// Viscous bound of an element with viscosity eps > 0.
template <typename R>
__device__ __forceinline__ R visc_bound(R eps, R gmax, const Phys<R> &P)
{
    return P.visc_c / (P.br1 * eps * gmax);
}

template <typename R> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename R>
struct StageArgs {
    Mesh<R> m;
    Phys<R> P;
    Tab<R> tab;                  // uniform entries (read as scalars)
    const Tab<R> *tg;            // the same tables in device memory: per-lane entries
    const R *h, *hu, *hv;        // stage input W
    const R *h0, *hu0, *hv0;     // SSP: W^n
    R *oh, *ohu, *ohv;           // output: R (rhs mode) or the new state
    R *dh, *dhu, *dhv;           // LSRK register dU (in place)
    int store_du;                // 0 on the last LSRK stage: the next step's first stage does not read dU
    // artificial viscosity (nullptr eps: off)
    const R *eps;                // [K] viscosity of the input state
    const R *vtr;                // [K][4][nf][4] face viscous fluxes of viscous elements
    const R *lv2, *lv3;          // [K][np] viscous terms of viscous elements
    R *eps_out;                  // [K] viscosity of the output state (update modes)
    int32_t *list_out;           // elements of the output state with eps > 0
    int *count_out;
    R *dtc_out, *dtv_out;        // last stage of a step: per-element CFL / viscous bounds of the output
    R *frec_out;                 // with them (limiter on): face records [K][4][nf][3] (h, u, v) of the output
    const int32_t *inst;         // [K] instance of each element (ensembles), nullptr: one instance
    const R *gmax;               // [K] max |grad xi|^2 + |grad eta|^2 (viscous bound)
    const double *dt;            // per instance k: the current step at dt[8k]
    R ca, cb;                    // LSRK a_k, b_k; SSP alpha_k, beta_k
    int *flags;                  // status flags (kFlag*)
    int *iflags;                 // ensembles with step retries: per-instance flags (1: negative mean), else nullptr
    const int *imask;            // with inst: only elements of instances k with imask[k] != 0 (a retry of
                                 // some instances), else nullptr
    int64_t ntiles;
    int variant;                 // compiled variant 0..kStageVariants-1 (launch side)
};

// Face slot data loaded ahead of the LDS staging (slots t, t + T, ... of lane t).
// Kept small (it is live across the LDS staging): the neighbour element as
// int32 and one packed word, the neighbour node's index recomputed from them.
template <typename R>
struct FacePrefetch {
    int32_t en = 0;          // neighbour element
    int code = 0;            // neighbour side | face node << 2 | (visc_nbr) << 8
    R h = 0, hu = 0, hv = 0, bo = 0, bn = 0;
    __device__ int ns() const { return code & 3; }
    __device__ int kk() const { return (code >> 2) & 63; }
    // with AV: the element has no viscosity, its neighbour has
    __device__ bool visc_nbr() const { return (code >> 8) & 1; }
};

template <int N, typename R, int E, int NF>
__device__ __forceinline__ void prefetch_face(const StageArgs<R> &a, int t, int64_t e0, FacePrefetch<R> &pf)
{
    constexpr int nf = N + 1, np = nf * nf;
    if (t >= NF) return;
    const int fel = t / (4 * nf), s = (t / nf) & 3, k = t - (t / nf) * nf;
    const int64_t fe = e0 + fel;
    if (fe >= a.m.K) return;
    int64_t en;
    int ns, kk;
    const int64_t qn = nbr_node<N>(a.m, fe, s, k, en, ns, kk);
    const int64_t ql = qn - e0 * np;
    if (!(ql >= 0 && ql < E * np)) {
        pf.h = a.h[qn];
        pf.hu = a.hu[qn];
        pf.hv = a.hv[qn];
    }
    pf.bo = a.m.bface[(fe * 4 + s) * nf + k];
    pf.bn = a.m.bface[(en * 4 + ns) * nf + kk];
    const bool vn = a.eps && !(a.eps[fe] > R(0)) && a.eps[en] > R(0);
    pf.en = (int32_t)en;
    pf.code = ns | (kk << 2) | ((int)vn << 8);
}

template <int N, typename R, int MODE, int V>
__global__ __launch_bounds__((StageCfg<N, V>::T), (StageWaves<N, R, MODE, V>::value)) void stage_kernel(StageArgs<R> a)
{
    using S = TileShape<N, StageCfg<N, V>::T>;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T, NF = S::NFACE;
    static_assert((T & (T - 1)) == 0, "workgroup size must be a power of two");
    using V2 = typename Vec2<R>::type;
    // one contiguous staging region: reused as reduction scratch at the end.
    // Pairs read together are stored together (one 16-byte LDS read in FP64).
    // Node (i, j) of tile element el sits at el*PS + i*RS + stage_col(i, j)
    // (RS = N + 1 + PAD); lanes past the tile's nodes write to spare slots
    // after them.
    constexpr int RS = nf + StageCfg<N, V>::PAD, PS = nf * RS, LEN = E * PS + (T - E * np);
    static_assert(LEN >= T, "staging rows");
    __shared__ __align__(16) R s_st[9 * LEN];
    V2 *const s_q = (V2 *)s_st;                 // (hu, hv)
    V2 *const s_w = (V2 *)(s_st + 2 * LEN);     // (u, v)
    V2 *const s_a = (V2 *)(s_st + 4 * LEN);     // J grad(xi)  = (Ax, Cx)
    V2 *const s_b = (V2 *)(s_st + 6 * LEN);     // J grad(eta) = (Ae, Ce)
    R *const s_h = s_st + 8 * LEN;
    __shared__ R s_fl[3][NF];
    __shared__ R s_lim[4 * E];
    __shared__ R s_vinv[nf * nf];       // V^{-1} for the indicator epilogue (with AV)
    __shared__ R s_dz[nf * nf];         // D with a zero diagonal (volume term)
    __shared__ R s_mref[kMetricRel<R> ? 4 * E : 1];  // the tile elements' Mesh::mref (single precision)

    const int64_t tile = xcd_tile(a.ntiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    // lanes past the last element's nodes shadow node 0 of the last slot
    // (all LDS indices stay in range; they never store)
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0, i = p / nf, j = p - i * nf;
    const int64_t e0 = tile * E, e = e0 + el;
    const bool act = lane && (e < a.m.K) && (!a.imask || a.imask[a.inst[e]] != 0);
    // a retry of some instances: tiles with none of their elements leave
    // every output as it is
    if (a.imask && !block_any<T>(act)) return;
    const int64_t q = e * np + p;
    const Phys<R> &P = a.P;
    const bool av = a.eps != nullptr;

    R h = 0, hu = 0, hv = 0, Ax = 0, Cx = 0, Ae = 0, Ce = 0;
    double xr = 0, yr = 0;
    if (act) {
        h = a.h[q]; hu = a.hu[q]; hv = a.hv[q];
        if constexpr (kMetricInKernel<N, R>) {
            xr = a.m.xr[q]; yr = a.m.yr[q];
        } else {
            Ax = a.m.Ax[q]; Cx = a.m.Cx[q]; Ae = a.m.Ae[q]; Ce = a.m.Ce[q];
        }
    }
    // single precision: the stored terms are relative to the element's
    // middle node (kMetricRel); staged and held as they are until the volume
    // sums, the element's reference in LDS (s_mref)
    if constexpr (kMetricRel<R>) {
        if (act && p == 0) {
            const R *r = a.m.mref + 4 * e;
            s_mref[4 * el + 0] = r[0]; s_mref[4 * el + 1] = r[1];
            s_mref[4 * el + 2] = r[2]; s_mref[4 * el + 3] = r[3];
        }
    }
    // The face slots' neighbour traces and face bathymetry are loaded here,
    // with the element's own data, so that their latency is not paid a second
    // time after the LDS staging; a lane holds NS slots (two at N = 2, where
    // seven elements' 84 face nodes outnumber the 64 lanes).
    // With more slots than lanes (N = 2) only the first slot is prefetched;
    // the few lanes with a further slot load it when they evaluate it.
    constexpr int NS = (NF + T - 1) / T;
    FacePrefetch<R> pf0;
    // (a one-trip loop here costs a VGPR and a dozen spilled SGPRs at N = 7)
    prefetch_face<N, R, E, NF>(a, t, e0, pf0);
    const R eps_e = (av && act) ? a.eps[e] : R(0);
    const R ih = rcp_wet(h, P.h_tol);
    const R u = hu * ih, v = hv * ih;
    const int st = lane ? el * PS + i * RS + stage_col<N, V>(i, j) : E * PS + (t - E * np);
    s_h[st] = h;
    s_q[st] = V2{hu, hv};
    s_w[st] = V2{u, v};
    if constexpr (kMetricInKernel<N, R>) {
        // metric terms from the staged coordinates: J grad(xi) = (y_eta, -x_eta),
        // J grad(eta) = (-y_xi, x_xi), each a derivative-matrix sum along a line
        // (eq. NablaRelation); D (with its diagonal) sits in the face-flux
        // slots until the face loop needs them
        static_assert(3 * NF >= nf * nf, "D in the face-flux slots");
        R *const s_D = &s_fl[0][0];
        s_a[st] = V2{xr, yr};
        for (int c = t; c < nf * nf; c += T) s_D[c] = a.tg->D[(c / nf) * kMaxNF + (c - (c / nf) * nf)];
        lds_sync<T>();
        const int base = el * PS;
        R xxi = 0, yxi = 0, xeta = 0, yeta = 0;
#pragma unroll 2
        for (int m = 0; m < nf; ++m) {
            const R di = s_D[i * nf + m], dj = s_D[j * nf + m];
            const V2 ci = s_a[base + m * RS + stage_col<N, V>(m, j)], cj = s_a[base + i * RS + stage_col<N, V>(i, m)];
            xxi += di * ci.x;
            yxi += di * ci.y;
            xeta += dj * cj.x;
            yeta += dj * cj.y;
        }
        Ax = yeta; Cx = -xeta; Ae = -yxi; Ce = xxi;
        lds_sync<T>();   // every lane's coordinate reads done before the metric replaces them
    }
    s_a[st] = V2{Ax, Cx};
    s_b[st] = V2{Ae, Ce};
    if constexpr (MODE != kModeRhs)
        if (av) stage_vinv<N, R, T>(s_vinv, *a.tg, t);
    // the per-lane table entries of the volume term from LDS rather than
    // through the vector memory path (3-6% faster)
    for (int c = t; c < nf * nf; c += T) s_dz[c] = a.tg->Dz[(c / nf) * kMaxNF + (c - (c / nf) * nf)];
    lds_sync<T>();

    // ---- interface: (1/w_0) J^surf F*(own, nbr, n_out) per face node; for
    // an element without viscosity next to one with viscosity, also its only
    // viscous term: (1/(2 w_0)) n_s . Fv_nbr (its own viscous fluxes are 0) ----
    auto face_slot = [&](const int f, const FacePrefetch<R> &pfr) {
        const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
        const int64_t fe = e0 + fel;
        R c0 = 0, c1 = 0, c2 = 0;
        if (fe < a.m.K) {
            int fi, fj;
            side_node<N>(s, k, fi, fj);
            const int lp = fel * PS + fi * RS + stage_col<N, V>(fi, fj);
            const int64_t en = pfr.en;
            const int ns = pfr.ns(), kk = pfr.kk();
            int ni, nj;
            side_node<N>(ns, kk, ni, nj);
            const int64_t qn = en * np + ni * nf + nj;
            // outward scaled normal: +-J grad(xi) on xi = +-1, +-J grad(eta) on eta = +-1
            V2 dir = (s & 1) ? s_a[lp] : s_b[lp];
            if constexpr (kMetricRel<R>) {
                dir.x += s_mref[4 * fel + ((s & 1) ? 0 : 2)];
                dir.y += s_mref[4 * fel + ((s & 1) ? 1 : 3)];
            }
            const R sg = (s == 0 || s == 3) ? R(-1) : R(1);
            const R snx = sg * dir.x, sny = sg * dir.y;
            const R js = sqrt(snx * snx + sny * sny);
            const R ijs = rcp_nr(js);
            // neighbour trace: from LDS when the neighbour is in this workgroup
            const int64_t ql = qn - e0 * np;
            R hn, un, vn, bo, bn;
            if (ql >= 0 && ql < E * np) {
                const int qe = (int)ql / np, qp = (int)ql - qe * np;
                const int qs = qe * PS + (qp / nf) * RS + stage_col<N, V>(qp / nf, qp - (qp / nf) * nf);
                hn = s_h[qs];
                const V2 w = s_w[qs];
                un = w.x;
                vn = w.y;
            } else {
                hn = pfr.h;
                const R in = rcp_wet(hn, P.h_tol);
                un = pfr.hu * in;
                vn = pfr.hv * in;
            }
            bo = pfr.bo;
            bn = pfr.bn;
            if (is_wall(a.m, fe, s)) wall_mirror(snx * ijs, sny * ijs, un, vn);
            R F0, F1, F2;
            const V2 wl = s_w[lp];
            if constexpr (kJumpForm<R>)
                interface_flux_delta<R>(s_h[lp], wl.x, wl.y, bo, hn, un, vn, bn, snx * ijs, sny * ijs, P,
                                        F0, F1, F2);
            else
                interface_flux<R>(s_h[lp], wl.x, wl.y, bo, hn, un, vn, bn, snx * ijs, sny * ijs, P, F0,
                                  F1, F2);
            const R sc = js * a.tab.iw0;
            c0 = sc * F0; c1 = sc * F1; c2 = sc * F2;
            // interface bathymetry penalty of eq. SourceDisc for a bottom
            // that jumps at the face, (1/w_0) (g/2) {h} [[b]] J^surf n in L
            // (zero for a continuous bottom and at walls, where bn = bo)
            const R pen = R(0.25) * P.g * a.tab.iw0 * (s_h[lp] + hn) * (bn - bo);
            c1 += pen * snx; c2 += pen * sny;
            if (av && pfr.visc_nbr()) {
                const R *vn = a.vtr + ((en * 4 + ns) * nf + kk) * 4;
                const R hw = R(0.5) * a.tab.iw0;
                c1 -= hw * (snx * vn[0] + sny * vn[2]);
                c2 -= hw * (snx * vn[1] + sny * vn[3]);
            }
        }
        s_fl[0][f] = c0; s_fl[1][f] = c1; s_fl[2][f] = c2;
    };
    if (t < NF) face_slot(t, pf0);
    if constexpr (NS > 1) {
        for (int f = t + T; f < NF; f += T) {
            FacePrefetch<R> pfl;
            prefetch_face<N, R, E, NF>(a, f, e0, pfl);
            face_slot(f, pfl);
        }
    }

    // ---- volume: sum_m 2 D_im F~(i,m) + sum_m 2 D_jm G~(j,m) (D~ has a zero
    // diagonal).  Per pair with contravariant direction (A, C):
    //   F1' = s_hu sA + s_hv sC,  F2' = s_u F1' + 2g h h_m sA,  F3' = s_v F1' + 2g h h_m sC
    // and 2 D F~ = D (F1'/2, F2'/4, F3'/4).  With s_u = u + u_m the sums split
    // into the own factors times partner sums, accumulated over both
    // directions at once:
    //   sum D F2' = u sum D F1' + sum D F1' u_m + 2g h sum D h_m sA   (F3' alike)
    R A1 = 0, A2 = 0, A3 = 0, C2 = 0, C3 = 0;
    if constexpr (kJumpForm<R>) {
        // single precision: the same sums taken over the partners' jumps
        // from the own node (dX = X_m - X, t = 2 x own metric pair).  With
        // F1'(own) = 4 (hu A + hv C) and F2'(own) the own momentum part,
        //   F1'_m - F1'(own) = s_hu dA + s_hv dC + tA dhu + tC dhv
        //   F2'_m - F2'(own) = 2u (F1'_m - F1'(own)) + du F1'_m + 2g h (h_m dA + tA dh)
        // (F3' alike), so sum_m D (F' - F'(own)) holds no term of the size of
        // the flux itself; the row-sum parts D~ 1 F'(own) left out are the
        // own-flux parts the face slots subtract (interface_flux_delta).
        const int base = el * PS;
        constexpr int VU = StageCfg<N, V>::VU;
        // (the staged and own terms are relative to the element's middle
        // node: the jumps from the own relative terms, t from the absolute
        // ones, the sums from the own plus twice the reference)
        const R *const mr = s_mref + 4 * el;
        {
            const R tA = R(2) * (Ax + mr[0]), tC = R(2) * (Cx + mr[1]);
            const R pA = Ax + R(2) * mr[0], pC = Cx + R(2) * mr[1];
#pragma unroll VU
            for (int mm = 0; mm < nf; ++mm) {
                const int qq = base + mm * RS + stage_col<N, V>(mm, j);
                const R d = s_dz[i * nf + mm];
                const V2 am = s_a[qq], qm = s_q[qq], wm = s_w[qq];
                const R hm = s_h[qq];
                const R dA = am.x - Ax, dC = am.y - Cx, dh = hm - h;
                const R s1 = hu + qm.x, s2 = hv + qm.y;
                const R F1 = s1 * (pA + am.x) + s2 * (pC + am.y);
                const R dF1 = s1 * dA + s2 * dC + tA * (qm.x - hu) + tC * (qm.y - hv);
                const R dF = d * F1;
                A1 += d * dF1;
                A2 += dF * (wm.x - u);
                A3 += dF * (wm.y - v);
                C2 += d * (hm * dA + tA * dh);
                C3 += d * (hm * dC + tC * dh);
            }
        }
        {
            const R tA = R(2) * (Ae + mr[2]), tC = R(2) * (Ce + mr[3]);
            const R pA = Ae + R(2) * mr[2], pC = Ce + R(2) * mr[3];
#pragma unroll VU
            for (int mm = 0; mm < nf; ++mm) {
                const int qq = base + i * RS + stage_col<N, V>(i, mm);
                const R d = s_dz[j * nf + mm];
                const V2 bm = s_b[qq], qm = s_q[qq], wm = s_w[qq];
                const R hm = s_h[qq];
                const R dA = bm.x - Ae, dC = bm.y - Ce, dh = hm - h;
                const R s1 = hu + qm.x, s2 = hv + qm.y;
                const R F1 = s1 * (pA + bm.x) + s2 * (pC + bm.y);
                const R dF1 = s1 * dA + s2 * dC + tA * (qm.x - hu) + tC * (qm.y - hv);
                const R dF = d * F1;
                A1 += d * dF1;
                A2 += dF * (wm.x - u);
                A3 += dF * (wm.y - v);
                C2 += d * (hm * dA + tA * dh);
                C3 += d * (hm * dC + tC * dh);
            }
        }
    } else {
        const int base = el * PS;
        // partner-loop unroll of the variant (StageCfg)
        constexpr int VU = StageCfg<N, V>::VU;
#pragma unroll VU
        for (int mm = 0; mm < nf; ++mm) {
            // the self pair has coefficient 0 (no branch: D~ has a zero diagonal)
            const int qq = base + mm * RS + stage_col<N, V>(mm, j);
            const R d = s_dz[i * nf + mm];
            const V2 am = s_a[qq], qm = s_q[qq], wm = s_w[qq];
            const R sA = Ax + am.x, sC = Cx + am.y;
            const R df = d * ((hu + qm.x) * sA + (hv + qm.y) * sC);
            const R dh = d * s_h[qq];
            A1 += df;
            A2 += df * wm.x;
            A3 += df * wm.y;
            C2 += dh * sA;
            C3 += dh * sC;
        }
#pragma unroll VU
        for (int mm = 0; mm < nf; ++mm) {
            const int qq = base + i * RS + stage_col<N, V>(i, mm);
            const R d = s_dz[j * nf + mm];
            const V2 bm = s_b[qq], qm = s_q[qq], wm = s_w[qq];
            const R sA = Ae + bm.x, sC = Ce + bm.y;
            const R df = d * ((hu + qm.x) * sA + (hv + qm.y) * sC);
            const R dh = d * s_h[qq];
            A1 += df;
            A2 += df * wm.x;
            A3 += df * wm.y;
            C2 += dh * sA;
            C3 += dh * sC;
        }
    }
    const R h2g = R(2) * P.g * h;
    // (the jump form's mass sum enters the momentum sums twice: 2u dF1)
    const R uA = kJumpForm<R> ? R(2) * u : u, vA = kJumpForm<R> ? R(2) * v : v;
    R L1 = R(0.5) * A1, L2 = R(0.25) * (uA * A1 + A2 + h2g * C2), L3 = R(0.25) * (vA * A1 + A3 + h2g * C3);
    lds_sync<T>();   // face slots complete; staging region free from here on
    {
        const int fb = el * 4 * nf;
        if (j == 0) { L1 += s_fl[0][fb + 0 * nf + i]; L2 += s_fl[1][fb + 0 * nf + i]; L3 += s_fl[2][fb + 0 * nf + i]; }
        if (i == N) { L1 += s_fl[0][fb + 1 * nf + j]; L2 += s_fl[1][fb + 1 * nf + j]; L3 += s_fl[2][fb + 1 * nf + j]; }
        if (j == N) { L1 += s_fl[0][fb + 2 * nf + i]; L2 += s_fl[1][fb + 2 * nf + i]; L3 += s_fl[2][fb + 2 * nf + i]; }
        if (i == 0) { L1 += s_fl[0][fb + 3 * nf + j]; L2 += s_fl[1][fb + 3 * nf + j]; L3 += s_fl[2][fb + 3 * nf + j]; }
    }
    if constexpr (kMetricRel<R>) {
        // the own terms absolute from here on
        const R *const mr = s_mref + 4 * el;
        Ax += mr[0]; Cx += mr[1]; Ae += mr[2]; Ce += mr[3];
    }
    const R J = Ce * Ax - Cx * Ae;

    // ---- R = (1/J)(-L + S + L^v), S = -(g/2) h (b_x, b_y) ----
    R bxv = 0, byv = 0, Lv2 = 0, Lv3 = 0;
    if (act) {
        bxv = a.m.bx[q]; byv = a.m.by[q];
        if (av && eps_e > R(0)) { Lv2 = a.lv2[q]; Lv3 = a.lv3[q]; }
    }
    const R iJ = act ? rcp_nr(J) : R(0);
    const R hg = R(0.5) * P.g * h;
    const R R1 = -L1 * iJ;
    const R R2 = (-L2 - hg * bxv + Lv2) * iJ;
    const R R3 = (-L3 - hg * byv + Lv3) * iJ;

    if constexpr (MODE == kModeRhs) {
        if (act) { a.oh[q] = R1; a.ohu[q] = R2; a.ohv[q] = R3; }
        return;
    } else {
        const R dt = (R)a.dt[a.inst ? 8 * (int64_t)a.inst[act ? e : e0] : 0];
        R nh, nhu, nhv;
        R d0 = 0, d1 = 0, d2 = 0;
        if constexpr (MODE == kModeLsrk) {
            // the first stage has a_1 = 0: the register is not read
            if (act && a.ca != R(0)) { d0 = a.dh[q]; d1 = a.dhu[q]; d2 = a.dhv[q]; }
            d0 = a.ca * d0 + dt * R1;
            d1 = a.ca * d1 + dt * R2;
            d2 = a.ca * d2 + dt * R3;
            nh = h + a.cb * d0; nhu = hu + a.cb * d1; nhv = hv + a.cb * d2;
        } else {
            R w0 = 0, w1 = 0, w2 = 0;
            if (act) { w0 = a.h0[q]; w1 = a.hu0[q]; w2 = a.hv0[q]; }
            nh = a.ca * w0 + a.cb * (h + dt * R1);
            nhu = a.ca * w1 + a.cb * (hu + dt * R2);
            nhv = a.ca * w2 + a.cb * (hv + dt * R3);
        }
        // positivity limiter (eq. PosPres) toward the J-weighted means; an
        // element without a negative node keeps theta = 1, so the means are
        // only formed when some element of the workgroup has one
        if (P.limiter_on && block_any<T>(act && nh < R(0))) {
            const R wq = act ? J * a.tg->w[i] * a.tg->w[j] : R(0);
            R vals[5] = {wq, wq * nh, wq * nhu, wq * nhv, act ? nh : R(3.0e38)};
            elem_totals_any<N, R, 5, true, T>(vals, s_st, t, el, p, lane);
            if (lane && p == 0) {
                const R area = vals[0];
                const R mh = vals[1] / area, mhu = vals[2] / area, mhv = vals[3] / area, mn = vals[4];
                R th = R(1);
                if (act && mn < R(0)) {
                    if (mh < R(0)) {
                        th = R(0);
                        atomicOr(&a.flags[kFlagNegMean], 1);
                        if (a.iflags) atomicOr(&a.iflags[a.inst ? a.inst[e] : 0], 1);
                    } else {
                        th = mh / (mh - mn);
                        th = th < R(1) ? th : R(1);
                    }
                    atomicAdd(&a.flags[kFlagLimited], 1);
                }
                s_lim[4 * el + 0] = th; s_lim[4 * el + 1] = mh;
                s_lim[4 * el + 2] = mhu; s_lim[4 * el + 3] = mhv;
            }
            lds_sync<T>();
            const R th = s_lim[4 * el];
            if (act && th != R(1)) {
                const R mh = s_lim[4 * el + 1], mhu = s_lim[4 * el + 2], mhv = s_lim[4 * el + 3];
                nh = th * (nh - mh) + mh;
                nhu = th * (nhu - mhu) + mhu;
                nhv = th * (nhv - mhv) + mhv;
            }
        }
        if (P.limiter_on && nh < P.h_tol) { nhu = R(0); nhv = R(0); }
        // a non-finite value in any of the three (an infinity or NaN makes
        // their sum non-finite) is reported once per esdg_step
        if (act && !__builtin_isfinite(nh + nhu + nhv)) atomicOr(&a.flags[kFlagNonFinite], 1);
        if (act) {
            a.oh[q] = nh; a.ohu[q] = nhu; a.ohv[q] = nhv;
            if constexpr (MODE == kModeLsrk) {
                if (a.store_du) { a.dh[q] = d0; a.dhu[q] = d1; a.dhv[q] = d2; }
            }
        }
        R en = R(0);
        if (av) {
            // viscosity of the new state for the next stage (appendix A)
            s_st[8 * T + t] = nh;
            lds_sync<T>();
            en = element_viscosity<N, R, T>(s_st + 8 * T, s_st, s_vinv, P, t, el, p, lane, nh);
            if (act && p == 0) {
                a.eps_out[e] = en;
                if (en > R(0)) a.list_out[atomicAdd(a.count_out, 1)] = (int32_t)e;
            }
        }
        if (a.dtc_out) {
            // face records of the new state for the Lemma 2 bounds of the
            // next step: per face node the height and both velocities, the
            // values the time-step pass would read from the state (corner
            // nodes write both sides)
            if (a.frec_out && act) {
                const R ihn = rcp_wet(nh, P.h_tol);
                const R un = nhu * ihn, vn = nhv * ihn;
                auto rec = [&](int s, int k) {
                    R *const r = a.frec_out + ((e * 4 + s) * nf + k) * 3;
                    r[0] = nh;
                    r[1] = un;
                    r[2] = vn;
                };
                if (j == 0) rec(0, i);
                if (i == N) rec(1, j);
                if (j == N) rec(2, i);
                if (i == 0) rec(3, j);
            }
            // CFL and viscous bounds of the new state for the next step
            R vals[1] = {act ? cfl_bound<N, R>(nh, nhu, nhv, Ax, Cx, Ae, Ce, J, P) : R(3.0e38)};
            lds_sync<T>();   // scratch free
            elem_totals_any<N, R, 1, true, T>(vals, s_st, t, el, p, lane);
            if (act && p == 0) {
                a.dtc_out[e] = vals[0];
                if (a.dtv_out) a.dtv_out[e] = en > R(0) ? visc_bound<R>(en, a.gmax[e], P) : R(3.0e38);
            }
        }
    }
}

// ------------------------------------------------------------------------
// Standalone limiter (initial data / esdg_limit)
// ------------------------------------------------------------------------
template <int N, typename R>
__global__ __launch_bounds__(Shape<N>::T) void limit_kernel(Mesh<R> m, Phys<R> P, Tab<R> tab, R *h_,
                                                            R *hu_, R *hv_, int *flags, int64_t ntiles)
{
    using S = Shape<N>;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T;
    __shared__ R s_red[5 * T];
    const int64_t tile = xcd_tile(ntiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0, i = p / nf, j = p - i * nf;
    const int64_t e = tile * E + el;
    const bool act = lane && (e < m.K);
    const int64_t q = e * np + p;
    R nh = 0, nhu = 0, nhv = 0, J = 0;
    if (act) {
        nh = h_[q]; nhu = hu_[q]; nhv = hv_[q];
        R Ax, Cx, Ae, Ce;
        metric_at(m, q, e, Ax, Cx, Ae, Ce);
        J = Ce * Ax - Cx * Ae;
    }
    const R wq = act ? J * tab.w[i] * tab.w[j] : R(0);
    R vals[5] = {wq, wq * nh, wq * nhu, wq * nhv, act ? nh : R(3.0e38)};
    ElemReduce<N, R, 5>::template run<true>(vals, s_red, t, el, p);
    const R area = vals[0];
    const R mh = vals[1] / area, mhu = vals[2] / area, mhv = vals[3] / area, mn = vals[4];
    if (!act) return;
    if (mn < R(0)) {
        R th;
        if (mh < R(0)) {
            th = R(0);
            if (p == 0) atomicOr(&flags[kFlagNegMean], 1);
        } else {
            th = mh / (mh - mn);
            th = th < R(1) ? th : R(1);
        }
        if (p == 0) atomicAdd(&flags[kFlagLimited], 1);
        nh = th * (nh - mh) + mh;
        nhu = th * (nhu - mhu) + mhu;
        nhv = th * (nhv - mhv) + mhv;
    }
    if (nh < P.h_tol) { nhu = R(0); nhv = R(0); }
    h_[q] = nh; hu_[q] = nhu; hv_[q] = nhv;
}

// ------------------------------------------------------------------------
// Time step bounds: CFL, viscous (AV), Lemma 2.  Minima go to 64 slots per
// bound by atomicMin on the bit patterns of non-negative doubles (which order
// like unsigned integers); dt_finalize_kernel reduces and resets them.
//
// The last stage of every step leaves the per-element CFL and viscous bounds
// of its output state in dtc/dtv (stage epilogue); the time-step pass then
// only reduces those and evaluates Lemma 2 at the face nodes.  For a state
// no stage produced (initial data, after a limiter call or a retry) the pass
// evaluates every bound itself.  All loops are flat over nodes, face nodes
// and elements, with a fixed grid: each XCD takes one contiguous range of
// each index space so that neighbour traces hit its L2.  Each workgroup
// issues one atomic per bound.
// ------------------------------------------------------------------------
constexpr int kDtThreads = 256;
constexpr int64_t kDtChunk = 256;   // elements per chunk of the ensemble time-step pass
constexpr unsigned kDtMaxBlocks = 2048;

template <typename R>
struct DtArgs {
    Mesh<R> m;
    Phys<R> P;
    const R *h, *hu, *hv;
    const R *eps;              // full pass with AV: element viscosity of the state
    const R *dtc, *dtv;        // per-element CFL / viscous bounds from the stage epilogue (nullptr: full pass)
    const R *gmax;             // [K] max over the element's nodes of |grad xi|^2 + |grad eta|^2
    const R *fgeo;             // [K][4][nf][3] outward unit normal and w_0 J / J^surf per face node
    const R *frec;             // with dtc: [K][4][nf][3] face records (h, u, v) of the state
    unsigned long long *slots; // [instance][3][kDtSlots]
    const int64_t *cstart;     // ensembles: element chunks [cstart[c], cstart[c+1]) inside one instance
    const int32_t *cinst;      //   and the instance of chunk c
    int64_t nchunks;
};

__device__ __forceinline__ void slot_min(unsigned long long *slot, double v)
{
    if (v >= 0.0 && v < __builtin_huge_val()) atomicMin(slot, (unsigned long long)__double_as_longlong(v));
}

template <typename R>
__device__ __forceinline__ R wave_min(R v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const R o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// Per-element max of |grad xi|^2 + |grad eta|^2 (mesh constant; used by the
// viscous bound).  One thread per element.
template <int N, typename R>
__global__ void gmax_kernel(Mesh<R> m, R *gmax)
{
    constexpr int np = (N + 1) * (N + 1);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.K) return;
    R gm = R(0);
    for (int p = 0; p < np; ++p) {
        const int64_t q = e * np + p;
        R Ax, Cx, Ae, Ce;
        metric_at(m, q, e, Ax, Cx, Ae, Ce);
        const R J = Ce * Ax - Cx * Ae;
        const R gg = (Ax * Ax + Cx * Cx + Ae * Ae + Ce * Ce) / (J * J);
        gm = gg > gm ? gg : gm;
    }
    gmax[e] = gm;
}

// Face geometry for Lemma 2 (mesh constant): per face node the outward unit
// normal and w_0 J / J^surf.  One thread per face node.
template <int N, typename R>
__global__ void face_geometry_kernel(Mesh<R> m, R w0, R *fgeo)
{
    constexpr int nf = N + 1, np = nf * nf;
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= m.K * 4 * nf) return;
    const int64_t e = f / (4 * nf);
    const int r = (int)(f - e * 4 * nf), s = r / nf, k = r - s * nf;
    int i, j;
    side_node<N>(s, k, i, j);
    const int64_t q = e * np + i * nf + j;
    R Ax, Cx, Ae, Ce;
    metric_at(m, q, e, Ax, Cx, Ae, Ce);
    R snx, sny;
    if (s == 1) { snx = Ax; sny = Cx; }
    else if (s == 3) { snx = -Ax; sny = -Cx; }
    else if (s == 2) { snx = Ae; sny = Ce; }
    else { snx = -Ae; sny = -Ce; }
    const R js = sqrt(snx * snx + sny * sny);
    const R J = Ce * Ax - Cx * Ae;
    fgeo[f * 3 + 0] = snx / js;
    fgeo[f * 3 + 1] = sny / js;
    fgeo[f * 3 + 2] = w0 * (J / js);
}

// Index range [b, e) and stride of this workgroup over n items: XCD x of 8
// takes the x-th contiguous eighth.
struct XcdRange {
    int64_t b, e, stride;
    __device__ XcdRange(int64_t n, int T)
    {
        const int64_t per = (n + kXcds - 1) / kXcds;
        const int64_t lo = (int64_t)(blockIdx.x % kXcds) * per;
        const int64_t hi = lo + per < n ? lo + per : n;
        b = lo + (int64_t)(blockIdx.x / kXcds) * T + threadIdx.x;
        e = hi;
        stride = (int64_t)(gridDim.x / kXcds) * T;
    }
};

// The two bounds of eq. CFLConstraints for own trace (hm, utm) and
// neighbour (hp, utp), normal velocities along the outward unit normal.
template <typename R>
__device__ __forceinline__ R lemma2_formula(R hm, R hp, R utm, R utp, R w0a, const Phys<R> &P)
{
    const R cm = sqrt(P.g * (hm > R(0) ? hm : R(0))), cp = sqrt(P.g * (hp > R(0) ? hp : R(0)));
    const R au = R(0.5) * (utm + utp), ac = R(0.5) * (cm + cp);
    const R A = fabs(au + ac) + fabs(au - ac), B = fabs(au + ac) - fabs(au - ac);
    R posb = R(3.0e38);
    const R den1 = A + R(2) * au;
    if (den1 > R(0)) { const R bnd = w0a / den1; posb = bnd < posb ? bnd : posb; }
    const R den2 = ac * B * (utp - utm);
    if (hm > R(0) && den2 < R(0)) { const R bnd = fabs(w0a * P.g * hm / den2); posb = bnd < posb ? bnd : posb; }
    return posb;
}

// Lemma 2 bounds at face node f (own trace '-', neighbour '+').
template <int N, typename R>
__device__ __forceinline__ R lemma2_bound(const DtArgs<R> &a, int64_t f)
{
    constexpr int nf = N + 1, np = nf * nf;
    const Phys<R> &P = a.P;
    const int64_t fe = f / (4 * nf);
    const int rr = (int)(f - fe * 4 * nf), s = rr / nf, k = rr - s * nf;
    int fi, fj, ns, kk;
    int64_t en;
    side_node<N>(s, k, fi, fj);
    const int64_t qo = fe * np + fi * nf + fj;
    const int64_t qn = nbr_node<N>(a.m, fe, s, k, en, ns, kk);
    const R nx = a.fgeo[f * 3 + 0], ny = a.fgeo[f * 3 + 1], w0a = a.fgeo[f * 3 + 2];
    const R hm = a.h[qo], hp = a.h[qn];
    const R im = rcp_wet(hm, P.h_tol), ip = rcp_wet(hp, P.h_tol);
    const R utm = nx * (a.hu[qo] * im) + ny * (a.hv[qo] * im);
    const R utp = is_wall(a.m, fe, s) ? -utm : nx * (a.hu[qn] * ip) + ny * (a.hv[qn] * ip);
    return lemma2_formula<R>(hm, hp, utm, utp, w0a, P);
}

// Lemma 2 bounds at face node f from the face records the last stage left:
// the same heights and velocities lemma2_bound reads from the state, so the
// same bounds bit for bit, without reading whole elements.
template <int N, typename R>
__device__ __forceinline__ R lemma2_bound_rec(const DtArgs<R> &a, int64_t f)
{
    constexpr int nf = N + 1;
    const int64_t fe = f / (4 * nf);
    const int rr = (int)(f - fe * 4 * nf), s = rr / nf, k = rr - s * nf;
    const int64_t en = a.m.nbr[fe * 4 + s];
    const int c = a.m.code[fe * 4 + s];
    const int ns = c & 3, kk = ((c >> 2) & 1) ? N - k : k;
    const R *const rm = a.frec + f * 3, *const rp = a.frec + ((en * 4 + ns) * nf + kk) * 3;
    const R nx = a.fgeo[f * 3 + 0], ny = a.fgeo[f * 3 + 1], w0a = a.fgeo[f * 3 + 2];
    const R hm = rm[0], hp = rp[0];
    const R utm = nx * rm[1] + ny * rm[2];
    const R utp = is_wall(a.m, fe, s) ? -utm : nx * rp[1] + ny * rp[2];
    return lemma2_formula<R>(hm, hp, utm, utp, w0a, a.P);
}

// Minimum of the Lemma 2 bounds over the face nodes of range r.  Each
// iteration takes U face nodes at once, with clamped indices and no branch,
// so that the loads of all U (face map, then both traces) are in flight
// together; the minimum does not depend on the order.
template <int N, typename R, bool REC>
__device__ __forceinline__ R lemma2_min(const DtArgs<R> &a, XcdRange r)
{
    constexpr int U = 4;
    R posb = R(3.0e38);
    for (; r.b < r.e; r.b += U * r.stride) {
        R v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t f = r.b + u * r.stride;
            const int64_t fc = f < r.e ? f : r.e - 1;
            if constexpr (REC) v[u] = lemma2_bound_rec<N, R>(a, fc);
            else v[u] = lemma2_bound<N, R>(a, fc);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = r.b + u * r.stride < r.e;
            posb = (in && v[u] < posb) ? v[u] : posb;
        }
    }
    return posb;
}

// CFL bound at node q from the stored state and metric.
template <int N, typename R>
__device__ __forceinline__ R cfl_node(const DtArgs<R> &a, int64_t q)
{
    R Ax, Cx, Ae, Ce;
    metric_at(a.m, q, q / ((N + 1) * (N + 1)), Ax, Cx, Ae, Ce);
    return cfl_bound<N, R>(a.h[q], a.hu[q], a.hv[q], Ax, Cx, Ae, Ce, Ce * Ax - Cx * Ae, a.P);
}

// Workgroup minima of the three bounds into slots[3][kDtSlots] (slot sl).
template <typename R>
__device__ __forceinline__ void dt_block_min(R cflb, R viscb, R posb, unsigned long long *slots, int sl)
{
    constexpr int T = kDtThreads;
    __shared__ R s_w[3][T / 64];
    cflb = wave_min(cflb);
    viscb = wave_min(viscb);
    posb = wave_min(posb);
    const int t = threadIdx.x, wv = t >> 6;
    if ((t & 63) == 0) {
        s_w[0][wv] = cflb;
        s_w[1][wv] = viscb;
        s_w[2][wv] = posb;
    }
    lds_sync<T>();
    if (t < 3) {
        R v = s_w[t][0];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) v = s_w[t][w] < v ? s_w[t][w] : v;
        if (v < R(1.0e38)) slot_min(&slots[t * kDtSlots + sl], (double)v);
    }
    lds_sync<T>();
}

template <int N, typename R>
__global__ __launch_bounds__(kDtThreads) void dt_kernel(DtArgs<R> a)
{
    constexpr int nf = N + 1, np = nf * nf, T = kDtThreads;
    const int64_t K = a.m.K;
    R cflb = R(3.0e38), viscb = R(3.0e38), posb = R(3.0e38);
    if (a.dtc) {
        // per-element bounds left by the stage epilogue
        for (XcdRange r(K, T); r.b < r.e; r.b += r.stride) {
            const R c = a.dtc[r.b];
            cflb = c < cflb ? c : cflb;
            if (a.dtv) {
                const R v = a.dtv[r.b];
                viscb = v < viscb ? v : viscb;
            }
        }
    } else {
        for (XcdRange r(K * np, T); r.b < r.e; r.b += r.stride) {
            const R c = cfl_node<N, R>(a, r.b);
            cflb = c < cflb ? c : cflb;
        }
        if (a.eps) {
            for (XcdRange r(K, T); r.b < r.e; r.b += r.stride) {
                const R eps = a.eps[r.b];
                if (eps > R(0)) {
                    const R v = visc_bound<R>(eps, a.gmax[r.b], a.P);
                    viscb = v < viscb ? v : viscb;
                }
            }
        }
    }
    if (a.P.limiter_on) {
        // after a step: the face records its last stage left (with dtc)
        posb = a.frec ? lemma2_min<N, R, true>(a, XcdRange(K * 4 * nf, T))
                      : lemma2_min<N, R, false>(a, XcdRange(K * 4 * nf, T));
    }
    dt_block_min<R>(cflb, viscb, posb, a.slots, blockIdx.x % kDtSlots);
}

// The same per instance of an ensemble: each workgroup takes whole chunks
// of elements (a chunk lies inside one instance) and adds its minima to that
// instance's slots.
template <int N, typename R>
__global__ __launch_bounds__(kDtThreads) void dt_batch_kernel(DtArgs<R> a)
{
    constexpr int nf = N + 1, np = nf * nf, T = kDtThreads;
    const int t = threadIdx.x;
    for (int64_t c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
        const int64_t lo = a.cstart[c], hi = a.cstart[c + 1];
        R cflb = R(3.0e38), viscb = R(3.0e38), posb = R(3.0e38);
        if (a.dtc) {
            for (int64_t e = lo + t; e < hi; e += T) {
                const R v = a.dtc[e];
                cflb = v < cflb ? v : cflb;
                if (a.dtv) {
                    const R w = a.dtv[e];
                    viscb = w < viscb ? w : viscb;
                }
            }
        } else {
            for (int64_t q = lo * np + t; q < hi * np; q += T) {
                const R v = cfl_node<N, R>(a, q);
                cflb = v < cflb ? v : cflb;
            }
            if (a.eps) {
                for (int64_t e = lo + t; e < hi; e += T) {
                    const R eps = a.eps[e];
                    if (eps > R(0)) {
                        const R v = visc_bound<R>(eps, a.gmax[e], a.P);
                        viscb = v < viscb ? v : viscb;
                    }
                }
            }
        }
        if (a.P.limiter_on) {
            for (int64_t f = lo * 4 * nf + t; f < hi * 4 * nf; f += T) {
                const R v = a.frec ? lemma2_bound_rec<N, R>(a, f) : lemma2_bound<N, R>(a, f);
                posb = v < posb ? v : posb;
            }
        }
        dt_block_min<R>(cflb, viscb, posb, a.slots + (int64_t)a.cinst[c] * 3 * kDtSlots, (int)(c % kDtSlots));
    }
}

// ------------------------------------------------------------------------
// Diagnostics: per-workgroup partial sums of J w w (h, hu, hv, e, q.R),
// min h, max h, #dry nodes.
// ------------------------------------------------------------------------
template <int N, typename R>
__global__ __launch_bounds__(Shape<N>::T) void diag_kernel(Mesh<R> m, Phys<R> P, Tab<R> tab, const R *h_,
                                                           const R *hu_, const R *hv_, const R *b_,
                                                           const R *r0, const R *r1, const R *r2,
                                                           double *part)
{
    using S = Shape<N>;
    constexpr int nf = S::nf, np = S::np, T = S::T;
    __shared__ double s[8][T];
    const int t = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * T + t;
    double v[8] = {0, 0, 0, 0, 0, 1e300, -1e300, 0};
    if (q < m.K * np) {
        const int p = (int)(q % np), i = p / nf, j = p - i * nf;
        R Ax, Cx, Ae, Ce;
        metric_at(m, q, q / np, Ax, Cx, Ae, Ce);
        const double J = (double)Ce * Ax - (double)Cx * Ae;
        const double wq = J * tab.w[i] * tab.w[j];
        const double h = h_[q], hu = hu_[q], hv = hv_[q], b = b_[q];
        const double ih = h > P.h_tol ? 1.0 / h : 0.0;
        const double u = hu * ih, vv = hv * ih, g = P.g;
        v[0] = wq * h;
        v[1] = wq * hu;
        v[2] = wq * hv;
        v[3] = wq * (0.5 * h * (u * u + vv * vv) + 0.5 * g * h * h + g * h * b);
        v[4] = wq * ((g * (h + b) - 0.5 * (u * u + vv * vv)) * r0[q] + u * r1[q] + vv * r2[q]);
        v[5] = h;
        v[6] = h;
        v[7] = h > P.h_tol ? 0.0 : 1.0;
    }
    for (int c = 0; c < 8; ++c) s[c][t] = v[c];
    lds_sync<T>();
    for (int st = T / 2; st > 0; st >>= 1) {
        if (t < st) {
            for (int c = 0; c < 5; ++c) s[c][t] += s[c][t + st];
            s[5][t] = fmin(s[5][t], s[5][t + st]);
            s[6][t] = fmax(s[6][t], s[6][t + st]);
            s[7][t] += s[7][t + st];
        }
        lds_sync<T>();
    }
    if (t < 8) part[blockIdx.x * 8 + t] = s[t][0];
}

// ------------------------------------------------------------------------
// Precision conversion
// ------------------------------------------------------------------------
template <typename A, typename B>
__global__ void convert_kernel(const A *__restrict__ src, B *__restrict__ dst, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = (B)src[q];
}

}  // namespace esdg
