// Discrete adjoint (reverse mode) of one inviscid Runge-Kutta stage, float64.
//
// An LSRK(5,4) stage computes, per node, d_k = A_k d_{k-1} + dt R(W_{k-1}) and
// W_k = W_{k-1} + B_k d_k with R = -(1/J)(L_xi + L_eta - S) (Lemma 1): the
// split-form volume term with the two-point fluxes of eq. volumeFluxes and
// the contravariant metric averages of eq. Fmij, the rotated interface flux
// of appendix B and the bathymetry source of eq. SourceDisc.  Its reverse,
// for the cotangents a = dL/dW_k and c = A_{k+1} dL/dd_{k+1} (zero on a
// step's last stage), is
//     l = c + B_k a                      (dL/dd_k)
//     a' = a + dt (dR/dW)^T l            (dL/dW_{k-1})
//     c' = A_k l
// The same kernel reverses an SSPRK(3,3) stage (eq. RKSSP),
// W_k = alpha_k W^n + beta_k (W_{k-1} + dt R(W_{k-1})): with c = 0 and
// B_k = beta_k, l = beta_k a and dL/dW_{k-1} = beta_k a + dt (dR/dW)^T l (a
// scaled by sa = beta_k), while co collects the alpha_k a terms of dL/dW^n
// (A_k = alpha_k / beta_k, added to the running sum y) and the first stage
// adds that sum to its output (x).  In both schemes the reverse stage adds
// the bathymetry cotangents dt (dR/db)^T l, accumulated in three node
// fields: of the split derivatives b_x, b_y (the source is linear in them)
// and of the face traces of b (the interface flux reads b through the jump
// of the entropy variables).  bathymetry_adjoint_kernel maps the first two
// back to nodal b once per sweep (the map b -> (b_x, b_y) is linear and the
// same in every stage).
//
// Every node gathers its own cotangent; nothing is scattered:
//  * volume: the two-point flux is symmetric, F#(a, b) = F#(b, a), so the
//    derivative of the pair (a, b) term of node b's row with respect to W_a
//    equals that of node a's row with respect to its first argument; node a
//    contracts that derivative with D~_ab mu_a + D~_ba mu_b (mu = -l/J);
//  * interface: a face node takes the derivative of its own face term with
//    respect to its own ('-') trace and of the neighbour's face term with
//    respect to the neighbour's '+' trace, which is this node; since the
//    interface flux is conservative, F*(W+, W-, -n) = -F*(W-, W+, n), both
//    are one reverse evaluation of the own term's flux.  At a solid wall the
//    outside trace is the own trace with the normal velocity reversed: the
//    outside cotangent returns to this node through that (symmetric) mirror,
//    and there is no neighbour term.  The interface bathymetry penalty of
//    eq. SourceDisc, linear in {h} and [[b]], is reversed the same way (its
//    b-partials are nonzero also where b is continuous).
// The derivative of |x| is taken as sign(x) with sign(0) = 0; velocities
// below the dry cut-off are constants (zero derivative).
#pragma once
#include "esdg_kernels.hpp"

namespace esdg {

template <typename R>
struct FluxBar {
    R h, u, v, b;   // cotangents of one trace: height, primitive velocities, bathymetry
};

template <typename R>
__device__ __forceinline__ R sgn(R x)
{
    return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

// Reverse mode of interface_flux: cotangent (z0, z1, z2) of (F0, F1, F2) in,
// cotangents of both traces out (the wave speed c = sqrt(g h) is folded into
// the height).
template <typename R>
__device__ __forceinline__ void interface_flux_vjp(R hm, R um, R vm, R bm, R hp, R up, R vp, R bp, R nx, R ny,
                                                   const Phys<R> &P, R z0, R z1, R z2, FluxBar<R> &gm,
                                                   FluxBar<R> &gp)
{
    const R g = P.g;
    const R utm = nx * um + ny * vm, vtm = nx * vm - ny * um;
    const R utp = nx * up + ny * vp, vtp = nx * vp - ny * up;
    const R cm = sqrt(g * fmax(hm, R(0)));
    const R cp = sqrt(g * fmax(hp, R(0)));
    const R ah = R(0.5) * (hm + hp), au = R(0.5) * (utm + utp), av = R(0.5) * (vtm + vtp);
    const R ac = R(0.5) * (cm + cp);
    // cotangent in the face frame: F1 = nx f1 - ny f2, F2 = ny f1 + nx f2
    const R f0 = z0, f1 = nx * z1 + ny * z2, f2 = nx * z2 - ny * z1;
    // EC part: f0 = ah au, f1 = ah au^2 + (g/2) ah2, f2 = ah au av
    R bah = f0 * au + f1 * au * au + f2 * au * av;
    R bau = f0 * ah + R(2) * f1 * ah * au + f2 * ah * av;
    R bav = f2 * ah * au;
    const R bah2 = R(0.5) * g * f1;
    R bac = 0, bhm = 0, bhp = 0, bbm = 0, bbp = 0, butm = 0, bvtm = 0, butp = 0, bvtp = 0;
    if (!P.ec) {
        // dissipation -1/2 R |Lambda| R^T [[q~]] in the closed form of interface_flux
        const R dq1 = g * ((hp + bp) - (hm + bm)) - R(0.5) * ((utp * utp + vtp * vtp) - (utm * utm + vtm * vtm));
        const R dq2 = utp - utm, dq3 = vtp - vtm;
        const R sp = au + ac, sm = au - ac;
        const R lp = fabs(sp) * P.i2g, l2 = fabs(ah * au), lm = fabs(sm) * P.i2g;
        const R s1 = dq1 + sp * dq2 + av * dq3, s3 = dq1 + sm * dq2 + av * dq3;
        const R r1 = lp * s1, r3 = lm * s3;
        // f0 -= (r1 + r3)/2, f1 -= (sp r1 + sm r3)/2, f2 -= (av (r1 + r3) + r2)/2
        const R br1 = R(-0.5) * (f0 + sp * f1 + av * f2);
        const R br3 = R(-0.5) * (f0 + sm * f1 + av * f2);
        const R br2 = R(-0.5) * f2;
        bau -= R(0.5) * f1 * (r1 + r3);
        bac -= R(0.5) * f1 * (r1 - r3);
        bav -= R(0.5) * f2 * (r1 + r3);
        // r1 = lp s1, r2 = l2 dq3, r3 = lm s3
        const R blp = br1 * s1, blm = br3 * s3, bl2 = br2 * dq3;
        const R bs1 = br1 * lp, bs3 = br3 * lm;
        const R bdq1 = bs1 + bs3;
        const R bdq2 = bs1 * sp + bs3 * sm;
        const R bdq3 = br2 * l2 + (bs1 + bs3) * av;
        bau += (bs1 + bs3) * dq2;
        bac += (bs1 - bs3) * dq2;
        bav += (bs1 + bs3) * dq3;
        // lp = |au + ac|/(2g), lm = |au - ac|/(2g), l2 = |ah au|
        const R gp_ = blp * sgn(sp) * P.i2g, gm_ = blm * sgn(sm) * P.i2g, g2 = bl2 * sgn(ah * au);
        bau += gp_ + gm_ + g2 * ah;
        bac += gp_ - gm_;
        bah += g2 * au;
        // jumps of the entropy variables
        bhp += g * bdq1; bbp += g * bdq1;
        bhm -= g * bdq1; bbm -= g * bdq1;
        butp += bdq2 - utp * bdq1; bvtp += bdq3 - vtp * bdq1;
        butm += utm * bdq1 - bdq2; bvtm += vtm * bdq1 - bdq3;
    }
    // averages: ah, au, av, ah2 = (hm^2 + hp^2)/2, ac = (cm + cp)/2
    bhm += R(0.5) * bah + hm * bah2;
    bhp += R(0.5) * bah + hp * bah2;
    butm += R(0.5) * bau; butp += R(0.5) * bau;
    bvtm += R(0.5) * bav; bvtp += R(0.5) * bav;
    if (cm > R(0)) bhm += R(0.25) * bac * g / cm;
    if (cp > R(0)) bhp += R(0.25) * bac * g / cp;
    // rotation: ut = nx u + ny v, vt = nx v - ny u
    gm.h = bhm; gm.u = nx * butm - ny * bvtm; gm.v = ny * butm + nx * bvtm; gm.b = bbm;
    gp.h = bhp; gp.u = nx * butp - ny * bvtp; gp.v = ny * butp + nx * bvtp; gp.b = bbp;
}

struct AdjArgs {
    Mesh<double> m;
    Phys<double> P;
    Tab<double> tab;               // uniform entries
    const Tab<double> *tg;         // the same in device memory (per-lane entries)
    const double *h, *hu, *hv;     // stage input W_{k-1}
    const double *a[3];            // dL/dW_k (nullptr: zero)
    const double *c[3];            // A_{k+1} dL/dd_{k+1} (nullptr: zero)
    double *ao[3];                 // dL/dW_{k-1}
    double *co[3];                 // A_k dL/dd_k (nullptr: not written)
    const double *x[3];            // added to ao (nullptr: zero)
    const double *y[3];            // added to co (nullptr: zero; may alias co)
    double *gbx, *gby, *gbn;       // bathymetry cotangents (accumulated)
    double ca, cb, dt;             // A_k, B_k, step
    double sa;                     // scale of a in ao (1 for LSRK)
    int64_t ntiles;
};

// Face slot data of the reverse stage, loaded with the element's own data
// ahead of the LDS staging so that their latency is paid once (as in the
// forward stage kernel): the neighbour's trace, cotangent inputs and metric
// at the shared node, and the face bathymetry of both sides.
struct AdjFacePrefetch {
    bool wall = false;
    double hn = 0, hun = 0, hvn = 0;
    double c0 = 0, c1 = 0, c2 = 0, a0 = 0, a1 = 0, a2 = 0;
    double nAx = 0, nCx = 0, nAe = 0, nCe = 0;
    double bo = 0, bn = 0;
};

template <int N>
__device__ __forceinline__ void adj_prefetch_face(const AdjArgs &a, int f, int64_t e0, AdjFacePrefetch &pf)
{
    constexpr int nf = N + 1;
    if (f >= Shape<N>::NFACE) return;
    const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
    const int64_t fe = e0 + fel;
    if (fe >= a.m.K) return;
    int ns, kk;
    int64_t en;
    const int64_t qn = nbr_node<N>(a.m, fe, s, k, en, ns, kk);
    pf.wall = is_wall(a.m, fe, s);
    pf.hn = a.h[qn]; pf.hun = a.hu[qn]; pf.hvn = a.hv[qn];
    if (!pf.wall) {
        pf.nAx = a.m.Ax[qn]; pf.nCx = a.m.Cx[qn]; pf.nAe = a.m.Ae[qn]; pf.nCe = a.m.Ce[qn];
        if (a.c[0]) { pf.c0 = a.c[0][qn]; pf.c1 = a.c[1][qn]; pf.c2 = a.c[2][qn]; }
        if (a.a[0]) { pf.a0 = a.a[0][qn]; pf.a1 = a.a[1][qn]; pf.a2 = a.a[2][qn]; }
    }
    pf.bo = a.m.bface[(fe * 4 + s) * nf + k];
    pf.bn = a.m.bface[(en * 4 + ns) * nf + kk];
}

// Register budget of four waves per SIMD (128 VGPRs, a few spilled) for
// N >= 3: unbounded it takes 132-134 VGPRs and three waves; measured 2.5%
// faster per launch at 128^2, N = 5, and 2.7% at 192^2, N = 3 (five waves
// spill 36 VGPRs and run 40% slower).  N = 2, with two face slots per lane,
// spills 20 VGPRs under that budget and runs 14% slower: no budget there
// (with each slot's loads grouped ahead of its evaluation it runs 12%
// faster than before, 40.8 against 46.4 us at 256^2).
template <int N>
struct AdjWaves {
    static constexpr int value = N == 2 ? 1 : 4;
};

template <int N>
__global__ __launch_bounds__(Shape<N>::T, AdjWaves<N>::value) void adjoint_stage_kernel(AdjArgs a)
{
    using S = Shape<N>;
    using R = double;
    constexpr int nf = S::nf, np = S::np, E = S::E, T = S::T, NF = S::NFACE;
    __shared__ R s_h[T];
    __shared__ double2 s_q[T], s_w[T], s_a[T], s_b[T];   // (hu, hv), (u, v), J grad(xi), J grad(eta)
    __shared__ R s_m[3][T];                              // mu = -l / J
    __shared__ R s_fg[4][NF];                            // face cotangents: h, u, v, b
    __shared__ R s_dz[nf * nf];                          // D with a zero diagonal

    const int64_t tile = xcd_tile(a.ntiles);
    if (tile < 0) return;
    const int t = threadIdx.x;
    const bool lane = t < E * np;
    const int el = lane ? t / np : E - 1, p = lane ? t - el * np : 0, i = p / nf, j = p - i * nf;
    const int64_t e0 = tile * E, e = e0 + el;
    const bool act = lane && (e < a.m.K);
    const int64_t q = e * np + p;
    const Phys<R> &P = a.P;

    R h = 0, hu = 0, hv = 0, Ax = 0, Cx = 0, Ae = 0, Ce = 0, A0 = 0, A1 = 0, A2 = 0, l0 = 0, l1 = 0, l2 = 0;
    if (act) {
        h = a.h[q]; hu = a.hu[q]; hv = a.hv[q];
        Ax = a.m.Ax[q]; Cx = a.m.Cx[q]; Ae = a.m.Ae[q]; Ce = a.m.Ce[q];
        if (a.a[0]) { A0 = a.a[0][q]; A1 = a.a[1][q]; A2 = a.a[2][q]; }
        if (a.c[0]) { l0 = a.c[0][q]; l1 = a.c[1][q]; l2 = a.c[2][q]; }
    }
    // one face slot per lane: its loads go out with the element's own (with
    // two per lane, at N = 2, holding both would spill; they load after the
    // staging as the slots are evaluated)
    constexpr int NS = (NF + T - 1) / T;
    AdjFacePrefetch pf0;
    if constexpr (NS == 1) adj_prefetch_face<N>(a, t, e0, pf0);
    if (act) { l0 += a.cb * A0; l1 += a.cb * A1; l2 += a.cb * A2; }
    const R ih = rcp_wet(h, P.h_tol);
    const R u = hu * ih, v = hv * ih;
    const R J = Ce * Ax - Cx * Ae;
    const R iJ = act ? R(1) / J : R(0);
    const R m0 = -l0 * iJ, m1 = -l1 * iJ, m2 = -l2 * iJ;
    s_h[t] = h;
    s_q[t] = double2{hu, hv};
    s_w[t] = double2{u, v};
    s_a[t] = double2{Ax, Cx};
    s_b[t] = double2{Ae, Ce};
    s_m[0][t] = m0; s_m[1][t] = m1; s_m[2][t] = m2;
    for (int c = t; c < nf * nf; c += T) s_dz[c] = a.tg->Dz[(c / nf) * kMaxNF + (c - (c / nf) * nf)];
    lds_sync<T>();

    // ---- interface: own term w.r.t. the '-' trace, neighbour's term w.r.t. its '+' trace ----
    auto face_slot = [&](const int f, const AdjFacePrefetch &pfr) {
        const int fel = f / (4 * nf), s = (f / nf) & 3, k = f - (f / nf) * nf;
        const int64_t fe = e0 + fel;
        R gh = 0, gu = 0, gv = 0, gb = 0;
        if (fe < a.m.K) {
            int fi, fj;
            side_node<N>(s, k, fi, fj);
            const int lp = fel * np + fi * nf + fj;
            // own outward normal and surface Jacobian
            const double2 dir = (s & 1) ? s_a[lp] : s_b[lp];
            const R sg = (s == 0 || s == 3) ? R(-1) : R(1);
            const R snx = sg * dir.x, sny = sg * dir.y;
            const R js = sqrt(snx * snx + sny * sny);
            const R nx = snx / js, ny = sny / js;
            const bool wall = pfr.wall;
            // neighbour's trace and cotangent mu_n = -l_n / J_n (a wall: the
            // own trace, mirrored, and no neighbour term)
            const R hn = pfr.hn;
            const R inn = rcp_wet(hn, P.h_tol);
            R un = pfr.hun * inn, vn = pfr.hvn * inn;
            R nm0 = 0, nm1 = 0, nm2 = 0;
            if (wall) {
                wall_mirror(nx, ny, un, vn);
            } else {
                const R nJ = pfr.nCe * pfr.nAx - pfr.nCx * pfr.nAe;
                R nl0 = pfr.c0, nl1 = pfr.c1, nl2 = pfr.c2;
                if (a.a[0]) { nl0 += a.cb * pfr.a0; nl1 += a.cb * pfr.a1; nl2 += a.cb * pfr.a2; }
                const R inJ = R(1) / nJ;
                nm0 = nl0 * inJ; nm1 = nl1 * inJ; nm2 = nl2 * inJ;
            }
            const R bo = pfr.bo;
            const R bn = pfr.bn;
            const R ho = s_h[lp];
            const double2 wo = s_w[lp];
            // Own term (J^surf / w_0) mu . F*(own, nbr, n) and the neighbour's
            // (J^surf / w_0) mu_n . F*(nbr, own, -n) = -(J^surf / w_0) mu_n . F*(own, nbr, n)
            // (the flux is conservative; on a conforming mesh both sides share
            // the face's normal up to sign and its surface Jacobian): one
            // reverse evaluation with the cotangent (J^surf / w_0)(mu - mu_n).
            const R so = js * a.tab.iw0;
            FluxBar<R> g1, g2;
            interface_flux_vjp<R>(ho, wo.x, wo.y, bo, hn, un, vn, bn, nx, ny, P, so * (s_m[0][lp] + nm0),
                                  so * (s_m[1][lp] + nm1), so * (s_m[2][lp] + nm2), g1, g2);
            gh = g1.h; gu = g1.u; gv = g1.v; gb = g1.b;
            if (!wall) {
                // interface bathymetry penalty (g/(4 w_0)) (h + h_n)(b_n - b) J^surf n
                // in L of both sides (the neighbour's with its own normal, -n
                // up to rounding): d/dh and d/db of this node from both terms
                const R wpen = R(0.25) * P.g * a.tab.iw0 *
                               ((s_m[1][lp] - nm1) * snx + (s_m[2][lp] - nm2) * sny);
                gh += wpen * (bn - bo);
                gb -= wpen * (ho + hn);
            }
            if (wall) {
                // the outside trace is (h, M(u, v), b), M = I - 2 n n^T = M^T:
                // its cotangent returns through the mirror
                wall_mirror(nx, ny, g2.u, g2.v);
                gh += g2.h; gu += g2.u; gv += g2.v; gb += g2.b;
            }
        }
        s_fg[0][f] = gh; s_fg[1][f] = gu; s_fg[2][f] = gv; s_fg[3][f] = gb;
    };
    if constexpr (NS == 1) {
        if (t < NF) face_slot(t, pf0);
    } else {
        for (int f = t; f < NF; f += T) {
            AdjFacePrefetch pfl;
            adj_prefetch_face<N>(a, f, e0, pfl);
            face_slot(f, pfl);
        }
    }

    // ---- volume: pairs along xi and eta; z = Dz_im mu_i + Dz_mi mu_m (D~ = 2 Dz).
    // Unrolled by two only: a full unroll hoists every partner's LDS reads
    // and needs more registers than one wave per SIMD leaves ----
    R P1 = 0, P2 = 0, Gh = 0, Tu = 0, Tv = 0;
    {
        const int base = el * np;
#pragma unroll 2
        for (int mm = 0; mm < nf; ++mm) {
            const int qq = base + mm * nf + j;
            const R da = s_dz[i * nf + mm], db = s_dz[mm * nf + i];
            const R z0 = da * m0 + db * s_m[0][qq], z1 = da * m1 + db * s_m[1][qq], z2 = da * m2 + db * s_m[2][qq];
            const double2 am = s_a[qq], qm = s_q[qq], wm = s_w[qq];
            const R sA = Ax + am.x, sC = Cx + am.y;
            const R Q = (hu + qm.x) * sA + (hv + qm.y) * sC;
            const R tt = z0 + R(0.5) * ((u + wm.x) * z1 + (v + wm.y) * z2);
            P1 += Q * z1; P2 += Q * z2;
            Gh += s_h[qq] * (sA * z1 + sC * z2);
            Tu += sA * tt; Tv += sC * tt;
        }
#pragma unroll 2
        for (int mm = 0; mm < nf; ++mm) {
            const int qq = base + i * nf + mm;
            const R da = s_dz[j * nf + mm], db = s_dz[mm * nf + j];
            const R z0 = da * m0 + db * s_m[0][qq], z1 = da * m1 + db * s_m[1][qq], z2 = da * m2 + db * s_m[2][qq];
            const double2 bm = s_b[qq], qm = s_q[qq], wm = s_w[qq];
            const R sA = Ae + bm.x, sC = Ce + bm.y;
            const R Q = (hu + qm.x) * sA + (hv + qm.y) * sC;
            const R tt = z0 + R(0.5) * ((u + wm.x) * z1 + (v + wm.y) * z2);
            P1 += Q * z1; P2 += Q * z2;
            Gh += s_h[qq] * (sA * z1 + sC * z2);
            Tu += sA * tt; Tv += sC * tt;
        }
    }
    lds_sync<T>();   // face slots complete

    // face cotangents of this node (primitive velocities), summed over its sides
    R fh = 0, fu = 0, fv = 0, fb = 0;
    {
        const int fb0 = el * 4 * nf;
        auto side = [&](int f) { fh += s_fg[0][f]; fu += s_fg[1][f]; fv += s_fg[2][f]; fb += s_fg[3][f]; };
        if (j == 0) side(fb0 + 0 * nf + i);
        if (i == N) side(fb0 + 1 * nf + j);
        if (j == N) side(fb0 + 2 * nf + i);
        if (i == 0) side(fb0 + 3 * nf + j);
    }
    if (!act) return;
    const R g = P.g;
    const R bxv = a.m.bx[q], byv = a.m.by[q];
    // u = hu/h: d/dhu = 1/h, d/dh = -u/h (zero below the dry cut-off: ih = 0)
    const R gh = R(-0.25) * (u * P1 + v * P2) * ih + R(0.5) * g * Gh + fh - (u * fu + v * fv) * ih +
                 R(0.5) * g * (m1 * bxv + m2 * byv);
    const R ghu = R(0.5) * Tu + R(0.25) * P1 * ih + fu * ih;
    const R ghv = R(0.5) * Tv + R(0.25) * P2 * ih + fv * ih;
    const R dt = a.dt;
    R x0 = 0, x1 = 0, x2 = 0;
    if (a.x[0]) { x0 = a.x[0][q]; x1 = a.x[1][q]; x2 = a.x[2][q]; }
    a.ao[0][q] = a.sa * A0 + dt * gh + x0;
    a.ao[1][q] = a.sa * A1 + dt * ghu + x1;
    a.ao[2][q] = a.sa * A2 + dt * ghv + x2;
    if (a.co[0]) {
        R y0 = 0, y1 = 0, y2 = 0;
        if (a.y[0]) { y0 = a.y[0][q]; y1 = a.y[1][q]; y2 = a.y[2][q]; }
        a.co[0][q] = a.ca * l0 + y0;
        a.co[1][q] = a.ca * l1 + y1;
        a.co[2][q] = a.ca * l2 + y2;
    }
    const R hs = R(0.5) * g * h * dt;
    a.gbx[q] += hs * m1;
    a.gby[q] += hs * m2;
    a.gbn[q] += dt * fb;
}

// gb = (d(b_x, b_y)/db)^T (gbx, gby) + gbn for the split derivatives of
// eq. SourceDisc, b_x = y_eta D_xi b + D_xi(y_eta b) - y_xi D_eta b - D_eta(y_xi b)
// and b_y alike: node (a, c) collects sum_i D_ia [(Ax_ic + Ax_ac) gbx_ic +
// (Cx_ic + Cx_ac) gby_ic] + sum_j D_jc [(Ae_aj + Ae_ac) gbx_aj + (Ce_aj + Ce_ac) gby_aj].
template <int N>
__global__ void bathymetry_adjoint_kernel(int64_t K, const double *__restrict__ Ax, const double *__restrict__ Cx,
                                          const double *__restrict__ Ae, const double *__restrict__ Ce,
                                          const double *__restrict__ gbx, const double *__restrict__ gby,
                                          const double *__restrict__ gbn, double *__restrict__ gb, Tab<double> tab)
{
    constexpr int nf = N + 1, np = nf * nf;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * np) return;
    const int64_t e = q / np;
    const int p = (int)(q - e * np), i = p / nf, j = p - i * nf;
    const int64_t o = e * np;
    const double ax = Ax[q], cx = Cx[q], ae = Ae[q], ce = Ce[q];
    double s = gbn[q];
#pragma unroll
    for (int m = 0; m < nf; ++m) {
        const int64_t qa = o + m * nf + j, qb = o + i * nf + m;
        s += tab.D[m * kMaxNF + i] * ((Ax[qa] + ax) * gbx[qa] + (Cx[qa] + cx) * gby[qa]);
        s += tab.D[m * kMaxNF + j] * ((Ae[qb] + ae) * gbx[qb] + (Ce[qb] + ce) * gby[qb]);
    }
    gb[q] = s;
}

}  // namespace esdg
