/*
 * Plain FP64 CPU oracle of the entropy-stable nodal DGSEM for the 2D shallow
 * water equations with artificial viscosity and the positivity limiter
 * (Wintermeyer, Winters, Gassner, Warburton, arXiv:1804.02221).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU library is checked against.  It shares no code, header,
 * table or helper with the HIP path; only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  Build: gcc -O2 -ffp-contract=off
 * (no fast-math), no OpenMP.
 *
 * Every function follows the paper's equations in the paper's order and
 * notation.  Where the printed formula is garbled or silent, the reading
 * taken is stated at the spot (the full list is kept with the design notes).
 *
 * Conventions.  Arrays are [K][(N+1)^2], node p = i*(N+1)+j, i <-> xi,
 * j <-> eta.  Local sides 0..3 are the paper's s=1..4: eta=-1, xi=+1,
 * eta=+1, xi=-1.  Face node k runs along increasing xi (sides 0,2) or eta
 * (sides 1,3).  nbr_elem/nbr_side/flip give the element and side sharing
 * each side; flip=1 reverses the neighbour's face-node order; nbr_elem = -1
 * marks a solid wall.
 *
 * Parity status of each part is listed in the test suite; functions whose
 * result no property of the paper fixes say so below ("parity unpinned").
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NMAX 16

typedef struct {
    double g;          /* gravitational constant                              */
    double h_tol;      /* velocity cut-off height, section 6.1 (1e-4)         */
    double eps0;       /* artificial-viscosity amplitude, appendix A          */
    double sigma_min;  /* indicator thresholds, appendix A (reading A12)      */
    double sigma_max;
    double cfl;        /* advective CFL number                                */
    double cfl_visc;   /* safety factor of the viscous time-step bound        */
    int surface_flux;  /* 0 = entropy stable (ES), 1 = entropy conservative   */
    int av_on;         /* artificial viscosity on                             */
    int limiter_on;    /* positivity limiter on                               */
    int integrator;    /* 0 = LSRK(5,4) 2N-storage, 1 = SSPRK(3,3)            */
    int max_dt_retries;
} orc_params;

typedef struct {
    int N;
    int64_t K;
    const double *x, *y;          /* nodal coordinates [K][np]             */
    const int32_t *nbr_elem;      /* [K][4]                                */
    const int8_t *nbr_side;       /* [K][4]                                */
    const int8_t *flip;           /* [K][4]                                */
} orc_mesh;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENEGMEAN = -5 };

/* ------------------------------------------------------------------------ */
/* Operators: LGL nodes and weights, derivative matrix, SBP matrices,        */
/* Vandermonde (section 2.2 and appendix A)                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N;
    double xi[ORC_NMAX + 1], w[ORC_NMAX + 1];
    double D[ORC_NMAX + 1][ORC_NMAX + 1];   /* D_ij = l_j'(xi_i)             */
    double Dt[ORC_NMAX + 1][ORC_NMAX + 1];  /* D~ = 2D + S                   */
    double Dh[ORC_NMAX + 1][ORC_NMAX + 1];  /* D^ = -M^{-1} D^T M            */
    double Vinv[ORC_NMAX + 1][ORC_NMAX + 1];/* nodal -> orthonormal modal    */
} orc_ops;

/* Legendre polynomial L_n(x) and its derivative, three-term recurrence. */
static void legendre(int n, long double x, long double *L, long double *dL)
{
    long double l0 = 1.0L, l1 = x;
    if (n == 0) { *L = 1.0L; *dL = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
        long double l2 = ((2 * k + 1) * x * l1 - k * l0) / (k + 1);
        l0 = l1;
        l1 = l2;
    }
    *L = l1;
    /* (1 - x^2) L_n' = n (L_{n-1} - x L_n) */
    if (fabsl(1.0L - x * x) > 0.0L)
        *dL = n * (l0 - x * l1) / (1.0L - x * x);
    else
        *dL = (x > 0 ? 1.0L : ((n % 2) ? 1.0L : -1.0L)) * 0.5L * n * (n + 1);
}

static void lgl_nodes_weights(int N, double *xi, double *w)
{
    /* Nodes: -1, +1 and the roots of L_N' (Newton, long double).
     * Weights: w_j = 2 / (N (N+1) L_N(xi_j)^2). */
    long double X[ORC_NMAX + 1];
    X[0] = -1.0L;
    X[N] = 1.0L;
    for (int j = 1; j < N; ++j) {
        long double x = -cosl(3.14159265358979323846264338327950288L * j / N);
        for (int it = 0; it < 100; ++it) {
            long double L, dL;
            legendre(N, x, &L, &dL);
            /* Legendre ODE: (1-x^2) L'' = 2 x L' - N(N+1) L */
            long double d2L = (2.0L * x * dL - (long double)N * (N + 1) * L) / (1.0L - x * x);
            long double dx = dL / d2L;
            x -= dx;
            if (fabsl(dx) < 1e-30L) break;
        }
        X[j] = x;
    }
    for (int j = 0; j <= N; ++j) {
        long double L, dL;
        legendre(N, X[j], &L, &dL);
        xi[j] = (double)X[j];
        w[j] = (double)(2.0L / ((long double)N * (N + 1) * L * L));
    }
}

static void gauss_nodes_weights(int n, long double *x, long double *w)
{
    /* n-point Legendre-Gauss rule: roots of L_n, w = 2/((1-x^2) L_n'(x)^2). */
    for (int l = 0; l < n; ++l) {
        long double t = -cosl(3.14159265358979323846264338327950288L * (l + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double L, dL;
            legendre(n, t, &L, &dL);
            long double dt = L / dL;
            t -= dt;
            if (fabsl(dt) < 1e-30L) break;
        }
        long double L, dL;
        legendre(n, t, &L, &dL);
        x[l] = t;
        w[l] = 2.0L / ((1.0L - t * t) * dL * dL);
    }
}

/* Lagrange basis l_j on the LGL nodes, evaluated at t (definition). */
static long double lagrange(int N, const double *xi, int j, long double t)
{
    long double p = 1.0L;
    for (int i = 0; i <= N; ++i)
        if (i != j) p *= (t - xi[i]) / ((long double)xi[j] - xi[i]);
    return p;
}

static void build_ops(int N, orc_ops *op)
{
    memset(op, 0, sizeof(*op));
    op->N = N;
    lgl_nodes_weights(N, op->xi, op->w);
    /* D_ij = l_j'(xi_i) (eq. DmatDef), barycentric form; the diagonal makes
     * every row sum to zero (derivative of a constant). */
    long double lam[ORC_NMAX + 1];
    for (int j = 0; j <= N; ++j) {
        long double p = 1.0L;
        for (int k = 0; k <= N; ++k)
            if (k != j) p *= ((long double)op->xi[j] - op->xi[k]);
        lam[j] = 1.0L / p;
    }
    for (int i = 0; i <= N; ++i) {
        long double diag = 0.0L;
        for (int j = 0; j <= N; ++j) {
            if (j == i) continue;
            long double d = (lam[j] / lam[i]) / ((long double)op->xi[i] - op->xi[j]);
            op->D[i][j] = (double)d;
            diag -= d;
        }
        op->D[i][i] = (double)diag;
    }
    /* S = diag(1/w_0, 0, ..., 0, -1/w_N); D~ = 2D + S (eq. Dmat_modification);
     * D^ = -M^{-1} D^T M (reading: the printed -M^{-1} D M is not the
     * matrix that satisfies D = -S + D^). */
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) {
            double S = 0.0;
            if (i == j && i == 0) S = 1.0 / op->w[0];
            if (i == j && i == N) S = -1.0 / op->w[N];
            op->Dt[i][j] = 2.0 * op->D[i][j] + S;
            op->Dh[i][j] = -(op->w[j] / op->w[i]) * op->D[j][i];
        }
    /* Vandermonde inverse by Gauss quadrature (appendix A, eq. Vandermonde):
     * Vinv_ij = sum_l Lt_i(xg_l) l_j(xg_l) wg_l with Lt_i = sqrt(i+1/2) L_i.
     * (Reading: the printed l_j(x^G_i) means the quadrature node x^G_l.) */
    long double xg[ORC_NMAX + 1], wg[ORC_NMAX + 1];
    gauss_nodes_weights(N + 1, xg, wg);
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) {
            long double s = 0.0L;
            for (int l = 0; l <= N; ++l) {
                long double Li, dLi;
                legendre(i, xg[l], &Li, &dLi);
                s += Li * lagrange(N, op->xi, j, xg[l]) * wg[l];
            }
            op->Vinv[i][j] = (double)(s * sqrtl(i + 0.5L));
        }
}

int orc_operators(int N, double *xi, double *w, double *D, double *Dtilde,
                  double *Dhat, double *Vinv)
{
    if (N < 1 || N > ORC_NMAX) return ORC_EINVAL;
    orc_ops op;
    build_ops(N, &op);
    int n1 = N + 1;
    for (int i = 0; i < n1; ++i) {
        if (xi) xi[i] = op.xi[i];
        if (w) w[i] = op.w[i];
        for (int j = 0; j < n1; ++j) {
            if (D) D[i * n1 + j] = op.D[i][j];
            if (Dtilde) Dtilde[i * n1 + j] = op.Dt[i][j];
            if (Dhat) Dhat[i * n1 + j] = op.Dh[i][j];
            if (Vinv) Vinv[i * n1 + j] = op.Vinv[i][j];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Geometry (section 2.1): metric terms by the derivative matrix, Jacobian   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *xxi, *xeta, *yxi, *yeta, *J;   /* [K][np] */
} orc_geom;

static int geom_alloc(orc_geom *G, int64_t n)
{
    G->xxi = malloc(sizeof(double) * n);
    G->xeta = malloc(sizeof(double) * n);
    G->yxi = malloc(sizeof(double) * n);
    G->yeta = malloc(sizeof(double) * n);
    G->J = malloc(sizeof(double) * n);
    return (G->xxi && G->xeta && G->yxi && G->yeta && G->J) ? 0 : -1;
}

static void geom_free(orc_geom *G)
{
    free(G->xxi); free(G->xeta); free(G->yxi); free(G->yeta); free(G->J);
}

static void geometry(const orc_ops *op, const orc_mesh *m, orc_geom *G)
{
    int N = op->N, n1 = N + 1, np = n1 * n1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->K; ++e) {
        const double *x = m->x + e * np, *y = m->y + e * np;
        /* The metric terms are derivatives of the mapping, so they do not
         * change when the element is translated: differentiate coordinates
         * relative to the element's first node, which keeps the sums at the
         * element's size instead of the domain's (no cancellation against
         * the absolute position). */
        const double x0 = x[0], y0 = y[0];
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                double xx = 0, xe = 0, yx = 0, ye = 0;
                for (int mm = 0; mm <= N; ++mm) {
                    xx += op->D[i][mm] * (x[mm * n1 + j] - x0);
                    yx += op->D[i][mm] * (y[mm * n1 + j] - y0);
                    xe += op->D[j][mm] * (x[i * n1 + mm] - x0);
                    ye += op->D[j][mm] * (y[i * n1 + mm] - y0);
                }
                int64_t q = e * np + i * n1 + j;
                G->xxi[q] = xx; G->xeta[q] = xe; G->yxi[q] = yx; G->yeta[q] = ye;
                G->J[q] = xx * ye - xe * yx;                 /* eq. JacobianDef */
            }
    }
}

int orc_geometry(int N, int64_t K, const double *x, const double *y, double *xxi,
                 double *xeta, double *yxi, double *yeta, double *J)
{
    if (N < 1 || N > ORC_NMAX || K < 0) return ORC_EINVAL;
    orc_ops op;
    build_ops(N, &op);
    orc_mesh m = {N, K, x, y, NULL, NULL, NULL};
    orc_geom G = {xxi, xeta, yxi, yeta, J};
    geometry(&op, &m, &G);
    return ORC_OK;
}

/* Face node k of local side s -> local (i, j). */
static void side_node(int N, int s, int k, int *i, int *j)
{
    switch (s) {
    case 0: *i = k; *j = 0; break;
    case 1: *i = N; *j = k; break;
    case 2: *i = k; *j = N; break;
    default: *i = 0; *j = k; break;
    }
}

/* Outward scaled normal of side s at node q: the contravariant direction
 * (+-xi or +-eta) written with the metric terms; its length is the surface
 * Jacobian of eq. SurfJac. */
static void scaled_normal(const orc_geom *G, int s, int64_t q, double *nx, double *ny)
{
    switch (s) {
    case 0: *nx = G->yxi[q]; *ny = -G->xxi[q]; break;     /* eta = -1 */
    case 1: *nx = G->yeta[q]; *ny = -G->xeta[q]; break;   /* xi  = +1 */
    case 2: *nx = -G->yxi[q]; *ny = G->xxi[q]; break;     /* eta = +1 */
    default: *nx = -G->yeta[q]; *ny = G->xeta[q]; break;  /* xi  = -1 */
    }
}

/* Is side s of element e a solid wall (no neighbour)? */
static int is_wall(const orc_mesh *m, int64_t e, int s)
{
    return m->nbr_elem[e * 4 + s] < 0;
}

/* The neighbour node matched to face node k of side s of element e; at a
 * wall, the element's own face node (its trace is then mirrored where the
 * flux needs the outside state). */
static int64_t nbr_node(const orc_mesh *m, int64_t e, int s, int k)
{
    int N = m->N, n1 = N + 1, np = n1 * n1;
    if (is_wall(m, e, s)) {
        int i, j;
        side_node(N, s, k, &i, &j);
        return e * np + i * n1 + j;
    }
    int64_t en = m->nbr_elem[e * 4 + s];
    int sn = m->nbr_side[e * 4 + s];
    int kk = m->flip[e * 4 + s] ? N - k : k;
    int i, j;
    side_node(N, sn, kk, &i, &j);
    return en * np + i * n1 + j;
}

/* ------------------------------------------------------------------------ */
/* Point-wise fluxes                                                         */
/* ------------------------------------------------------------------------ */
/* Velocity with the dry cut-off of section 6.1: zero where h <= h_tol. */
static double velocity(double hq, double h, double h_tol)
{
    return (h > h_tol) ? hq / h : 0.0;
}

/* Outside state of a solid wall with unit outward normal n: the same water
 * height and the discharge with its normal component reversed (reading: the
 * usual reflecting wall; the interface flux then carries no mass through the
 * wall and, for the EC flux, no entropy). */
static void wall_state(const double *wm, double nx, double ny, double *wp)
{
    double dn = wm[1] * nx + wm[2] * ny;
    wp[0] = wm[0];
    wp[1] = wm[1] - 2.0 * dn * nx;
    wp[2] = wm[2] - 2.0 * dn * ny;
}

/* Entropy-conservative two-point volume fluxes F#, G# (eq. volumeFluxes). */
void orc_volume_flux(double g, double h_tol, const double *wa, const double *wb,
                     double *Fs, double *Gs)
{
    double ha = wa[0], hb = wb[0];
    double ua = velocity(wa[1], ha, h_tol), ub = velocity(wb[1], hb, h_tol);
    double va = velocity(wa[2], ha, h_tol), vb = velocity(wb[2], hb, h_tol);
    double avg_h = 0.5 * (ha + hb);
    double avg_h2 = 0.5 * (ha * ha + hb * hb);
    double avg_hu = 0.5 * (wa[1] + wb[1]);
    double avg_hv = 0.5 * (wa[2] + wb[2]);
    double avg_u = 0.5 * (ua + ub);
    double avg_v = 0.5 * (va + vb);
    double p = g * avg_h * avg_h - 0.5 * g * avg_h2;
    Fs[0] = avg_hu;
    Fs[1] = avg_hu * avg_u + p;
    Fs[2] = avg_hu * avg_v;
    Gs[0] = avg_hv;
    Gs[1] = avg_hv * avg_u;
    Gs[2] = avg_hv * avg_v + p;
}

/* Numerical interface flux in the direction of the unit normal n (pointing
 * from the '-' state into the '+' state), evaluated in the rotated frame
 * (appendix B, eqs. rotatingVelocities, surfaceFlux2DRotated,
 * surfaceFlux2DCurved, RightEigenvectors2DCurved, ScalingMatrix2DCurved).
 * Entropy-stable: the EC flux minus 1/2 R|Lambda|R^T [[q~]], evaluated as
 * the matrix product; entropy-conservative: the first term only
 * (eq. surfaceFluxes).  Reading: {c} is the mean of c = sqrt(g h). */
void orc_surface_flux(const orc_params *P, const double *wm, double bm, const double *wp,
                      double bp, double nx, double ny, double *F)
{
    double g = P->g;
    double hm = wm[0], hp = wp[0];
    double um = velocity(wm[1], hm, P->h_tol), vm = velocity(wm[2], hm, P->h_tol);
    double up = velocity(wp[1], hp, P->h_tol), vp = velocity(wp[2], hp, P->h_tol);
    /* rotate: u~ = n.u, v~ = t.u with t = (-ny, nx) */
    double utm = nx * um + ny * vm, vtm = -ny * um + nx * vm;
    double utp = nx * up + ny * vp, vtp = -ny * up + nx * vp;
    double cm = sqrt(g * fmax(hm, 0.0)), cp = sqrt(g * fmax(hp, 0.0));
    double ah = 0.5 * (hm + hp), au = 0.5 * (utm + utp), av = 0.5 * (vtm + vtp);
    double ah2 = 0.5 * (hm * hm + hp * hp), ac = 0.5 * (cm + cp);
    double Fr[3];
    Fr[0] = ah * au;
    Fr[1] = ah * au * au + 0.5 * g * ah2;
    Fr[2] = ah * au * av;
    if (P->surface_flux == 0) {
        /* jump of the entropy variables q = (g(h+b) - (u^2+v^2)/2, u, v) */
        double qm[3] = {g * (hm + bm) - 0.5 * (utm * utm + vtm * vtm), utm, vtm};
        double qp[3] = {g * (hp + bp) - 0.5 * (utp * utp + vtp * vtp), utp, vtp};
        double dq[3] = {qp[0] - qm[0], qp[1] - qm[1], qp[2] - qm[2]};
        double R[3][3] = {{1.0, 0.0, 1.0},
                          {au + ac, 0.0, au - ac},
                          {av, 1.0, av}};
        double Lam[3] = {fabs(au + ac) / (2.0 * g),
                         2.0 * g * fabs(ah * au) / (2.0 * g),
                         fabs(au - ac) / (2.0 * g)};
        double RTdq[3], dis[3];
        for (int a = 0; a < 3; ++a) {
            RTdq[a] = 0.0;
            for (int c = 0; c < 3; ++c) RTdq[a] += R[c][a] * dq[c];
            RTdq[a] *= Lam[a];
        }
        for (int a = 0; a < 3; ++a) {
            dis[a] = 0.0;
            for (int c = 0; c < 3; ++c) dis[a] += R[a][c] * RTdq[c];
            Fr[a] -= 0.5 * dis[a];
        }
    }
    /* rotate back */
    F[0] = Fr[0];
    F[1] = nx * Fr[1] - ny * Fr[2];
    F[2] = ny * Fr[1] + nx * Fr[2];
}

/* ------------------------------------------------------------------------ */
/* Shock indicator and viscosity (appendix A)                                */
/* ------------------------------------------------------------------------ */
static double viscosity_of_element(const orc_params *P, const orc_ops *op, const double *h)
{
    int N = op->N, n1 = N + 1;
    double hmax = -INFINITY;
    for (int q = 0; q < n1 * n1; ++q) hmax = fmax(hmax, h[q]);
    if (!(hmax > P->h_tol)) return 0.0;   /* dry element: no indicator (reading) */
    /* Q^ = V^{-1} Q V^{-T}, Q = nodal water height (reading A12: Q = h) */
    double T[ORC_NMAX + 1][ORC_NMAX + 1], Qh[ORC_NMAX + 1][ORC_NMAX + 1];
    for (int a = 0; a <= N; ++a)
        for (int j = 0; j <= N; ++j) {
            double s = 0.0;
            for (int i = 0; i <= N; ++i) s += op->Vinv[a][i] * h[i * n1 + j];
            T[a][j] = s;
        }
    for (int a = 0; a <= N; ++a)
        for (int c = 0; c <= N; ++c) {
            double s = 0.0;
            for (int j = 0; j <= N; ++j) s += T[a][j] * op->Vinv[c][j];
            Qh[a][c] = s;
        }
    /* energy in the highest mode shell over all modes, and in the next shell
     * over the modes up to N-1 (eq. sigmadof, simplified form) */
    double topN = Qh[N][N] * Qh[N][N], all = 0.0;
    for (int i = 0; i < N; ++i) topN += Qh[i][N] * Qh[i][N] + Qh[N][i] * Qh[N][i];
    for (int a = 0; a <= N; ++a)
        for (int c = 0; c <= N; ++c) all += Qh[a][c] * Qh[a][c];
    double topM = Qh[N - 1][N - 1] * Qh[N - 1][N - 1], allM = 0.0;
    for (int i = 0; i < N - 1; ++i)
        topM += Qh[i][N - 1] * Qh[i][N - 1] + Qh[N - 1][i] * Qh[N - 1][i];
    for (int a = 0; a < N; ++a)
        for (int c = 0; c < N; ++c) allM += Qh[a][c] * Qh[a][c];
    double r1 = all > 0 ? topN / all : 0.0;
    double r2 = allM > 0 ? topM / allM : 0.0;
    double rmax = fmax(r1, r2);
    if (!(rmax > 0.0)) return 0.0;          /* sigma = -infinity */
    double sigma = log10(rmax);
    /* piecewise ramp; reading: the middle branch is sigma_min < sigma < sigma_max */
    if (sigma <= P->sigma_min) return 0.0;
    if (sigma >= P->sigma_max) return P->eps0;
    double pi = 3.14159265358979323846;
    double Delta = 1.0 + sin(pi * (sigma - 0.5 * (P->sigma_max + P->sigma_min)) /
                             (P->sigma_max - P->sigma_min));
    return 0.5 * P->eps0 * Delta;
}

int orc_indicator(const orc_params *P, int N, int64_t K, const double *h, double *eps)
{
    if (N < 1 || N > ORC_NMAX) return ORC_EINVAL;
    orc_ops op;
    build_ops(N, &op);
    int np = (N + 1) * (N + 1);
    for (int64_t e = 0; e < K; ++e) eps[e] = viscosity_of_element(P, &op, h + e * np);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side R = -(1/J)(L_xi + L_eta - S - L^v_xi - L^v_eta)           */
/* (Lemma 1, eq. RKSSP operator, Theorem 1)                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *Lvol[3];   /* optional [K][np]: L_xi + L_eta (volume + surface)  */
    double *S[3];      /* optional: source S~                                */
    double *Lv[3];     /* optional: L^v_xi + L^v_eta                         */
    double *grad[4];   /* optional: U1, U2, V1, V2 (physical gradients)      */
} orc_parts;

/* need: NULL (all elements) or a [K] mask of elements whose R is wanted. */
static int rhs_impl(const orc_params *P, const orc_ops *op, const orc_mesh *m,
                    const orc_geom *G, const double *b, const double *h, const double *hu,
                    const double *hv, double *Rh, double *Rhu, double *Rhv, double *eps_out,
                    const uint8_t *need, orc_parts *parts)
{
    const int N = op->N, n1 = N + 1, np = n1 * n1;
    const int64_t K = m->K, n = K * np;
    const double g = P->g, htol = P->h_tol;
    double *u = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double *eps = calloc((size_t)K, sizeof(double));
    uint8_t *needv = NULL;     /* elements whose viscous fluxes are needed */
    double *Fv2 = NULL, *Fv3 = NULL, *Gv2 = NULL, *Gv3 = NULL;
    if (!u || !v || !eps) { free(u); free(v); free(eps); return ORC_ENOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        u[q] = velocity(hu[q], h[q], htol);
        v[q] = velocity(hv[q], h[q], htol);
    }
    if (P->av_on) {
        needv = calloc((size_t)K, 1);
        Fv2 = calloc((size_t)n, sizeof(double));
        Fv3 = calloc((size_t)n, sizeof(double));
        Gv2 = calloc((size_t)n, sizeof(double));
        Gv3 = calloc((size_t)n, sizeof(double));
        if (!needv || !Fv2 || !Fv3 || !Gv2 || !Gv3) {
            free(u); free(v); free(eps); free(needv);
            free(Fv2); free(Fv3); free(Gv2); free(Gv3);
            return ORC_ENOMEM;
        }
        for (int64_t e = 0; e < K; ++e) {
            if (need && !need[e]) continue;
            needv[e] = 1;
            for (int s = 0; s < 4; ++s)
                if (!is_wall(m, e, s)) needv[m->nbr_elem[e * 4 + s]] = 1;
        }
        /* viscosity per element from the stage state (appendix A) */
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < K; ++e)
            if (needv[e]) eps[e] = viscosity_of_element(P, op, h + e * np);
        /* BR1 gradients of the gradient variables u, v (eq. BR1).  Readings:
         * the printed formula lacks the division by J; the lifted reference
         * derivative (D^ w)_i + (delta_iN W*_N - delta_i0 W*_0)/w_i enters the
         * chain rule of eq. NablaRelation with the same metric signs as the
         * volume part (the printed signs of the eta-surface term in U1/V1 and
         * the xi-surface term in U2/V2 are inconsistent with it). */
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < K; ++e) {
            if (!needv[e]) continue;
            double Us[4][ORC_NMAX + 1], Vs[4][ORC_NMAX + 1];   /* U* = {u} per side */
            for (int s = 0; s < 4; ++s)
                for (int k = 0; k <= N; ++k) {
                    int i, j;
                    side_node(N, s, k, &i, &j);
                    int64_t q = e * np + i * n1 + j, qn = nbr_node(m, e, s, k);
                    Us[s][k] = 0.5 * (u[q] + u[qn]);
                    Vs[s][k] = 0.5 * (v[q] + v[qn]);
                }
            for (int i = 0; i <= N; ++i)
                for (int j = 0; j <= N; ++j) {
                    int64_t q = e * np + i * n1 + j;
                    double dxu = 0, deu = 0, dxv = 0, dev = 0;
                    for (int mm = 0; mm <= N; ++mm) {
                        dxu += op->Dh[i][mm] * u[e * np + mm * n1 + j];
                        dxv += op->Dh[i][mm] * v[e * np + mm * n1 + j];
                        deu += op->Dh[j][mm] * u[e * np + i * n1 + mm];
                        dev += op->Dh[j][mm] * v[e * np + i * n1 + mm];
                    }
                    /* xi-surface: (delta_iN U*_Nj - delta_i0 U*_0j)/w_i,
                     * U*_Nj on side 1 (k=j), U*_0j on side 3 (k=j) */
                    if (i == N) { dxu += Us[1][j] / op->w[i]; dxv += Vs[1][j] / op->w[i]; }
                    if (i == 0) { dxu -= Us[3][j] / op->w[i]; dxv -= Vs[3][j] / op->w[i]; }
                    /* eta-surface: U*_iN on side 2 (k=i), U*_i0 on side 0 */
                    if (j == N) { deu += Us[2][i] / op->w[j]; dev += Vs[2][i] / op->w[j]; }
                    if (j == 0) { deu -= Us[0][i] / op->w[j]; dev -= Vs[0][i] / op->w[j]; }
                    double J = G->J[q];
                    double U1 = (G->yeta[q] * dxu - G->yxi[q] * deu) / J;
                    double U2 = (-G->xeta[q] * dxu + G->xxi[q] * deu) / J;
                    double V1 = (G->yeta[q] * dxv - G->yxi[q] * dev) / J;
                    double V2 = (-G->xeta[q] * dxv + G->xxi[q] * dev) / J;
                    /* viscous fluxes f^v = h eps (0, U1, V1), g^v = h eps (0, U2, V2) */
                    double he = h[q] * eps[e];
                    Fv2[q] = he * U1; Fv3[q] = he * V1;
                    Gv2[q] = he * U2; Gv3[q] = he * V2;
                    if (parts && parts->grad[0]) {
                        parts->grad[0][q] = U1; parts->grad[1][q] = U2;
                        parts->grad[2][q] = V1; parts->grad[3][q] = V2;
                    }
                }
        }
    }
    if (eps_out)
        for (int64_t e = 0; e < K; ++e) eps_out[e] = eps[e];

    /* every element writes its own nodes only: the loop is element-parallel
     * and bitwise the same at any thread count */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < K; ++e) {
        if (need && !need[e]) continue;
        const int64_t o = e * np;
        double L[3][(ORC_NMAX + 1) * (ORC_NMAX + 1)];
        double Sx[(ORC_NMAX + 1) * (ORC_NMAX + 1)], Sy[(ORC_NMAX + 1) * (ORC_NMAX + 1)];
        double Lv2[(ORC_NMAX + 1) * (ORC_NMAX + 1)], Lv3[(ORC_NMAX + 1) * (ORC_NMAX + 1)];
        /* --- volume: sum_m D~_im F~_(i,m),j + sum_m D~_jm G~_i,(j,m) (Lemma 1,
         * eqs. fluxDiffFormF and Fmij).  Readings: G~ uses the metric
         * averages {y_xi}, {x_xi} in the order of the contravariant flux
         * g~ = -y_xi f + x_xi g (eq. ContravariantFluxes), and L_eta sums over
         * D~_jm (the node's own row, as in eq. VolInt). */
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int p = i * n1 + j;
                double acc[3] = {0, 0, 0};
                double wij[3] = {h[o + p], hu[o + p], hv[o + p]};
                for (int mm = 0; mm <= N; ++mm) {
                    int pm = mm * n1 + j;
                    double wmj[3] = {h[o + pm], hu[o + pm], hv[o + pm]};
                    double Fs[3], Gs[3];
                    orc_volume_flux(g, htol, wij, wmj, Fs, Gs);
                    double ay = 0.5 * (G->yeta[o + p] + G->yeta[o + pm]);
                    double ax = 0.5 * (G->xeta[o + p] + G->xeta[o + pm]);
                    for (int c = 0; c < 3; ++c)
                        acc[c] += op->Dt[i][mm] * (Fs[c] * ay - Gs[c] * ax);
                }
                for (int mm = 0; mm <= N; ++mm) {
                    int pm = i * n1 + mm;
                    double wim[3] = {h[o + pm], hu[o + pm], hv[o + pm]};
                    double Fs[3], Gs[3];
                    orc_volume_flux(g, htol, wij, wim, Fs, Gs);
                    double ay = 0.5 * (G->yxi[o + p] + G->yxi[o + pm]);
                    double ax = 0.5 * (G->xxi[o + p] + G->xxi[o + pm]);
                    for (int c = 0; c < 3; ++c)
                        acc[c] += op->Dt[j][mm] * (-Fs[c] * ay + Gs[c] * ax);
                }
                for (int c = 0; c < 3; ++c) L[c][p] = acc[c];
            }
        /* --- interface: (1/w_i)(delta_iN F~*_Nj - delta_i0 F~*_0j) and the eta
         * analogue (Lemma 1).  F~* is the contravariant numerical flux in the
         * +xi (+eta) direction; it equals J^surf times the numerical flux
         * along the element's outward unit normal on sides xi=+1 / eta=+1 and
         * minus that on xi=-1 / eta=-1.  The element's own trace is the '-'
         * state (the normal points from '-' to '+'). */
        for (int s = 0; s < 4; ++s)
            for (int k = 0; k <= N; ++k) {
                int i, j;
                side_node(N, s, k, &i, &j);
                int p = i * n1 + j;
                int64_t q = o + p, qn = nbr_node(m, e, s, k);
                double snx, sny;
                scaled_normal(G, s, q, &snx, &sny);
                double Js = sqrt(snx * snx + sny * sny);   /* eq. SurfJac */
                double wm[3] = {h[q], hu[q], hv[q]}, wp[3] = {h[qn], hu[qn], hv[qn]};
                if (is_wall(m, e, s)) wall_state(wm, snx / Js, sny / Js, wp);
                double Fn[3];
                orc_surface_flux(P, wm, b[q], wp, b[qn], snx / Js, sny / Js, Fn);
                for (int c = 0; c < 3; ++c) {
                    double Fcontra = (s == 1 || s == 2) ? Js * Fn[c] : -Js * Fn[c];
                    if (s == 1) L[c][p] += Fcontra / op->w[N];   /* + F~*_Nj / w_N */
                    if (s == 3) L[c][p] -= Fcontra / op->w[0];   /* - F~*_0j / w_0 */
                    if (s == 2) L[c][p] += Fcontra / op->w[N];   /* + G~*_iN / w_N */
                    if (s == 0) L[c][p] -= Fcontra / op->w[0];   /* - G~*_i0 / w_0 */
                }
            }
        /* --- source (eq. SourceDisc): the split-form bathymetry derivatives
         * and the interface penalty S^{.,*}.  Readings: the split derivative
         * carries D (the printed 2D doubles it: lake at rest then fails), and
         * b_y follows the chain rule J b_y = -x_eta b_xi + x_xi b_eta. */
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int p = i * n1 + j;
                double Db_xi = 0, Dyb_xi = 0, Dxb_xi = 0, Db_eta = 0, Dyb_eta = 0, Dxb_eta = 0;
                for (int mm = 0; mm <= N; ++mm) {
                    int pa = mm * n1 + j, pb = i * n1 + mm;
                    Db_xi += op->D[i][mm] * b[o + pa];
                    Dyb_xi += op->D[i][mm] * (G->yeta[o + pa] * b[o + pa]);
                    Dxb_xi += op->D[i][mm] * (G->xeta[o + pa] * b[o + pa]);
                    Db_eta += op->D[j][mm] * b[o + pb];
                    Dyb_eta += op->D[j][mm] * (G->yxi[o + pb] * b[o + pb]);
                    Dxb_eta += op->D[j][mm] * (G->xxi[o + pb] * b[o + pb]);
                }
                double bx = G->yeta[o + p] * Db_xi + Dyb_xi - G->yxi[o + p] * Db_eta - Dyb_eta;
                double by = -G->xeta[o + p] * Db_xi - Dxb_xi + G->xxi[o + p] * Db_eta + Dxb_eta;
                Sx[p] = 0.5 * g * (-h[o + p] * bx);
                Sy[p] = 0.5 * g * (-h[o + p] * by);
            }
        /* Interface penalty S^{x,*}, S^{y,*} of eq. SourceDisc for a bottom
         * that jumps across a face (the paper defers its form to its earlier
         * work).  Reading, derived here from Lemma 1.3 and 1.2: at every face
         * node, with the element's own outward unit normal n and the surface
         * Jacobian of eq. SurfJac,
         *     S^{.,*} = -(1/w_0) J^surf {h} [[b]] n,   [[b]] = b_nbr - b_own,
         * entering S as (g/2) S^{.,*}.  At rest (h + b constant, u = 0) the
         * interface flux leaves (1/w_0) J^surf (g/2) {h}[[h]] n in L, which
         * this term cancels ([[h]] = -[[b]]); and it adds -g {h}[[b]]{u.n}
         * J^surf per face node to the entropy rate, cancelling the g[[b]]F_1
         * term of the Tadmor condition of the EC flux.  Zero where b is
         * continuous and at solid walls (the wall's outside bottom is the
         * element's own). */
        for (int s = 0; s < 4; ++s)
            for (int k = 0; k <= N; ++k) {
                int i, j;
                side_node(N, s, k, &i, &j);
                int p = i * n1 + j;
                int64_t q = o + p, qn = nbr_node(m, e, s, k);
                double jb = b[qn] - b[q];
                if (jb == 0.0) continue;
                double snx, sny;
                scaled_normal(G, s, q, &snx, &sny);
                double Js = sqrt(snx * snx + sny * sny);
                double avg_h = 0.5 * (h[q] + h[qn]);
                double sxs = -(Js / op->w[0]) * avg_h * jb * (snx / Js);
                double sys = -(Js / op->w[0]) * avg_h * jb * (sny / Js);
                Sx[p] += 0.5 * g * sxs;
                Sy[p] += 0.5 * g * sys;
            }
        /* --- viscous divergence (Theorem 1, eq. ViscTermsDisc) on the
         * momentum rows: D applied to the contravariant viscous fluxes plus
         * (F~v* - F~v)/w at the faces, F~v* = {F~v}.  Reading: the interface
         * average is the mean of both sides' physical viscous fluxes at the
         * shared node, contracted with this element's metric terms. */
        for (int p = 0; p < np; ++p) { Lv2[p] = 0.0; Lv3[p] = 0.0; }
        if (P->av_on) {
            for (int i = 0; i <= N; ++i)
                for (int j = 0; j <= N; ++j) {
                    int p = i * n1 + j;
                    double a2 = 0, a3 = 0;
                    for (int mm = 0; mm <= N; ++mm) {
                        int64_t qa = o + mm * n1 + j, qb = o + i * n1 + mm;
                        double Ft2 = G->yeta[qa] * Fv2[qa] - G->xeta[qa] * Gv2[qa];
                        double Ft3 = G->yeta[qa] * Fv3[qa] - G->xeta[qa] * Gv3[qa];
                        double Gt2 = -G->yxi[qb] * Fv2[qb] + G->xxi[qb] * Gv2[qb];
                        double Gt3 = -G->yxi[qb] * Fv3[qb] + G->xxi[qb] * Gv3[qb];
                        a2 += op->D[i][mm] * Ft2 + op->D[j][mm] * Gt2;
                        a3 += op->D[i][mm] * Ft3 + op->D[j][mm] * Gt3;
                    }
                    Lv2[p] = a2;
                    Lv3[p] = a3;
                }
            for (int s = 0; s < 4; ++s)
                for (int k = 0; k <= N; ++k) {
                    int i, j;
                    side_node(N, s, k, &i, &j);
                    int p = i * n1 + j;
                    int64_t q = o + p, qn = nbr_node(m, e, s, k);
                    double f2a = 0.5 * (Fv2[q] + Fv2[qn]), f3a = 0.5 * (Fv3[q] + Fv3[qn]);
                    double g2a = 0.5 * (Gv2[q] + Gv2[qn]), g3a = 0.5 * (Gv3[q] + Gv3[qn]);
                    double t2s, t3s, t2, t3;   /* contravariant fluxes (+xi or +eta) */
                    if (s == 1 || s == 3) {
                        t2s = G->yeta[q] * f2a - G->xeta[q] * g2a;
                        t3s = G->yeta[q] * f3a - G->xeta[q] * g3a;
                        t2 = G->yeta[q] * Fv2[q] - G->xeta[q] * Gv2[q];
                        t3 = G->yeta[q] * Fv3[q] - G->xeta[q] * Gv3[q];
                    } else {
                        t2s = -G->yxi[q] * f2a + G->xxi[q] * g2a;
                        t3s = -G->yxi[q] * f3a + G->xxi[q] * g3a;
                        t2 = -G->yxi[q] * Fv2[q] + G->xxi[q] * Gv2[q];
                        t3 = -G->yxi[q] * Fv3[q] + G->xxi[q] * Gv3[q];
                    }
                    double sg = (s == 1 || s == 2) ? 1.0 : -1.0;   /* delta_N - delta_0 */
                    double wgt = (s == 1 || s == 2) ? op->w[N] : op->w[0];
                    Lv2[p] += sg * (t2s - t2) / wgt;
                    Lv3[p] += sg * (t3s - t3) / wgt;
                }
        }
        /* --- R = -(1/J)(L_xi + L_eta - S) + (1/J) L^v */
        for (int p = 0; p < np; ++p) {
            double J = G->J[o + p];
            Rh[o + p] = -(L[0][p]) / J;
            Rhu[o + p] = -(L[1][p] - Sx[p] - Lv2[p]) / J;
            Rhv[o + p] = -(L[2][p] - Sy[p] - Lv3[p]) / J;
            if (parts) {
                for (int c = 0; c < 3; ++c)
                    if (parts->Lvol[c]) parts->Lvol[c][o + p] = L[c][p];
                if (parts->S[0]) { parts->S[0][o + p] = 0.0; parts->S[1][o + p] = Sx[p]; parts->S[2][o + p] = Sy[p]; }
                if (parts->Lv[0]) { parts->Lv[0][o + p] = 0.0; parts->Lv[1][o + p] = Lv2[p]; parts->Lv[2][o + p] = Lv3[p]; }
            }
        }
    }
    free(u); free(v); free(eps); free(needv);
    free(Fv2); free(Fv3); free(Gv2); free(Gv3);
    return ORC_OK;
}

static int check_mesh(const orc_mesh *m)
{
    if (!m || m->N < 1 || m->N > ORC_NMAX || m->K < 1 || !m->x || !m->y || !m->nbr_elem ||
        !m->nbr_side || !m->flip)
        return ORC_EINVAL;
    for (int64_t e = 0; e < m->K; ++e)
        for (int s = 0; s < 4; ++s) {
            int32_t en = m->nbr_elem[e * 4 + s];
            int sn = m->nbr_side[e * 4 + s];
            if (en < 0) continue;                               /* solid wall */
            if (en >= m->K || sn < 0 || sn > 3) return ORC_EINVAL;
        }
    return ORC_OK;
}

int orc_rhs(const orc_params *P, const orc_mesh *m, const double *b, const double *h,
            const double *hu, const double *hv, double *Rh, double *Rhu, double *Rhv,
            double *eps_out, const uint8_t *need, orc_parts *parts)
{
    int st = check_mesh(m);
    if (st) return st;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    int64_t n = m->K * (int64_t)(m->N + 1) * (m->N + 1);
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    st = rhs_impl(P, &op, m, &G, b, h, hu, hv, Rh, Rhu, Rhv, eps_out, need, parts);
    geom_free(&G);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Positivity limiter (eq. PosPres) with the velocity cut-off of 6.1         */
/* ------------------------------------------------------------------------ */
static int limit_impl(const orc_params *P, const orc_ops *op, const orc_mesh *m,
                      const orc_geom *G, double *h, double *hu, double *hv, int64_t *n_limited)
{
    const int N = op->N, n1 = N + 1, np = n1 * n1;
    int negmean = 0;
    int64_t nl = 0;
#pragma omp parallel for schedule(static) reduction(+ : nl) reduction(| : negmean)
    for (int64_t e = 0; e < m->K; ++e) {
        const int64_t o = e * np;
        /* Jacobian-weighted element means and the minimum (eq. AverageTerm) */
        double area = 0, mh = 0, mhu = 0, mhv = 0, hmin = INFINITY;
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int64_t q = o + i * n1 + j;
                double wq = G->J[q] * op->w[i] * op->w[j];
                area += wq;
                mh += h[q] * wq;
                mhu += hu[q] * wq;
                mhv += hv[q] * wq;
                hmin = fmin(hmin, h[q]);
            }
        mh /= area; mhu /= area; mhv /= area;
        /* theta = min(1, hbar/(hbar - m)); reading: theta = 1 whenever m >= 0
         * (no division at m = hbar), theta = 0 and an error flag if hbar < 0. */
        double theta = 1.0;
        if (hmin < 0.0) {
            if (mh < 0.0) { theta = 0.0; negmean = 1; }
            else theta = fmin(1.0, mh / (mh - hmin));
            ++nl;
        }
        for (int p = 0; p < np; ++p) {
            int64_t q = o + p;
            if (theta != 1.0) {
                h[q] = theta * (h[q] - mh) + mh;
                hu[q] = theta * (hu[q] - mhu) + mhu;
                hv[q] = theta * (hv[q] - mhv) + mhv;
            }
            /* velocities (hence discharges) set to zero below h_tol */
            if (h[q] < P->h_tol) { hu[q] = 0.0; hv[q] = 0.0; }
        }
    }
    if (n_limited) *n_limited = nl;
    return negmean ? ORC_ENEGMEAN : ORC_OK;
}

int orc_limit(const orc_params *P, const orc_mesh *m, double *h, double *hu, double *hv,
              int64_t *n_limited)
{
    int st = check_mesh(m);
    if (st) return st;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    int64_t n = m->K * (int64_t)(m->N + 1) * (m->N + 1);
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    st = limit_impl(P, &op, m, &G, h, hu, hv, n_limited);
    geom_free(&G);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Time step: advective CFL, viscous bound, Lemma 2 positivity bounds        */
/* ------------------------------------------------------------------------ */
/* Spectral radius of the 1D BR1 operator at dx = 1, eps = 1, per N (derived
 * numerically for N = 2..8; the paper gives no values), and the real-axis
 * stability limit of LSRK(5,4) rounded down.  Both are checked against their
 * definitions by a CPU test that assembles the operator and the stability
 * function independently. */
static const double ORC_BR1_RADIUS[9] = {0, 0, 25.6, 82.9, 203.0, 425.0, 800.0, 1383.0, 2244.0};
static const double ORC_LSRK_REAL_LIMIT = 4.6;

static void dt_impl(const orc_params *P, const orc_ops *op, const orc_mesh *m,
                    const orc_geom *G, const double *b, const double *h, const double *hu,
                    const double *hv, double out[4])
{
    const int N = op->N, n1 = N + 1, np = n1 * n1;
    const double g = P->g, htol = P->h_tol;
    double dt_cfl = INFINITY, dt_visc = INFINITY, dt_pos = INFINITY;
    (void)b;
    /* minima are exact: the same bounds at any thread count */
#pragma omp parallel for schedule(static) reduction(min : dt_cfl, dt_visc, dt_pos)
    for (int64_t e = 0; e < m->K; ++e) {
        const int64_t o = e * np;
        double gmax = 0.0;
        for (int p = 0; p < np; ++p) {
            int64_t q = o + p;
            double u = velocity(hu[q], h[q], htol), v = velocity(hv[q], h[q], htol);
            double c = sqrt(g * fmax(h[q], 0.0));
            double lx = fabs(G->yeta[q] * u - G->xeta[q] * v) +
                        c * sqrt(G->yeta[q] * G->yeta[q] + G->xeta[q] * G->xeta[q]);
            double le = fabs(-G->yxi[q] * u + G->xxi[q] * v) +
                        c * sqrt(G->yxi[q] * G->yxi[q] + G->xxi[q] * G->xxi[q]);
            if (lx + le > 0.0)
                dt_cfl = fmin(dt_cfl, P->cfl * (2.0 / n1) * G->J[q] / (lx + le));
            double J2 = G->J[q] * G->J[q];
            double gg = (G->yeta[q] * G->yeta[q] + G->xeta[q] * G->xeta[q] +
                         G->yxi[q] * G->yxi[q] + G->xxi[q] * G->xxi[q]) / J2;
            gmax = fmax(gmax, gg);
        }
        if (P->av_on) {
            double eps = viscosity_of_element(P, op, h + o);
            if (eps > 0.0 && N >= 2 && N <= 8)
                dt_visc = fmin(dt_visc, P->cfl_visc * 4.0 * ORC_LSRK_REAL_LIMIT /
                                            (ORC_BR1_RADIUS[N] * eps * gmax));
        }
        /* Lemma 2 (eq. CFLConstraints), at every face node of every side,
         * own trace '-', neighbour '+', own outward unit normal, a = J/J^surf,
         * w_0 = 2/(N(N+1)) (reading: the printed N(N-1)/2 is not the LGL
         * end weight). */
        for (int s = 0; s < 4; ++s)
            for (int k = 0; k <= N; ++k) {
                int i, j;
                side_node(N, s, k, &i, &j);
                int64_t q = o + i * n1 + j, qn = nbr_node(m, e, s, k);
                double snx, sny;
                scaled_normal(G, s, q, &snx, &sny);
                double Js = sqrt(snx * snx + sny * sny);
                double nx = snx / Js, ny = sny / Js;
                double a = G->J[q] / Js;
                double hm = h[q], hp = h[qn];
                double utm = nx * velocity(hu[q], hm, htol) + ny * velocity(hv[q], hm, htol);
                double utp = nx * velocity(hu[qn], hp, htol) + ny * velocity(hv[qn], hp, htol);
                if (is_wall(m, e, s)) utp = -utm;        /* the wall's mirror state */
                double cm = sqrt(g * fmax(hm, 0.0)), cp = sqrt(g * fmax(hp, 0.0));
                double au = 0.5 * (utm + utp), ac = 0.5 * (cm + cp);
                double A = fabs(au + ac) + fabs(au - ac);
                double B = fabs(au + ac) - fabs(au - ac);
                double w0 = op->w[0];
                if (A + 2.0 * au > 0.0) dt_pos = fmin(dt_pos, w0 * a / (A + 2.0 * au));
                double den = ac * B * (utp - utm);
                if (hm > 0.0 && den < 0.0) dt_pos = fmin(dt_pos, fabs(w0 * a * g * hm / den));
            }
    }
    double dt = fmin(dt_cfl, dt_visc);
    if (P->limiter_on) dt = fmin(dt, dt_pos);
    out[0] = dt; out[1] = dt_cfl; out[2] = dt_visc; out[3] = dt_pos;
}

int orc_dt(const orc_params *P, const orc_mesh *m, const double *b, const double *h,
           const double *hu, const double *hv, double out[4])
{
    int st = check_mesh(m);
    if (st) return st;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    int64_t n = m->K * (int64_t)(m->N + 1) * (m->N + 1);
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    dt_impl(P, &op, m, &G, b, h, hu, hv, out);
    geom_free(&G);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Time integration                                                          */
/* ------------------------------------------------------------------------ */
/* Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage RK, the
 * low-storage scheme of the paper's earlier work (section 2.2, before eq. RKSSP). */
static const double LSRK_A[5] = {0.0, -567301805773.0 / 1357537059087.0,
                                 -2404267990393.0 / 2016746695238.0,
                                 -3550918686646.0 / 2091501179385.0,
                                 -1275806237668.0 / 842570457699.0};
static const double LSRK_B[5] = {1432997174477.0 / 9575080441755.0,
                                 5161836677717.0 / 13612068292357.0,
                                 1720146321549.0 / 2090206949498.0,
                                 3134564353537.0 / 4481467310338.0,
                                 2277821191437.0 / 14882151754819.0};

/* Threads of the element loops (OpenMP); the results do not depend on it. */
int orc_set_threads(int n)
{
    if (n < 1) return ORC_EINVAL;
    omp_set_num_threads(n);
    return ORC_OK;
}

int orc_get_threads(void) { return omp_get_max_threads(); }

int orc_lsrk_coefficients(double *a, double *b)
{
    for (int k = 0; k < 5; ++k) { a[k] = LSRK_A[k]; b[k] = LSRK_B[k]; }
    return ORC_OK;
}

/* One step of size dt from W (in place); returns ORC_ENEGMEAN if a limiter
 * call met a negative element mean. */
static int one_step(const orc_params *P, const orc_ops *op, const orc_mesh *m,
                    const orc_geom *G, const double *b, double *h, double *hu, double *hv,
                    double dt, double *work)
{
    const int64_t n = m->K * (int64_t)(op->N + 1) * (op->N + 1);
    double *R0 = work, *R1 = work + n, *R2 = work + 2 * n;
    int status = ORC_OK, st;
    if (P->integrator == 0) {
        double *d0 = work + 3 * n, *d1 = work + 4 * n, *d2 = work + 5 * n;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) { d0[q] = 0; d1[q] = 0; d2[q] = 0; }
        for (int k = 0; k < 5; ++k) {
            st = rhs_impl(P, op, m, G, b, h, hu, hv, R0, R1, R2, NULL, NULL, NULL);
            if (st) return st;
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < n; ++q) {
                d0[q] = LSRK_A[k] * d0[q] + dt * R0[q];
                d1[q] = LSRK_A[k] * d1[q] + dt * R1[q];
                d2[q] = LSRK_A[k] * d2[q] + dt * R2[q];
                h[q] += LSRK_B[k] * d0[q];
                hu[q] += LSRK_B[k] * d1[q];
                hv[q] += LSRK_B[k] * d2[q];
            }
            if (P->limiter_on) {
                st = limit_impl(P, op, m, G, h, hu, hv, NULL);
                if (st) status = st;
            }
        }
    } else {
        /* SSPRK(3,3) in the Shu-Osher form of eq. RKSSP */
        double *W0 = work + 3 * n, *W1 = work + 4 * n, *W2 = work + 5 * n;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n; ++q) { W0[q] = h[q]; W1[q] = hu[q]; W2[q] = hv[q]; }
        static const double alpha[3] = {0.0, 0.75, 1.0 / 3.0};
        static const double beta[3] = {1.0, 0.25, 2.0 / 3.0};
        for (int k = 0; k < 3; ++k) {
            st = rhs_impl(P, op, m, G, b, h, hu, hv, R0, R1, R2, NULL, NULL, NULL);
            if (st) return st;
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < n; ++q) {
                h[q] = alpha[k] * W0[q] + beta[k] * (h[q] + dt * R0[q]);
                hu[q] = alpha[k] * W1[q] + beta[k] * (hu[q] + dt * R1[q]);
                hv[q] = alpha[k] * W2[q] + beta[k] * (hv[q] + dt * R2[q]);
            }
            if (P->limiter_on) {
                st = limit_impl(P, op, m, G, h, hu, hv, NULL);
                if (st) status = st;
            }
        }
    }
    return status;
}

/* nsteps steps; dt_fixed > 0 gives a fixed step, otherwise the step is
 * min(CFL, viscous, positivity) bound evaluated at the start of each step.
 * The step (adaptive or fixed) is redone from W^n with half its size, at
 * most max_dt_retries times, when it proves too large (reading of the
 * section 6 remark that the step is adjusted when a smaller one is found to
 * be needed):
 *   - a negative element mean in the limiter;
 *   - a step larger than ORC_STEP_BOUND_FACTOR times the smaller of the CFL
 *     and viscous bounds of the state it produced (the bounds hold the
 *     factors cfl and cfl_visc), i.e. the wave speeds or the viscosity grew
 *     so much within the step that its CFL number, measured on its result,
 *     is above twice the one an adaptive step is chosen for.
 * Out of retries the step is kept (a negative mean is reported).  t (in/out)
 * accumulates the time. */
#define ORC_STEP_BOUND_FACTOR 2.0
int orc_step(const orc_params *P, const orc_mesh *m, const double *b, double *h, double *hu,
             double *hv, int nsteps, double dt_fixed, double *t, double *last_dt)
{
    int st = check_mesh(m);
    if (st) return st;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    int64_t n = m->K * (int64_t)(m->N + 1) * (m->N + 1);
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    double *work = malloc(sizeof(double) * 9 * n);
    if (!work) { geom_free(&G); return ORC_ENOMEM; }
    double *s0 = work + 6 * n, *s1 = work + 7 * n, *s2 = work + 8 * n;
    int status = ORC_OK;
    const int adaptive = !(dt_fixed > 0.0);
    double next[4];          /* bounds of the current state when already known */
    int have_next = 0;
    for (int it = 0; it < nsteps; ++it) {
        double dt = dt_fixed;
        if (adaptive) {
            if (!have_next) dt_impl(P, &op, m, &G, b, h, hu, hv, next);
            dt = next[0];
            have_next = 0;
        }
        memcpy(s0, h, sizeof(double) * n);
        memcpy(s1, hu, sizeof(double) * n);
        memcpy(s2, hv, sizeof(double) * n);
        int tries = 0;
        for (;;) {
            st = one_step(P, &op, m, &G, b, h, hu, hv, dt, work);
            int redo = st == ORC_ENEGMEAN;
            if (!redo && st == ORC_OK && P->max_dt_retries > 0) {
                /* the bounds of the result: the check, and the next adaptive step */
                dt_impl(P, &op, m, &G, b, h, hu, hv, next);
                have_next = 1;
                redo = dt > ORC_STEP_BOUND_FACTOR * fmin(next[1], next[2]);
            }
            if (redo && tries < P->max_dt_retries) {
                memcpy(h, s0, sizeof(double) * n);
                memcpy(hu, s1, sizeof(double) * n);
                memcpy(hv, s2, sizeof(double) * n);
                dt *= 0.5;
                ++tries;
                have_next = 0;
                continue;
            }
            break;
        }
        if (t) *t += dt;
        if (last_dt) *last_dt = dt;
        if (st) { status = st; if (st != ORC_ENEGMEAN) break; }
    }
    free(work);
    geom_free(&G);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: mass, momentum, total energy (the entropy, eq.               */
/* entropyFunction) and its semi-discrete rate sum J w w q.R                 */
/* ------------------------------------------------------------------------ */
int orc_diagnostics(const orc_params *P, const orc_mesh *m, const double *b, const double *h,
                    const double *hu, const double *hv, double out[8])
{
    int st = check_mesh(m);
    if (st) return st;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    const int N = m->N, n1 = N + 1, np = n1 * n1;
    int64_t n = m->K * (int64_t)np;
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    double *R = malloc(sizeof(double) * 3 * n);
    if (!R) { geom_free(&G); return ORC_ENOMEM; }
    st = rhs_impl(P, &op, m, &G, b, h, hu, hv, R, R + n, R + 2 * n, NULL, NULL, NULL);
    double mass = 0, mx = 0, my = 0, E = 0, dE = 0, hmin = INFINITY, hmax = -INFINITY;
    int64_t ndry = 0;
    for (int64_t e = 0; e < m->K; ++e)
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int64_t q = e * np + i * n1 + j;
                double wq = G.J[q] * op.w[i] * op.w[j];
                double u = velocity(hu[q], h[q], P->h_tol), v = velocity(hv[q], h[q], P->h_tol);
                double ent = 0.5 * h[q] * (u * u + v * v) + 0.5 * P->g * h[q] * h[q] +
                             P->g * h[q] * b[q];
                double q1 = P->g * (h[q] + b[q]) - 0.5 * (u * u + v * v);
                mass += wq * h[q];
                mx += wq * hu[q];
                my += wq * hv[q];
                E += wq * ent;
                dE += wq * (q1 * R[q] + u * R[n + q] + v * R[2 * n + q]);
                hmin = fmin(hmin, h[q]);
                hmax = fmax(hmax, h[q]);
                if (!(h[q] > P->h_tol)) ++ndry;
            }
    out[0] = mass; out[1] = mx; out[2] = my; out[3] = E; out[4] = dE;
    out[5] = hmin; out[6] = hmax; out[7] = (double)ndry;
    free(R);
    geom_free(&G);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint: reverse mode of the inviscid right-hand side and of     */
/* LSRK(5,4) steps, for a gauge-misfit loss in the bathymetry.               */
/*                                                                            */
/* Scope of the adjoint: artificial viscosity off (the viscosity is frozen   */
/* at zero) and a limiter that never acts (all elements wet, so theta = 1    */
/* and no velocity is cut off).  The derivative of |x| is sign(x) with       */
/* sign(0) = 0; velocities below the dry cut-off are constants.              */
/* ------------------------------------------------------------------------ */

/* Forward-mode dual numbers with 8 tangent slots.  The local Jacobians of
 * the two-point volume flux (6 inputs) and of the interface flux (8 inputs:
 * own h, hu, hv, b, neighbour h, hu, hv, b) are obtained by evaluating the
 * flux formulas on duals, so the chain rule is applied mechanically. */
#define ORC_ND 8
typedef struct { double v, d[ORC_ND]; } dn;

static dn dn_c(double v) { dn r; r.v = v; for (int k = 0; k < ORC_ND; ++k) r.d[k] = 0.0; return r; }
static dn dn_var(double v, int k) { dn r = dn_c(v); r.d[k] = 1.0; return r; }
static dn dn_add(dn a, dn b) { dn r; r.v = a.v + b.v; for (int k = 0; k < ORC_ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dn dn_sub(dn a, dn b) { dn r; r.v = a.v - b.v; for (int k = 0; k < ORC_ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dn dn_scl(double s, dn a) { dn r; r.v = s * a.v; for (int k = 0; k < ORC_ND; ++k) r.d[k] = s * a.d[k]; return r; }
static dn dn_mul(dn a, dn b)
{
    dn r; r.v = a.v * b.v;
    for (int k = 0; k < ORC_ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dn dn_div(dn a, dn b)
{
    dn r; r.v = a.v / b.v;
    for (int k = 0; k < ORC_ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
static dn dn_sqrt(dn a)   /* a.v > 0 where the derivative is used */
{
    dn r; r.v = sqrt(a.v);
    for (int k = 0; k < ORC_ND; ++k) r.d[k] = r.v > 0.0 ? 0.5 * a.d[k] / r.v : 0.0;
    return r;
}
static dn dn_abs(dn a)
{
    double s = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
    return dn_scl(s, a);
}

/* velocity with the dry cut-off (constant zero where h <= h_tol) */
static dn dn_velocity(dn hq, dn h, double h_tol)
{
    return (h.v > h_tol) ? dn_div(hq, h) : dn_c(0.0);
}

/* Two-point volume fluxes F#, G# (eq. volumeFluxes) on duals. */
static void volume_flux_dn(double g, double h_tol, const dn *wa, const dn *wb, dn *Fs, dn *Gs)
{
    dn ua = dn_velocity(wa[1], wa[0], h_tol), ub = dn_velocity(wb[1], wb[0], h_tol);
    dn va = dn_velocity(wa[2], wa[0], h_tol), vb = dn_velocity(wb[2], wb[0], h_tol);
    dn avg_h = dn_scl(0.5, dn_add(wa[0], wb[0]));
    dn avg_h2 = dn_scl(0.5, dn_add(dn_mul(wa[0], wa[0]), dn_mul(wb[0], wb[0])));
    dn avg_hu = dn_scl(0.5, dn_add(wa[1], wb[1]));
    dn avg_hv = dn_scl(0.5, dn_add(wa[2], wb[2]));
    dn avg_u = dn_scl(0.5, dn_add(ua, ub));
    dn avg_v = dn_scl(0.5, dn_add(va, vb));
    dn p = dn_sub(dn_scl(g, dn_mul(avg_h, avg_h)), dn_scl(0.5 * g, avg_h2));
    Fs[0] = avg_hu;
    Fs[1] = dn_add(dn_mul(avg_hu, avg_u), p);
    Fs[2] = dn_mul(avg_hu, avg_v);
    Gs[0] = avg_hv;
    Gs[1] = dn_mul(avg_hv, avg_u);
    Gs[2] = dn_add(dn_mul(avg_hv, avg_v), p);
}

/* Interface flux along the unit normal (appendix B) on duals: the same
 * rotated EC flux and, for the ES flux, the dissipation R|Lambda|R^T [[q~]]
 * as a matrix product. */
static void surface_flux_dn(const orc_params *P, const dn *wm, dn bm, const dn *wp, dn bp,
                            double nx, double ny, dn *F)
{
    double g = P->g;
    dn hm = wm[0], hp = wp[0];
    dn um = dn_velocity(wm[1], hm, P->h_tol), vm = dn_velocity(wm[2], hm, P->h_tol);
    dn up = dn_velocity(wp[1], hp, P->h_tol), vp = dn_velocity(wp[2], hp, P->h_tol);
    dn utm = dn_add(dn_scl(nx, um), dn_scl(ny, vm)), vtm = dn_add(dn_scl(-ny, um), dn_scl(nx, vm));
    dn utp = dn_add(dn_scl(nx, up), dn_scl(ny, vp)), vtp = dn_add(dn_scl(-ny, up), dn_scl(nx, vp));
    dn cm = hm.v > 0.0 ? dn_sqrt(dn_scl(g, hm)) : dn_c(0.0);
    dn cp = hp.v > 0.0 ? dn_sqrt(dn_scl(g, hp)) : dn_c(0.0);
    dn ah = dn_scl(0.5, dn_add(hm, hp)), au = dn_scl(0.5, dn_add(utm, utp));
    dn av = dn_scl(0.5, dn_add(vtm, vtp));
    dn ah2 = dn_scl(0.5, dn_add(dn_mul(hm, hm), dn_mul(hp, hp))), ac = dn_scl(0.5, dn_add(cm, cp));
    dn Fr[3];
    Fr[0] = dn_mul(ah, au);
    Fr[1] = dn_add(dn_mul(ah, dn_mul(au, au)), dn_scl(0.5 * g, ah2));
    Fr[2] = dn_mul(ah, dn_mul(au, av));
    if (P->surface_flux == 0) {
        dn qm0 = dn_sub(dn_scl(g, dn_add(hm, bm)),
                        dn_scl(0.5, dn_add(dn_mul(utm, utm), dn_mul(vtm, vtm))));
        dn qp0 = dn_sub(dn_scl(g, dn_add(hp, bp)),
                        dn_scl(0.5, dn_add(dn_mul(utp, utp), dn_mul(vtp, vtp))));
        dn dq[3] = {dn_sub(qp0, qm0), dn_sub(utp, utm), dn_sub(vtp, vtm)};
        dn R[3][3] = {{dn_c(1.0), dn_c(0.0), dn_c(1.0)},
                      {dn_add(au, ac), dn_c(0.0), dn_sub(au, ac)},
                      {av, dn_c(1.0), av}};
        dn Lam[3] = {dn_scl(1.0 / (2.0 * g), dn_abs(dn_add(au, ac))),
                     dn_abs(dn_mul(ah, au)),
                     dn_scl(1.0 / (2.0 * g), dn_abs(dn_sub(au, ac)))};
        dn RTdq[3];
        for (int a = 0; a < 3; ++a) {
            RTdq[a] = dn_c(0.0);
            for (int c = 0; c < 3; ++c) RTdq[a] = dn_add(RTdq[a], dn_mul(R[c][a], dq[c]));
            RTdq[a] = dn_mul(Lam[a], RTdq[a]);
        }
        for (int a = 0; a < 3; ++a) {
            dn dis = dn_c(0.0);
            for (int c = 0; c < 3; ++c) dis = dn_add(dis, dn_mul(R[a][c], RTdq[c]));
            Fr[a] = dn_sub(Fr[a], dn_scl(0.5, dis));
        }
    }
    F[0] = Fr[0];
    F[1] = dn_sub(dn_scl(nx, Fr[1]), dn_scl(ny, Fr[2]));
    F[2] = dn_add(dn_scl(ny, Fr[1]), dn_scl(nx, Fr[2]));
}

/* Adds scale * (dR/dW)^T lam to gw and scale * (dR/db)^T lam to gb, R the
 * inviscid right-hand side of rhs_impl.  Every term of the forward
 * computation is visited in the forward's order and its local partial
 * derivatives are scattered to the nodes it reads (reverse mode). */
static int rhs_vjp_acc(const orc_params *P, const orc_ops *op, const orc_mesh *m,
                       const orc_geom *G, const double *b, const double *h, const double *hu,
                       const double *hv, const double *const lam[3], double scale,
                       double *const gw[3], double *gb)
{
    if (P->av_on) return ORC_EINVAL;
    const int N = op->N, n1 = N + 1, np = n1 * n1;
    const double g = P->g, htol = P->h_tol;
    for (int64_t e = 0; e < m->K; ++e) {
        const int64_t o = e * np;
        /* R = -(1/J)(L - S): dPhi/dL_p = mu_p, dPhi/dS_p = -mu_p for
         * Phi = scale * sum_p lam_p . R_p */
        double mu[3][(ORC_NMAX + 1) * (ORC_NMAX + 1)];
        for (int p = 0; p < np; ++p)
            for (int c = 0; c < 3; ++c) mu[c][p] = -scale * lam[c][o + p] / G->J[o + p];
        /* volume: L[c][p] += D~_im (F#[c] {y_eta} - G#[c] {x_eta}) along xi and
         * D~_jm (-F#[c] {y_xi} + G#[c] {x_xi}) along eta */
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int p = i * n1 + j;
                for (int dir = 0; dir < 2; ++dir)
                    for (int mm = 0; mm <= N; ++mm) {
                        int pm = dir == 0 ? mm * n1 + j : i * n1 + mm;
                        dn wa[3] = {dn_var(h[o + p], 0), dn_var(hu[o + p], 1), dn_var(hv[o + p], 2)};
                        dn wb[3] = {dn_var(h[o + pm], 3), dn_var(hu[o + pm], 4), dn_var(hv[o + pm], 5)};
                        dn Fs[3], Gs[3];
                        volume_flux_dn(g, htol, wa, wb, Fs, Gs);
                        double cF, cG, dcoef;
                        if (dir == 0) {
                            cF = 0.5 * (G->yeta[o + p] + G->yeta[o + pm]);
                            cG = -0.5 * (G->xeta[o + p] + G->xeta[o + pm]);
                            dcoef = op->Dt[i][mm];
                        } else {
                            cF = -0.5 * (G->yxi[o + p] + G->yxi[o + pm]);
                            cG = 0.5 * (G->xxi[o + p] + G->xxi[o + pm]);
                            dcoef = op->Dt[j][mm];
                        }
                        for (int c = 0; c < 3; ++c) {
                            double coef = dcoef * mu[c][p];
                            for (int k = 0; k < 3; ++k) {
                                gw[k][o + p] += coef * (cF * Fs[c].d[k] + cG * Gs[c].d[k]);
                                gw[k][o + pm] += coef * (cF * Fs[c].d[3 + k] + cG * Gs[c].d[3 + k]);
                            }
                        }
                    }
            }
        /* interface: L[c][p] += (+-) J^surf F*_n[c] / w at the face nodes, with
         * the signs of rhs_impl (own trace '-', neighbour '+') */
        for (int s = 0; s < 4; ++s)
            for (int k = 0; k <= N; ++k) {
                int i, j;
                side_node(N, s, k, &i, &j);
                int p = i * n1 + j;
                int64_t q = o + p, qn = nbr_node(m, e, s, k);
                double snx, sny;
                scaled_normal(G, s, q, &snx, &sny);
                double Js = sqrt(snx * snx + sny * sny);
                dn wm[3] = {dn_var(h[q], 0), dn_var(hu[q], 1), dn_var(hv[q], 2)};
                dn wp[3] = {dn_var(h[qn], 4), dn_var(hu[qn], 5), dn_var(hv[qn], 6)};
                dn bm = dn_var(b[q], 3), bp = dn_var(b[qn], 7);
                if (is_wall(m, e, s)) {
                    /* the outside state is the own trace with its normal
                     * discharge reversed, b unchanged: the chain rule runs
                     * through the mirror, and nothing reaches a neighbour */
                    double ux = snx / Js, uy = sny / Js;
                    dn dnrm = dn_add(dn_scl(ux, wm[1]), dn_scl(uy, wm[2]));
                    wp[0] = wm[0];
                    wp[1] = dn_sub(wm[1], dn_scl(2.0 * ux, dnrm));
                    wp[2] = dn_sub(wm[2], dn_scl(2.0 * uy, dnrm));
                    bp = bm;
                }
                dn Fn[3];
                surface_flux_dn(P, wm, bm, wp, bp, snx / Js, sny / Js, Fn);
                double contra = (s == 1 || s == 2) ? Js : -Js;       /* F~* = +-J^surf F*_n */
                double fac = (s == 1 || s == 2) ? contra / op->w[N] : -contra / op->w[0];
                for (int c = 0; c < 3; ++c) {
                    double coef = fac * mu[c][p];
                    for (int kk = 0; kk < 3; ++kk) {
                        gw[kk][q] += coef * Fn[c].d[kk];
                        gw[kk][qn] += coef * Fn[c].d[4 + kk];
                    }
                    gb[q] += coef * Fn[c].d[3];
                    gb[qn] += coef * Fn[c].d[7];
                }
            }
        /* source S = (g/2)(-h b_x, -h b_y) (eq. SourceDisc) with the split
         * derivatives of rhs_impl, reversed term by term */
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                int p = i * n1 + j;
                double Db_xi = 0, Dyb_xi = 0, Dxb_xi = 0, Db_eta = 0, Dyb_eta = 0, Dxb_eta = 0;
                for (int mm = 0; mm <= N; ++mm) {
                    int pa = mm * n1 + j, pb = i * n1 + mm;
                    Db_xi += op->D[i][mm] * b[o + pa];
                    Dyb_xi += op->D[i][mm] * (G->yeta[o + pa] * b[o + pa]);
                    Dxb_xi += op->D[i][mm] * (G->xeta[o + pa] * b[o + pa]);
                    Db_eta += op->D[j][mm] * b[o + pb];
                    Dyb_eta += op->D[j][mm] * (G->yxi[o + pb] * b[o + pb]);
                    Dxb_eta += op->D[j][mm] * (G->xxi[o + pb] * b[o + pb]);
                }
                double bx = G->yeta[o + p] * Db_xi + Dyb_xi - G->yxi[o + p] * Db_eta - Dyb_eta;
                double by = -G->xeta[o + p] * Db_xi - Dxb_xi + G->xxi[o + p] * Db_eta + Dxb_eta;
                double sx_bar = -mu[1][p], sy_bar = -mu[2][p];          /* dPhi/dS */
                gw[0][o + p] += sx_bar * (-0.5 * g * bx) + sy_bar * (-0.5 * g * by);
                double bx_bar = sx_bar * (-0.5 * g * h[o + p]);
                double by_bar = sy_bar * (-0.5 * g * h[o + p]);
                double Db_xi_bar = G->yeta[o + p] * bx_bar - G->xeta[o + p] * by_bar;
                double Dyb_xi_bar = bx_bar, Dxb_xi_bar = -by_bar;
                double Db_eta_bar = -G->yxi[o + p] * bx_bar + G->xxi[o + p] * by_bar;
                double Dyb_eta_bar = -bx_bar, Dxb_eta_bar = by_bar;
                for (int mm = 0; mm <= N; ++mm) {
                    int pa = mm * n1 + j, pb = i * n1 + mm;
                    gb[o + pa] += op->D[i][mm] * (Db_xi_bar + G->yeta[o + pa] * Dyb_xi_bar +
                                                  G->xeta[o + pa] * Dxb_xi_bar);
                    gb[o + pb] += op->D[j][mm] * (Db_eta_bar + G->yxi[o + pb] * Dyb_eta_bar +
                                                  G->xxi[o + pb] * Dxb_eta_bar);
                }
            }
        /* interface penalty of rhs_impl, S += (g/2) c {h} [[b]] with
         * c = -(J^surf/w_0) n per component: linear in [[b]] and in {h}, so
         * its partials are taken where [[b]] = 0 too */
        for (int s = 0; s < 4; ++s)
            for (int k = 0; k <= N; ++k) {
                int i, j;
                side_node(N, s, k, &i, &j);
                int p = i * n1 + j;
                int64_t q = o + p, qn = nbr_node(m, e, s, k);
                double snx, sny;
                scaled_normal(G, s, q, &snx, &sny);
                double Js = sqrt(snx * snx + sny * sny);
                double cx = 0.5 * g * (-(Js / op->w[0]) * (snx / Js));
                double cy = 0.5 * g * (-(Js / op->w[0]) * (sny / Js));
                double avg_h = 0.5 * (h[q] + h[qn]), jb = b[qn] - b[q];
                double sx_bar = -mu[1][p], sy_bar = -mu[2][p];
                double avg_bar = (sx_bar * cx + sy_bar * cy) * jb;
                double jb_bar = (sx_bar * cx + sy_bar * cy) * avg_h;
                gw[0][q] += 0.5 * avg_bar;
                gw[0][qn] += 0.5 * avg_bar;
                gb[qn] += jb_bar;
                gb[q] -= jb_bar;
            }
    }
    return ORC_OK;
}

/* (dR/dW)^T lam and (dR/db)^T lam of the inviscid right-hand side at (W, b). */
int orc_rhs_vjp(const orc_params *P, const orc_mesh *m, const double *b, const double *h,
                const double *hu, const double *hv, const double *lh, const double *lhu,
                const double *lhv, double *gh, double *ghu, double *ghv, double *gb)
{
    int st = check_mesh(m);
    if (st) return st;
    if (P->av_on) return ORC_EINVAL;
    orc_ops op;
    build_ops(m->N, &op);
    orc_geom G;
    int64_t n = m->K * (int64_t)(m->N + 1) * (m->N + 1);
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    memset(gh, 0, sizeof(double) * n);
    memset(ghu, 0, sizeof(double) * n);
    memset(ghv, 0, sizeof(double) * n);
    memset(gb, 0, sizeof(double) * n);
    const double *lam[3] = {lh, lhu, lhv};
    double *gw[3] = {gh, ghu, ghv};
    st = rhs_vjp_acc(P, &op, m, &G, b, h, hu, hv, lam, 1.0, gw, gb);
    geom_free(&G);
    return st;
}

/* Gauge-misfit loss over nsteps fixed steps of size dt from (h0, hu0, hv0),
 * LSRK(5,4) or SSPRK(3,3) as P->integrator selects:
 *     L = 1/2 sum_{n=1..nsteps} sum_g (H_g(t_n) - target[n-1][g])^2 dt,
 * H_g the water surface h + b interpolated at reference point (xi_g, eta_g)
 * of element gelem[g] with the LGL Lagrange basis.  H_out [nsteps][ng]
 * receives H_g(t_n).  With gb != NULL also the gradient: gb = dL/db for the
 * initial state held fixed, and g{h,hu,hv}0 = dL/dW(0) (each may be NULL
 * except gb).  All stage states are kept (no checkpointing): a plain
 * reverse sweep.  Returns ORC_EINVAL if the limiter would act in any stage
 * (the adjoint assumes it inactive) or the setup is out of scope. */
int orc_gauge_adjoint(const orc_params *P, const orc_mesh *m, const double *b,
                      const double *h0, const double *hu0, const double *hv0, int nsteps,
                      double dt, int ng, const int32_t *gelem, const double *gxi,
                      const double *geta, const double *target, double *loss, double *H_out,
                      double *gb, double *gh0, double *ghu0, double *ghv0)
{
    int st = check_mesh(m);
    if (st) return st;
    if (P->av_on || P->integrator < 0 || P->integrator > 1 || nsteps < 1 || ng < 0 || !(dt > 0.0))
        return ORC_EINVAL;
    const int N = m->N, n1 = N + 1, np = n1 * n1;
    /* stages per step: LSRK(5,4) or SSPRK(3,3) (eq. RKSSP) */
    const int ssp = P->integrator == 1, S = ssp ? 3 : 5;
    static const double SSP_ALPHA[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double SSP_BETA[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int gg = 0; gg < ng; ++gg)
        if (gelem[gg] < 0 || gelem[gg] >= m->K) return ORC_EINVAL;
    orc_ops op;
    build_ops(N, &op);
    orc_geom G;
    const int64_t n = m->K * (int64_t)np;
    if (geom_alloc(&G, n)) { geom_free(&G); return ORC_ENOMEM; }
    geometry(&op, m, &G);
    /* gauge weights l_i(xi_g) l_j(eta_g) */
    double *gw = malloc(sizeof(double) * (size_t)(ng > 0 ? ng : 1) * np);
    /* every stage input of every step, plus the final state */
    const int64_t nslot = (int64_t)nsteps * S + 1;
    double *Ws = malloc(sizeof(double) * 3 * n * nslot);
    double *R = malloc(sizeof(double) * 3 * n), *d = malloc(sizeof(double) * 3 * n);
    double *Hg = malloc(sizeof(double) * (size_t)nsteps * (ng > 0 ? ng : 1));
    if (!gw || !Ws || !R || !d || !Hg) {
        free(gw); free(Ws); free(R); free(d); free(Hg); geom_free(&G);
        return ORC_ENOMEM;
    }
    for (int gg = 0; gg < ng; ++gg)
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j)
                gw[gg * np + i * n1 + j] = (double)(lagrange(N, op.xi, i, gxi[gg]) *
                                                    lagrange(N, op.xi, j, geta[gg]));
    memcpy(Ws, h0, sizeof(double) * n);
    memcpy(Ws + n, hu0, sizeof(double) * n);
    memcpy(Ws + 2 * n, hv0, sizeof(double) * n);
    double L = 0.0;
    st = ORC_OK;
    for (int64_t q = 0; q < n; ++q)
        if (!(h0[q] >= P->h_tol)) st = ORC_EINVAL;   /* the initial state must be wet too */
    for (int it = 0; it < nsteps && st == ORC_OK; ++it) {
        memset(d, 0, sizeof(double) * 3 * n);
        for (int k = 0; k < S && st == ORC_OK; ++k) {
            const int64_t s = (int64_t)it * S + k;
            const double *W = Ws + s * 3 * n;
            const double *Wstep = Ws + (int64_t)it * S * 3 * n;   /* W^n */
            double *Wn = Ws + (s + 1) * 3 * n;
            st = rhs_impl(P, &op, m, &G, b, W, W + n, W + 2 * n, R, R + n, R + 2 * n, NULL, NULL,
                          NULL);
            if (st) break;
            if (ssp) {
                for (int64_t q = 0; q < 3 * n; ++q)
                    Wn[q] = SSP_ALPHA[k] * Wstep[q] + SSP_BETA[k] * (W[q] + dt * R[q]);
            } else {
                for (int64_t q = 0; q < 3 * n; ++q) {
                    d[q] = LSRK_A[k] * d[q] + dt * R[q];
                    Wn[q] = W[q] + LSRK_B[k] * d[q];
                }
            }
            if (P->limiter_on) {
                int64_t nl = 0;
                double *hh = Wn, *hhu = Wn + n, *hhv = Wn + 2 * n;
                for (int64_t q = 0; q < n; ++q)
                    if (!(hh[q] >= P->h_tol)) st = ORC_EINVAL;   /* cut-off or limiter would act */
                if (st == ORC_OK) {
                    st = limit_impl(P, &op, m, &G, hh, hhu, hhv, &nl);
                    if (st == ORC_OK && nl > 0) st = ORC_EINVAL;
                }
            }
        }
        if (st) break;
        const double *W = Ws + ((int64_t)it * S + S) * 3 * n;
        for (int gg = 0; gg < ng; ++gg) {
            double H = 0.0;
            for (int p = 0; p < np; ++p) {
                int64_t q = (int64_t)gelem[gg] * np + p;
                H += gw[gg * np + p] * (W[q] + b[q]);
            }
            Hg[(int64_t)it * ng + gg] = H;
            double r = H - target[(int64_t)it * ng + gg];
            L += 0.5 * r * r * dt;
        }
    }
    if (st == ORC_OK) {
        if (loss) *loss = L;
        if (H_out) memcpy(H_out, Hg, sizeof(double) * (size_t)nsteps * ng);
    }
    if (st == ORC_OK && gb) {
        /* reverse sweep: a = dL/dW (running), c = dL/d(register) for LSRK;
         * for SSPRK c holds the stage's cotangent and z collects dL/dW^n
         * from the alpha_k W^n terms */
        double *a = calloc((size_t)(3 * n), sizeof(double));
        double *c = calloc((size_t)(3 * n), sizeof(double));
        double *z = calloc((size_t)(3 * n), sizeof(double));
        if (!a || !c || !z) st = ORC_ENOMEM;
        memset(gb, 0, sizeof(double) * n);
        for (int it = nsteps - 1; it >= 0 && st == ORC_OK; --it) {
            /* the loss reads W(t_{it+1}) = h + b at the gauges */
            for (int gg = 0; gg < ng; ++gg) {
                double r = (Hg[(int64_t)it * ng + gg] - target[(int64_t)it * ng + gg]) * dt;
                for (int p = 0; p < np; ++p) {
                    int64_t q = (int64_t)gelem[gg] * np + p;
                    a[q] += r * gw[gg * np + p];
                    gb[q] += r * gw[gg * np + p];
                }
            }
            const double *lam[3] = {c, c + n, c + 2 * n};
            double *ga[3] = {a, a + n, a + 2 * n};
            if (ssp) {
                /* W_k = alpha_k W^n + beta_k (W_{k-1} + dt R(W_{k-1})):
                 * dL/dW_{k-1} = beta_k (a + dt (dR/dW)^T a), dL/dW^n += alpha_k a */
                memset(z, 0, sizeof(double) * 3 * n);
                for (int k = 2; k >= 0 && st == ORC_OK; --k) {
                    const double *W = Ws + ((int64_t)it * S + k) * 3 * n;
                    for (int64_t q = 0; q < 3 * n; ++q) {
                        z[q] += SSP_ALPHA[k] * a[q];
                        c[q] = SSP_BETA[k] * a[q];
                        a[q] = c[q];
                    }
                    st = rhs_vjp_acc(P, &op, m, &G, b, W, W + n, W + 2 * n, lam, dt, ga, gb);
                }
                for (int64_t q = 0; q < 3 * n; ++q) a[q] += z[q];
                continue;
            }
            /* W_k = W_{k-1} + B_k d_k,  d_k = A_k d_{k-1} + dt R(W_{k-1}),
             * with d_{-1} = 0 at the start of the step */
            memset(c, 0, sizeof(double) * 3 * n);
            for (int k = 4; k >= 0 && st == ORC_OK; --k) {
                const int64_t s = (int64_t)it * 5 + k;
                const double *W = Ws + s * 3 * n;
                for (int64_t q = 0; q < 3 * n; ++q) c[q] += LSRK_B[k] * a[q];
                st = rhs_vjp_acc(P, &op, m, &G, b, W, W + n, W + 2 * n, lam, dt, ga, gb);
                for (int64_t q = 0; q < 3 * n; ++q) c[q] *= LSRK_A[k];
            }
        }
        if (st == ORC_OK) {
            if (gh0) memcpy(gh0, a, sizeof(double) * n);
            if (ghu0) memcpy(ghu0, a + n, sizeof(double) * n);
            if (ghv0) memcpy(ghv0, a + 2 * n, sizeof(double) * n);
        }
        free(a); free(c); free(z);
    }
    free(gw); free(Ws); free(R); free(d); free(Hg);
    geom_free(&G);
    return st;
}
