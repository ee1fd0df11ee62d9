// Host-side operator tables of the nodal DGSEM on Legendre-Gauss-Lobatto
// nodes (section 2.2) and the orthonormal-Legendre Vandermonde inverse used
// by the shock indicator (appendix A).  Computed once per context in long
// double, then rounded to the compute precision and passed to the kernels by
// value (kernel-argument constant buffer).
#pragma once
#include <cmath>
#include <cstring>

namespace esdg {

constexpr int kMaxN = 8;
constexpr int kMaxNF = kMaxN + 1;

struct HostTables {
    int N;
    long double x[kMaxNF], w[kMaxNF];
    long double D[kMaxNF][kMaxNF];     // D_ij = l_j'(x_i)
    long double Vinv[kMaxNF][kMaxNF];  // nodal values -> orthonormal Legendre coefficients
};

// Legendre P_n(t) and P_{n-1}(t) by the three-term recurrence.
inline void legendre_pair(int n, long double t, long double &pn, long double &pnm1)
{
    long double a = 1.0L, b = t;
    if (n == 0) { pn = 1.0L; pnm1 = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        long double c = ((2 * k - 1) * t * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pnm1 = a;
}

inline void build_tables(int N, HostTables &T)
{
    std::memset(&T, 0, sizeof(T));
    T.N = N;
    const int n1 = N + 1;
    // LGL nodes: Newton iteration on (1 - t^2) P_N'(t) written with the
    // identity (1 - t^2) P_N' = N (P_{N-1} - t P_N), started from the
    // Chebyshev-Gauss-Lobatto points; the derivative of the residual
    // t P_N - P_{N-1} is (N+1) P_N.
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i <= N; ++i) {
        long double t = -cosl(pi * i / N);
        if (i > 0 && i < N) {
            for (int it = 0; it < 200; ++it) {
                long double pn, pm;
                legendre_pair(N, t, pn, pm);
                long double step = (t * pn - pm) / ((N + 1) * pn);
                t -= step;
                if (fabsl(step) < 1e-32L) break;
            }
        }
        T.x[i] = t;
    }
    // symmetric placement
    for (int i = 0; i <= N / 2; ++i) {
        long double s = 0.5L * (T.x[N - i] - T.x[i]);
        T.x[i] = -s;
        T.x[N - i] = s;
    }
    if (N % 2 == 0) T.x[N / 2] = 0.0L;
    long double PN[kMaxNF];
    for (int i = 0; i <= N; ++i) {
        long double pn, pm;
        legendre_pair(N, T.x[i], pn, pm);
        PN[i] = pn;
        T.w[i] = 2.0L / ((long double)N * (N + 1) * pn * pn);
    }
    // Differentiation matrix, closed form for LGL nodes:
    // D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)), D_00 = -N(N+1)/4, D_NN = N(N+1)/4.
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) {
            if (i != j) T.D[i][j] = PN[i] / (PN[j] * (T.x[i] - T.x[j]));
            else if (i == 0) T.D[i][j] = -(long double)N * (N + 1) / 4.0L;
            else if (i == N) T.D[i][j] = (long double)N * (N + 1) / 4.0L;
            else T.D[i][j] = 0.0L;
        }
    // Vandermonde V_ij = sqrt(j + 1/2) P_j(x_i), inverted by Gauss-Jordan with
    // partial pivoting.
    long double A[kMaxNF][2 * kMaxNF];
    for (int i = 0; i <= N; ++i) {
        for (int j = 0; j <= N; ++j) {
            long double pj, pm;
            legendre_pair(j, T.x[i], pj, pm);
            A[i][j] = sqrtl(j + 0.5L) * pj;
            A[i][n1 + j] = (i == j) ? 1.0L : 0.0L;
        }
    }
    for (int c = 0; c <= N; ++c) {
        int piv = c;
        for (int r = c + 1; r <= N; ++r)
            if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 2 * n1; ++k) { long double tmp = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = tmp; }
        long double d = A[c][c];
        for (int k = 0; k < 2 * n1; ++k) A[c][k] /= d;
        for (int r = 0; r <= N; ++r) {
            if (r == c) continue;
            long double f = A[r][c];
            if (f != 0.0L)
                for (int k = 0; k < 2 * n1; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) T.Vinv[i][j] = A[i][n1 + j];
}

// Spectral radius of the one-dimensional BR1 diffusion operator at unit
// element width and unit viscosity, per degree (measured numerically), and
// the real-axis stability limit of LSRK(5,4); they size the explicit
// viscous step.
constexpr double kBR1Radius[kMaxN + 1] = {0, 0, 25.6, 82.9, 203.0, 425.0, 800.0, 1383.0, 2244.0};
constexpr double kLsrkRealLimit = 4.6;

// Carpenter-Kennedy five-stage fourth-order 2N-storage Runge-Kutta.
constexpr double kLsrkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                              -2404267990393.0 / 2016746695238.0,
                              -3550918686646.0 / 2091501179385.0,
                              -1275806237668.0 / 842570457699.0};
constexpr double kLsrkB[5] = {1432997174477.0 / 9575080441755.0,
                              5161836677717.0 / 13612068292357.0,
                              1720146321549.0 / 2090206949498.0,
                              3134564353537.0 / 4481467310338.0,
                              2277821191437.0 / 14882151754819.0};

}  // namespace esdg
