"""Pins of the oracle's operators (section 2.2, appendix A) against textbook
values, the SBP property and exactness on polynomials."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg


# Textbook LGL nodes and weights (closed forms).
TEXTBOOK = {
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [2, 3, 4])
def test_lgl_textbook(orc, N):
    op = orc.operators(N)
    x, w = TEXTBOOK[N]
    assert np.allclose(op["xi"], x, rtol=0, atol=2e-16)
    assert np.allclose(op["w"], w, rtol=0, atol=4e-16)


@pytest.mark.parametrize("N", range(2, 9))
def test_quadrature_exactness_and_end_weight(orc, N):
    op = orc.operators(N)
    xi, w = op["xi"], op["w"]
    assert abs(w.sum() - 2.0) < 1e-14
    # LGL quadrature is exact to degree 2N-1
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14
    # end weight 2/(N(N+1)) (the printed N(N-1)/2 is not a quadrature weight)
    assert abs(w[0] - 2.0 / (N * (N + 1))) < 1e-16
    assert abs(w[-1] - w[0]) < 1e-16


@pytest.mark.parametrize("N", range(2, 9))
def test_derivative_matrix_exact_on_polynomials(orc, N):
    op = orc.operators(N)
    xi, D = op["xi"], op["D"]
    rng = np.random.default_rng(N)
    for _ in range(5):
        c = rng.standard_normal(N + 1)           # degree-N polynomial
        p = np.polynomial.Polynomial(c)
        assert np.max(np.abs(D @ p(xi) - p.deriv()(xi))) < 1e-12 * (1 + np.abs(c).sum() * N * N)


@pytest.mark.parametrize("N", range(2, 9))
def test_sbp_and_modified_operators(orc, N):
    op = orc.operators(N)
    D, w = op["D"], op["w"]
    M = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(M @ D + (M @ D).T - B)) < 1e-13        # eq. SBP_def
    S = np.zeros_like(D)
    S[0, 0], S[N, N] = 1.0 / w[0], -1.0 / w[N]
    assert np.max(np.abs(D - (-S + op["Dhat"]))) < 1e-12 * N * N  # D = -S + D^
    assert np.max(np.abs(op["Dtilde"] - (2 * D + S))) < 1e-13    # eq. Dmat_modification
    # D~ has a zero diagonal on LGL nodes (the endpoint parts cancel)
    assert np.max(np.abs(np.diag(op["Dtilde"]))) < 1e-12 * N * N


@pytest.mark.parametrize("N", range(2, 9))
def test_vandermonde_inverse(orc, N):
    op = orc.operators(N)
    xi = op["xi"]
    # V_ij = sqrt(j+1/2) L_j(xi_i), evaluated here with numpy's Legendre series
    V = np.stack([np.sqrt(j + 0.5) * npleg.legval(xi, np.eye(N + 1)[j]) for j in range(N + 1)], 1)
    assert np.max(np.abs(op["Vinv"] @ V - np.eye(N + 1))) < 1e-13


def _mode(N, xi, a, bb):
    La = np.sqrt(a + 0.5) * npleg.legval(xi, np.eye(N + 1)[a])
    Lb = np.sqrt(bb + 0.5) * npleg.legval(xi, np.eye(N + 1)[bb])
    return np.outer(La, Lb).reshape(-1)   # node p = i*(N+1)+j


@pytest.mark.parametrize("N", [3, 5, 7])
def test_indicator_modes(orc, N):
    """A pure top mode gives sigma = 0 (full viscosity); degree <= N-2 data
    give zero energy in both shells (no viscosity); a known mix gives the
    ramp value of appendix A."""
    op = orc.operators(N)
    xi = op["xi"]
    smin, smax = -3.0, -1.0
    P = orc.params(N, eps0=0.7, sigma_min=smin, sigma_max=smax, av_on=1)
    h_top = 1.0 + 0.0 * xi[0] + _mode(N, xi, N, 1)
    h_low = 2.0 + 0.3 * _mode(N, xi, N - 2, N - 2) + 0.1 * _mode(N, xi, 1, 0)
    eps = orc.indicator(P, N, np.stack([h_top, h_low]))
    assert eps[0] == pytest.approx(0.7, abs=1e-15)
    assert eps[1] == 0.0
    # mix: Q = 1 + alpha * mode(N,0).  Q = 1 is 2 * Lt_0(xi) Lt_0(eta)
    # (Lt_0 = sqrt(1/2)), so its modal energy is 4 and r1 = a^2/(4 + a^2), r2 = 0
    for alpha in [0.03, 0.1, 0.2]:
        Q = 1.0 + alpha * _mode(N, xi, N, 0)
        r = alpha ** 2 / (4.0 + alpha ** 2)
        s = np.log10(r)
        if s <= smin:
            want = 0.0
        elif s >= smax:
            want = 0.7
        else:
            want = 0.35 * (1 + np.sin(np.pi * (s - 0.5 * (smax + smin)) / (smax - smin)))
        got = orc.indicator(P, N, Q[None, :])[0]
        assert got == pytest.approx(want, rel=1e-12, abs=1e-15)
    # a dry element gets no viscosity
    assert orc.indicator(P, N, np.zeros((1, (N + 1) ** 2)))[0] == 0.0


def test_lsrk_coefficients_fourth_order(orc):
    """The 2N-storage coefficients give a fourth-order method: error ratios on
    the nonlinear ODE y' = -y^2 (exact solution 1/(1+t))."""
    a, b = orc.lsrk_coefficients()

    def run(nsteps, T=1.0):
        dt = T / nsteps
        y = 1.0
        for _ in range(nsteps):
            du = 0.0
            for k in range(5):
                du = a[k] * du + dt * (-y * y)
                y = y + b[k] * du
        return y

    errs = [abs(run(n) - 0.5) for n in (8, 16, 32)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.8, rates


@pytest.mark.parametrize("N", [3, 5, 7])
def test_indicator_second_shell(orc, N):
    """The second energy ratio of appendix A: the energy in the mode shell
    N-1 over the energy of the modes up to N-1 (the top shell N left out of
    the denominator).  Q = 1 + beta mode(N-1, 0) has no top-shell energy
    (r1 = 0) and r2 = beta^2 / (4 + beta^2); with a top-shell part alpha
    mode(N, 0) as well, r1 = alpha^2 / (4 + alpha^2 + beta^2) while r2 keeps
    its value (a denominator over all modes would give beta^2 / (4 + alpha^2
    + beta^2)); the transposed mode(0, N-1) is in the same shell."""
    op = orc.operators(N)
    xi = op["xi"]
    smin, smax = -4.0, 0.0
    P = orc.params(N, eps0=1.0, sigma_min=smin, sigma_max=smax, av_on=1)

    def ramp(r):
        s = np.log10(r)
        return 0.5 * (1 + np.sin(np.pi * (s - 0.5 * (smax + smin)) / (smax - smin)))

    for beta in [0.05, 0.3]:
        r2 = beta ** 2 / (4.0 + beta ** 2)
        for Q in (1.0 + beta * _mode(N, xi, N - 1, 0), 1.0 + beta * _mode(N, xi, 0, N - 1)):
            got = orc.indicator(P, N, Q[None, :])[0]
            assert got == pytest.approx(ramp(r2), rel=1e-10)
        alpha = 0.5 * beta
        Q = 1.0 + alpha * _mode(N, xi, N, 0) + beta * _mode(N, xi, N - 1, 1)
        r1 = alpha ** 2 / (4.0 + alpha ** 2 + beta ** 2)
        assert r2 > r1
        got = orc.indicator(P, N, Q[None, :])[0]
        assert got == pytest.approx(ramp(r2), rel=1e-10)
        assert abs(got - ramp(beta ** 2 / (4.0 + alpha ** 2 + beta ** 2))) > 1e-6
