"""Pins of the oracle's positivity machinery: the limiter of eq. PosPres
(mean preservation, non-negative nodes, Lemma 3), the Lemma 2 time-step
bound (non-negative element means after an Euler step at that bound, and a
violation well above it), and end-to-end runs: lake at rest over 100 LSRK
steps and a wet/dry dam break (non-negative depth, mass conservation,
decreasing entropy)."""
import numpy as np
import pytest

from paper_1804_02221_amd.inputs import dam_break, lake_bump, make_periodic_mesh, periodic_gaussians

G = 9.81


def means(orc, mesh, *fields):
    op = orc.operators(mesh.N)
    geo = orc.geometry(mesh)
    wq = geo["J"] * np.outer(op["w"], op["w"]).reshape(-1)[None, :]
    area = wq.sum(1)
    return [(wq * f).sum(1) / area for f in fields], wq


def _rough_state(mesh, seed, neg=True):
    rng = np.random.default_rng(seed)
    K, npn = mesh.K, mesh.n_p
    h = rng.uniform(0.0, 1.0, (K, npn)) * rng.uniform(0.2, 2.0, (K, 1))
    if neg:
        h[rng.uniform(size=(K, npn)) < 0.2] *= -0.3
    hu = rng.uniform(-0.5, 0.5, (K, npn))
    hv = rng.uniform(-0.5, 0.5, (K, npn))
    return h, hu, hv


def test_limiter_means_and_positivity(orc):
    mesh = make_periodic_mesh(5, 4, 4, 10.0, 10.0, amp=0.1, rotate_seed=1)
    h, hu, hv = _rough_state(mesh, 3)
    (mh, mhu, mhv), wq = means(orc, mesh, h, hu, hv)
    assert mh.min() > 0
    P = orc.params(5, limiter_on=1, h_tol=-1.0)   # no cut-off: pure scaling
    h2, hu2, hv2, nl, st = orc.limit(P, mesh, h, hu, hv)
    assert st == 0 and nl == np.sum(h.min(1) < 0)
    (mh2, mhu2, mhv2), _ = means(orc, mesh, h2, hu2, hv2)
    assert np.allclose(mh2, mh, rtol=1e-14, atol=0)
    assert np.allclose(mhu2, mhu, rtol=0, atol=1e-15 * np.abs(hu).max() * mesh.n_p)
    assert np.allclose(mhv2, mhv, rtol=0, atol=1e-15 * np.abs(hv).max() * mesh.n_p)
    assert h2.min() >= -1e-15 * mh.max()
    # the minimum of every limited element sits at zero (theta is the largest admissible)
    lim = h.min(1) < 0
    assert np.abs(h2[lim].min(1)).max() < 1e-15 * mh.max()
    # elements with non-negative nodes are untouched
    assert np.array_equal(h2[~lim], h[~lim]) and np.array_equal(hu2[~lim], hu[~lim])


def test_limiter_velocity_cutoff_and_negative_mean(orc):
    mesh = make_periodic_mesh(3, 3, 3, 10.0, 10.0)
    h, hu, hv = _rough_state(mesh, 4, neg=False)
    h[0, :] = 5e-5                      # below h_tol everywhere
    h[1, :] = -1.0                      # negative mean
    P = orc.params(3, limiter_on=1)
    h2, hu2, hv2, nl, st = orc.limit(P, mesh, h, hu, hv)
    assert st == orc.ENEGMEAN
    assert np.all(hu2[0] == 0) and np.all(hv2[0] == 0)
    small = h2 < 1e-4
    assert np.all(hu2[small] == 0) and np.all(hv2[small] == 0)


def test_limiter_entropy_lemma3(orc):
    """Lemma 3 on states at rest over flat bathymetry: the element entropy
    sum J w w (g h^2/2 + g h b) does not grow under the limiter."""
    mesh = make_periodic_mesh(4, 4, 4, 10.0, 10.0, amp=0.1)
    h, _, _ = _rough_state(mesh, 5)
    z = np.zeros_like(h)
    b = np.full_like(h, 0.3)
    P = orc.params(4, limiter_on=1, h_tol=0.0)
    h2, _, _, nl, st = orc.limit(P, mesh, h, z, z)
    assert nl > 0
    _, wq = means(orc, mesh, h)
    E0 = (wq * (0.5 * G * h * h + G * h * b)).sum(1)
    E1 = (wq * (0.5 * G * h2 * h2 + G * h2 * b)).sum(1)
    assert np.all(E1 <= E0 + 1e-14 * np.abs(E0))
    assert np.any(E1 < E0 - 1e-6)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_lemma2_positive_means(orc, N):
    """Lemma 2: with h >= 0 at every node (dry nodes included) one forward
    Euler step of the ES scheme at dt = dt_pos keeps every element mean
    non-negative; four times that step does not."""
    mesh = make_periodic_mesh(N, 5, 5, 10.0, 10.0, amp=0.1, rotate_seed=N)
    rng = np.random.default_rng(N)
    K, npn = mesh.K, mesh.n_p
    h = rng.uniform(0, 1, (K, npn)) ** 3 * (rng.uniform(size=(K, 1)) < 0.6)
    h[rng.uniform(size=(K, npn)) < 0.3] = 0.0
    u = rng.uniform(-3, 3, (K, npn))
    v = rng.uniform(-3, 3, (K, npn))
    hu, hv = h * u, h * v
    b = periodic_gaussians(mesh, [(4.0, 6.0)], [0.5], [2.0])
    P = orc.params(N, limiter_on=1)
    dts = orc.dt(P, mesh, b, h, hu, hv)
    dt_pos = dts[3]
    assert np.isfinite(dt_pos) and dt_pos > 0 and dts[0] == min(dts[1], dts[3])
    Rh = orc.rhs(P, mesh, b, h, hu, hv)[0]
    (m0,), _ = means(orc, mesh, h)
    (m1,), _ = means(orc, mesh, h + dt_pos * Rh)
    assert m1.min() >= -1e-15 * max(1.0, m0.max())


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_lemma2_bound_is_nearly_sharp(orc, N):
    """The case the proof of Lemma 2 is built on: all water of an element
    sits on one face and flows out into dry neighbours.  At dt_pos the mean
    stays positive; at four times dt_pos it is negative."""
    mesh = make_periodic_mesh(N, 5, 5, 10.0, 10.0, amp=0.1)
    n1 = N + 1
    h = np.zeros((mesh.K, mesh.n_p))
    hu, hv = np.zeros_like(h), np.zeros_like(h)
    e = 12
    h[e, N * n1:(N + 1) * n1] = 1.0
    hu[e, N * n1:(N + 1) * n1] = 3.0
    b = np.zeros_like(h)
    P = orc.params(N, limiter_on=1)
    dt_pos = orc.dt(P, mesh, b, h, hu, hv)[3]
    Rh = orc.rhs(P, mesh, b, h, hu, hv)[0]
    (m1,), _ = means(orc, mesh, h + dt_pos * Rh)
    (m4,), _ = means(orc, mesh, h + 4 * dt_pos * Rh)
    assert m1.min() >= 0.0 and m1[e] > 0
    assert m4[e] < 0


@pytest.mark.parametrize("N", [3, 5])
def test_lemma2_second_bound_only_where_it_can_bind(orc, N):
    """Reading of Lemma 2's second bound (eq. CFLConstraints): the proof
    (eq. UpdateConditions) shows that the third term, h^- + dt/(g w_0 a)
    {c} B [[u~]], can only turn negative where {c} B [[u~]] < 0, so the bound
    is enforced there only.  State: an element holding a thin film
    (h = 1e-3, u~ = 0.1) beside a deep, fast neighbour (h = 1, u~ = 3) that
    moves away from it: B [[u~]] > 0 at their shared face, where the printed
    formula taken unconditionally would allow a step about two orders of
    magnitude smaller.  One Euler step at the oracle's dt_pos keeps every
    element mean non-negative, and the film's mean grows."""
    nx = 4
    mesh = make_periodic_mesh(N, nx, nx, 4.0, 4.0)      # Cartesian: unit normals +-x, +-y
    K, npn = mesh.K, mesh.n_p
    h = np.full((K, npn), 0.5)
    u = np.zeros((K, npn))
    e_film, e_deep = 5, 6                                # e = iy*nx + ix: e_deep is the +x neighbour
    h[e_film], u[e_film] = 1e-3, 0.1
    h[e_deep], u[e_deep] = 1.0, 3.0
    hu, hv = h * u, np.zeros_like(h)
    b = np.zeros_like(h)
    P = orc.params(N, limiter_on=1)
    dt_pos = orc.dt(P, mesh, b, h, hu, hv)[3]
    # the printed second bound at the shared face (side xi = +1 of the film):
    # a = J / J^surf = dx / 2 on this mesh, w_0 = 2 / (N (N + 1))
    w0, a = 2.0 / (N * (N + 1)), 0.5
    um, up = 0.1, 3.0
    cbar = 0.5 * (np.sqrt(G * 1e-3) + np.sqrt(G * 1.0))
    ubar = 0.5 * (um + up)
    B = abs(ubar + cbar) - abs(ubar - cbar)
    assert B * (up - um) > 0
    printed = abs(w0 * a * G * 1e-3 / (cbar * B * (up - um)))
    assert dt_pos > 50 * printed
    Rh = orc.rhs(P, mesh, b, h, hu, hv)[0]
    (m0,), _ = means(orc, mesh, h)
    (m1,), _ = means(orc, mesh, h + dt_pos * Rh)
    assert m1.min() >= 0.0
    assert m1[e_film] > m0[e_film]


def test_lake_at_rest_100_steps(orc):
    """End to end: 16x16 N=3 lake at rest (no bump) stays at rest over 100
    LSRK(5,4) steps at CFL 0.5."""
    w = lake_bump(16, 3, bump=False)
    P = orc.params(3, cfl=0.5)
    h, hu, hv, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 100, 0.0)
    assert st == 0 and t > 0
    # accumulated round-off of 500 right-hand sides, relative to H and H sqrt(gH)
    H = 2.0
    assert np.abs(h - w.h).max() < 1e-12 * H
    assert max(np.abs(hu).max(), np.abs(hv).max()) < 1e-12 * H * np.sqrt(G * H)


def test_entropy_conserving_run_drift(orc):
    """Bump on the lake, EC volume and surface fluxes: the total entropy drift
    after 20 steps is a time-integration error (fourth order), far below the
    ES run's dissipation."""
    w = lake_bump(16, 3, seed=1)
    res = {}
    for sf in (0, 1):
        P = orc.params(3, surface_flux=sf)
        E0 = orc.diagnostics(P, w.mesh, w.b, w.h, w.hu, w.hv)[3]
        h, hu, hv, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 20, 0.0)
        E1 = orc.diagnostics(P, w.mesh, w.b, h, hu, hv)[3]
        res[sf] = (E1 - E0) / abs(E0)
    assert res[0] < 0
    assert abs(res[1]) < 1e-3 * abs(res[0])


def test_dam_break_positivity_mass_entropy(orc):
    """Curved wet/dry dam break with AV and the limiter at the combined
    CFL / viscous / Lemma-2 step: non-negative depth after every step and
    mass conserved to round-off with SSPRK(3,3); over flat bathymetry (where
    Lemma 3 applies: the entropy function does not depend on position) the
    LSRK(5,4) run's entropy decreases monotonically, cf. the dry dam break of
    section 6.1."""
    w = dam_break(12, 3, seed=2)
    P = orc.params(3, av_on=1, limiter_on=1, eps0=0.05, integrator=1)
    d0 = orc.diagnostics(P, w.mesh, w.b, w.h, w.hu, w.hv)
    h, hu, hv = w.h, w.hu, w.hv
    for it in range(15):
        h, hu, hv, t, st = orc.step(P, w.mesh, w.b, h, hu, hv, 1, 0.0)
        assert st == 0
        d = orc.diagnostics(P, w.mesh, w.b, h, hu, hv)
        assert d[5] >= -1e-15
        assert abs(d[0] - d0[0]) < 1e-13 * d0[0]
    assert d[3] < d0[3]
    flat = np.zeros_like(w.b)
    P = orc.params(3, av_on=1, limiter_on=1, eps0=0.05, integrator=0)
    h, hu, hv = w.h, w.hu, w.hv
    Es = [orc.diagnostics(P, w.mesh, flat, h, hu, hv)[3]]
    for it in range(20):
        h, hu, hv, t, st = orc.step(P, w.mesh, flat, h, hu, hv, 1, 0.0)
        assert st == 0
        d = orc.diagnostics(P, w.mesh, flat, h, hu, hv)
        assert d[5] >= -1e-15
        Es.append(d[3])
    assert np.all(np.diff(Es) < 0)


def test_limiter_can_raise_entropy_over_varying_bathymetry(orc):
    """Lemma 3 assumes a position-independent entropy function; with
    varying b the term g h b is not, and limiting can move water uphill.
    Documented as a limit of the lemma: a state at rest whose water sits in
    the low part of a sloped element gains entropy when limited."""
    mesh = make_periodic_mesh(3, 3, 3, 10.0, 10.0)
    n1 = 4
    b = np.zeros((mesh.K, mesh.n_p))
    h = np.zeros_like(b)
    for i in range(n1):
        for j in range(n1):
            b[:, i * n1 + j] = 0.5 * i           # slope along xi inside each element
            h[:, i * n1 + j] = 1.0 - 0.6 * i     # deep where b is low, negative at the top
    z = np.zeros_like(h)
    P = orc.params(3, limiter_on=1, h_tol=0.0)
    h2, _, _, nl, st = orc.limit(P, mesh, h, z, z)
    assert nl == mesh.K and st == 0
    E0 = orc.diagnostics(P, mesh, b, h, z, z)[3]
    E1 = orc.diagnostics(P, mesh, b, h2, z, z)[3]
    assert E1 > E0
