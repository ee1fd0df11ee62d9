"""Pins of the oracle's discrete adjoint against the forward oracle and the
mathematics, not against itself:

* the reverse mode of the right-hand side against central differences of the
  (separately pinned) forward right-hand side, per input kind (h, hu, hv, b)
  and for both interface fluxes, so a dropped, mis-signed or transposed term
  in any part fails;
* the gradient of the total mass rate, which vanishes identically by the
  discrete conservation of Lemma 1, is zero;
* the gauge-misfit loss and its gradient through LSRK(5,4) and SSPRK(3,3)
  steps against a loss assembled independently here (one oracle step at a
  time, gauges interpolated with a Lagrange basis built from numpy's
  Legendre roots) and its central differences along random directions in b
  and in W(0);
* all of the above also on basins with solid walls, whose outside state is
  the mirror of the own trace (the reverse mode runs through the mirror).
"""
import numpy as np
import pytest

from paper_1804_02221_amd.inputs import lgl_positions, make_box_mesh, make_periodic_mesh, periodic_gaussians, smooth_sweep


def _dot(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def _state(rot=None, N=3, n=4):
    w = smooth_sweep(n, N, seed=21, rotate_seed=rot)
    return w.mesh, w.b, w.h, w.hu, w.hv


def _box_state(N, wx, wy, rot, seed=0):
    """A wet state in a walled box with a flow through the walls' normals
    (so the mirror matters) on a curved mesh."""
    mesh = make_box_mesh(N, 4, 5, -2.0, -2.0, 4.0, 4.0, amp=0.1, walls_x=wx, walls_y=wy, rotate_seed=rot)
    rng = np.random.default_rng(seed)
    x, y = mesh.x, mesh.y
    c = rng.uniform(0.3, 0.7, 6)
    b = 0.3 * np.exp(-((x - c[0] * 4 + 2) ** 2 + (y - c[1] * 4 + 2) ** 2))
    h = 1.0 + 0.2 * np.sin(1.3 * x + c[2]) * np.cos(0.9 * y + c[3]) - b
    return mesh, b, h, h * (0.3 * np.cos(0.7 * x + c[4]) + 0.2), h * (0.2 * np.sin(0.8 * y + c[5]) - 0.15)


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("N,rot", [(3, None), (4, 7), (2, 3)])
@pytest.mark.parametrize("kind", ["h", "hu", "hv", "b"])
def test_rhs_vjp_against_central_differences(orc, flux, N, rot, kind):
    mesh, b, h, hu, hv = _state(rot, N)
    P = orc.params(N, surface_flux=flux)
    rng = np.random.default_rng(5 + N + 10 * flux)
    lam = [rng.standard_normal(h.shape) for _ in range(3)]
    gh, ghu, ghv, gb = orc.rhs_vjp(P, mesh, b, h, hu, hv, *lam)
    d = rng.standard_normal(h.shape)
    args = dict(h=h, hu=hu, hv=hv, b=b)
    grad = dict(h=gh, hu=ghu, hv=ghv, b=gb)[kind]
    eps = 1e-5 * np.abs(args[kind]).max()

    def R(sign):
        a = dict(args)
        a[kind] = args[kind] + sign * eps * d
        return orc.rhs(P, mesh, a["b"], a["h"], a["hu"], a["hv"])[:3]

    fd = (_dot(lam, R(1)) - _dot(lam, R(-1))) / (2 * eps)
    ad = float(np.sum(grad * d))
    assert abs(fd - ad) <= 2e-7 * abs(ad) + 1e-9 * np.abs(grad).max() * np.abs(d).sum() / d.size, (fd, ad)


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("N,wx,wy,rot", [(3, True, True, None), (4, True, False, 7), (2, False, True, 3)])
@pytest.mark.parametrize("kind", ["h", "hu", "hv", "b"])
def test_rhs_vjp_with_walls_against_central_differences(orc, flux, N, wx, wy, rot, kind):
    mesh, b, h, hu, hv = _box_state(N, wx, wy, rot, seed=N)
    assert (mesh.nbr_elem < 0).any()
    P = orc.params(N, surface_flux=flux)
    rng = np.random.default_rng(50 + N + 10 * flux)
    lam = [rng.standard_normal(h.shape) for _ in range(3)]
    gh, ghu, ghv, gb = orc.rhs_vjp(P, mesh, b, h, hu, hv, *lam)
    d = rng.standard_normal(h.shape)
    args = dict(h=h, hu=hu, hv=hv, b=b)
    grad = dict(h=gh, hu=ghu, hv=ghv, b=gb)[kind]
    eps = 1e-5 * np.abs(args[kind]).max()

    def R(sign):
        a = dict(args)
        a[kind] = args[kind] + sign * eps * d
        return orc.rhs(P, mesh, a["b"], a["h"], a["hu"], a["hv"])[:3]

    fd = (_dot(lam, R(1)) - _dot(lam, R(-1))) / (2 * eps)
    ad = float(np.sum(grad * d))
    assert abs(fd - ad) <= 2e-7 * abs(ad) + 1e-9 * np.abs(grad).max() * np.abs(d).sum() / d.size, (fd, ad)


def test_rhs_vjp_at_walls_only_through_the_mirror(orc):
    """Cotangents placed on the wall face nodes only: the VJP there equals
    central differences of R restricted to those nodes' own traces, and a
    wall face node's gradient does not leak to the far side of the box (the
    periodic image it would have had without the wall)."""
    N = 3
    mesh, b, h, hu, hv = _box_state(N, True, False, None, seed=9)
    P = orc.params(N)
    n1 = N + 1
    walls = np.argwhere(mesh.nbr_elem < 0)
    lam = [np.zeros_like(h) for _ in range(3)]
    rng = np.random.default_rng(3)
    for e, s in walls:
        for k in range(n1):
            i, j = {0: (k, 0), 1: (N, k), 2: (k, N), 3: (0, k)}[int(s)]
            for c in range(3):
                lam[c][e, i * n1 + j] = rng.standard_normal()
    g = orc.rhs_vjp(P, mesh, b, h, hu, hv, *lam)
    # the two inner columns of the 4-column box (no wall side) receive nothing
    cx = mesh.x.mean(axis=1)
    far = np.abs(cx) < 1.0
    assert far.any()
    for a in g:
        assert np.abs(a[far]).max() == 0.0
    d = rng.standard_normal(h.shape)
    eps = 1e-6

    def R(sign):
        return orc.rhs(P, mesh, b, h, hu + sign * eps * d, hv)[:3]

    fd = (_dot(lam, R(1)) - _dot(lam, R(-1))) / (2 * eps)
    ad = float(np.sum(g[1] * d))
    assert abs(fd - ad) <= 1e-7 * abs(ad), (fd, ad)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("rot", [None, 13])
def test_total_mass_rate_has_zero_gradient(orc, rot, walls):
    """sum J w_i w_j R_h = 0 for every state (Lemma 1, conservation; no mass
    crosses a wall), so its gradient with respect to W and b vanishes."""
    mesh, b, h, hu, hv = _box_state(3, True, True, rot) if walls else _state(rot, 3)
    P = orc.params(3)
    op = orc.operators(3)
    J = orc.geometry(mesh)["J"]
    wq = J * np.outer(op["w"], op["w"]).reshape(-1)[None, :]
    z = np.zeros_like(h)
    g = orc.rhs_vjp(P, mesh, b, h, hu, hv, wq, z, z)
    rng = np.random.default_rng(0)
    ref = orc.rhs_vjp(P, mesh, b, h, hu, hv, wq * rng.uniform(0.5, 1.5, wq.shape), z, z)
    for a, r in zip(g, ref):
        assert np.abs(a).max() <= 1e-12 * np.abs(r).max() + 1e-300


def test_rhs_vjp_rejects_viscosity(orc):
    mesh, b, h, hu, hv = _state(None, 3)
    P = orc.params(3, av_on=1, eps0=0.05)
    with pytest.raises(RuntimeError):
        orc.rhs_vjp(P, mesh, b, h, hu, hv, h, h, h)


# ---------------------------------------------------------------------------
# Loss through time steps
# ---------------------------------------------------------------------------
def _lagrange_weights(N, xi, eta):
    x = lgl_positions(N)

    def basis(t):
        out = np.ones(N + 1)
        for j in range(N + 1):
            for m in range(N + 1):
                if m != j:
                    out[j] *= (t - x[m]) / (x[j] - x[m])
        return out

    return np.outer(basis(xi), basis(eta)).reshape(-1)


def _small_case(N=3, n=4, steps=6, ng=5, seed=3):
    mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1, rotate_seed=seed)
    rng = np.random.default_rng(seed)
    b = periodic_gaussians(mesh, [tuple(rng.uniform(0, 10, 2)) for _ in range(3)],
                           rng.uniform(0.1, 0.3, 3), rng.uniform(1.5, 3.0, 3))
    H0 = 1.0 + periodic_gaussians(mesh, [tuple(rng.uniform(2, 8, 2))], [0.05], [2.0])
    db = periodic_gaussians(mesh, [tuple(rng.uniform(0, 10, 2))], [0.02], [2.0])
    gelem = rng.integers(0, mesh.x.shape[0], ng).astype(np.int32)
    gxi, geta = rng.uniform(-1, 1, ng), rng.uniform(-1, 1, ng)
    return mesh, b, H0, db, gelem, gxi, geta, steps


def _small_box_case(N=3, steps=6, ng=5, seed=3):
    """_small_case in the walled box [-2, 2]^2 (walls on both axes), fields
    evaluated at the nodal coordinates."""
    mesh = make_box_mesh(N, 4, 4, -2.0, -2.0, 4.0, 4.0, amp=0.1, rotate_seed=seed)
    rng = np.random.default_rng(seed)
    x, y = mesh.x, mesh.y

    def bumps(k, lo, hi, amps, width):
        c = rng.uniform(lo, hi, (k, 2))
        return sum(a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / width ** 2) for (cx, cy), a in zip(c, amps))

    b = bumps(3, -1.5, 1.5, rng.uniform(0.1, 0.3, 3), 0.8)
    H0 = 1.0 + bumps(1, -1.0, 1.0, [0.05], 0.8)
    db = bumps(1, -1.5, 1.5, [0.02], 0.8)
    gelem = rng.integers(0, mesh.x.shape[0], ng).astype(np.int32)
    gxi, geta = rng.uniform(-1, 1, ng), rng.uniform(-1, 1, ng)
    return mesh, b, H0, db, gelem, gxi, geta, steps


def _loss_by_steps(orc, P, mesh, b, h0, hu0, hv0, steps, dt, gelem, gxi, geta, target):
    N = mesh.N
    Wg = [_lagrange_weights(N, a, c) for a, c in zip(gxi, geta)]
    h, hu, hv = h0, hu0, hv0
    L, Hs = 0.0, []
    for n in range(steps):
        h, hu, hv, _, st = orc.step(P, mesh, b, h, hu, hv, 1, dt_fixed=dt)
        assert st == 0
        H = np.array([np.dot(wg, (h + b)[e]) for wg, e in zip(Wg, gelem)])
        Hs.append(H)
        L += 0.5 * dt * np.sum((H - target[n]) ** 2)
    return L, np.array(Hs)


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("flux", [0, 1])
def test_gauge_loss_and_gradient(orc, flux, walls, integrator):
    mesh, b, H0, db, gelem, gxi, geta, steps = _small_box_case() if walls else _small_case()
    N = mesh.N
    P = orc.params(N, surface_flux=flux, limiter_on=1, integrator=integrator)
    z = np.zeros_like(b)
    dt = 0.5 * orc.dt(P, mesh, b, H0 - b, z, z)[1]
    # target: the same run over the perturbed bed b + db, plus gauge noise
    # (keeps the misfits well above round-off on so short a run)
    tgt = orc.gauge_adjoint(P, mesh, b + db, H0 - b - db, z, z, steps, dt, gelem, gxi, geta,
                            np.zeros((steps, len(gelem))), gradient=False)["H"]
    tgt = tgt + 1e-3 * np.random.default_rng(2).standard_normal(tgt.shape)
    r = orc.gauge_adjoint(P, mesh, b, H0 - b, z, z, steps, dt, gelem, gxi, geta, tgt)
    L2, H2 = _loss_by_steps(orc, P, mesh, b, H0 - b, z, z, steps, dt, gelem, gxi, geta, tgt)
    assert np.abs(r["H"] - H2).max() <= 1e-13 * np.abs(H2).max()
    assert abs(r["loss"] - L2) <= 1e-12 * L2
    assert L2 > 0
    rng = np.random.default_rng(1)
    # directions in b (initial state held fixed) and in each component of W(0)
    for which in ("b", "h0", "hu0", "hv0"):
        d = rng.standard_normal(b.shape)
        eps = 1e-6

        def L(s):
            bb, hh, uu, vv = b, H0 - b, z, z
            if which == "b":
                bb = b + s * eps * d
            elif which == "h0":
                hh = hh + s * eps * d
            elif which == "hu0":
                uu = uu + s * eps * d
            else:
                vv = vv + s * eps * d
            return _loss_by_steps(orc, P, mesh, bb, hh, uu, vv, steps, dt, gelem, gxi, geta, tgt)[0]

        fd = (L(1) - L(-1)) / (2 * eps)
        g = dict(b=r["gb"], h0=r["gh0"], hu0=r["ghu0"], hv0=r["ghv0"])[which]
        ad = float(np.sum(g * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-8 * L2, (which, fd, ad)


def test_gauge_adjoint_refuses_an_active_limiter(orc):
    """A dry node (the velocity cut-off or the limiter would act) is outside
    the adjoint's scope."""
    mesh, b, H0, db, gelem, gxi, geta, steps = _small_case(steps=2)
    P = orc.params(mesh.N, limiter_on=1)
    h0 = H0 - b
    h0[0, 0] = 0.0
    z = np.zeros_like(b)
    with pytest.raises(RuntimeError):
        orc.gauge_adjoint(P, mesh, b, h0, z, z, 2, 1e-3, gelem, gxi, geta, np.zeros((2, len(gelem))))
