"""GPU parity of the discrete adjoint (through the C ABI) against the oracle
adjoint, element by element, plus properties that hold at any size: central
differences of the GPU's own loss along random directions, independence of
the checkpoint interval, and the torch.autograd wrappers.

Tolerances (FP64): the reverse mode of R to 1e-12 of the largest oracle
value per field (the forward bar); the gradient through time steps to 1e-10
of the largest oracle value per field (a reverse sweep over tens of stages,
each a sum of the same cancelling terms as R).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02221_amd.inputs import (bathymetry_gradient, make_box_mesh, make_periodic_mesh, periodic_gaussians,
                                         smooth_sweep)

TOL_VJP = 1e-12
TOL_GRAD = 1e-10
# Richardson-extrapolated central differences (steps 1e-4 and 5e-5) of the
# full-size loss along continuous random directions (bathymetries stay
# continuous): the loss is smooth along them and the extrapolation is
# accurate to ~1e-9 relative.  (Along directions that differ between
# coincident nodes, b jumps across faces and the velocities of the resting
# water cross zero at the |.| kinks of the dissipation: differences then
# carry an O(eps) error.)
FD_TOL = 1e-6


@pytest.fixture(scope="module")
def esdg():
    from paper_1804_02221_amd import esdg as m
    m.lib()
    return m


def make_solver(esdg, mesh, b, h, hu, hv, N, **kw):
    s = esdg.Solver(0, 64)
    s.upload_mesh(mesh)
    P = esdg.default_params(N)
    for k, v in kw.items():
        setattr(P, k, v)
    s.set_params(P)
    s.set_bathymetry(b)
    s.set_state(h, hu, hv)
    return s, P


def oparams(orc, P):
    return orc.params(3, **P.as_dict())


def check(got, want, tol, what):
    for c, (g_, w_) in enumerate(zip(got, want)):
        S = np.abs(w_).max()
        err = np.abs(g_ - w_).max()
        print(f"{what} field {c}: err {err:.3e} scale {S:.3e}", flush=True)
        assert err <= tol * S, f"{what} field {c}: err {err:.3e} > {tol:.0e} * {S:.3e}"


@pytest.mark.parametrize("N,n,ec,rot", [(2, 5, 0, 2), (3, 5, 0, None), (4, 4, 1, 4), (5, 5, 0, 5),
                                        (6, 3, 1, None), (7, 4, 0, 7), (8, 3, 0, 8)])
def test_rhs_vjp_parity(esdg, orc, N, n, ec, rot):
    w = smooth_sweep(n, N, seed=40 + N, rotate_seed=rot)
    s, P = make_solver(esdg, w.mesh, w.b, w.h, w.hu, w.hv, N, surface_flux=ec, limiter_on=1)
    rng = np.random.default_rng(N)
    lam = [rng.standard_normal(w.h.shape) for _ in range(3)]
    print(f"rhs_vjp N={N} K={w.h.shape[0]} ec={ec} rot={rot}", flush=True)
    got = s.rhs_vjp(*lam)
    want = orc.rhs_vjp(oparams(orc, P), w.mesh, w.b, w.h, w.hu, w.hv, *lam)
    check(got, want, TOL_VJP, f"N={N}")
    s.close()


@pytest.mark.parametrize("N,rot,ec", [(3, 3, 0), (6, None, 1), (8, 8, 0)])
def test_rhs_vjp_parity_jumping_bottom(esdg, orc, N, rot, ec):
    """A bottom that jumps at every face: the reverse mode of the interface
    bathymetry penalty (eq. SourceDisc) on both sides of each face."""
    w = smooth_sweep(4, N, seed=90 + N, rotate_seed=rot)
    b = w.b + 0.15 * np.random.default_rng(N).uniform(size=(w.mesh.K, 1))
    s, P = make_solver(esdg, w.mesh, b, w.h, w.hu, w.hv, N, surface_flux=ec, limiter_on=1)
    rng = np.random.default_rng(200 + N)
    lam = [rng.standard_normal(w.h.shape) for _ in range(3)]
    got = s.rhs_vjp(*lam)
    want = orc.rhs_vjp(oparams(orc, P), w.mesh, b, w.h, w.hu, w.hv, *lam)
    check(got, want, TOL_VJP, f"jumping bottom N={N}")
    s.close()


def box_state(N, nx, ny, wx, wy, rot, seed):
    """A wet state in a walled box with flow through the walls' normals."""
    mesh = make_box_mesh(N, nx, ny, -2.0, -2.0, 4.0, 4.0, amp=0.1, walls_x=wx, walls_y=wy, rotate_seed=rot)
    rng = np.random.default_rng(seed)
    x, y = mesh.x, mesh.y
    c = rng.uniform(0.3, 0.7, 6)
    b = 0.3 * np.exp(-((x - c[0] * 4 + 2) ** 2 + (y - c[1] * 4 + 2) ** 2))
    h = 1.0 + 0.2 * np.sin(1.3 * x + c[2]) * np.cos(0.9 * y + c[3]) - b
    return mesh, b, h, h * (0.3 * np.cos(0.7 * x + c[4]) + 0.2), h * (0.2 * np.sin(0.8 * y + c[5]) - 0.15)


@pytest.mark.parametrize("N,wx,wy,ec,rot", [(2, 1, 1, 0, 2), (3, 1, 0, 0, None), (4, 0, 1, 1, 4),
                                            (5, 1, 1, 0, 5), (7, 1, 1, 1, 7), (8, 1, 0, 0, 8)])
def test_rhs_vjp_parity_with_walls(esdg, orc, N, wx, wy, ec, rot):
    mesh, b, h, hu, hv = box_state(N, 5, 4, bool(wx), bool(wy), rot, N)
    s, P = make_solver(esdg, mesh, b, h, hu, hv, N, surface_flux=ec, limiter_on=1)
    rng = np.random.default_rng(100 + N)
    lam = [rng.standard_normal(h.shape) for _ in range(3)]
    print(f"rhs_vjp walls N={N} x={wx} y={wy} ec={ec} rot={rot}", flush=True)
    got = s.rhs_vjp(*lam)
    want = orc.rhs_vjp(oparams(orc, P), mesh, b, h, hu, hv, *lam)
    check(got, want, TOL_VJP, f"walls N={N}")
    s.close()


def test_rhs_vjp_device_arrays(esdg, orc):
    import torch
    w = smooth_sweep(4, 3, seed=7)
    s, P = make_solver(esdg, w.mesh, w.b, w.h, w.hu, w.hv, 3)
    rng = np.random.default_rng(1)
    lam = [rng.standard_normal(w.h.shape) for _ in range(3)]
    host = s.rhs_vjp(*lam)
    dev = s.rhs_vjp(*[torch.tensor(x, device="cuda:0") for x in lam])
    for a, b in zip(host, dev):
        assert np.array_equal(a, b.cpu().numpy().reshape(a.shape))
    s.close()


def small_case(N=3, n=5, steps=13, ng=7, seed=3, rot=3):
    mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1, rotate_seed=rot)
    rng = np.random.default_rng(seed)
    b = periodic_gaussians(mesh, [tuple(rng.uniform(0, 10, 2)) for _ in range(3)],
                           rng.uniform(0.1, 0.3, 3), rng.uniform(1.5, 3.0, 3))
    H0 = 1.0 + periodic_gaussians(mesh, [tuple(rng.uniform(2, 8, 2))], [0.05], [2.0])
    db = periodic_gaussians(mesh, [tuple(rng.uniform(0, 10, 2))], [0.05], [2.0])
    gelem = rng.integers(0, mesh.x.shape[0], ng).astype(np.int32)
    gelem[1] = gelem[0]   # two gauges in one element
    gxi, geta = rng.uniform(-1, 1, ng), rng.uniform(-1, 1, ng)
    return mesh, b, H0, db, gelem, gxi, geta, steps


@pytest.mark.parametrize("N,ec,every,integ", [(3, 0, 4, 0), (5, 1, 5, 0), (7, 0, 13, 0), (3, 1, 4, 1),
                                               (5, 0, 13, 1), (8, 1, 5, 1)])
def test_gauge_gradient_parity(esdg, orc, N, ec, every, integ):
    """integ 0: LSRK(5,4), 1: SSPRK(3,3)."""
    mesh, b, H0, db, gelem, gxi, geta, steps = small_case(N=N)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, N, surface_flux=ec, limiter_on=1, integrator=integ)
    op = oparams(orc, P)
    dt = 0.5 * orc.dt(op, mesh, b, H0 - b, z, z)[1]
    # target from the oracle's run over b + db (no oracle input from the GPU)
    # plus gauge noise: on so short a run the misfits H - target are small
    # enough that the rounding of H (1e-16 of H) would set their relative error
    tgt = orc.gauge_adjoint(op, mesh, b + db, H0 - b - db, z, z, steps, dt, gelem, gxi, geta,
                            np.zeros((steps, len(gelem))), gradient=False)["H"]
    tgt = tgt + 1e-3 * np.random.default_rng(N).standard_normal(tgt.shape)
    ref = orc.gauge_adjoint(op, mesh, b, H0 - b, z, z, steps, dt, gelem, gxi, geta, tgt)
    print(f"gauge gradient N={N} ec={ec} every={every} steps={steps} integrator={integ}", flush=True)
    s.set_gauges(gelem, gxi, geta)
    loss, H = s.adjoint_forward(steps, dt, every, tgt, want_H=True)
    assert np.abs(H - ref["H"]).max() <= 1e-13 * np.abs(ref["H"]).max()
    assert abs(loss - ref["loss"]) <= 1e-9 * ref["loss"]
    gb, gh0, ghu0, ghv0 = s.adjoint_backward()
    check([gb, gh0, ghu0, ghv0], [ref["gb"], ref["gh0"], ref["ghu0"], ref["ghv0"]], TOL_GRAD,
          f"grad N={N}")
    # the forward left the final state as esdg_step would; the backward leaves it alone
    h1 = s.get_state()[0]
    ref1 = orc.step(op, mesh, b, H0 - b, z, z, steps, dt_fixed=dt)[0]
    assert np.abs(h1 - ref1).max() <= 1e-13 * np.abs(ref1).max()
    s.close()


@pytest.mark.parametrize("N,ec,every,integ", [(3, 0, 4, 0), (7, 1, 5, 0), (5, 0, 4, 1)])
def test_gauge_gradient_parity_with_walls(esdg, orc, N, ec, every, integ):
    """A closed basin (walls on both axes): waves from the initial surface
    bump reflect off the walls within the run."""
    mesh = make_box_mesh(N, 5, 5, -2.0, -2.0, 4.0, 4.0, amp=0.1, rotate_seed=N)
    rng = np.random.default_rng(N)
    x, y = mesh.x, mesh.y
    b = 0.25 * np.exp(-((x - 0.6) ** 2 + (y + 0.4) ** 2) / 0.5) + 0.05 * x
    H0 = 1.0 + 0.05 * np.exp(-((x + 1.2) ** 2 + (y - 1.0) ** 2) / 0.3)
    db = 0.03 * np.exp(-((x + 0.3) ** 2 + (y + 1.1) ** 2) / 0.4)
    ng, steps = 6, 30
    gelem = rng.integers(0, mesh.K, ng).astype(np.int32)
    gxi, geta = rng.uniform(-1, 1, ng), rng.uniform(-1, 1, ng)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, N, surface_flux=ec, limiter_on=1, integrator=integ)
    op = oparams(orc, P)
    dt = 0.8 * orc.dt(op, mesh, b, H0 - b, z, z)[1]
    tgt = orc.gauge_adjoint(op, mesh, b + db, H0 - b - db, z, z, steps, dt, gelem, gxi, geta,
                            np.zeros((steps, ng)), gradient=False)["H"]
    tgt = tgt + 1e-3 * rng.standard_normal(tgt.shape)
    ref = orc.gauge_adjoint(op, mesh, b, H0 - b, z, z, steps, dt, gelem, gxi, geta, tgt)
    print(f"gauge gradient with walls N={N} ec={ec} every={every} steps={steps}", flush=True)
    s.set_gauges(gelem, gxi, geta)
    loss, H = s.adjoint_forward(steps, dt, every, tgt, want_H=True)
    assert np.abs(H - ref["H"]).max() <= 1e-13 * np.abs(ref["H"]).max()
    assert abs(loss - ref["loss"]) <= 1e-9 * ref["loss"]
    gb, gh0, ghu0, ghv0 = s.adjoint_backward()
    check([gb, gh0, ghu0, ghv0], [ref["gb"], ref["gh0"], ref["ghu0"], ref["ghv0"]], TOL_GRAD,
          f"walls grad N={N}")
    s.close()


@pytest.mark.parametrize("integ", [0, 1])
def test_checkpoint_interval_is_invisible(esdg, integ):
    mesh, b, H0, db, gelem, gxi, geta, steps = small_case(N=4, steps=11)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, 4, limiter_on=1, integrator=integ)
    s.set_gauges(gelem, gxi, geta)
    dt = 0.5 * s.compute_dt()[1]
    tgt = np.full((steps, len(gelem)), 1.01)
    out = []
    for every in (1, 3, 11, 50):
        s.set_state(H0 - b, z, z)
        L = s.adjoint_forward(steps, dt, every, tgt)
        out.append((L, s.adjoint_backward()))
    for L, g in out[1:]:
        assert L == out[0][0]
        for a, c in zip(g, out[0][1]):
            assert np.array_equal(a, c)
    s.close()


def test_adjoint_argument_errors(esdg):
    mesh, b, H0, db, gelem, gxi, geta, steps = small_case(N=3, steps=2)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, 3, limiter_on=1)
    with pytest.raises((ValueError, esdg.EsdgError)):
        s.adjoint_forward(2, 1e-3, 1, np.zeros(2))          # no gauges yet
    with pytest.raises(esdg.EsdgError):
        s.set_gauges([0], [1.5], [0.0])                      # outside the element
    s.set_gauges(gelem, gxi, geta)
    with pytest.raises(esdg.EsdgError):
        s.adjoint_backward()                                 # no forward sweep
    with pytest.raises(esdg.EsdgError):
        s.adjoint_forward(2, -1.0, 1, np.zeros((2, len(gelem))))
    s.adjoint_forward(2, 1e-3, 1, np.zeros((2, len(gelem))))
    s.set_bathymetry(b)                                      # invalidates the sweep
    with pytest.raises(esdg.EsdgError):
        s.adjoint_backward()
    s.adjoint_forward(2, 1e-3, 1, np.zeros((2, len(gelem))))
    s.set_params(s.get_params(), integrator=1)               # so does another scheme
    with pytest.raises(esdg.EsdgError):
        s.adjoint_backward()
    s.set_params(s.get_params(), integrator=0)               # the recorded one again
    s.adjoint_backward()
    s.set_params(s.get_params(), av_on=1, eps0=0.05)
    with pytest.raises(esdg.EsdgError):
        s.rhs_vjp(z, z, z)
    s.close()
    s32 = esdg.Solver(0, 32)
    s32.upload_mesh(mesh)
    s32.set_bathymetry(b)
    s32.set_state(H0 - b, z, z)
    with pytest.raises(esdg.EsdgError):
        s32.rhs_vjp(z, z, z)
    s32.close()


def test_limiter_activity_is_reported(esdg):
    """A state that dries out is outside the adjoint: the forward sweep
    reports it instead of returning a gradient of a non-smooth map."""
    mesh, b, H0, db, gelem, gxi, geta, steps = small_case(N=3, steps=2)
    z = np.zeros_like(b)
    h = np.maximum(0.6 - b, 0.0) + 0.0
    h[: h.shape[0] // 2] = 0.0        # half the domain dry: the dam-break front
    s, P = make_solver(esdg, mesh, b, h, z, z, 3, limiter_on=1)
    s.set_gauges(gelem, gxi, geta)
    dt = 0.2 * s.compute_dt()[0]
    with pytest.raises(esdg.EsdgError):
        s.adjoint_forward(5, dt, 2, np.zeros((5, len(gelem))))
    s.close()


def test_autograd_wrappers(esdg):
    import torch
    from paper_1804_02221_amd.autograd import Rhs, gauge_misfit
    mesh, b, H0, db, gelem, gxi, geta, steps = small_case(N=3, steps=6)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, 3, limiter_on=1)
    s.set_gauges(gelem, gxi, geta)
    dt = 0.5 * s.compute_dt()[1]
    dev = "cuda:0"
    T = lambda a: torch.tensor(a, device=dev, dtype=torch.float64)
    # Rhs: grad of sum(lam . R) equals the library's reverse mode
    rng = np.random.default_rng(2)
    h = T(H0 - b).requires_grad_()
    hu = T(0.1 * rng.standard_normal(b.shape)).requires_grad_()
    hv = T(0.1 * rng.standard_normal(b.shape)).requires_grad_()
    bb = T(b).requires_grad_()
    lam = [T(rng.standard_normal(b.shape)) for _ in range(3)]
    R = Rhs.apply(h, hu, hv, bb, s)
    sum(torch.sum(l * r.reshape(l.shape)) for l, r in zip(lam, R)).backward()
    s.set_bathymetry(b)
    s.set_state(H0 - b, hu.detach().cpu().numpy(), hv.detach().cpu().numpy())
    ref = s.rhs_vjp(*[l.cpu().numpy() for l in lam])
    for t_, r_ in zip((h, hu, hv, bb), ref):
        assert np.array_equal(t_.grad.cpu().numpy(), r_)
    # GaugeMisfit: d/db with H0 fixed is gb - gh0
    tgt = np.full((steps, len(gelem)), 1.02)
    bt = T(b).requires_grad_()
    L = gauge_misfit(s, bt, T(H0), T(z), T(z), tgt, steps, dt, every=4)
    L.backward()
    s.set_bathymetry(b)
    s.set_state(H0 - b, z, z)
    L2 = s.adjoint_forward(steps, dt, 4, tgt)
    gb, gh0, _, _ = s.adjoint_backward()
    assert float(L.detach()) == L2
    assert np.array_equal(bt.grad.cpu().numpy(), gb - gh0)
    s.close()


def test_full_size_gradient(esdg, orc):
    """The bathymetry-gradient workload at full size (128 x 128 elements,
    N = 5, 400 steps, checkpoints every 20, 32 gauges): the reverse mode of R
    against the oracle on the whole field, and the gradient (initial surface
    held fixed, h(0) = H0 - b) against central differences of the GPU loss
    along 20 random continuous directions, with a dot-product check in the
    initial discharge."""
    w, x = bathymetry_gradient()
    N, steps, every = 5, 400, 20
    s, P = make_solver(esdg, w.mesh, w.b, w.h, w.hu, w.hv, N, **w.params)
    rng = np.random.default_rng(11)
    lam = [rng.standard_normal(w.h.shape) for _ in range(3)]
    print("full size: reverse mode of R against the oracle", flush=True)
    got = s.rhs_vjp(*lam)
    want = orc.rhs_vjp(oparams(orc, P), w.mesh, w.b, w.h, w.hu, w.hv, *lam)
    check(got, want, TOL_VJP, "C5 vjp")
    s.set_gauges(x["gelem"], x["gxi"], x["geta"])
    dt = s.compute_dt()[0]
    # target run over b + db
    zero = np.zeros_like(w.h)
    s.set_bathymetry(w.b + x["db"])
    s.set_state(x["H0"] - w.b - x["db"], zero, zero)
    _, tgt = s.adjoint_forward(steps, dt, every, np.zeros((steps, 32)), want_H=True)

    def loss(b, h0=None, hu0=zero):
        s.set_bathymetry(b)
        s.set_state(x["H0"] - b if h0 is None else h0, hu0, zero)
        return s.adjoint_forward(steps, dt, every, tgt)

    print("full size: forward and reverse sweep", flush=True)
    L0 = loss(w.b)
    gb, gh0, ghu0, _ = s.adjoint_backward()
    gtot = gb - gh0
    assert L0 > 0

    def richardson(f, eps=1e-4):
        # central differences at eps and eps/2 combined so that the eps^2
        # term cancels: the loss is far from linear on the scale where plain
        # central differences would reach 1e-6
        d1 = (f(eps) - f(-eps)) / (2 * eps)
        d2 = (f(eps / 2) - f(-eps / 2)) / eps
        return (4 * d2 - d1) / 3

    m = w.mesh

    def direction():
        return m.gather(rng.standard_normal((m.nx * m.N, m.ny * m.N)))

    errs = []
    for k in range(20):
        d = direction()
        fd = richardson(lambda e: loss(w.b + e * d))
        ad = float(np.sum(gtot * d))
        errs.append(abs(fd - ad) / abs(ad))
        print(f"direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {errs[-1]:.2e}", flush=True)
        assert abs(fd - ad) <= FD_TOL * abs(ad), (k, fd, ad)
    print(f"full size: 20 directions, max rel err {max(errs):.2e}", flush=True)
    # dot-product check in the initial discharge.  The run starts at rest,
    # where the dissipation's |ah au| has its kink: the loss then has an
    # |eps| eps part along discharge directions, differentiable with the
    # derivative sign(0) = 0 gives, but central differences carry an O(eps)
    # error; the bound adds the differences' own change between the steps.
    d = direction()
    e = 1e-5
    D1 = (loss(w.b, hu0=e * d) - loss(w.b, hu0=-e * d)) / (2 * e)
    D2 = (loss(w.b, hu0=0.5 * e * d) - loss(w.b, hu0=-0.5 * e * d)) / e
    fd = (4 * D2 - D1) / 3
    ad = float(np.sum(ghu0 * d))
    print(f"full size: discharge direction rel err {abs(fd - ad) / abs(ad):.2e}, "
          f"step change {abs(D1 - D2) / abs(ad):.2e}", flush=True)
    assert abs(fd - ad) <= FD_TOL * abs(ad) + abs(D1 - D2), (fd, ad, D1, D2)
    s.close()


def test_ssprk_gradient_in_a_walled_basin_against_differences(esdg):
    """SSPRK(3,3) steps in a closed basin (walls on both axes, 24 x 24
    elements, N = 4, 120 steps, checkpoints every 10): the gradient of the
    gauge misfit against Richardson-extrapolated central differences of the
    GPU loss along continuous random directions in b, after the waves from
    the initial surface bump have reached the walls."""
    N, steps, every = 4, 120, 10
    mesh = make_box_mesh(N, 24, 24, -2.0, -2.0, 4.0, 4.0, amp=0.1, rotate_seed=4)
    rng = np.random.default_rng(21)
    x, y = mesh.x, mesh.y
    b = 0.25 * np.exp(-((x - 0.6) ** 2 + (y + 0.4) ** 2) / 0.5) + 0.05 * x
    H0 = 1.0 + 0.05 * np.exp(-((x + 1.2) ** 2 + (y - 1.0) ** 2) / 0.3)
    db = 0.03 * np.exp(-((x + 0.3) ** 2 + (y + 1.1) ** 2) / 0.4)
    ng = 12
    gelem = rng.integers(0, mesh.K, ng).astype(np.int32)
    gxi, geta = rng.uniform(-1, 1, ng), rng.uniform(-1, 1, ng)
    z = np.zeros_like(b)
    s, P = make_solver(esdg, mesh, b, H0 - b, z, z, N, limiter_on=1, integrator=1)
    s.set_gauges(gelem, gxi, geta)
    dt = 0.8 * s.compute_dt()[1]
    s.set_bathymetry(b + db)
    s.set_state(H0 - b - db, z, z)
    _, tgt = s.adjoint_forward(steps, dt, every, np.zeros((steps, ng)), want_H=True)

    def loss(bb):
        s.set_bathymetry(bb)
        s.set_state(H0 - bb, z, z)
        return s.adjoint_forward(steps, dt, every, tgt)

    print(f"SSPRK walled basin: {steps} steps to t = {steps * dt:.3f}", flush=True)
    L0 = loss(b)
    gb, gh0, _, _ = s.adjoint_backward()
    gtot = gb - gh0
    assert L0 > 0
    # the waves reached the walls: the surface moved at the wall nodes
    h_end = s.get_state()[0]
    wall = (np.abs(np.abs(x) - 2.0) < 1e-9) | (np.abs(np.abs(y) - 2.0) < 1e-9)
    assert np.abs((h_end + b - H0)[wall]).max() > 1e-3

    def richardson(f, eps=1e-4):
        d1 = (f(eps) - f(-eps)) / (2 * eps)
        d2 = (f(eps / 2) - f(-eps / 2)) / eps
        return (4 * d2 - d1) / 3

    for k in range(5):
        d = mesh.gather(rng.standard_normal((mesh.nx * N, mesh.ny * N)))
        fd = richardson(lambda e: loss(b + e * d))
        ad = float(np.sum(gtot * d))
        print(f"direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}", flush=True)
        assert abs(fd - ad) <= FD_TOL * abs(ad), (k, fd, ad)
    s.close()
