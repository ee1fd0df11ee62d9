"""Pins of the oracle's solid walls (reflecting outside state) against what
the method fixes on a closed basin: the lake at rest stays at rest (Lemma 1.3
with walls), no mass crosses a wall, the EC flux produces no entropy at a
wall and the ES flux dissipates, the wall flux has its closed form, mirror
symmetry of a symmetric state in a box, and the oscillating lake of the
paper's test section against its closed-form solution."""
import numpy as np
import pytest

from paper_1804_02221_amd.inputs import make_box_mesh, oscillating_lake

G = 9.81


def weights(orc, mesh):
    op = orc.operators(mesh.N)
    geo = orc.geometry(mesh)
    return geo["J"] * np.outer(op["w"], op["w"]).reshape(-1)[None, :], geo


def smooth_state(mesh, seed=0, wet=True):
    rng = np.random.default_rng(seed)
    x, y = mesh.x, mesh.y
    c = rng.uniform(0.3, 0.7, 6)
    b = 0.3 * np.exp(-((x - c[0] * 4 - 2) ** 2 + (y - c[1] * 4 + 2) ** 2))
    h = 1.0 + 0.2 * np.sin(1.3 * x + c[2]) * np.cos(0.9 * y + c[3]) - b
    u = 0.3 * np.cos(0.7 * x + c[4])
    v = 0.2 * np.sin(0.8 * y + c[5])
    return b, h, h * u, h * v


@pytest.mark.parametrize("N,rot", [(3, None), (4, 5), (5, 9)])
def test_lake_at_rest_in_a_walled_basin(orc, N, rot):
    mesh = make_box_mesh(N, 5, 4, -2.0, -2.0, 4.0, 4.0, amp=0.1, rotate_seed=rot)
    x, y = mesh.x, mesh.y
    b = 0.4 * np.exp(-((x - 0.5) ** 2 + (y + 0.3) ** 2)) + 0.1 * x * y
    h = 1.5 - b
    z = np.zeros_like(h)
    P = orc.params(N, av_on=1, limiter_on=1, eps0=0.05)
    R = orc.rhs(P, mesh, b, h, z, z)[:3]
    scale = G * 1.5 * 1.5 * 40.0
    assert max(np.abs(r).max() for r in R) < 1e-13 * scale


@pytest.mark.parametrize("flux", [0, 1])
def test_walls_carry_no_mass_and_entropy_sign(orc, flux):
    mesh = make_box_mesh(3, 5, 5, -2.0, -2.0, 4.0, 4.0, amp=0.1, rotate_seed=2)
    b, h, hu, hv = smooth_state(mesh)
    P = orc.params(3, surface_flux=flux)
    Rh, Rhu, Rhv, _ = orc.rhs(P, mesh, b, h, hu, hv)
    wq, _ = weights(orc, mesh)
    mass_rate = np.sum(wq * Rh)
    assert abs(mass_rate) < 1e-13 * np.sum(wq * np.abs(Rh))
    d = orc.diagnostics(P, mesh, b, h, hu, hv)
    terms = np.sum(wq * (np.abs(Rh) + np.abs(Rhu) + np.abs(Rhv))) * G * 2.0
    if flux == 1:
        assert abs(d[4]) < 1e-12 * terms          # EC: no entropy produced, walls included
    else:
        assert d[4] < -1e-8 * terms               # ES: dissipative


def test_wall_flux_closed_form(orc):
    """With the reflected outside state the ES flux is n (g h^2/2 + h sqrt(g h) u.n)
    in the momentum and zero in the mass; the EC flux is n g h^2/2."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        h = rng.uniform(0.1, 2.0)
        u, v = rng.uniform(-1, 1, 2)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        un = u * nx + v * ny
        wm = np.array([h, h * u, h * v])
        wp = np.array([h, h * (u - 2 * un * nx), h * (v - 2 * un * ny)])
        b = rng.uniform(0, 1)
        for flux, fn in ((0, 0.5 * G * h * h + h * np.sqrt(G * h) * un), (1, 0.5 * G * h * h)):
            F = orc.surface_flux(orc.params(3, surface_flux=flux), wm, b, wp, b, nx, ny)
            assert abs(F[0]) < 1e-14
            assert np.allclose(F[1:], [fn * nx, fn * ny], rtol=1e-13, atol=1e-13)


def test_mirror_symmetry_in_a_box(orc):
    """A state symmetric under x -> -x in the box [-2,2]^2 (hu odd) has an
    odd R_hu and even R_h, R_hv: both walls reflect alike."""
    N = 3
    mesh = make_box_mesh(N, 6, 5, -2.0, -2.0, 4.0, 4.0)
    x, y = mesh.x, mesh.y
    b = 0.2 * np.exp(-(x ** 2 + (y - 0.4) ** 2))
    h = 1.0 + 0.1 * np.cos(1.1 * x) * np.sin(y + 0.3) - b
    hu = h * 0.3 * np.sin(0.9 * x)
    hv = h * 0.2 * np.cos(0.7 * x) * np.cos(y)
    P = orc.params(N, av_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-29.0)  # viscosity everywhere
    Rh, Rhu, Rhv, _ = orc.rhs(P, mesh, b, h, hu, hv)
    # mirror of node (i, j) of element (ix, iy): node (N-i, j) of element (nx-1-ix, iy)
    nx_, n1 = 6, N + 1
    e = np.arange(mesh.K)
    em = (e // nx_) * nx_ + (nx_ - 1 - e % nx_)
    i, j = np.divmod(np.arange(n1 * n1), n1)
    mir = (em[:, None] * n1 * n1 + ((N - i) * n1 + j)[None, :]).ravel()
    assert np.allclose(x.ravel()[mir], -x.ravel()) and np.allclose(y.ravel()[mir], y.ravel())
    sc = max(np.abs(Rh).max(), np.abs(Rhu).max())
    assert np.abs(Rh.ravel() - Rh.ravel()[mir]).max() < 1e-12 * sc
    assert np.abs(Rhu.ravel() + Rhu.ravel()[mir]).max() < 1e-12 * sc
    assert np.abs(Rhv.ravel() - Rhv.ravel()[mir]).max() < 1e-12 * sc


def lake_error(orc, n, t_end):
    """L1 error of the water height over the basin relative to the exact
    water volume, after running the oscillating lake to t_end (adaptive
    steps, the last one clipped)."""
    w = oscillating_lake(n, 3)
    P = orc.params(3, **w.params)
    h, hu, hv, t = w.h, w.hu, w.hv, 0.0
    while t < t_end - 1e-12:
        dt = min(orc.dt(P, w.mesh, w.b, h, hu, hv)[0], t_end - t)
        h, hu, hv, _, st = orc.step(P, w.mesh, w.b, h, hu, hv, 1, dt_fixed=dt)
        assert st == 0
        t += dt
    ex = oscillating_lake(n, 3, t=t_end)
    wq, _ = weights(orc, w.mesh)
    assert h.min() >= -1e-14
    return np.sum(wq * np.abs(h - ex.h)) / np.sum(wq * ex.h)


def test_oscillating_lake_against_closed_form(orc):
    """The planar oscillation in the parabolic bowl (walls at |x|, |y| = 2,
    never reached): at t = T/6 the water height is close to the closed form
    and closer on the finer mesh."""
    T = 2 * np.pi / np.sqrt(2 * G * 0.1)
    e1 = lake_error(orc, 10, T / 6)
    e2 = lake_error(orc, 20, T / 6)
    print("relative L1 errors", e1, e2)
    assert e2 < 0.06
    assert e2 < 0.7 * e1


def test_three_mound_dam_break_coarse(orc):
    """The dam break over three mounds on a 15 x 10 mesh, 20 adaptive
    SSPRK(3,3) steps: the bed is the maximum of the three cones (apex heights
    1, 1, 2.8 at their centres), no mass is gained or lost in the closed
    basin, no height turns negative and the total entropy decreases."""
    from paper_1804_02221_amd.inputs import three_mound_dam_break
    w = three_mound_dam_break(15, 10, 3)
    x, y = w.mesh.x, w.mesh.y
    cone = lambda a, s, cx, cy: a - s * np.hypot(x - cx, y - cy)
    want = np.maximum.reduce([np.zeros_like(x), cone(1, 0.1, 30, 22.5), cone(1, 0.1, 30, 7.5),
                              cone(2.8, 0.28, 47.5, 15)])
    assert np.abs(w.b - want).max() <= 1e-14
    assert (w.mesh.nbr_elem < 0).sum() == 2 * (15 + 10)
    P = orc.params(3, **w.params)
    d0 = orc.diagnostics(P, w.mesh, w.b, w.h, w.hu, w.hv)
    h, hu, hv, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 20, 0.0)
    assert st == 0 and t > 0
    d1 = orc.diagnostics(P, w.mesh, w.b, h, hu, hv)
    assert abs(d1[0] - d0[0]) <= 1e-13 * d0[0]
    assert h.min() >= 0.0
    assert d1[3] < d0[3]


def test_conical_island_initial_state(orc):
    """The island case's initial data against its closed forms: the cone's
    apex height and radius, the solitary wave's crest A above h0 at x = 2.5
    with the long-wave speed sqrt(g/h0) in its discharge, a dry island top,
    and 20 adaptive steps on a 10 x 12 mesh that keep the mass and h >= 0."""
    from paper_1804_02221_amd.inputs import conical_island
    w = conical_island(10, 12, 3)
    x, y = w.mesh.x, w.mesh.y
    r = np.hypot(x - 12.5, y - 15.0)
    assert np.abs(w.b - np.where(r <= 3.6, 0.93 * (1 - r / 3.6), 0.0)).max() <= 1e-15
    crest = np.abs(x - 2.5) < 1e-12
    assert crest.any() and np.allclose(w.h[crest], 0.32 + 0.064, rtol=0, atol=1e-14)
    assert np.allclose(w.hu[crest], w.h[crest] * 0.064 * np.sqrt(9.81 / 0.32), rtol=1e-14)
    assert (w.h[w.b > 0.4] == 0).all() and (w.hv == 0).all()
    P = orc.params(3, **w.params)
    d0 = orc.diagnostics(P, w.mesh, w.b, w.h, w.hu, w.hv)
    h, hu, hv, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 20, 0.0)
    d1 = orc.diagnostics(P, w.mesh, w.b, h, hu, hv)
    assert st == 0 and abs(d1[0] - d0[0]) <= 1e-13 * d0[0] and h.min() >= 0.0
