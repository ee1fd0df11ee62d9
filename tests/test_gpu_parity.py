"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
element by element, on the same seeded inputs.

Bar (FP64): per field, max |GPU - oracle| <= 16 x floor, the floor being the
oracle's own response to a random 1-ulp perturbation of its inputs
(tests/parity_floor.py; no GPU value enters it).  On the 512^2, N = 7
workload the floor is ~5e-16 of the size of the terms that cancel in R and
3e-12 to 1e-11 of max |R|; a plain 1e-12 max |R| would sit below it there.

With artificial viscosity the element viscosity comes from log10 of a modal
energy ratio formed by cancellation, so on the sine ramp of the indicator
its rounding noise (~1e-9 relative) reaches R.  The viscous cases therefore
come in two kinds: saturated (thresholds chosen from the state so that every
element's viscosity is exactly 0 or eps0; the floor is then the inviscid
one's kind) and ramp (thresholds spread over the states; the floor contains
the indicator's conditioning, and eps is checked against its own floor).

FP32: the single-precision stage kernel forms its two-point sums and
interface fluxes from jumps to the own node.  On small curvilinear meshes R
agrees with the FP64 oracle on the FP64 state to 1e-5 of max |R| (and of the
term scale g |h| |h+b| |D| |metric| / J); on an affine mesh with metric
terms exact in FP32 and the state and bathymetry rounded to FP32 on both
sides, to 1e-5 of max |R| as well: there the comparison sees the FP32
arithmetic alone.  (On fine meshes the rounding of the stored state alone
moves R by more than 1e-5 of max |R|: 1e-4 at 512^2, N = 7.)
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02221_amd.inputs import (dam_break, fourier_field, lake_bump, make_periodic_mesh,
                                         periodic_gaussians, smooth_sweep)
from parity_floor import check, rhs_floor, step_floor

G = 9.81
TOL32 = 1e-5


@pytest.fixture(scope="module")
def esdg():
    from paper_1804_02221_amd import esdg as m
    m.lib()
    return m


def term_scale(orc, mesh, h, b):
    op = orc.operators(mesh.N)
    geo = orc.geometry(mesh)
    met = max(np.abs(geo[k]).max() for k in ("xxi", "xeta", "yxi", "yeta"))
    return G * np.abs(h).max() * np.abs(h + b).max() * np.abs(op["D"]).max() * met / geo["J"].min()


def make_solver(esdg, w, prec=64, **kw):
    s = esdg.Solver(0, prec)
    s.upload_mesh(w.mesh)
    P = esdg.default_params(w.mesh.N)
    for k, v in {**w.params, **kw}.items():
        setattr(P, k, v)
    s.set_params(P)
    s.set_bathymetry(w.b)
    s.set_state(w.h, w.hu, w.hv)
    return s, P


def oparams(orc, P):
    return orc.params(3, **P.as_dict())


def element_sigma(orc, N, h):
    """log10 of the indicator's larger modal energy ratio per element (test
    side, from the oracle's V^{-1}; used only to place the thresholds)."""
    V = orc.operators(N)["Vinv"]
    nf = N + 1
    Q = np.einsum("ai,eij,cj->eac", V, h.reshape(-1, nf, nf), V)
    q2 = Q ** 2
    shell = np.maximum.outer(np.arange(nf), np.arange(nf))
    top, tot = q2[:, shell == N].sum(1), q2.sum((1, 2))
    topM, totM = q2[:, shell == N - 1].sum(1), q2[:, :N, :N].sum((1, 2))
    r = np.maximum(top / tot, np.where(totM > 0, topM / np.where(totM > 0, totM, 1.0), 0.0))
    return np.log10(np.maximum(r, 1e-300))


def saturating_thresholds(orc, N, h, rough):
    """(sigma_min, sigma_max) that leave every element's viscosity at exactly
    0 or eps0: inside the gap between smooth and rough elements when there is
    one, else below every element (all viscous)."""
    sg = element_sigma(orc, N, h)
    lo, hi = sg[~rough].max(), sg[rough].min()
    if hi - lo > 1.0:
        return lo + 0.3, hi - 0.3
    return sg.min() - 1.3, sg.min() - 0.3


def rough_state(w, N, seed, frac=0.4, amp=0.3):
    rng = np.random.default_rng(seed)
    rough = rng.uniform(size=w.mesh.K) < frac
    w.h = w.h + amp * rng.uniform(-1.0, 1.0, size=w.h.shape) * rough[:, None]
    w.hu = w.hu + 0.05 * rng.standard_normal(w.hu.shape)   # ES dissipation active
    return rough


def test_geometry(esdg, orc):
    for N in (2, 5, 8):
        mesh = make_periodic_mesh(N, 5, 3, 10.0, 10.0, amp=0.1, rotate_seed=N)
        s = esdg.Solver()
        s.upload_mesh(mesh)
        geo = s.get_geometry()
        ref = orc.geometry(mesh)
        for k in ("xxi", "xeta", "yxi", "yeta", "J"):
            assert np.abs(geo[k] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max(), k
        s.close()


CASES = [  # (N, n elements per side, av, surface flux EC?, rotate)
    (2, 5, 0, 0, None), (3, 5, 1, 0, 3), (4, 4, 0, 1, 4), (5, 5, 1, 0, None),
    (6, 3, 1, 1, 6), (7, 5, 1, 0, 7), (8, 4, 1, 0, 8), (7, 3, 0, 0, None),
]


@pytest.mark.parametrize("N,n,av,ec,rot", CASES)
def test_rhs_parity(esdg, orc, N, n, av, ec, rot):
    """R at every node; with AV, saturated viscosities (exactly 0 or eps0)."""
    w = smooth_sweep(n, N, seed=20 + N, rotate_seed=rot)
    rough = rough_state(w, N, seed=N)
    kw = dict(av_on=av, surface_flux=ec, eps0=0.05)
    if av:
        kw["sigma_min"], kw["sigma_max"] = saturating_thresholds(orc, N, w.h, rough)
    s, P = make_solver(esdg, w, **kw)
    got = s.rhs()
    Po = oparams(orc, P)
    Ro, fl = rhs_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv)
    check(got, Ro[:3], fl, f"rhs N={N} av={av} ec={ec}")
    if av:
        eps = s.get_eps()
        assert set(np.unique(Ro[3])) <= {0.0, 0.05}, "viscosity not saturated"
        assert (Ro[3] > 0).sum() > 0
        assert np.array_equal(eps, Ro[3])
    s.close()


@pytest.mark.parametrize("N", [3, 5, 8])
def test_rhs_parity_indicator_ramp(esdg, orc, N):
    """Viscosities spread over the indicator's sine ramp (thresholds -30,
    -1): eps against its own floor, R against a floor that contains the
    indicator's conditioning."""
    w = smooth_sweep(4, N, seed=60 + N, rotate_seed=N)
    rough_state(w, N, seed=100 + N, amp=0.1)
    s, P = make_solver(esdg, w, av_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    got = s.rhs()
    eps = s.get_eps()
    Ro, fl = rhs_floor(orc, oparams(orc, P), w.mesh, w.b, w.h, w.hu, w.hv)
    on_ramp = ((Ro[3] > 0) & (Ro[3] < 0.05)).sum()
    assert on_ramp > 0.5 * w.mesh.K
    check([eps], [Ro[3]], [max(fl[3], 1e-17)], f"eps ramp N={N}", names=("eps",))
    check(got, Ro[:3], fl, f"rhs ramp N={N}")
    s.close()


@pytest.mark.parametrize("N,jump", [(3, False), (7, False), (3, True), (6, True)])
def test_lake_at_rest(esdg, orc, N, jump):
    """Lemma 1.3 on the GPU: R = 0 to the floor, with a continuous bottom and
    with one that jumps at every face (interface penalty of eq. SourceDisc)."""
    mesh = make_periodic_mesh(N, 6, 5, 10.0, 10.0, amp=0.1, rotate_seed=1)
    b = periodic_gaussians(mesh, [(3.0, 4.0), (7.0, 2.0)], [0.4, 0.3], [1.5, 1.0])
    if jump:
        b = b + 0.2 * np.random.default_rng(N).uniform(size=(mesh.K, 1))
    h = 2.0 - b
    z = np.zeros_like(h)
    s = esdg.Solver()
    s.upload_mesh(mesh)
    P = esdg.default_params(N, av_on=1, limiter_on=1, eps0=0.05)
    s.set_params(P)
    s.set_bathymetry(b)
    s.set_state(h, z, z)
    R = s.rhs()
    Ro, fl = rhs_floor(orc, oparams(orc, P), mesh, b, h, z, z)
    check(R, Ro[:3], fl, f"lake at rest N={N} jump={jump}")
    sc = term_scale(orc, mesh, h, b)
    assert max(np.abs(r).max() for r in R) < 1e-13 * sc
    s.close()


@pytest.mark.parametrize("N,rot,ec", [(2, 3, 0), (4, None, 1), (5, 5, 0), (8, 8, 0)])
def test_rhs_and_steps_over_a_jumping_bottom(esdg, orc, N, rot, ec):
    """The interface bathymetry penalty: R and two adaptive LSRK steps over a
    bottom with a random jump at every face, against the oracle."""
    w = smooth_sweep(4, N, seed=70 + N, rotate_seed=rot)
    w.b = w.b + 0.15 * np.random.default_rng(N).uniform(size=(w.mesh.K, 1))
    s, P = make_solver(esdg, w, surface_flux=ec, limiter_on=1)
    Po = oparams(orc, P)
    Ro, fl = rhs_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv)
    check(s.rhs(), Ro[:3], fl, f"rhs jump N={N}")
    t_gpu, _ = s.step(2, 0.0)
    (h, hu, hv, t_orc, _), fls = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 2, 0.0)
    assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    check(s.get_state(), (h, hu, hv), fls, f"steps jump N={N}")
    s.close()


def test_dt_limiter_eps_diagnostics(esdg, orc):
    w = dam_break(10, 4, seed=2, rotate_seed=5)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05, integrator=1)
    Po = oparams(orc, P)
    # take a few oracle steps so the data has fronts, then compare pieces there
    h, hu, hv, t, st = orc.step(Po, w.mesh, w.b, w.h, w.hu, w.hv, 3, 0.0)
    s.set_state(h, hu, hv)
    dts = s.compute_dt()
    dto = orc.dt(Po, w.mesh, w.b, h, hu, hv)
    assert np.allclose(dts, dto, rtol=1e-12, atol=0)
    eps = s.get_eps()
    Ro, fl = rhs_floor(orc, Po, w.mesh, w.b, h, hu, hv)
    check([eps], [Ro[3]], [max(fl[3], 1e-17)], "eps dam break", names=("eps",))
    d = s.diagnostics()
    do = orc.diagnostics(Po, w.mesh, w.b, h, hu, hv)
    # global sums: their rounding is that of the summation order (1e-13 of
    # the summed magnitudes); the entropy rate sum J w w q.R in addition
    # inherits R's floor through |q|
    op = orc.operators(4)
    wq = orc.geometry(w.mesh)["J"] * np.outer(op["w"], op["w"]).reshape(-1)[None, :]
    ih = np.where(h > 1e-4, 1.0 / np.where(h > 1e-4, h, 1.0), 0.0)
    u, v = hu * ih, hv * ih
    q1 = G * (h + w.b) - 0.5 * (u * u + v * v)
    mags = [np.sum(wq * np.abs(h)), np.sum(wq * np.abs(hu)), np.sum(wq * np.abs(hv)),
            np.sum(wq * (0.5 * h * (u * u + v * v) + 0.5 * G * h * h + G * h * np.abs(w.b)))]
    for k in range(4):
        assert abs(d[k] - do[k]) <= 1e-13 * mags[k], (k, d[k], do[k])
    rate_bar = 16.0 * np.sum(wq * (np.abs(q1) * fl[0] + np.abs(u) * fl[1] + np.abs(v) * fl[2])) + \
        1e-13 * np.sum(wq * (np.abs(q1 * Ro[0]) + np.abs(u * Ro[1]) + np.abs(v * Ro[2])))
    print(f"[parity] dE/dt err {abs(d[4] - do[4]):.3e} bar {rate_bar:.3e}", flush=True)
    assert abs(d[4] - do[4]) <= rate_bar
    assert d[5] == do[5] and d[6] == do[6] and d[7] == do[7]
    # limiter on a state with negative nodes
    from parity_floor import perturbed_inputs
    rng = np.random.default_rng(3)
    hn = h - 0.3 * rng.uniform(size=h.shape) * (rng.uniform(size=(h.shape[0], 1)) < 0.5)
    s.set_state(hn, hu, hv)
    nl, st = s.limit()
    ho, huo, hvo, nlo, sto = orc.limit(Po, w.mesh, hn, hu, hv)
    assert nl == nlo and st == sto
    lfl = np.zeros(3)
    for k in range(2):
        _, hk, huk, hvk = perturbed_inputs(w.mesh, w.b, hn, hu, hv, 60 + k)
        o = orc.limit(Po, w.mesh, hk, huk, hvk)
        lfl = np.maximum(lfl, [np.abs(o[c] - (ho, huo, hvo)[c]).max() for c in range(3)])
    if orc.host_has_fma():
        with orc.rounding_twin():
            o = orc.limit(Po, w.mesh, hn, hu, hv)
        lfl = np.maximum(lfl, [np.abs(o[c] - (ho, huo, hvo)[c]).max() for c in range(3)])
    check(s.get_state(), (ho, huo, hvo), lfl, "limiter")
    s.close()


@pytest.mark.parametrize("N,integrator", [(3, 0), (4, 1), (7, 0)])
def test_dt_bounds_left_by_the_last_stage(esdg, orc, N, integrator):
    """After a step the time-step pass reduces the per-element CFL and
    viscous bounds the last stage left; they must equal the bounds of the
    full pass on the same state and the oracle's after the same step."""
    w = dam_break(6, N, seed=4, rotate_seed=3)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05, integrator=integrator)
    Po = oparams(orc, P)
    s.step(1, 0.0)
    fused = s.compute_dt()
    h, hu, hv = s.get_state()
    s.set_state(h, hu, hv)             # invalidates the stage's bounds: full pass
    full = s.compute_dt()
    assert np.allclose(fused, full, rtol=1e-14, atol=0), (fused, full)
    ho, huo, hvo, _, _ = orc.step(Po, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0)
    dto = orc.dt(Po, w.mesh, w.b, ho, huo, hvo)
    assert np.allclose(fused, dto, rtol=1e-11, atol=0), (fused, dto)
    assert np.isfinite(fused[2]) and fused[2] < 1e30, "viscous bound expected on the dam break"
    s.close()


@pytest.mark.parametrize("integrator,adaptive", [(0, False), (0, True), (1, True)])
def test_step_parity_dam_break(esdg, orc, integrator, adaptive):
    w = dam_break(8, 5, seed=2, rotate_seed=2)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05, integrator=integrator)
    Po = oparams(orc, P)
    dt = 0.0 if adaptive else 0.5 * orc.dt(Po, w.mesh, w.b, w.h, w.hu, w.hv)[0]
    t_gpu, st = s.step(4, dt)
    (h, hu, hv, t_orc, sto), fl = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 4, dt)
    assert st == 0 and sto == 0
    assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    check(s.get_state(), (h, hu, hv), fl, f"dam-break steps integ={integrator} adaptive={adaptive}")
    s.close()


def test_step_parity_lake_bump_lsrk(esdg, orc):
    """The plain-method workload (16 x 16, N = 3, EC volume / ES surface flux,
    no AV or limiter, LSRK(5,4) at CFL 0.5): 100 steps against the oracle."""
    w = lake_bump(16, 3, seed=1)
    s, P = make_solver(esdg, w)
    Po = oparams(orc, P)
    t_gpu, _ = s.step(100, 0.0)
    (h, hu, hv, t_orc, _), fl = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 100, 0.0)
    assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    check(s.get_state(), (h, hu, hv), fl, "lake bump 100 steps")
    s.close()


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_step_parity_every_degree(esdg, orc, N):
    """Two adaptive LSRK(5,4) steps with AV (on the ramp) and the limiter at
    every degree (every workgroup shape, ragged last tiles, rotated frames)."""
    w = smooth_sweep(5, N, seed=40 + N, rotate_seed=N)
    rng = np.random.default_rng(100 + N)
    w.hu = w.hu + 0.05 * rng.standard_normal(w.hu.shape)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    Po = oparams(orc, P)
    t_gpu, _ = s.step(2, 0.0)
    (h, hu, hv, t_orc, _), fl = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 2, 0.0)
    assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    check(s.get_state(), (h, hu, hv), fl, f"steps N={N}")
    s.close()


@pytest.mark.parametrize("N", [2, 5, 8])
def test_two_by_two_mesh(esdg, orc, N):
    """2 x 2 periodic elements: each element meets the same neighbour across
    two opposite sides (and itself nowhere); RHS and one step."""
    w = smooth_sweep(2, N, seed=50 + N, rotate_seed=N)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    Po = oparams(orc, P)
    Ro, fl = rhs_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, draws=4)
    check(s.rhs(), Ro[:3], fl, f"2x2 rhs N={N}")
    t_gpu, _ = s.step(1, 0.0)
    (h, hu, hv, t_orc, _), fls = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0, draws=3)
    check(s.get_state(), (h, hu, hv), fls, f"2x2 step N={N}")
    s.close()


def test_full_size_step_parity(esdg, orc):
    """One adaptive LSRK(5,4) step with AV and limiter on the 512 x 512
    curvilinear N = 7 workload the benchmark times, every node against the
    oracle."""
    w = smooth_sweep(512, 7, seed=3)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.025)
    Po = oparams(orc, P)
    t_gpu, _ = s.step(1, 0.0)
    got = s.get_state()
    s.close()
    (h, hu, hv, t_orc, _), fl = step_floor(orc, Po, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0)
    assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    check(got, (h, hu, hv), fl, "full-size step")


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_fp32_variant(esdg, orc, N):
    """FP32 on a curvilinear mesh against the FP64 oracle on the FP64 state:
    within 1e-5 of the term scale and of max |R|.  Its error against the
    oracle on the FP32-rounded state and bathymetry is printed beside it
    (what remains of the FP32 metric terms and arithmetic)."""
    w = smooth_sweep(5, N, seed=30 + N)
    s, P = make_solver(esdg, w, prec=32, av_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    got = s.rhs()
    s.close()
    Po = oparams(orc, P)
    Ro = orc.rhs(Po, w.mesh, w.b, w.h, w.hu, w.hv)
    Rr = orc.rhs(Po, w.mesh, _f32(w.b), _f32(w.h), _f32(w.hu), _f32(w.hv))
    sc = term_scale(orc, w.mesh, w.h, w.b)
    for c in range(3):
        mx = np.abs(Ro[c]).max()
        err = np.abs(got[c] - Ro[c]).max()
        print(f"[parity] fp32 N={N} field {c}: err {err:.3e} err/term-scale {err / sc:.2e} err/max {err / mx:.2e}"
              f" (input rounding alone {np.abs(Rr[c] - Ro[c]).max() / mx:.2e},"
              f" vs the rounded inputs {np.abs(got[c] - Rr[c]).max() / mx:.2e})", flush=True)
        assert err <= TOL32 * sc
        assert err <= TOL32 * mx


@pytest.mark.parametrize("av", ["off", "on"])
@pytest.mark.parametrize("N", [3, 7])
def test_fp32_fine_curvilinear_mesh(esdg, orc, N, av):
    """The throughput recipe at 256 x 256 curvilinear elements (a quarter
    of the benchmark's element size): the FP32 R against the FP64 oracle on
    the FP32-rounded state and bathymetry within 1e-5 of max |R| per field
    (measured 3e-7 to 3.3e-6).  On elements this small the metric terms vary
    little across an element; rounded at their own size they would move R by
    some 1e-4 of max |R| (the discrete metric identities the volume sums rely
    on would hold only to that rounding), stored relative to each element's
    middle node they are rounded at the size of their variation.  AV off, or
    on with the benchmark's parameters (no element of this smooth state gets
    viscosity, on either side).  With every element at eps0 the viscous term,
    a second derivative of the velocity, turns the FP32 rounding of u = hu/h
    into errors growing like 1 / element size^2: up to 5% of the viscous term
    at element corners here (4e-4 of max |R|), 0.3% at 64 x 64; that case is
    left to the coarse meshes of the tests below."""
    w = smooth_sweep(256, N, seed=3)
    b, h, hu, hv = _f32(w.b), _f32(w.h), _f32(w.hu), _f32(w.hv)
    kw = dict(av_on=0) if av == "off" else dict(av_on=1, eps0=0.025)
    s = esdg.Solver(0, 32)
    s.upload_mesh(w.mesh)
    P = esdg.default_params(N, limiter_on=1, **kw)
    s.set_params(P)
    s.set_bathymetry(b)
    s.set_state(h, hu, hv)
    got = s.rhs()
    s.close()
    Ro = orc.rhs(oparams(orc, P), w.mesh, b, h, hu, hv)
    for c in range(3):
        mx = np.abs(Ro[c]).max()
        rel = np.abs(got[c] - Ro[c]).max() / mx
        print(f"[parity] fp32 256x256 N={N} av={av} field {c}: err/max {rel:.2e}", flush=True)
        assert rel <= TOL32


@pytest.mark.parametrize("av", ["off", "saturated"])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_fp32_arithmetic(esdg, orc, N, av):
    """The FP32 kernels' own arithmetic: an affine 8 x 8 mesh of [0,10]^2,
    whose metric terms (0.625) and Jacobian are exact in FP32, state and
    bathymetry rounded to FP32 before both sides see them; the FP32 R
    against the FP64 oracle on those same inputs within 1e-5 of max |R|
    per field (measured: 1e-7 to 6e-7), limiter on, AV off or saturated
    (thresholds that give every element the full eps0).  On the indicator's
    sine ramp the FP32 rounding of the small modal energies moves eps
    itself, by up to 1e-3 relative at N = 8, which is the indicator's
    conditioning rather than the kernels' arithmetic; the curvilinear case
    above covers the ramp."""
    mesh = make_periodic_mesh(N, 8, 8, 10.0, 10.0, amp=0.0)
    rng = np.random.default_rng(60 + N)
    h = _f32(fourier_field(mesh, rng, 4, 0.5, 2.0))
    u = fourier_field(mesh, rng, 4, -0.49, 0.49)
    v = fourier_field(mesh, rng, 4, -0.49, 0.49)
    b = _f32(fourier_field(mesh, rng, 4, 0.0, 1.0))
    hu, hv = _f32(h * u), _f32(h * v)
    s = esdg.Solver(0, 32)
    s.upload_mesh(mesh)
    kw = dict(av_on=0) if av == "off" else dict(av_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-29.0)
    P = esdg.default_params(N, limiter_on=1, **kw)
    s.set_params(P)
    s.set_bathymetry(b)
    s.set_state(h, hu, hv)
    got = s.rhs()
    s.close()
    Ro = orc.rhs(oparams(orc, P), mesh, b, h, hu, hv)
    for c in range(3):
        mx = np.abs(Ro[c]).max()
        rel = np.abs(got[c] - Ro[c]).max() / mx
        print(f"[parity] fp32 arithmetic N={N} AV {av} field {c}: err/max {rel:.2e}", flush=True)
        assert rel <= TOL32


def test_full_size_sampled_parity(esdg, orc):
    """512 x 512 curvilinear elements, N = 7, AV and limiter on: the GPU
    right-hand side on the whole mesh, the oracle on 48 sampled elements."""
    w = smooth_sweep(512, 7, seed=3)
    s, P = make_solver(esdg, w)
    got = s.rhs()
    s.close()
    rng = np.random.default_rng(0)
    K = w.mesh.K
    sel = np.concatenate([[0, K - 1, 511, K - 512], rng.integers(0, K, 44)])
    need = np.zeros(K, bool)
    need[sel] = True
    Ro, fl = rhs_floor(orc, oparams(orc, P), w.mesh, w.b, w.h, w.hu, w.hv, need=need)
    check(got, Ro[:3], fl, "512^2 N=7 sampled rhs", sel=sel)


def test_nonfinite_state_is_reported(esdg):
    """A NaN in the state: the kernels run to completion and esdg_step
    reports ESDG_ENONFINITE (before the missing admissible step it causes)."""
    w = smooth_sweep(4, 3, seed=9)
    s, P = make_solver(esdg, w, av_on=1, limiter_on=1, eps0=0.05)
    s.step(1, 0.0)
    h = w.h.copy()
    h[5, 3] = np.nan
    s.set_state(h, w.hu, w.hv)
    for dt in (0.0, 1e-3):
        s.set_state(h, w.hu, w.hv)
        with pytest.raises(esdg.EsdgError) as ei:
            s.step(2, dt)
        assert ei.value.code == esdg.ENONFINITE, ei.value
    # a finite state afterwards steps normally
    s.set_state(w.h, w.hu, w.hv)
    t, st = s.step(1, 0.0)
    assert st == 0 and t > 0
    s.close()


def test_error_paths(esdg):
    mesh = make_periodic_mesh(3, 3, 3, 10.0, 10.0)
    s = esdg.Solver()
    with pytest.raises(esdg.EsdgError) as ei:
        s.rhs()
    assert ei.value.code == esdg.EINVAL
    bad = mesh.nbr_elem.copy()
    bad[0, 1] = 4
    with pytest.raises(esdg.EsdgError) as ei:
        s.upload_mesh(3, mesh.K, mesh.x, mesh.y, bad, mesh.nbr_side, mesh.flip)
    assert ei.value.code == esdg.EMESH
    # mirrored element -> negative Jacobian
    x = mesh.x.copy()
    x[4] = x[4].reshape(4, 4)[::-1].reshape(-1)
    with pytest.raises(esdg.EsdgError) as ei:
        s.upload_mesh(3, mesh.K, x, mesh.y, mesh.nbr_elem, mesh.nbr_side, mesh.flip)
    assert ei.value.code == esdg.EMESH
    # an empty mesh and degrees outside 2..8 are refused
    e0 = np.zeros((0, 16))
    with pytest.raises(esdg.EsdgError) as ei:
        s.upload_mesh(3, 0, e0, e0, np.zeros((0, 4), np.int32), np.zeros((0, 4), np.int8), np.zeros((0, 4), np.int8))
    assert ei.value.code == esdg.EINVAL
    for N in (1, 9):
        z = np.zeros((mesh.K, (N + 1) ** 2))
        with pytest.raises(esdg.EsdgError) as ei:
            s.upload_mesh(N, mesh.K, z, z, mesh.nbr_elem, mesh.nbr_side, mesh.flip)
        assert ei.value.code == esdg.EINVAL
    s.close()
