"""GPU: graph replay of esdg_step (esdg_set_graphs) against eager launches.

Two contexts on the same problem, one replaying captured step graphs, one
launching every kernel; after every call the states and times must be
bitwise equal.  Between the calls the program does its own eager work and
synchronises (state downloads, diagnostics, a parameter change, a new state,
a stage-variant change, fixed steps of two sizes), so every replay is
checked, not only the first."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02221_amd.inputs import dam_break, smooth_sweep


@pytest.fixture(scope="module")
def esdg():
    from paper_1804_02221_amd import esdg as m
    m.lib()
    return m


def pair(esdg, w, **kw):
    out = []
    for graphs in (True, False):
        s = esdg.Solver(0, 64)
        s.set_graphs(graphs)
        s.upload_mesh(w.mesh)
        P = esdg.default_params(w.mesh.N)
        for k, v in {**w.params, **kw}.items():
            setattr(P, k, v)
        s.set_params(P)
        s.set_bathymetry(w.b)
        s.set_state(w.h, w.hu, w.hv)
        out.append(s)
    return out


def same(a, b, what):
    ga, gb = a.get_state(), b.get_state()
    for c in range(3):
        assert np.array_equal(ga[c], gb[c]), f"{what}: field {c} differs by {np.abs(ga[c] - gb[c]).max():.3e}"
    assert a.get_time() == b.get_time(), what


@pytest.mark.parametrize("integrator", [0, 1])
def test_graph_steps_equal_eager_steps(esdg, integrator):
    w = dam_break(10, 4, seed=2, rotate_seed=1)
    g, e = pair(esdg, w, av_on=1, limiter_on=1, eps0=0.05, integrator=integrator)
    calls = [("first step (eager in both)", lambda s: s.step(1, 0.0, raise_negmean=False)),
             ("three adaptive steps", lambda s: s.step(3, 0.0, raise_negmean=False)),
             ("diagnostics", lambda s: s.diagnostics()),
             ("four adaptive steps", lambda s: s.step(4, 0.0, raise_negmean=False)),
             ("fixed step", lambda s: s.step(3, 2e-4, raise_negmean=False)),
             ("another fixed step", lambda s: s.step(2, 1e-4, raise_negmean=False)),
             ("adaptive again", lambda s: s.step(5, 0.0, raise_negmean=False)),
             ("stage variant 1", lambda s: (s.set_stage_variant(1), s.step(3, 0.0, raise_negmean=False))),
             ("stage variant 0", lambda s: (s.set_stage_variant(0), s.step(2, 0.0, raise_negmean=False)))]
    for what, f in calls:
        f(g)
        f(e)
        same(g, e, what)
    # a parameter change (the captured graphs hold the parameters by value)
    for s in (g, e):
        P = s.get_params()
        P.cfl = 0.3
        P.eps0 = 0.02
        s.set_params(P)
        s.step(4, 0.0, raise_negmean=False)
    same(g, e, "after set_params")
    # a new state (the graphs stay valid: they hold buffer addresses, not data)
    h2 = w.h * 0.9
    for s in (g, e):
        s.set_state(h2, w.hu, w.hv)
        s.step(6, 0.0, raise_negmean=False)
    same(g, e, "after set_state")
    g.close()
    e.close()


def test_graph_steps_plain_method(esdg):
    """The plain method (no AV, no limiter, LSRK(5,4)) on a smooth state."""
    w = smooth_sweep(8, 5, seed=3, rotate_seed=2)
    g, e = pair(esdg, w, av_on=0, limiter_on=0)
    for n in (1, 2, 5, 1, 7):
        g.step(n, 0.0)
        e.step(n, 0.0)
        same(g, e, f"{n} steps")
    g.close()
    e.close()


def test_ensemble_graph_steps_equal_eager_steps(esdg):
    """An ensemble (three degrees, uneven grids) stepping with graph replay
    per degree group against the same ensemble launching every kernel."""
    from paper_1804_02221_amd.inputs import ensemble_member
    specs = [(8, 3, True, 41), (12, 5, False, 42), (6, 7, True, 43), (10, 3, False, 44)]
    members = [ensemble_member(*sp) for sp in specs]
    ens = []
    for graphs in (True, False):
        e = esdg.Ensemble(0, 64)
        for w in members:
            e.add_workload(w)
        e.set_graphs(graphs)
        ens.append(e)
    for n in (1, 4, 2, 6):
        for e in ens:
            e.step(n, raise_negmean=False)
        for i in range(len(members)):
            a, b = ens[0].get_state(i), ens[1].get_state(i)
            for c in range(3):
                assert np.array_equal(a[c], b[c]), (n, i, c)
            assert ens[0].get_time(i) == ens[1].get_time(i)
    for e in ens:
        e.close()
