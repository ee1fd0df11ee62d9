"""The oracle's element loops run under OpenMP; every element writes only its
own nodes and the time-step reductions are minima, so its results must be
bitwise the same at any thread count.  Checked at 1 and at 4 threads on a
rough curved dam break (AV, limiter, wet/dry nodes, adaptive step)."""
import numpy as np
import pytest

from paper_1804_02221_amd.inputs import dam_break, smooth_sweep


@pytest.fixture
def threads(orc):
    keep = orc.get_threads()
    yield
    orc.set_threads(keep)


def run_all(orc, w, P):
    R = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    dt = orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)
    st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 3, 0.0)
    rng = np.random.default_rng(0)
    hn = w.h - 0.3 * rng.uniform(size=w.h.shape)
    lim = orc.limit(P, w.mesh, hn, w.hu, w.hv)
    return [*R, dt, *st[:3], np.array([st[3], st[4]]), *lim[:3], np.array([lim[3], lim[4]])]


@pytest.mark.parametrize("integrator", [0, 1])
def test_bitwise_at_any_thread_count(orc, threads, integrator):
    w = dam_break(12, 4, seed=2, rotate_seed=5)
    P = orc.params(4, av_on=1, limiter_on=1, eps0=0.05, integrator=integrator)
    orc.set_threads(1)
    one = run_all(orc, w, P)
    orc.set_threads(4)
    four = run_all(orc, w, P)
    for a, b in zip(one, four):
        assert np.array_equal(a, b)


def test_bitwise_rough_ramp(orc, threads):
    w = smooth_sweep(9, 6, seed=4, rotate_seed=2)
    w.hu = w.hu + 0.05 * np.random.default_rng(1).standard_normal(w.hu.shape)
    P = orc.params(6, av_on=1, limiter_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    orc.set_threads(1)
    one = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    orc.set_threads(3)
    three = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    assert (one[3] > 0).sum() > 10
    for a, b in zip(one, three):
        assert np.array_equal(a, b)
