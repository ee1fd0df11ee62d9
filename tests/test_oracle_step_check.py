"""Pins of the oracle's step adjustment (section 6: the step is chosen by a
CFL condition and adjusted when a smaller one proves necessary).  Reading:
a step (adaptive or fixed) is redone from W^n with half its size, at most
max_dt_retries times, when the limiter meets a negative element mean or when
the step is larger than twice the smaller of the CFL and viscous bounds of
the state it produced.  Each accepted or rejected size is re-derived here
from separate single steps of that size (no retries) and the bounds of their
results."""
import numpy as np
import pytest

from paper_1804_02221_amd import esdg as _esdg_params
from paper_1804_02221_amd.inputs import dam_break


def _params(orc, w, **kw):
    P = _esdg_params.default_params(3)
    for k, v in {**w.params, "eps0": 0.05, **kw}.items():
        setattr(P, k, v)
    return orc.params(3, **P.as_dict())


def _too_large(orc, P0, w, dt):
    """A single step of size dt (no retries): is it above twice the smaller
    CFL / viscous bound of its result, or does it meet a negative mean?"""
    h, hu, hv, _, st = orc.step(P0, w.mesh, w.b, w.h, w.hu, w.hv, 1, dt)
    bn = orc.dt(P0, w.mesh, w.b, h, hu, hv)
    return st != 0 or dt > 2.0 * min(bn[1], bn[2]), (h, hu, hv)


def test_adaptive_step_halved_until_admissible_for_its_result(orc):
    """SSPRK(3,3) on a dam break at rest: the flow starts within the first
    step, its result's CFL bound is 2.4 times below the step the start state
    allows, so the step is redone once at half the size."""
    w = dam_break(6, 3, seed=4, rotate_seed=3)
    P = _params(orc, w, integrator=1, max_dt_retries=4)
    P0 = _params(orc, w, integrator=1, max_dt_retries=0)
    dt0 = orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)[0]
    h, hu, hv, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0)
    assert st == 0
    k = int(round(np.log2(dt0 / t)))
    assert t == dt0 / 2 ** k and 1 <= k <= 4
    for j in range(k):
        assert _too_large(orc, P0, w, dt0 / 2 ** j)[0]
    bad, direct = _too_large(orc, P0, w, t)
    assert not bad
    # the kept result is the single step of the accepted size
    for a, b in zip((h, hu, hv), direct):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("integrator,cfl,lo,hi", [(0, 0.5, 0.0, 1.0), (1, 1.0, 1.0, 2.0)])
def test_adaptive_step_kept_when_admissible_for_its_result(orc, integrator, cfl, lo, hi):
    """The same state under LSRK(5,4) (step / result's bound 0.69) and under
    SSPRK(3,3) with cfl = 1 (1.20: above the result's bound, below twice
    it): the step the start state allows is kept as it is."""
    w = dam_break(6, 3, seed=4, rotate_seed=3)
    P = _params(orc, w, integrator=integrator, cfl=cfl, max_dt_retries=4)
    P0 = _params(orc, w, integrator=integrator, cfl=cfl, max_dt_retries=0)
    dt0 = orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)[0]
    h, hu, hv, _, _ = orc.step(P0, w.mesh, w.b, w.h, w.hu, w.hv, 1, dt0)
    bn = orc.dt(P0, w.mesh, w.b, h, hu, hv)
    assert lo < dt0 / min(bn[1], bn[2]) < hi
    _, _, _, t, st = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 1, 0.0)
    assert st == 0 and t == dt0


def test_fixed_step_is_checked_too(orc):
    """A caller's fixed step meets the same check: the SSPRK(3,3) step the
    start state allows, given as a fixed step, is redone once at half the
    size (callers clip the step to reach an end time this way)."""
    w = dam_break(6, 3, seed=4, rotate_seed=3)
    P = _params(orc, w, integrator=1, max_dt_retries=4)
    dt0 = orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)[0]
    _, _, _, t, _ = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 1, dt0)
    assert t == dt0 / 2


@pytest.mark.parametrize("fixed", [False, True])
def test_no_retries_no_check(orc, fixed):
    """Without retries a step is never redone, adaptive or fixed."""
    w = dam_break(6, 3, seed=4, rotate_seed=3)
    P = _params(orc, w, integrator=1, max_dt_retries=0)
    dt0 = orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)[0]
    _, _, _, t, _ = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 1, dt0 if fixed else 0.0)
    assert t == dt0


def test_next_step_takes_the_bounds_of_the_kept_state(orc):
    """Three adaptive steps in one call equal three calls of one step (the
    bounds evaluated for the check serve as the next step's)."""
    w = dam_break(6, 3, seed=4, rotate_seed=3)
    P = _params(orc, w, integrator=1, max_dt_retries=3)
    h3, hu3, hv3, t3, _ = orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 3, 0.0)
    h, hu, hv, t = w.h, w.hu, w.hv, 0.0
    for _ in range(3):
        h, hu, hv, t, _ = orc.step(P, w.mesh, w.b, h, hu, hv, 1, 0.0, t0=t)
    assert t == t3
    for a, b in zip((h, hu, hv), (h3, hu3, hv3)):
        assert np.array_equal(a, b)
