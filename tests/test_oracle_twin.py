"""The oracle's rounding twin (the same C source built with fused
multiply-adds), which the GPU parity floors use as the size of a pure
rounding-order difference: it must really round differently (else it adds
nothing to a floor), and it must agree with the plain build to rounding on
smooth states (else it would be a different method and widen the floors
beyond rounding)."""
import numpy as np
import pytest

import oracle as orc
from paper_1804_02221_amd.inputs import smooth_sweep

pytestmark = pytest.mark.skipif(not orc.host_has_fma(), reason="host CPU without FMA")


def _p(N, **kw):
    return orc.params(N, **kw)


@pytest.mark.parametrize("N,av", [(3, 0), (5, 1), (7, 0)])
def test_twin_rounds_differently_and_agrees_to_rounding(N, av):
    w = smooth_sweep(6, N, seed=11 + N, rotate_seed=N)
    P = _p(N, av_on=av, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    R0 = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    with orc.rounding_twin():
        R1 = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    assert orc.lib() is not None
    differs = False
    for c in range(3):
        d = np.abs(R1[c] - R0[c]).max()
        differs |= d > 0
        # the flux terms that cancel into R are ~1e3 |R| on these meshes
        assert d <= 1e-11 * np.abs(R0[c]).max(), (c, d)
    assert differs, "the twin build rounds exactly as the plain build"


def test_twin_switch_is_scoped():
    w = smooth_sweep(4, 3, seed=1)
    P = _p(3)
    a = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    with orc.rounding_twin():
        pass
    b = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv)
    for c in range(3):
        assert np.array_equal(a[c], b[c])
