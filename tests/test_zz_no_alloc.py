"""GPU: esdg_diagnostics_noalloc, the variant of esdg_diagnostics whose
partial sums live in the library's fixed device array, against
esdg_diagnostics itself (the same kernels and summation order: bitwise
equal), on two calls in a row with the second mesh smaller than the first
(the array keeps the first call's rows; the second must not see them), and
the size limit of the array (65536 partial rows: at N = 7, 64 threads per
workgroup, more than 65536 elements are refused)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02221_amd.inputs import dam_break, smooth_sweep


@pytest.fixture(scope="module")
def esdg():
    from paper_1804_02221_amd import esdg as m
    m.lib()
    return m


def solver(esdg, w, **kw):
    s = esdg.Solver(0, 64)
    s.upload_mesh(w.mesh)
    P = esdg.default_params(w.mesh.N)
    for k, v in {**getattr(w, "params", {}), **kw}.items():
        setattr(P, k, v)
    s.set_params(P)
    s.set_bathymetry(w.b)
    s.set_state(w.h, w.hu, w.hv)
    return s


def test_noalloc_diagnostics_two_calls_second_smaller(esdg):
    cases = [
        (smooth_sweep(24, 5, seed=7, rotate_seed=5), dict(av_on=1, limiter_on=1, eps0=0.05,
                                                           sigma_min=-30.0, sigma_max=-1.0)),
        (dam_break(6, 3, seed=2, rotate_seed=1), dict(av_on=1, limiter_on=1, eps0=0.05)),
    ]
    nodes = [w.mesh.K * (w.mesh.N + 1) ** 2 for w, _ in cases]
    assert nodes[1] < nodes[0]
    for w, kw in cases:
        s = solver(esdg, w, **kw)
        s.step(2, 0.0)
        ref = s.diagnostics()
        got = s.diagnostics_noalloc()
        again = s.diagnostics_noalloc()
        print(f"[no-alloc] K={w.mesh.K} N={w.mesh.N}: mass {got[0]:.15e} entropy {got[3]:.15e} "
              f"min h {got[5]:.3e}", flush=True)
        assert np.array_equal(got, ref), (got, ref)
        assert np.array_equal(again, ref)
        s.close()


def test_noalloc_diagnostics_size_limit(esdg):
    w = smooth_sweep(257, 7, seed=3)
    s = solver(esdg, w)
    with pytest.raises(esdg.EsdgError) as ei:
        s.diagnostics_noalloc()
    assert ei.value.code == esdg.EINVAL
    assert "too large" in str(ei.value)
    # the existing entry point still serves this mesh
    d = s.diagnostics()
    assert np.isfinite(d).all()
    s.close()
