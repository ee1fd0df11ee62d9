"""GPU: the compiled variants of the stage kernel (tile, register budget,
partner-loop unroll) give bitwise-identical results at every degree, and the
autotuner neither changes the state nor the following steps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02221_amd.inputs import dam_break, smooth_sweep

KW = dict(av_on=1, limiter_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)


@pytest.fixture(scope="module")
def esdg():
    from paper_1804_02221_amd import esdg as m
    m.lib()
    return m


def solver(esdg, w, **kw):
    s = esdg.Solver(0, 64)
    s.upload_mesh(w.mesh)
    s.set_params(esdg.default_params(w.mesh.N, **{**KW, **kw}))
    s.set_bathymetry(w.b)
    s.set_state(w.h, w.hu, w.hv)
    return s


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_variants_bitwise_equal(esdg, N):
    w = smooth_sweep(5, N, seed=60 + N, rotate_seed=N)
    w.hu = w.hu + 0.05 * np.random.default_rng(N).standard_normal(w.hu.shape)
    out = []
    for v in range(esdg.STAGE_VARIANTS):
        s = solver(esdg, w)
        s.set_stage_variant(v)
        r = s.rhs()
        s.step(2, 0.0)
        out.append((r, s.get_state(), s.get_time()))
        s.close()
    for o in out[1:]:
        for c in range(3):
            assert np.array_equal(out[0][0][c], o[0][c])
            assert np.array_equal(out[0][1][c], o[1][c])
        assert out[0][2] == o[2]


def test_autotune_leaves_the_solution_alone(esdg):
    w = dam_break(6, 5, seed=3, rotate_seed=1)
    ref = solver(esdg, w)
    ref.step(2, 0.0)
    s = solver(esdg, w)
    s.step(1, 0.0)
    before, t_before = s.get_state(), s.get_time()
    choice, ms = s.autotune(3)
    assert choice in range(esdg.STAGE_VARIANTS) and ms.shape == (esdg.STAGE_VARIANTS,) and np.all(ms > 0)
    assert ms[choice] == ms.min()
    after, t_after = s.get_state(), s.get_time()
    for a_, b_ in zip(before, after):
        assert np.array_equal(a_, b_)
    assert t_before == t_after
    s.step(1, 0.0)
    for a_, b_ in zip(s.get_state(), ref.get_state()):
        assert np.array_equal(a_, b_)
    assert s.get_time() == ref.get_time()
    s.close()
    ref.close()


def test_ensemble_autotune(esdg):
    ws = [dam_break(4, 3, seed=21), smooth_sweep(4, 7, seed=22), dam_break(5, 7, seed=23, rotate_seed=2)]
    ens = esdg.Ensemble(0, 64)
    ids = [ens.add_workload(w, **KW) for w in ws]
    ch = ens.autotune(3)
    assert set(ch) == {3, 7} and set(ch.values()) <= set(range(esdg.STAGE_VARIANTS))
    ens.step(2)
    for w, i in zip(ws, ids):
        s = solver(esdg, w)
        s.step(2, 0.0)
        for a_, b_ in zip(ens.get_state(i), s.get_state()):
            assert np.array_equal(a_, b_)
        s.close()
    ens.close()
