"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, -fno-sanitize-recover): its entry points -- operators, geometry, the
right-hand side with AV, its reverse mode, limiter, time-step bounds, steps
of both integrators, diagnostics, the gauge-loss adjoint -- on small
periodic and walled meshes, in a child process that preloads the ASan
runtime.  Any out-of-bounds access, use after free or undefined behaviour
aborts the child with a report."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np, sys
sys.path.insert(0, ROOT)
import oracle as orc
orc.use_sanitized()
orc.set_threads(2)
from paper_1804_02221_amd.inputs import smooth_sweep, dam_break, make_box_mesh
for N in (2, 3, 5):
    orc.operators(N)
    w = smooth_sweep(4, N, seed=N, rotate_seed=N)
    P = orc.params(N, av_on=1, limiter_on=1, eps0=0.05, sigma_min=-30.0, sigma_max=-1.0)
    orc.geometry(w.mesh)
    R = orc.rhs(P, w.mesh, w.b, w.h, w.hu, w.hv, parts=True)
    Pi = orc.params(N, limiter_on=1)
    orc.rhs_vjp(Pi, w.mesh, w.b, w.h, w.hu, w.hv, R[0], R[1], R[2])
    orc.dt(P, w.mesh, w.b, w.h, w.hu, w.hv)
    orc.limit(P, w.mesh, w.h - 0.9, w.hu, w.hv)
    for integ in (0, 1):
        P.integrator = integ
        orc.step(P, w.mesh, w.b, w.h, w.hu, w.hv, 2, 0.0)
    orc.diagnostics(P, w.mesh, w.b, w.h, w.hu, w.hv)
d = dam_break(4, 3, seed=2, rotate_seed=1)
Pd = orc.params(3, **{k: v for k, v in d.params.items() if k in ("g", "eps0", "cfl", "av_on", "limiter_on")})
orc.step(Pd, d.mesh, d.b, d.h, d.hu, d.hv, 3, 0.0)
m = make_box_mesh(3, 3, 3, -1.0, -1.0, 2.0, 2.0, amp=0.1, walls_x=True, walls_y=True, rotate_seed=1)
h = 1.0 + 0.1 * np.sin(m.x) * np.cos(m.y)
b = 0.1 * np.cos(m.x)
Pw = orc.params(3, limiter_on=1)
orc.rhs(Pw, m, b, h, 0.2 * h, -0.1 * h)
orc.step(Pw, m, b, h, 0.2 * h, -0.1 * h, 2, 0.0)
rng = np.random.default_rng(0)
ge = rng.integers(0, m.K, 3).astype(np.int32)
gx, gy = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
orc.gauge_adjoint(Pw, m, b, h, 0.2 * h, -0.1 * h, 3, 1e-3, ge, gx, gy, np.zeros((3, 3)))
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_ub_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime not found")
    oracle.build_sanitized(force=False)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHILD.replace("ROOT", repr(ROOT))], capture_output=True, text=True,
                       env=env, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "sanitized oracle ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
