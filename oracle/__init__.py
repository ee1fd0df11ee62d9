"""CPU oracle of the entropy-stable DGSEM shallow-water right-hand side.

TEST INFRASTRUCTURE ONLY: this package is the plain FP64 reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

The arithmetic lives in ``esdg_oracle.c`` (plain C, built with
``gcc -O2 -ffp-contract=off``; OpenMP over elements, bitwise independent of
the thread count); this module only marshals numpy arrays.

A second build of the same source, the *rounding twin*, lets the compiler
fuse multiplies and adds (``-ffp-contract=fast -mfma``): the same formulas
in the same order, rounded differently.  The tests use the spread between
the two builds as the size of a pure rounding-order difference (see
``tests/parity_floor.py``); ``rounding_twin()`` switches every function of
this module to it for the duration of a ``with`` block.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esdg_oracle.c")
_LIB = os.path.join(_HERE, "libesdg_oracle.so")
_LIB_TWIN = os.path.join(_HERE, "libesdg_oracle_fma.so")
_LIB_ASAN = os.path.join(_HERE, "libesdg_oracle_asan.so")

OK, EINVAL, ENOMEM, ENEGMEAN = 0, -1, -2, -5


_FLAGS = {_LIB: ["-ffp-contract=off"], _LIB_TWIN: ["-ffp-contract=fast", "-mfma", "-mavx2"],
          # AddressSanitizer + UndefinedBehaviorSanitizer build (tests load it in a
          # process that preloads the ASan runtime; see use_sanitized)
          _LIB_ASAN: ["-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                      "-fno-omit-frame-pointer", "-g"]}


def _build_one(path: str, force: bool) -> None:
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", *_FLAGS[path], "-fno-fast-math", "-std=c11",
                               "-fopenmp", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile the oracle shared library and its rounding twin in place (gcc,
    no fast-math)."""
    _build_one(_LIB, force)
    _build_one(_LIB_TWIN, force)
    return _LIB


def build_sanitized(force: bool = True) -> str:
    """Compile the AddressSanitizer/UBSan build of the oracle in place."""
    _build_one(_LIB_ASAN, force)
    return _LIB_ASAN


def use_sanitized() -> None:
    """Switch every function of this module to the sanitizer build, for the
    rest of the process.  The process must have the ASan runtime loaded
    first (LD_PRELOAD of gcc's libasan.so)."""
    global _active
    _active = _LIB_ASAN


def host_has_fma() -> bool:
    """True when the host CPU executes the twin's fused multiply-adds."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    fl = line.split()
                    return "fma" in fl and "avx2" in fl
    except OSError:
        pass
    return False


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("h_tol", C.c_double), ("eps0", C.c_double),
                ("sigma_min", C.c_double), ("sigma_max", C.c_double), ("cfl", C.c_double),
                ("cfl_visc", C.c_double), ("surface_flux", C.c_int), ("av_on", C.c_int),
                ("limiter_on", C.c_int), ("integrator", C.c_int), ("max_dt_retries", C.c_int)]


class _Mesh(C.Structure):
    _fields_ = [("N", C.c_int), ("K", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p),
                ("nbr_elem", C.c_void_p), ("nbr_side", C.c_void_p), ("flip", C.c_void_p)]


class _Parts(C.Structure):
    _fields_ = [("Lvol", C.c_void_p * 3), ("S", C.c_void_p * 3), ("Lv", C.c_void_p * 3),
                ("grad", C.c_void_p * 4)]


_libs = {}
_active = _LIB


@contextlib.contextmanager
def rounding_twin():
    """Within the block every function of this module runs the twin build."""
    global _active
    if not host_has_fma():
        raise RuntimeError("the rounding twin needs a host CPU with FMA and AVX2")
    prev, _active = _active, _LIB_TWIN
    try:
        yield
    finally:
        _active = prev


def lib():
    path = _active
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _build_one(path, force=True)
        L = C.CDLL(path)
        P, I, I64 = C.c_void_p, C.c_int, C.c_int64
        L.orc_operators.argtypes = [I, P, P, P, P, P, P]
        L.orc_geometry.argtypes = [I, I64, P, P, P, P, P, P, P]
        L.orc_volume_flux.argtypes = [C.c_double, C.c_double, P, P, P, P]
        L.orc_volume_flux.restype = None
        L.orc_surface_flux.argtypes = [P, P, C.c_double, P, C.c_double, C.c_double, C.c_double, P]
        L.orc_surface_flux.restype = None
        L.orc_indicator.argtypes = [P, I, I64, P, P]
        L.orc_rhs.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_limit.argtypes = [P, P, P, P, P, P]
        L.orc_dt.argtypes = [P, P, P, P, P, P, P]
        L.orc_step.argtypes = [P, P, P, P, P, P, I, C.c_double, P, P]
        L.orc_diagnostics.argtypes = [P, P, P, P, P, P, P]
        L.orc_lsrk_coefficients.argtypes = [P, P]
        L.orc_set_threads.argtypes = [I]
        L.orc_get_threads.argtypes = []
        L.orc_rhs_vjp.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_gauge_adjoint.argtypes = [P, P, P, P, P, P, I, C.c_double, I, P, P, P, P, P, P,
                                        P, P, P, P]
        _libs[path] = L
    return _libs[path]


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_sigma(N: int):
    """Indicator thresholds s0 -+ 1 with s0 = -4 log10(N) (the paper gives no
    values; this follows the N^-4 scaling of the indicator it cites)."""
    s0 = -4.0 * math.log10(N)
    return s0 - 1.0, s0 + 1.0


def params(N: int = 3, **kw) -> Params:
    smin, smax = default_sigma(N)
    d = dict(g=9.81, h_tol=1e-4, eps0=0.0, sigma_min=smin, sigma_max=smax, cfl=0.5,
             cfl_visc=0.5, surface_flux=0, av_on=0, limiter_on=0, integrator=0,
             max_dt_retries=0)
    d.update(kw)
    return Params(**d)


class _MeshRef:
    """Keeps the contiguous arrays alive while C holds pointers to them."""

    def __init__(self, mesh):
        self.N = int(mesh.N)
        self.x = _f64(mesh.x)
        self.y = _f64(mesh.y)
        self.ne = np.ascontiguousarray(mesh.nbr_elem, dtype=np.int32)
        self.ns = np.ascontiguousarray(mesh.nbr_side, dtype=np.int8)
        self.fl = np.ascontiguousarray(mesh.flip, dtype=np.int8)
        self.K = self.x.shape[0]
        self.c = _Mesh(self.N, self.K, _p(self.x), _p(self.y), _p(self.ne), _p(self.ns), _p(self.fl))


def _check(st, what):
    if st not in (OK,):
        raise RuntimeError(f"oracle {what} failed with status {st}")


def operators(N: int) -> dict:
    n1 = N + 1
    out = {k: np.zeros((n1, n1)) for k in ("D", "Dtilde", "Dhat", "Vinv")}
    xi, w = np.zeros(n1), np.zeros(n1)
    _check(lib().orc_operators(N, _p(xi), _p(w), _p(out["D"]), _p(out["Dtilde"]),
                               _p(out["Dhat"]), _p(out["Vinv"])), "operators")
    out["xi"], out["w"] = xi, w
    return out


def geometry(mesh) -> dict:
    M = _MeshRef(mesh)
    out = {k: np.zeros_like(M.x) for k in ("xxi", "xeta", "yxi", "yeta", "J")}
    _check(lib().orc_geometry(M.N, M.K, _p(M.x), _p(M.y), _p(out["xxi"]), _p(out["xeta"]),
                              _p(out["yxi"]), _p(out["yeta"]), _p(out["J"])), "geometry")
    return out


def volume_flux(g, h_tol, wa, wb):
    wa, wb = _f64(wa), _f64(wb)
    F, G = np.zeros(3), np.zeros(3)
    lib().orc_volume_flux(g, h_tol, _p(wa), _p(wb), _p(F), _p(G))
    return F, G


def surface_flux(P: Params, wm, bm, wp, bp, nx, ny):
    wm, wp = _f64(wm), _f64(wp)
    F = np.zeros(3)
    lib().orc_surface_flux(C.byref(P), _p(wm), float(bm), _p(wp), float(bp), float(nx),
                           float(ny), _p(F))
    return F


def indicator(P: Params, N: int, h) -> np.ndarray:
    h = _f64(h)
    K = h.shape[0]
    eps = np.zeros(K)
    _check(lib().orc_indicator(C.byref(P), N, K, _p(h), _p(eps)), "indicator")
    return eps


def rhs(P: Params, mesh, b, h, hu, hv, need=None, parts: bool = False):
    """R = dW/dt.  ``need``: optional boolean [K] mask of elements to
    evaluate (others are left zero).  With ``parts`` also returns the volume
    + surface operator L, the source S, the viscous term L^v and the BR1
    gradients (U1, U2, V1, V2)."""
    M = _MeshRef(mesh)
    b, h, hu, hv = _f64(b), _f64(h), _f64(hu), _f64(hv)
    Rh, Rhu, Rhv = np.zeros_like(h), np.zeros_like(h), np.zeros_like(h)
    eps = np.zeros(M.K)
    nd = None if need is None else np.ascontiguousarray(need, dtype=np.uint8)
    pr, keep = None, None
    if parts:
        keep = {k: [np.zeros_like(h) for _ in range(n)] for k, n in
                (("L", 3), ("S", 3), ("Lv", 3), ("grad", 4))}
        pr = _Parts((C.c_void_p * 3)(*[a.ctypes.data for a in keep["L"]]),
                    (C.c_void_p * 3)(*[a.ctypes.data for a in keep["S"]]),
                    (C.c_void_p * 3)(*[a.ctypes.data for a in keep["Lv"]]),
                    (C.c_void_p * 4)(*[a.ctypes.data for a in keep["grad"]]))
    st = lib().orc_rhs(C.byref(P), C.byref(M.c), _p(b), _p(h), _p(hu), _p(hv), _p(Rh),
                       _p(Rhu), _p(Rhv), _p(eps), _p(nd), C.byref(pr) if pr is not None else None)
    _check(st, "rhs")
    if parts:
        return Rh, Rhu, Rhv, eps, keep
    return Rh, Rhu, Rhv, eps


def limit(P: Params, mesh, h, hu, hv):
    M = _MeshRef(mesh)
    h, hu, hv = _f64(h).copy(), _f64(hu).copy(), _f64(hv).copy()
    nl = C.c_int64(0)
    st = lib().orc_limit(C.byref(P), C.byref(M.c), _p(h), _p(hu), _p(hv), C.byref(nl))
    if st not in (OK, ENEGMEAN):
        _check(st, "limit")
    return h, hu, hv, int(nl.value), st


def dt(P: Params, mesh, b, h, hu, hv):
    M = _MeshRef(mesh)
    out = np.zeros(4)
    _check(lib().orc_dt(C.byref(P), C.byref(M.c), _p(_f64(b)), _p(_f64(h)), _p(_f64(hu)),
                        _p(_f64(hv)), _p(out)), "dt")
    return out  # dt, dt_cfl, dt_visc, dt_pos


def step(P: Params, mesh, b, h, hu, hv, nsteps: int, dt_fixed: float = 0.0, t0: float = 0.0):
    M = _MeshRef(mesh)
    h, hu, hv = _f64(h).copy(), _f64(hu).copy(), _f64(hv).copy()
    t = C.c_double(t0)
    last = C.c_double(0.0)
    st = lib().orc_step(C.byref(P), C.byref(M.c), _p(_f64(b)), _p(h), _p(hu), _p(hv),
                        int(nsteps), float(dt_fixed), C.byref(t), C.byref(last))
    if st not in (OK, ENEGMEAN):
        _check(st, "step")
    return h, hu, hv, t.value, st


def diagnostics(P: Params, mesh, b, h, hu, hv):
    """mass, mom_x, mom_y, entropy E, dE/dt, min h, max h, #dry nodes."""
    M = _MeshRef(mesh)
    out = np.zeros(8)
    _check(lib().orc_diagnostics(C.byref(P), C.byref(M.c), _p(_f64(b)), _p(_f64(h)),
                                 _p(_f64(hu)), _p(_f64(hv)), _p(out)), "diagnostics")
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's element loops (results do not depend on it)."""
    _check(lib().orc_set_threads(int(n)), "set_threads")


def get_threads() -> int:
    return int(lib().orc_get_threads())


def lsrk_coefficients():
    a, b = np.zeros(5), np.zeros(5)
    lib().orc_lsrk_coefficients(_p(a), _p(b))
    return a, b


def rhs_vjp(P: Params, mesh, b, h, hu, hv, lh, lhu, lhv):
    """Reverse mode of the inviscid right-hand side at (W, b): returns
    (dR/dW)^T lam as (gh, ghu, ghv) and (dR/db)^T lam as gb."""
    M = _MeshRef(mesh)
    args = [_f64(a) for a in (b, h, hu, hv, lh, lhu, lhv)]
    out = [np.zeros_like(args[1]) for _ in range(4)]
    _check(lib().orc_rhs_vjp(C.byref(P), C.byref(M.c), *[_p(a) for a in args],
                             *[_p(o) for o in out]), "rhs_vjp")
    return tuple(out)


def gauge_adjoint(P: Params, mesh, b, h0, hu0, hv0, nsteps: int, dt: float, gelem, gxi, geta,
                  target, gradient: bool = True) -> dict:
    """Gauge-misfit loss L = 1/2 sum_n sum_g (H_g(t_n) - target[n-1, g])^2 dt over
    nsteps fixed LSRK(5,4) or SSPRK(3,3) steps (P.integrator), the surface
    H = h + b at the gauges (element gelem[g], reference point (gxi[g],
    geta[g])).  Returns loss, H [nsteps, ng] and, with gradient, gb = dL/db
    (initial state fixed) and gW0 = dL/dW(0)."""
    M = _MeshRef(mesh)
    b, h0, hu0, hv0 = _f64(b), _f64(h0), _f64(hu0), _f64(hv0)
    gelem = np.ascontiguousarray(gelem, dtype=np.int32)
    gxi, geta = _f64(gxi), _f64(geta)
    ng = gelem.shape[0]
    target = _f64(target).reshape(nsteps, ng)
    loss = np.zeros(1)
    H = np.zeros((nsteps, ng))
    out = [np.zeros_like(h0) for _ in range(4)] if gradient else [None] * 4
    st = lib().orc_gauge_adjoint(C.byref(P), C.byref(M.c), _p(b), _p(h0), _p(hu0), _p(hv0),
                                 int(nsteps), float(dt), int(ng), _p(gelem), _p(gxi), _p(geta),
                                 _p(target), _p(loss), _p(H), *[_p(o) for o in out])
    _check(st, "gauge_adjoint")
    r = dict(loss=float(loss[0]), H=H)
    if gradient:
        r.update(gb=out[0], gh0=out[1], ghu0=out[2], ghv0=out[3])
    return r
