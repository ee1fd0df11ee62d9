"""ctypes binding of the C ABI in ``include/esdg.h`` (argument marshalling only).

Every computation runs in the HIP library ``libesdg.so`` next to this file;
there is no CPU fallback: if the library is missing, loading it raises.
Arrays may be numpy float64 arrays (host memory) or contiguous float64 torch
CUDA tensors (device memory, passed by pointer; the copy is ordered on the
solver's stream).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesdg.so")

OK, EINVAL, ENOMEM, EHIP, EMESH, ENEGMEAN, EDTPOS, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
STAGE_VARIANTS = 5   # ESDG_STAGE_VARIANTS of include/esdg.h
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", EMESH: "EMESH", ENEGMEAN: "ENEGMEAN",
          EDTPOS: "EDTPOS", ENONFINITE: "ENONFINITE"}


class EsdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("h_tol", C.c_double), ("eps0", C.c_double),
                ("sigma_min", C.c_double), ("sigma_max", C.c_double), ("cfl", C.c_double),
                ("cfl_visc", C.c_double), ("surface_flux", C.c_int), ("av_on", C.c_int),
                ("limiter_on", C.c_int), ("integrator", C.c_int), ("max_dt_retries", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def use_sanitized_build() -> None:
    """Load libesdg_hostsan.so instead: the same kernels, with the host code
    built under AddressSanitizer (``build.py --sanitize``).  Call before the
    first use, in a process that preloads gcc's ASan runtime."""
    global LIB_PATH
    if _lib is not None:
        raise RuntimeError("the library is already loaded")
    LIB_PATH = os.path.join(os.path.dirname(LIB_PATH), "libesdg_hostsan.so")


def lib() -> C.CDLL:
    """Load libesdg.so (built by ``paper_1804_02221_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1804_02221_amd/build.py "
                              "(there is no fallback implementation)")
        # torch ships its own HIP runtime; loaded first, it is the one runtime
        # of the process and the library binds to it (loaded after the
        # library, a second runtime would come up beside it and torch would
        # see no GPU)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
        sig = {
            "esdg_default_params": ([P, I], None),
            "esdg_create": ([P, I, I], I),
            "esdg_destroy": ([P], I),
            "esdg_set_stream": ([P, P], I),
            "esdg_set_params": ([P, P], I),
            "esdg_get_params": ([P, P], I),
            "esdg_upload_mesh": ([P, I, I64, P, P, P, P, P, I], I),
            "esdg_set_bathymetry": ([P, P, I], I),
            "esdg_set_state": ([P, P, P, P, I], I),
            "esdg_get_state": ([P, P, P, P, I], I),
            "esdg_rhs": ([P, P, P, P, I], I),
            "esdg_limit": ([P, P], I),
            "esdg_compute_dt": ([P, P], I),
            "esdg_step": ([P, I, D, P], I),
            "esdg_get_time": ([P, P], I),
            "esdg_set_time": ([P, D], I),
            "esdg_diagnostics": ([P, P], I),
            "esdg_diagnostics_noalloc": ([P, P], I),
            "esdg_get_eps": ([P, P, I], I),
            "esdg_step_stats": ([P, P, P], I),
            "esdg_get_geometry": ([P, P, P, P, P, P, I], I),
            "esdg_profile": ([P, I], I),
            "esdg_profile_read": ([P, P, P, P, P], I),
            "esdg_last_error": ([P], C.c_char_p),
            "esdg_abi_version": ([], I),
            "esdg_ensemble_create": ([P, I, I], I),
            "esdg_ensemble_destroy": ([P], I),
            "esdg_ensemble_add": ([P, P, I, I64, P, P, P, P, P, P, P, P, P, P], I),
            "esdg_ensemble_build": ([P], I),
            "esdg_ensemble_step": ([P, I], I),
            "esdg_ensemble_set_graphs": ([P, I], I),
            "esdg_ensemble_size": ([P, P], I),
            "esdg_ensemble_get_state": ([P, I, P, P, P, I], I),
            "esdg_ensemble_get_time": ([P, I, P], I),
            "esdg_ensemble_last_error": ([P], C.c_char_p),
            "esdg_ensemble_degrees": ([P, P, P], I),
            "esdg_ensemble_autotune": ([P, I, P], I),
            "esdg_autotune": ([P, I, P, P], I),
            "esdg_set_stage_variant": ([P, I], I),
            "esdg_set_graphs": ([P, I], I),
            "esdg_rhs_vjp": ([P, P, P, P, P, P, P, P, I], I),
            "esdg_set_gauges": ([P, I, P, P, P], I),
            "esdg_gauge_values": ([P, P, I], I),
            "esdg_adjoint_forward": ([P, I, D, I, P, I, P, P], I),
            "esdg_adjoint_backward": ([P, D, P, P, P, P, I], I),
            "esdg_profile_read_adjoint": ([P, P, P], I),
            "esdg_profile_read_kernels": ([P, P, P], I),
            "esdg_lds_bandwidth": ([I, P], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    """Names of the ABI entry points the binding expects."""
    lib()
    return [n for n in dir(_lib) if n.startswith("esdg_")]


def default_params(N: int = 3, **kw) -> Params:
    p = Params()
    lib().esdg_default_params(C.byref(p), int(N))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def lds_bandwidth(device: int = 0) -> float:
    """Measured LDS read bandwidth (bytes/s) in the volume term's pattern."""
    out = C.c_double(0.0)
    st = lib().esdg_lds_bandwidth(int(device), C.byref(out))
    if st != OK:
        raise EsdgError(st, "esdg_lds_bandwidth failed")
    return out.value


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Arg:
    """Pointer + memory kind of a float64 array argument."""

    def __init__(self, a, n=None, dtype=np.float64):
        if _is_torch(a):
            import torch
            want = {np.float64: torch.float64, np.int32: torch.int32, np.int8: torch.int8}[dtype]
            if a.dtype != want or not a.is_contiguous() or not a.is_cuda:
                raise TypeError(f"expected a contiguous CUDA tensor of {want}")
            self.keep = a
            self.ptr = C.c_void_p(a.data_ptr())
            self.mem = 1
            size = a.numel()
        else:
            arr = np.ascontiguousarray(a, dtype=dtype)
            self.keep = arr
            self.ptr = arr.ctypes.data_as(C.c_void_p)
            self.mem = 0
            size = arr.size
        if n is not None and size != n:
            raise ValueError(f"array has {size} entries, expected {n}")


class Solver:
    """One solver context (one mesh, one degree) on one GPU."""

    def __init__(self, device: int = 0, precision: int = 64, stream=None):
        self._ctx = C.c_void_p()
        st = lib().esdg_create(C.byref(self._ctx), int(device), int(precision))
        if st != OK:
            raise EsdgError(st, "esdg_create failed")
        self.device = device
        self.precision = precision
        self.N = None
        self.K = None
        self.n_gauges = 0
        if stream is not None:
            self.set_stream(stream)

    # -- plumbing -------------------------------------------------------
    def _check(self, st):
        if st != OK:
            raise EsdgError(st, lib().esdg_last_error(self._ctx).decode())
        return st

    def close(self):
        if self._ctx:
            lib().esdg_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def n_nodes(self):
        return 0 if self.N is None else self.K * (self.N + 1) ** 2

    def set_stream(self, stream):
        """stream: an int handle or a torch.cuda.Stream."""
        h = getattr(stream, "cuda_stream", stream)
        self._check(lib().esdg_set_stream(self._ctx, C.c_void_p(int(h) if h else 0)))

    def set_params(self, P: Params | None = None, **kw):
        if P is None:
            P = default_params(self.N or 3)
        for k, v in kw.items():
            setattr(P, k, v)
        self._check(lib().esdg_set_params(self._ctx, C.byref(P)))
        return P

    def get_params(self) -> Params:
        P = Params()
        self._check(lib().esdg_get_params(self._ctx, C.byref(P)))
        return P

    # -- setup ----------------------------------------------------------
    def upload_mesh(self, N, K=None, x=None, y=None, nbr_elem=None, nbr_side=None, flip=None):
        """upload_mesh(mesh) with a mesh object (N, x, y, nbr_elem, nbr_side,
        flip attributes) or upload_mesh(N, K, x, y, nbr_elem, nbr_side, flip)."""
        if not isinstance(N, int):
            m = N
            N, x, y, nbr_elem, nbr_side, flip = m.N, m.x, m.y, m.nbr_elem, m.nbr_side, m.flip
            K = x.shape[0]
        n = K * (N + 1) ** 2
        ax, ay = _Arg(x, n), _Arg(y, n)
        ne = _Arg(nbr_elem, 4 * K, np.int32)
        ns = _Arg(nbr_side, 4 * K, np.int8)
        fl = _Arg(flip, 4 * K, np.int8)
        mems = {ax.mem, ay.mem, ne.mem, ns.mem, fl.mem}
        if len(mems) != 1:
            raise ValueError("mix of host and device arrays")
        self._check(lib().esdg_upload_mesh(self._ctx, int(N), int(K), ax.ptr, ay.ptr, ne.ptr, ns.ptr,
                                           fl.ptr, ax.mem))
        self.N, self.K = int(N), int(K)
        self.n_gauges = 0

    def set_bathymetry(self, b):
        a = _Arg(b, self.n_nodes)
        self._check(lib().esdg_set_bathymetry(self._ctx, a.ptr, a.mem))

    def set_state(self, h, hu, hv):
        a, b, c = _Arg(h, self.n_nodes), _Arg(hu, self.n_nodes), _Arg(hv, self.n_nodes)
        if len({a.mem, b.mem, c.mem}) != 1:
            raise ValueError("mix of host and device arrays")
        self._check(lib().esdg_set_state(self._ctx, a.ptr, b.ptr, c.ptr, a.mem))

    # -- outputs ----------------------------------------------------------
    def _outs(self, count, size, device):
        if device:
            import torch
            return [torch.empty(size, dtype=torch.float64, device=f"cuda:{self.device}") for _ in range(count)]
        return [np.empty(size) for _ in range(count)]

    def _shape(self, arrs):
        if self.N is None:
            return arrs
        return [a.reshape(self.K, (self.N + 1) ** 2) for a in arrs]

    def get_state(self, device: bool = False):
        outs = self._outs(3, self.n_nodes, device)
        ps = [_Arg(o) for o in outs]
        self._check(lib().esdg_get_state(self._ctx, ps[0].ptr, ps[1].ptr, ps[2].ptr, ps[0].mem))
        return self._shape(outs)

    def rhs(self, device: bool = False):
        outs = self._outs(3, self.n_nodes, device)
        ps = [_Arg(o) for o in outs]
        self._check(lib().esdg_rhs(self._ctx, ps[0].ptr, ps[1].ptr, ps[2].ptr, ps[0].mem))
        return self._shape(outs)

    def limit(self):
        """Returns (n_limited, status); status ENEGMEAN is not raised."""
        n = C.c_int64(0)
        st = lib().esdg_limit(self._ctx, C.byref(n))
        if st not in (OK, ENEGMEAN):
            self._check(st)
        return int(n.value), st

    def compute_dt(self):
        out = np.zeros(4)
        self._check(lib().esdg_compute_dt(self._ctx, out.ctypes.data_as(C.c_void_p)))
        return out

    def step(self, nsteps: int, dt: float = 0.0, raise_negmean: bool = True):
        t = C.c_double(0.0)
        st = lib().esdg_step(self._ctx, int(nsteps), float(dt), C.byref(t))
        if st == ENEGMEAN and not raise_negmean:
            return t.value, st
        self._check(st)
        return t.value, st

    def get_time(self):
        t = C.c_double(0.0)
        self._check(lib().esdg_get_time(self._ctx, C.byref(t)))
        return t.value

    def set_time(self, t: float):
        self._check(lib().esdg_set_time(self._ctx, float(t)))

    def diagnostics(self):
        out = np.zeros(8)
        self._check(lib().esdg_diagnostics(self._ctx, out.ctypes.data_as(C.c_void_p)))
        return out

    def diagnostics_noalloc(self):
        """esdg_diagnostics_noalloc: the same outputs, no device allocation."""
        out = np.zeros(8)
        self._check(lib().esdg_diagnostics_noalloc(self._ctx, out.ctypes.data_as(C.c_void_p)))
        return out

    def step_stats(self):
        """(limited element-stages of the last step call, viscous elements now)."""
        lim, vis = C.c_int64(0), C.c_int64(0)
        self._check(lib().esdg_step_stats(self._ctx, C.byref(lim), C.byref(vis)))
        return int(lim.value), int(vis.value)

    def get_eps(self, device: bool = False):
        (o,) = self._outs(1, self.K, device)
        a = _Arg(o)
        self._check(lib().esdg_get_eps(self._ctx, a.ptr, a.mem))
        return o

    def get_geometry(self):
        outs = self._outs(5, self.n_nodes, False)
        ps = [_Arg(o) for o in outs]
        self._check(lib().esdg_get_geometry(self._ctx, *[p.ptr for p in ps], 0))
        return dict(zip(("xxi", "xeta", "yxi", "yeta", "J"), self._shape(outs)))

    def autotune(self, reps: int = 5):
        """Pick the fastest compiled stage-kernel variant; returns (choice,
        mean ms per variant)."""
        c = C.c_int(0)
        ms = np.zeros(STAGE_VARIANTS)
        self._check(lib().esdg_autotune(self._ctx, int(reps), C.byref(c), ms.ctypes.data_as(C.c_void_p)))
        return c.value, ms

    def set_stage_variant(self, variant: int):
        self._check(lib().esdg_set_stage_variant(self._ctx, int(variant)))

    def set_graphs(self, enable: bool = True):
        """esdg_set_graphs: replay each step as one captured HIP graph."""
        self._check(lib().esdg_set_graphs(self._ctx, int(bool(enable))))

    def profile(self, enable: bool = True):
        self._check(lib().esdg_profile(self._ctx, int(bool(enable))))

    def profile_read(self):
        sm, sn, am, an = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
        self._check(lib().esdg_profile_read(self._ctx, C.byref(sm), C.byref(sn), C.byref(am), C.byref(an)))
        return dict(stage_ms=sm.value, stage_launches=sn.value, av_ms=am.value, av_launches=an.value)

    KERNEL_CLASSES = ("stage", "indicator", "av_faces", "av_div", "dt", "adjoint")

    def profile_read_kernels(self):
        """Summed event milliseconds and launch counts per kernel class since
        the last read (then reset): {class: (ms, launches)}."""
        ms = np.zeros(6)
        n = np.zeros(6, dtype=np.int64)
        self._check(lib().esdg_profile_read_kernels(self._ctx, ms.ctypes.data_as(C.c_void_p),
                                                    n.ctypes.data_as(C.c_void_p)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNEL_CLASSES)}

    def profile_read_adjoint(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(lib().esdg_profile_read_adjoint(self._ctx, C.byref(ms), C.byref(n)))
        return dict(ms=ms.value, launches=n.value)


    # -- discrete adjoint -------------------------------------------------
    def rhs_vjp(self, lh, lhu, lhv, device: bool | None = None):
        """(dR/dW)^T lam and (dR/db)^T lam at the current state: returns
        (gh, ghu, ghv, gb).  Outputs on the device when the inputs are CUDA
        tensors (or device=True)."""
        a = [_Arg(x, self.n_nodes) for x in (lh, lhu, lhv)]
        if len({x.mem for x in a}) != 1:
            raise ValueError("mix of host and device arrays")
        dev = bool(a[0].mem) if device is None else device
        if dev != bool(a[0].mem):
            raise ValueError("inputs and outputs must both be host or both device arrays")
        outs = self._outs(4, self.n_nodes, dev)
        ps = [_Arg(o) for o in outs]
        self._check(lib().esdg_rhs_vjp(self._ctx, *[x.ptr for x in a], *[p.ptr for p in ps], a[0].mem))
        return self._shape(outs)

    def set_gauges(self, elem, xi, eta):
        e = np.ascontiguousarray(elem, dtype=np.int32)
        x = np.ascontiguousarray(xi, dtype=np.float64)
        y = np.ascontiguousarray(eta, dtype=np.float64)
        if not (e.size == x.size == y.size):
            raise ValueError("gauge arrays differ in length")
        self._check(lib().esdg_set_gauges(self._ctx, int(e.size), e.ctypes.data_as(C.c_void_p),
                                          x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p)))
        self.n_gauges = int(e.size)

    def gauge_values(self):
        out = np.zeros(self.n_gauges)
        self._check(lib().esdg_gauge_values(self._ctx, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def adjoint_forward(self, nsteps: int, dt: float, every: int, target, want_H: bool = False):
        """Gauge-misfit loss over nsteps fixed steps (checkpoints every
        `every` steps); target [nsteps, ng] host or device.  Returns the loss
        (and the gauge values [nsteps, ng] with want_H)."""
        t = _Arg(target, int(nsteps) * self.n_gauges)
        loss = C.c_double(0.0)
        H = np.zeros((int(nsteps), self.n_gauges)) if want_H else None
        if want_H and t.mem:
            raise ValueError("want_H needs a host target")
        self._check(lib().esdg_adjoint_forward(self._ctx, int(nsteps), float(dt), int(every), t.ptr, t.mem,
                                               C.byref(loss),
                                               H.ctypes.data_as(C.c_void_p) if want_H else None))
        return (loss.value, H) if want_H else loss.value

    def adjoint_backward(self, seed: float = 1.0, device: bool = False):
        """seed * (dL/db, dL/dh0, dL/dhu0, dL/dhv0) of the last forward sweep."""
        outs = self._outs(4, self.n_nodes, device)
        ps = [_Arg(o) for o in outs]
        self._check(lib().esdg_adjoint_backward(self._ctx, float(seed), *[p.ptr for p in ps], ps[0].mem))
        return self._shape(outs)


class Ensemble:
    """Independent instances (own mesh, degree, bathymetry, state, step and
    time) advanced together: one launch per stage covers all instances of a
    degree (``esdg_ensemble_*`` in include/esdg.h)."""

    def __init__(self, device: int = 0, precision: int = 64):
        self._h = C.c_void_p()
        st = lib().esdg_ensemble_create(C.byref(self._h), int(device), int(precision))
        if st != OK:
            raise EsdgError(st, "esdg_ensemble_create failed")
        self.device = device
        self._shapes = []

    def _check(self, st):
        if st != OK:
            raise EsdgError(st, lib().esdg_ensemble_last_error(self._h).decode())
        return st

    def close(self):
        if self._h:
            lib().esdg_ensemble_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, mesh, b, h, hu, hv, params: Params) -> int:
        """Add one instance (host arrays); returns its id."""
        N, K = mesh.N, mesh.x.shape[0]
        n = K * (N + 1) ** 2
        args = [_Arg(mesh.x, n), _Arg(mesh.y, n), _Arg(mesh.nbr_elem, 4 * K, np.int32),
                _Arg(mesh.nbr_side, 4 * K, np.int8), _Arg(mesh.flip, 4 * K, np.int8),
                _Arg(b, n), _Arg(h, n), _Arg(hu, n), _Arg(hv, n)]
        if any(a.mem for a in args):
            raise ValueError("ensemble instances are added from host arrays")
        i = C.c_int(-1)
        self._check(lib().esdg_ensemble_add(self._h, C.byref(params), int(N), int(K), *[a.ptr for a in args],
                                            C.byref(i)))
        self._shapes.append((N, K))
        return i.value

    def add_workload(self, w, **params) -> int:
        P = default_params(w.mesh.N)
        for k, v in {**w.params, **params}.items():
            setattr(P, k, v)
        return self.add(w.mesh, w.b, w.h, w.hu, w.hv, P)

    def build(self):
        self._check(lib().esdg_ensemble_build(self._h))

    def step(self, nsteps: int, raise_negmean: bool = True) -> int:
        """Advance every instance nsteps steps; returns the status (ENEGMEAN
        only with raise_negmean=False: an element mean went negative, the
        limiter set it to its mean, the states are finite)."""
        st = lib().esdg_ensemble_step(self._h, int(nsteps))
        if st == ENEGMEAN and not raise_negmean:
            return st
        self._check(st)
        return st

    def set_graphs(self, enable: bool = True):
        """esdg_ensemble_set_graphs: graph replay per degree group."""
        self._check(lib().esdg_ensemble_set_graphs(self._h, int(bool(enable))))

    def __len__(self):
        n = C.c_int(0)
        self._check(lib().esdg_ensemble_size(self._h, C.byref(n)))
        return n.value

    def get_state(self, i: int):
        N, K = self._shapes[i]
        outs = [np.empty((K, (N + 1) ** 2)) for _ in range(3)]
        self._check(lib().esdg_ensemble_get_state(self._h, int(i), *[o.ctypes.data_as(C.c_void_p) for o in outs],
                                                  0))
        return outs

    def get_time(self, i: int) -> float:
        t = C.c_double(0.0)
        self._check(lib().esdg_ensemble_get_time(self._h, int(i), C.byref(t)))
        return t.value

    def degrees(self):
        n = C.c_int(0)
        Ns = (C.c_int * 16)()
        self._check(lib().esdg_ensemble_degrees(self._h, C.byref(n), Ns))
        return [Ns[g] for g in range(n.value)]

    def autotune(self, reps: int = 5):
        """Autotune every degree's stage kernel; returns {N: choice}."""
        degs = self.degrees() if self._built_or_build() else []
        ch = (C.c_int * 16)()
        self._check(lib().esdg_ensemble_autotune(self._h, int(reps), ch))
        return {N: ch[g] for g, N in enumerate(degs)}

    def _built_or_build(self):
        self.build()
        return True


def solver_for(workload, device: int = 0, precision: int = 64, **params) -> Solver:
    """Solver with a workload's mesh, bathymetry and state uploaded."""
    s = Solver(device, precision)
    s.upload_mesh(workload.mesh)
    P = default_params(workload.mesh.N)
    for k, v in {**workload.params, **params}.items():
        setattr(P, k, v)
    s.set_params(P)
    s.set_bathymetry(workload.b)
    s.set_state(workload.h, workload.hu, workload.hv)
    return s
