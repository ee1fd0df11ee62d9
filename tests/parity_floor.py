"""FP64 parity bars tied to the oracle's own rounding floor (test helper).

A GPU result and the oracle's differ by rounding only: the two evaluate the
same formulas in different orders (the kernels' factored two-point sums,
fused multiply-adds, their own metric and bathymetry-derivative passes).
How far rounding can move an output is measured on the oracle alone, on the
CPU: the output's response to a random 1-ulp perturbation of the inputs --
every nodal value of h, hu, hv nudged to a neighbouring double, and the bottom
b nudged once per physical node, so that it stays continuous across faces as
the inputs are.  That response, the *floor*, already contains every
amplification the method applies to rounding: the cancellation of the
flux-differencing terms (their size, g h (h+b) |D| |metric| / J, is ~1e5
times R on the 512^2, N = 7 workload) and, with artificial viscosity on the
ramp of the indicator, the ill-conditioned log10 of the modal energy ratio.
Input nudges do not excite every ill-conditioned decision equally: on a
wet/dry front the limiter's theta = mean / (mean - min) and the viscosity
ramp amplify rounding made *inside* the evaluation, which a nudge of the
inputs reaches only now and then (on the 8 x 8, N = 5 dam break one draw in
two moves h by 7e-16 after four steps, the other by 8e-15).  So the floor also
takes the spread between the oracle and its rounding twin -- the same C
source built with fused multiply-adds (oracle.rounding_twin()), i.e. the same
formulas rounded in another order, which is exactly the kind of difference a
GPU evaluation has (on that dam break the twin differs by 1e-12 in h after
four steps).  The floor of a field is the largest of these responses.  A GPU
output is accepted when

    max |GPU - oracle| <= FLOOR_MULT * floor       (per field)

Nothing here depends on a GPU value: floors come from oracle runs only.
Every check prints err, floor, err/floor and err/max|R| for the record.
"""
from __future__ import annotations

import numpy as np

FLOOR_MULT = 16.0
DRAWS = 2


def nudge(a: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Every entry moved to a neighbouring double, up or down at random."""
    d = np.where(rng.integers(0, 2, size=a.shape) == 1, np.inf, -np.inf)
    return np.nextafter(a, d)


def nudge_continuous(mesh, b: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """b nudged by one ulp per physical node (coincident DG nodes alike), so
    that a continuous bottom stays continuous; meshes without a node lattice
    keep b unchanged."""
    ax, ay = getattr(mesh, "ax", None), getattr(mesh, "ay", None)
    if ax is None or ay is None:
        return b
    up = rng.integers(0, 2, size=(int(ax.max()) + 1, int(ay.max()) + 1)) == 1
    d = np.where(up[ax, ay], np.inf, -np.inf)
    out = np.nextafter(b, d)
    # a lattice node shared by elements of a walled mesh (no periodic wrap)
    # holds bitwise-equal b in every copy, so the nudge keeps them equal
    return out


def perturbed_inputs(mesh, b, h, hu, hv, seed: int):
    rng = np.random.default_rng(seed)
    return nudge_continuous(mesh, b, rng), nudge(h, rng), nudge(hu, rng), nudge(hv, rng)


def _twin(orc, fn):
    """fn() evaluated by the oracle's rounding twin (None where the host
    cannot run it)."""
    if not orc.host_has_fma():
        return None
    with orc.rounding_twin():
        return fn()


def rhs_floor(orc, P, mesh, b, h, hu, hv, need=None, draws: int = DRAWS, seed: int = 1234):
    """Oracle R (and eps) and the per-field floor [R_h, R_hu, R_hv, eps]."""
    R0 = orc.rhs(P, mesh, b, h, hu, hv, need=need)
    fl = np.zeros(4)
    runs = [orc.rhs(P, mesh, *perturbed_inputs(mesh, b, h, hu, hv, seed + k), need=need)
            for k in range(draws)]
    runs.append(_twin(orc, lambda: orc.rhs(P, mesh, b, h, hu, hv, need=need)))
    for Rk in runs:
        if Rk is None:
            continue
        for c in range(4):
            fl[c] = max(fl[c], float(np.abs(Rk[c] - R0[c]).max()))
    return R0, fl


def step_floor(orc, P, mesh, b, h, hu, hv, nsteps: int, dt: float, draws: int = 1, seed: int = 4321):
    """Oracle state after nsteps steps (and t, status) and the floor of each
    of h, hu, hv (the run repeated from nudged inputs; with an adaptive step
    the nudged run also picks its own steps)."""
    out = orc.step(P, mesh, b, h, hu, hv, nsteps, dt)
    fl = np.zeros(3)
    runs = [orc.step(P, mesh, *perturbed_inputs(mesh, b, h, hu, hv, seed + k), nsteps, dt)
            for k in range(draws)]
    runs.append(_twin(orc, lambda: orc.step(P, mesh, b, h, hu, hv, nsteps, dt)))
    for o in runs:
        if o is None:
            continue
        for c in range(3):
            fl[c] = max(fl[c], float(np.abs(o[c] - out[c]).max()))
    return out, fl


def check(got, want, floor, what: str, mult: float = FLOOR_MULT, sel=None, names=("h", "hu", "hv")):
    """Assert max|got - want| <= mult * floor for every field; print the
    ratios.  sel: optional index selecting the compared entries."""
    msgs = []
    for c, (g_, w_) in enumerate(zip(got, want)):
        g_ = np.asarray(g_)
        w_ = np.asarray(w_)
        if sel is not None:
            g_, w_ = g_[sel], w_[sel]
        err = float(np.abs(g_ - w_).max()) if w_.size else 0.0
        mx = float(np.abs(w_).max()) if w_.size else 0.0
        fl = float(floor[c])
        ratio = err / fl if fl > 0 else (0.0 if err == 0 else np.inf)
        msgs.append(f"{names[c]}: err {err:.3e} floor {fl:.3e} err/floor {ratio:.2f} "
                    f"err/max {err / mx if mx > 0 else 0.0:.2e}")
        print(f"[parity] {what} {msgs[-1]}", flush=True)
        assert err <= mult * fl or err == 0.0, f"{what} {msgs[-1]} (bar {mult:g} x floor)"
    return msgs
