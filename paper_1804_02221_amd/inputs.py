"""Seeded synthetic workloads for the entropy-stable DGSEM shallow-water solver.

This module builds *inputs only*: periodic quadrilateral meshes (nodal
coordinates at Legendre-Gauss-Lobatto points plus the face-connectivity map)
and smooth or discontinuous initial data and bathymetry.  It holds none of the
method's arithmetic (no derivative operators, fluxes, metric terms or time
integration); the same arrays are handed to the GPU library and to the CPU
oracle, so random-number parity never matters.

Layout conventions (shared with the C ABI in ``include/esdg.h``):

* arrays are structure-of-arrays ``[K][(N+1)^2]`` (float64, C order), node
  ``p = i*(N+1) + j`` with ``i`` the xi-index and ``j`` the eta-index
  (the paper's coalesced index order, GPU-implementation section, version 4);
* element sides are numbered 0..3 = the paper's s=1..4
  (eta=-1, xi=+1, eta=+1, xi=-1; the paper fixes only which axis each side
  lies on, Lemma 2);
* face node ``k`` on a side runs along increasing xi (sides 0, 2) or
  increasing eta (sides 1, 3): side 0 -> (k, 0), side 1 -> (N, k),
  side 2 -> (k, N), side 3 -> (0, k);
* ``nbr_elem[e, s]``, ``nbr_side[e, s]`` name the element and local side that
  share side ``s`` of element ``e``; ``flip[e, s] = 1`` when the neighbour's
  face-node order runs the other way (neighbour node index ``N - k``).

Curvilinear mesh: nodal coordinates are the map
``x = X + a sin(2 pi X/Lx) sin(2 pi Y/Ly)``, ``y = Y + (same)`` evaluated at
each element's LGL nodes (for ``[0,10]^2`` this is ``0.1 sin(pi X/5)
sin(pi Y/5)``), so the mesh is conforming and periodic.  Every field is
evaluated on the lattice of unique periodic node positions and gathered into
the DG arrays, so coincident nodes hold bitwise-identical values (in
particular the bathymetry is continuous, which Lemma 2 and the well-balanced
property assume).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Face node k of local side s -> local node (i, j).  Topology only.
def _side_node(N: int, s: int, k):
    if s == 0:
        return k, 0 * k
    if s == 1:
        return N + 0 * k, k
    if s == 2:
        return k, N + 0 * k
    return 0 * k, k


def lgl_positions(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto positions in [-1, 1] (ascending), used only to
    place nodal coordinates.  Endpoints +-1 and the roots of L_N', found with
    numpy's Legendre root finder and symmetrised so that x_{N-i} = -x_i."""
    if N < 1:
        raise ValueError("N must be >= 1")
    inner = np.sort(np.real(np.polynomial.legendre.Legendre.basis(N).deriv().roots()))
    x = np.concatenate(([-1.0], inner, [1.0]))
    x = 0.5 * (x - x[::-1])
    if N % 2 == 0:
        x[N // 2] = 0.0
    return x


@dataclass
class PeriodicMesh:
    N: int
    nx: int
    ny: int
    Lx: float
    Ly: float
    amp: float
    x: np.ndarray          # [K, np] physical x (unwrapped within each element)
    y: np.ndarray
    ax: np.ndarray         # [K, np] wrapped lattice index in x
    ay: np.ndarray
    nbr_elem: np.ndarray   # [K, 4] int32
    nbr_side: np.ndarray   # [K, 4] int8
    flip: np.ndarray       # [K, 4] int8
    rot: np.ndarray        # [K] int8, quarter turns of each element's local frame
    lat_x: np.ndarray = field(repr=False)   # [nx*N] wrapped lattice X positions
    lat_y: np.ndarray = field(repr=False)

    @property
    def K(self) -> int:
        return self.x.shape[0]

    @property
    def n_p(self) -> int:
        return (self.N + 1) ** 2

    def gather(self, lattice_field: np.ndarray) -> np.ndarray:
        """Lattice field [nx*N, ny*N] -> DG nodal array [K, np]."""
        return np.ascontiguousarray(lattice_field[self.ax, self.ay])

    def lattice_xy(self):
        """Physical (wrapped) coordinates on the unique-node lattice."""
        X, Y = np.meshgrid(self.lat_x, self.lat_y, indexing="ij")
        pert = self.amp * np.sin(2 * np.pi * X / self.Lx) * np.sin(2 * np.pi * Y / self.Ly)
        return X + pert, Y + pert

    def element_centroid_ref(self):
        """Undeformed element centroids (X, Y), shape [K]."""
        K = self.K
        e = np.arange(K)
        ix, iy = e % self.nx, e // self.nx
        return (ix + 0.5) * self.Lx / self.nx, (iy + 0.5) * self.Ly / self.ny


def make_periodic_mesh(N: int, nx: int, ny: int, Lx: float, Ly: float,
                       amp: float = 0.0, rotate_seed: int | None = None) -> PeriodicMesh:
    """Periodic nx-by-ny quad mesh of [0,Lx]x[0,Ly], elements ordered
    e = iy*nx + ix.  With ``rotate_seed`` every element's local (xi, eta) frame
    is turned by a random multiple of 90 degrees (orientation kept, J > 0),
    which exercises the face map and the flip flags."""
    if N < 2:
        raise ValueError("mesh generator needs N >= 2 (face keys use an interior face node)")
    if nx < 2 or ny < 2:
        raise ValueError("periodic mesh needs nx, ny >= 2")
    n1 = N + 1
    K = nx * ny
    xi = lgl_positions(N)
    dx, dy = Lx / nx, Ly / ny
    MX, MY = nx * N, ny * N
    a = np.arange(MX)
    lat_x = (a // N + 0.5 * (xi[a % N] + 1.0)) * dx
    c = np.arange(MY)
    lat_y = (c // N + 0.5 * (xi[c % N] + 1.0)) * dy

    e = np.arange(K)
    ix, iy = e % nx, e // nx
    if rotate_seed is None:
        rot = np.zeros(K, dtype=np.int8)
    else:
        rot = np.random.default_rng(rotate_seed).integers(0, 4, size=K).astype(np.int8)

    ip, jp = np.meshgrid(np.arange(n1), np.arange(n1), indexing="ij")
    ip = ip.reshape(-1)
    jp = jp.reshape(-1)  # local node p = i'*(N+1)+j'

    def unrot(r, i_, j_):
        # local (i', j') of a frame turned r quarter turns -> unrotated (i, j)
        if r == 0:
            return i_, j_
        if r == 1:
            return N - j_, i_
        if r == 2:
            return N - i_, N - j_
        return j_, N - i_

    I = np.empty((K, n1 * n1), dtype=np.int64)
    J = np.empty((K, n1 * n1), dtype=np.int64)
    for r in range(4):
        sel = rot == r
        if not np.any(sel):
            continue
        ii, jj = unrot(r, ip, jp)
        I[sel] = ii[None, :]
        J[sel] = jj[None, :]
    AX = ix[:, None] * N + I            # unwrapped lattice index
    AY = iy[:, None] * N + J
    ax = AX % MX
    ay = AY % MY
    Xu = lat_x[ax] + Lx * (AX // MX)
    Yu = lat_y[ay] + Ly * (AY // MY)
    Xw = lat_x[ax]
    Yw = lat_y[ay]
    pert = amp * np.sin(2 * np.pi * Xw / Lx) * np.sin(2 * np.pi * Yw / Ly)
    x = np.ascontiguousarray(Xu + pert)
    y = np.ascontiguousarray(Yu + pert)

    # ---- face map: match sides through the lattice keys of the interior
    # face nodes k=1 and k=N-1 (orientation independent), orient via k=0 ----
    key1 = np.empty((K, 4), dtype=np.int64)
    keyM = np.empty((K, 4), dtype=np.int64)
    key0 = np.empty((K, 4), dtype=np.int64)
    keyN = np.empty((K, 4), dtype=np.int64)
    for s in range(4):
        for kk, dst in ((1, key1), (N - 1, keyM), (0, key0), (N, keyN)):
            li, lj = _side_node(N, s, kk)
            p = li * n1 + lj
            dst[:, s] = ax[:, p] * MY + ay[:, p]
    key1 = np.minimum(key1, keyM)
    flat = key1.reshape(-1)
    order = np.argsort(flat, kind="stable")
    sk = flat[order]
    if sk.size % 2 or not np.all(sk[0::2] == sk[1::2]) or (
            sk.size > 2 and np.any(sk[2::2] == sk[1:-1:2])):
        raise RuntimeError("face matching failed: mesh is not conforming")
    A = order[0::2]
    B = order[1::2]
    nbr_elem = np.empty(4 * K, dtype=np.int32)
    nbr_side = np.empty(4 * K, dtype=np.int8)
    nbr_elem[A] = B // 4
    nbr_side[A] = B % 4
    nbr_elem[B] = A // 4
    nbr_side[B] = A % 4
    nbr_elem = nbr_elem.reshape(K, 4)
    nbr_side = nbr_side.reshape(K, 4)
    own0 = key0
    nb0 = key0[nbr_elem, nbr_side]
    nbN = keyN[nbr_elem, nbr_side]
    flip = np.where(own0 == nb0, 0, 1).astype(np.int8)
    if not np.all((own0 == nb0) | (own0 == nbN)):
        raise RuntimeError("face orientation could not be resolved")
    return PeriodicMesh(N=N, nx=nx, ny=ny, Lx=Lx, Ly=Ly, amp=amp, x=x, y=y,
                        ax=ax, ay=ay, nbr_elem=np.ascontiguousarray(nbr_elem),
                        nbr_side=np.ascontiguousarray(nbr_side),
                        flip=np.ascontiguousarray(flip), rot=rot,
                        lat_x=lat_x, lat_y=lat_y)


def make_box_mesh(N: int, nx: int, ny: int, x0: float, y0: float, Lx: float, Ly: float,
                  amp: float = 0.0, walls_x: bool = True, walls_y: bool = True,
                  rotate_seed: int | None = None) -> PeriodicMesh:
    """Mesh of [x0, x0+Lx] x [y0, y0+Ly] with solid walls (nbr_elem = -1) on the
    sides x = const (walls_x) and/or y = const (walls_y), periodic in the
    other direction: the periodic mesh with the faces across the seams cut.
    The sin perturbation vanishes on the boundary, so walls are straight.
    Fields on such a mesh are evaluated at the nodal coordinates (x, y), not
    through the periodic lattice."""
    if nx < 3 or ny < 3:
        raise ValueError("box mesh needs nx, ny >= 3")
    m = make_periodic_mesh(N, nx, ny, Lx, Ly, amp=amp, rotate_seed=rotate_seed)
    cx, cy = m.element_centroid_ref()
    ne = m.nbr_elem.copy()
    for s in range(4):
        nb = ne[:, s]
        cut = np.zeros(m.K, dtype=bool)
        if walls_x:
            cut |= np.abs(cx[nb] - cx) > 0.5 * Lx
        if walls_y:
            cut |= np.abs(cy[nb] - cy) > 0.5 * Ly
        ne[cut, s] = -1
    m.nbr_elem = np.ascontiguousarray(ne)
    m.x = np.ascontiguousarray(m.x + x0)
    m.y = np.ascontiguousarray(m.y + y0)
    return m


# --------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------
def periodic_gaussians(mesh: PeriodicMesh, centers, amps, widths) -> np.ndarray:
    """sum_k a_k exp(-|x - c_k|^2 / w_k^2), periodised over the 3x3 images,
    evaluated at physical node positions; returns [K, np]."""
    PX, PY = mesh.lattice_xy()
    out = np.zeros_like(PX)
    for (cx, cy), a_, w_ in zip(centers, amps, widths):
        for ox in (-mesh.Lx, 0.0, mesh.Lx):
            for oy in (-mesh.Ly, 0.0, mesh.Ly):
                out += a_ * np.exp(-((PX - cx - ox) ** 2 + (PY - cy - oy) ** 2) / w_ ** 2)
    return mesh.gather(out)


def fourier_field(mesh: PeriodicMesh, rng: np.random.Generator, kmax: int,
                  lo: float, hi: float) -> np.ndarray:
    """Smooth periodic random field: Fourier modes |k| <= kmax with random
    amplitudes and phases in the reference coordinates, affinely mapped onto
    [lo, hi]; evaluated as a rank-(2kmax+1) tensor product on the lattice."""
    ks = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(ks, ks, indexing="ij")
    mask = (KX ** 2 + KY ** 2 <= kmax ** 2) & ~((KX == 0) & (KY == 0))
    amp = rng.standard_normal(KX.shape) * mask
    ph = rng.uniform(0.0, 2 * np.pi, KX.shape)
    C = amp * np.exp(1j * ph)
    EX = np.exp(2j * np.pi * np.outer(mesh.lat_x / mesh.Lx, ks))
    EY = np.exp(2j * np.pi * np.outer(mesh.lat_y / mesh.Ly, ks))
    F = np.real(EX @ C @ EY.T)
    F = (F - F.min()) / (F.max() - F.min())
    return mesh.gather(lo + (hi - lo) * F)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: PeriodicMesh
    b: np.ndarray
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    params: dict


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lake_bump(n: int = 16, N: int = 3, seed: int = 1, bump: bool = True,
              amp: float = 0.0, rotate_seed: int | None = None) -> Workload:
    """Plain-method case: [0,2]^2 periodic, n x n quads, g=9.81,
    b = 0.5 exp(-40((x-1)^2+(y-1)^2)), lake at rest H=2 plus a seeded Gaussian
    surface bump of amplitude 1e-2 (width 0.2, centre ~ U([0.5,1.5]^2))."""
    mesh = make_periodic_mesh(N, n, n, 2.0, 2.0, amp=amp * 0.2, rotate_seed=rotate_seed)
    rng = np.random.default_rng(seed)
    b = periodic_gaussians(mesh, [(1.0, 1.0)], [0.5], [1.0 / np.sqrt(40.0)])
    H = np.full_like(b, 2.0)
    if bump:
        c0 = rng.uniform(0.5, 1.5, size=2)
        H = H + periodic_gaussians(mesh, [tuple(c0)], [1e-2], [0.2])
    h = H - b
    z = np.zeros_like(h)
    return Workload("lake_bump", mesh, _c(b), _c(h), _c(z), _c(z.copy()),
                    dict(g=9.81, surface_flux=0, av_on=0, limiter_on=0, cfl=0.5))


def dam_break(n: int = 128, N: int = 7, seed: int = 2, rotate_seed: int | None = None) -> Workload:
    """Curvilinear wet/dry dam break on [0,10]^2 (periodic): sin-perturbed
    map with amplitude 0.1; h = 1 in elements whose undeformed centroid has
    X < 5, else dry; u = v = 0; bathymetry = 8 periodised Gaussians with
    amplitude U(0,0.3), width U(0.5,2), centre U([0,10]^2)."""
    mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1, rotate_seed=rotate_seed)
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, 0.3, 8)
    widths = rng.uniform(0.5, 2.0, 8)
    centers = rng.uniform(0.0, 10.0, (8, 2))
    b = periodic_gaussians(mesh, [tuple(cc) for cc in centers], amps, widths)
    cx, _ = mesh.element_centroid_ref()
    h = np.where((cx < 5.0)[:, None], 1.0, 0.0) * np.ones((1, mesh.n_p))
    z = np.zeros_like(h)
    return Workload("dam_break", mesh, _c(b), _c(h), _c(z), _c(z.copy()),
                    dict(g=9.81, surface_flux=0, av_on=1, limiter_on=1, eps0=0.025, cfl=0.5))


def smooth_sweep(n: int = 512, N: int = 7, seed: int = 3, rotate_seed: int | None = None) -> Workload:
    """Throughput workload: [0,10]^2 periodic, n x n curvilinear elements
    (same sin map), independent smooth random Fourier fields (|k| <= 4):
    h in [0.5, 2], u, v in [-0.49, 0.49], b in [0, 1]."""
    mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1, rotate_seed=rotate_seed)
    rng = np.random.default_rng(seed)
    h = fourier_field(mesh, rng, 4, 0.5, 2.0)
    u = fourier_field(mesh, rng, 4, -0.49, 0.49)
    v = fourier_field(mesh, rng, 4, -0.49, 0.49)
    b = fourier_field(mesh, rng, 4, 0.0, 1.0)
    return Workload("smooth_sweep", mesh, _c(b), _c(h), _c(h * u), _c(h * v),
                    dict(g=9.81, surface_flux=0, av_on=1, limiter_on=1, eps0=0.025, cfl=0.5))


def ensemble_member(n: int, N: int, dam: bool, seed: int) -> Workload:
    """One instance of the batched-ensemble recipe: n x n curvilinear
    periodic elements of [0,10]^2 (the sin map of dam_break), bathymetry of 8
    periodised Gaussians (amplitude U(0,0.3), width U(0.5,2)); initial data
    the dam break (h = 1 for undeformed centroid X < 5, else dry) or, when
    not dam, a wet Gaussian surface bump H = 1.2 + 0.1 exp(-|x - x0|^2) over
    the bed (h = max(H - b, 0)); at rest.  AV and limiter on; eps0 = 0.05 at
    N = 3, 0.025 otherwise; SSPRK(3,3), the integrator the paper adopts for
    wet/dry runs because Lemma 2's mean positivity covers it (section 2.2,
    eq. RKSSP)."""
    if dam:
        w = dam_break(n, N, seed=seed)
    else:
        mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1)
        rng = np.random.default_rng(seed)
        amps = rng.uniform(0.0, 0.3, 8)
        widths = rng.uniform(0.5, 2.0, 8)
        centers = rng.uniform(0.0, 10.0, (8, 2))
        b = periodic_gaussians(mesh, [tuple(cc) for cc in centers], amps, widths)
        x0 = tuple(rng.uniform(2.0, 8.0, 2))
        H = 1.2 + periodic_gaussians(mesh, [x0], [0.1], [1.0])
        h = np.maximum(H - b, 0.0)
        z = np.zeros_like(h)
        w = Workload("bump", mesh, _c(b), _c(h), _c(z), _c(z.copy()),
                     dict(g=9.81, surface_flux=0, av_on=1, limiter_on=1, eps0=0.025, cfl=0.5))
    w.name = f"{'dam' if dam else 'bump'}_{n}x{n}_N{N}"
    w.params = dict(w.params, eps0=0.05 if N == 3 else 0.025, integrator=1)
    return w


def bathymetry_gradient(n: int = 128, N: int = 5, seed: int = 4, target_seed: int = 5,
                        n_gauges: int = 32):
    """Adjoint workload: n x n curvilinear periodic elements of [0,10]^2 (the
    sin map of dam_break), degree N; bathymetry of 8 periodised Gaussians
    (amplitude U(0,0.3), width U(0.5,2)) scaled down to max b <= 0.8; water
    surface H0 = 1 + 0.05 exp(-|x - x0|^2) (x0 ~ U([2,8]^2)), so h = H0 - b
    >= 0.2 everywhere; at rest.  Gauges: n_gauges points, each a uniformly
    drawn element and reference point (xi, eta) ~ U([-1,1]^2).  The target
    run uses the bed b + db, db = 4 periodised Gaussians (amplitude
    U(-0.05,0.05), width U(0.5,1.5)) drawn from target_seed.  AV off, limiter
    on (it never acts on this wet state).

    Returns (Workload, extras) with extras = dict(H0, db, gelem, gxi, geta)."""
    mesh = make_periodic_mesh(N, n, n, 10.0, 10.0, amp=0.1)
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, 0.3, 8)
    widths = rng.uniform(0.5, 2.0, 8)
    centers = rng.uniform(0.0, 10.0, (8, 2))
    b = periodic_gaussians(mesh, [tuple(cc) for cc in centers], amps, widths)
    if b.max() > 0.8:
        b = b * (0.8 / b.max())
    x0 = tuple(rng.uniform(2.0, 8.0, 2))
    H0 = 1.0 + periodic_gaussians(mesh, [x0], [0.05], [1.0])
    K = mesh.x.shape[0]
    gelem = rng.integers(0, K, n_gauges).astype(np.int32)
    gxi = rng.uniform(-1.0, 1.0, n_gauges)
    geta = rng.uniform(-1.0, 1.0, n_gauges)
    rt = np.random.default_rng(target_seed)
    db = periodic_gaussians(mesh, [tuple(cc) for cc in rt.uniform(0.0, 10.0, (4, 2))],
                            rt.uniform(-0.05, 0.05, 4), rt.uniform(0.5, 1.5, 4))
    h = H0 - b
    z = np.zeros_like(h)
    w = Workload(f"bathymetry_gradient_{n}x{n}_N{N}", mesh, _c(b), _c(h), _c(z), _c(z.copy()),
                 dict(g=9.81, surface_flux=0, av_on=0, limiter_on=1, cfl=0.5))
    return w, dict(H0=_c(H0), db=_c(db), gelem=gelem, gxi=_c(gxi), geta=_c(geta))


def oscillating_lake(n: int = 200, N: int = 3, t: float = 0.0, h0: float = 0.1, a: float = 1.0,
                     sigma: float = 0.5, g: float = 9.81) -> Workload:
    """The paper's oscillating lake: [-2,2]^2 with solid walls, n x n Cartesian
    elements, parabolic bowl b = h0 (x^2+y^2)/a^2 and the planar oscillation
    of its closed form at time t (omega = sqrt(2 g h0)/a): h = max(0, sigma
    h0/a^2 (2x cos wt + 2y sin wt - sigma) + h0 - b), u = -sigma w sin wt,
    v = sigma w cos wt (zero where dry); eps0 = 0.01, AV and limiter on,
    SSPRK(3,3) (the integrator the mean-positivity bound of Lemma 2 covers)."""
    mesh = make_box_mesh(N, n, n, -2.0, -2.0, 4.0, 4.0)
    x, y = mesh.x, mesh.y
    w = np.sqrt(2.0 * g * h0) / a
    b = h0 * (x * x + y * y) / (a * a)
    h = np.maximum(0.0, sigma * h0 / (a * a) * (2 * x * np.cos(w * t) + 2 * y * np.sin(w * t) - sigma) + h0 - b)
    u = np.where(h > 0, -sigma * w * np.sin(w * t), 0.0)
    v = np.where(h > 0, sigma * w * np.cos(w * t), 0.0)
    return Workload(f"oscillating_lake_{n}x{n}_N{N}", mesh, _c(b), _c(h), _c(h * u), _c(h * v),
                    dict(g=g, surface_flux=0, av_on=1, limiter_on=1, eps0=0.01, cfl=0.5, integrator=1))


def dry_dam_break(n: int = 50, N: int = 3) -> Workload:
    """The paper's dry dam break: [-20,20]^2, n x n Cartesian elements, solid
    walls at x = -20 and 20, periodic in y; h = 10 where x < 0, else dry;
    at rest; flat bed; eps0 = 0.1, AV and limiter on, SSPRK(3,3); a step
    whose stages meet a negative element mean is redone with half the step
    (up to three times: the Lemma 2 bound is evaluated at the step's start,
    the later stages' states can need less)."""
    mesh = make_box_mesh(N, n, n, -20.0, -20.0, 40.0, 40.0, walls_x=True, walls_y=False)
    h = np.where(mesh.x < 0.0, 10.0, 0.0)
    z = np.zeros_like(h)
    return Workload(f"dry_dam_break_{n}x{n}_N{N}", mesh, _c(z.copy()), _c(h), _c(z.copy()), _c(z.copy()),
                    dict(g=9.81, surface_flux=0, av_on=1, limiter_on=1, eps0=0.1, cfl=0.5, integrator=1,
                         max_dt_retries=3))


def three_mound_dam_break(nx: int = 150, ny: int = 100, N: int = 3) -> Workload:
    """The paper's dam break over three mounds: [0,75] x [0,45] (the domain as
    the paper states it), nx x ny Cartesian elements, solid walls on all four
    sides; h = 1.875 where x < 16 (the dam sits on the element interface
    x = 16 at the paper's mesh, whose nodes take the dry side, as the strict
    inequality reads), else dry; at rest; bed b = max(0, M1, M2, M3) with the
    cones M1 = 1 - 0.1 |x - (30, 22.5)|, M2 = 1 - 0.1 |x - (30, 7.5)|,
    M3 = 2.8 - 0.28 |x - (47.5, 15)|; eps0 = 0.2, g = 9.81, AV and limiter
    on, SSPRK(3,3) with step halving as in dry_dam_break."""
    mesh = make_box_mesh(N, nx, ny, 0.0, 0.0, 75.0, 45.0, walls_x=True, walls_y=True)
    x, y = mesh.x, mesh.y
    m1 = 1.0 - 0.1 * np.sqrt((x - 30.0) ** 2 + (y - 22.5) ** 2)
    m2 = 1.0 - 0.1 * np.sqrt((x - 30.0) ** 2 + (y - 7.5) ** 2)
    m3 = 2.8 - 0.28 * np.sqrt((x - 47.5) ** 2 + (y - 15.0) ** 2)
    b = np.maximum(np.maximum(0.0, m1), np.maximum(m2, m3))
    h = np.where(x < 16.0, 1.875, 0.0)
    z = np.zeros_like(h)
    return Workload(f"three_mound_dam_break_{nx}x{ny}_N{N}", mesh, _c(b), _c(h), _c(z.copy()), _c(z.copy()),
                    dict(g=9.81, surface_flux=0, av_on=1, limiter_on=1, eps0=0.2, cfl=0.5, integrator=1,
                         max_dt_retries=3))


def conical_island(nx: int = 50, ny: int = 50, N: int = 3) -> Workload:
    """The paper's solitary-wave run-up on a conical island: [0,25] x [0,30],
    nx x ny Cartesian elements, solid walls everywhere; still water of depth
    h0 = 0.32 with a solitary wave of amplitude A = 0.064 centred at x = 2.5,
    eta = A sech^2(gamma (x - 2.5)) with gamma = sqrt(3 A / (4 h0^3)) (the
    paper prints the same wave in lengths scaled by h0), u = eta sqrt(g / h0),
    v = 0; the island b = 0.93 (1 - r / 3.6) for r <= 3.6 around (12.5, 15),
    else 0, and h = max(0, h0 + eta - b); eps0 = 0.1, g = 9.81, AV and
    limiter on, SSPRK(3,3) with step halving as in dry_dam_break."""
    mesh = make_box_mesh(N, nx, ny, 0.0, 0.0, 25.0, 30.0, walls_x=True, walls_y=True)
    x, y = mesh.x, mesh.y
    g, h0, A = 9.81, 0.32, 0.064
    gam = np.sqrt(3.0 * A / (4.0 * h0 ** 3))
    eta = A / np.cosh(gam * (x - 2.5)) ** 2
    r = np.sqrt((x - 12.5) ** 2 + (y - 15.0) ** 2)
    b = np.where(r <= 3.6, 0.93 * (1.0 - r / 3.6), 0.0)
    h = np.maximum(0.0, h0 + eta - b)
    u = np.where(h > 0.0, eta * np.sqrt(g / h0), 0.0)
    z = np.zeros_like(h)
    return Workload(f"conical_island_{nx}x{ny}_N{N}", mesh, _c(b), _c(h), _c(h * u), _c(z),
                    dict(g=g, surface_flux=0, av_on=1, limiter_on=1, eps0=0.1, cfl=0.5, integrator=1,
                         max_dt_retries=3))


def random_states(rng: np.random.Generator, n: int, dry_fraction: float = 0.0,
                  hmax: float = 2.0, umax: float = 1.0):
    """Independent random point states (h, hu, hv, b) for flux-level tests."""
    h = rng.uniform(0.05, hmax, n)
    if dry_fraction > 0:
        h[rng.uniform(size=n) < dry_fraction] = 0.0
    u = rng.uniform(-umax, umax, n)
    v = rng.uniform(-umax, umax, n)
    u[h == 0] = 0.0
    v[h == 0] = 0.0
    b = rng.uniform(0.0, 1.0, n)
    return h, h * u, h * v, b
