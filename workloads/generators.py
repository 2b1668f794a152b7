"""Seeded generators for macro meshes, boundary data and RVE microstructures.

Conventions shared by every consumer of a :class:`Problem`:

* Macro nodes are numbered lexicographically (x fastest); DOFs are node-major,
  ``dof = node * dim + component``.
* Q4 connectivity is counter-clockwise starting at the lower-left node; hex8
  lists the bottom face counter-clockwise, then the top face.
* One RVE per macro Gauss point: ``b = element * n_gp + g`` with the 2-point
  Gauss points ordered xi fastest, then eta (then zeta).  A problem with
  ``macro_basis == "element"`` (piecewise-constant macro basis of the
  fluctuation) has one RVE per macro element instead: ``b = element``.
* An RVE is a structured grid of n1 x n2 (x n3) square/cubic elements on a cube
  cell of side ``rve_size``; ``phase_id`` stores one byte per RVE element in
  lexicographic order (i fastest), RVE after RVE, starting at ``rve_off[b]``.
* ``phase_params[b, p]`` holds the parameters of phase p of RVE b: Lame
  (lambda, mu) for the linear and Neo-Hookean laws, (alpha, beta, kappa) for
  the Mooney-Rivlin family.
* ``dir_vals`` and ``f_ext`` are the prescribed displacements and external
  nodal forces at load factor 1.

Nothing here evaluates the method: the functions only place geometry, draw
random parameters from a seeded ``numpy.random.default_rng`` and convert
Young's modulus / Poisson ratio to Lame parameters.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

SEED_BASE = 12771


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    kinematics: str          # "small" | "finite"
    material: str            # "linear" | "neohooke" | "mooney_rivlin"
    X: np.ndarray            # (n_nodes, dim) float64
    conn: np.ndarray         # (n_elems, 2**dim) int32
    dir_dofs: np.ndarray     # (n_dir,) int32
    dir_vals: np.ndarray     # (n_dir,) float64, at load factor 1
    f_ext: np.ndarray        # (n_dofs,) float64, at load factor 1
    rve_res: np.ndarray      # (n_rve, dim) int32
    rve_off: np.ndarray      # (n_rve + 1,) int64
    phase_id: np.ndarray     # (rve_off[-1],) uint8
    phase_params: np.ndarray  # (n_rve, 2, n_params) float64
    rve_size: float = 1.0
    load_factors: Sequence[float] = (1.0,)
    macro_basis: str = "dirac"  # "dirac" (RVE per Gauss point) | "element" (RVE per element)
    macro_order: int = 1        # 1: Q4 / hex8 with 2 Gauss points per direction; 2: Q9 (2D) with 3
    seed: int = 0
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_gp(self) -> int:
        return (self.macro_order + 1) ** self.dim

    @property
    def n_qp(self) -> int:
        return self.n_elems * self.n_gp

    @property
    def n_rve(self) -> int:
        return int(self.rve_res.shape[0])

    @property
    def n_dofs(self) -> int:
        return self.n_nodes * self.dim

    def rve_phases(self, b: int) -> np.ndarray:
        """Phase ids of RVE b reshaped to (n3,) n2, n1 (x fastest)."""
        res = self.rve_res[b]
        ph = self.phase_id[self.rve_off[b]:self.rve_off[b + 1]]
        return ph.reshape(tuple(int(r) for r in res[::-1]))


# --------------------------------------------------------------------------
# material parameter conversion
# --------------------------------------------------------------------------

def lame_from_young(E, nu):
    """Lame parameters (lambda, mu) from Young's modulus and Poisson ratio."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


# --------------------------------------------------------------------------
# macro meshes
# --------------------------------------------------------------------------

def macro_q4_grid(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0):
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    XX, YY = np.meshgrid(xs, ys, indexing="xy")
    X = np.stack([XX.ravel(), YY.ravel()], axis=1)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    n0 = j * (nx + 1) + i
    conn = np.stack([n0, n0 + 1, n0 + nx + 2, n0 + nx + 1], axis=1).astype(np.int32)
    return X, conn


def macro_q9_grid(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0):
    """Biquadratic 9-node elements on a (2nx+1) x (2ny+1) node lattice (x
    fastest).  Per element: the corners counter-clockwise from the lower left,
    the mid-side nodes (bottom, right, top, left), then the centre."""
    mx, my = 2 * nx + 1, 2 * ny + 1
    XX, YY = np.meshgrid(np.linspace(0.0, Lx, mx), np.linspace(0.0, Ly, my), indexing="xy")
    X = np.stack([XX.ravel(), YY.ravel()], axis=1)
    conn = []
    for ey in range(ny):
        for ex in range(nx):
            i0, j0 = 2 * ex, 2 * ey
            n = lambda di, dj: (j0 + dj) * mx + i0 + di
            conn.append([n(0, 0), n(2, 0), n(2, 2), n(0, 2), n(1, 0), n(2, 1), n(1, 2), n(0, 1), n(1, 1)])
    return X, np.array(conn, dtype=np.int32)


def macro_hex8_grid(nx: int, ny: int, nz: int, L=(1.0, 1.0, 1.0)):
    xs = np.linspace(0.0, L[0], nx + 1)
    ys = np.linspace(0.0, L[1], ny + 1)
    zs = np.linspace(0.0, L[2], nz + 1)
    ZZ, YY, XX = np.meshgrid(zs, ys, xs, indexing="ij")
    X = np.stack([XX.ravel(), YY.ravel(), ZZ.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    sx, sy = 1, nx + 1
    sz = (nx + 1) * (ny + 1)
    n0 = k * sz + j * sy + i
    conn = np.stack([n0, n0 + sx, n0 + sx + sy, n0 + sy,
                     n0 + sz, n0 + sz + sx, n0 + sz + sx + sy, n0 + sz + sy],
                    axis=1).astype(np.int32)
    return X, conn


def macro_q4_cook(n: int = 20):
    """Mapped n x n Q4 mesh of Cook's membrane (corners (0,0), (480,440),
    (480,600), (0,440), the geometry of the paper's Sec. 5.2, Eq. (57))."""
    P1 = np.array([0.0, 0.0])
    P2 = np.array([480.0, 440.0])
    P3 = np.array([480.0, 600.0])
    P4 = np.array([0.0, 440.0])
    s = np.linspace(0.0, 1.0, n + 1)
    S, T = np.meshgrid(s, s, indexing="xy")
    S = S.ravel()[:, None]
    T = T.ravel()[:, None]
    X = (1 - S) * (1 - T) * P1 + S * (1 - T) * P2 + S * T * P3 + (1 - S) * T * P4
    _, conn = macro_q4_grid(n, n)
    return X, conn


# --------------------------------------------------------------------------
# RVE microstructures (phase id per element, lexicographic, x fastest)
# --------------------------------------------------------------------------

def _centroids(res: Sequence[int]):
    axes = [(np.arange(n) + 0.5) / n for n in res]
    grids = np.meshgrid(*axes[::-1], indexing="ij")   # (z,) y, x
    return [g for g in grids[::-1]]                     # x, y (, z)


def phases_laminate(n1: int, n2: int) -> np.ndarray:
    """Two layers normal to the second axis: rows j < n2/2 are phase 0."""
    j = np.arange(n2)[:, None] * np.ones((1, n1))
    return (j >= n2 // 2).astype(np.uint8).ravel()


def phases_circle(n1: int, n2: int, radius: float) -> np.ndarray:
    """Phase 1 where the element centroid lies inside the centred circle."""
    cx, cy = _centroids((n1, n2))
    inside = (cx - 0.5) ** 2 + (cy - 0.5) ** 2 < radius ** 2
    return inside.astype(np.uint8).ravel()


def phases_sphere(n: int, radius: float) -> np.ndarray:
    cx, cy, cz = _centroids((n, n, n))
    inside = (cx - 0.5) ** 2 + (cy - 0.5) ** 2 + (cz - 0.5) ** 2 < radius ** 2
    return inside.astype(np.uint8).ravel()


def phases_cross(n: int, half_width: float) -> np.ndarray:
    """Cross of half width ``half_width`` (relative to the unit cell)
    centred in the cell: phase 1 where |x-1/2| < hw or |y-1/2| < hw."""
    cx, cy = _centroids((n, n))
    inside = (np.abs(cx - 0.5) < half_width) | (np.abs(cy - 0.5) < half_width)
    return inside.astype(np.uint8).ravel()


# --------------------------------------------------------------------------
# boundary data
# --------------------------------------------------------------------------

def rollers_2d(X: np.ndarray, Lx: float, disp: float):
    """u_x = 0 on x = 0, u_y = 0 at the origin, u_x = disp on x = Lx."""
    tol = 1e-12 * max(1.0, Lx)
    left = np.where(np.abs(X[:, 0]) < tol)[0]
    right = np.where(np.abs(X[:, 0] - Lx) < tol)[0]
    origin = np.where((np.abs(X[:, 0]) < tol) & (np.abs(X[:, 1]) < tol))[0]
    dofs = np.concatenate([2 * left, 2 * origin + 1, 2 * right])
    vals = np.concatenate([np.zeros(len(left)), np.zeros(len(origin)),
                           np.full(len(right), disp)])
    order = np.argsort(dofs, kind="stable")
    return dofs[order].astype(np.int32), vals[order]


def rollers_3d(X: np.ndarray, Lx: float, disp: float):
    """Symmetry planes x = 0, y = 0, z = 0 and u_x = disp on x = Lx."""
    tol = 1e-12 * max(1.0, Lx)
    parts_d, parts_v = [], []
    for c in range(3):
        nodes = np.where(np.abs(X[:, c]) < tol)[0]
        parts_d.append(3 * nodes + c)
        parts_v.append(np.zeros(len(nodes)))
    right = np.where(np.abs(X[:, 0] - Lx) < tol)[0]
    parts_d.append(3 * right)
    parts_v.append(np.full(len(right), disp))
    dofs = np.concatenate(parts_d)
    vals = np.concatenate(parts_v)
    order = np.argsort(dofs, kind="stable")
    return dofs[order].astype(np.int32), vals[order]


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def _pack_phases(per_rve: List[np.ndarray]):
    off = np.zeros(len(per_rve) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(p) for p in per_rve])
    return off, np.concatenate(per_rve).astype(np.uint8)


def _problem(name, dim, kin, mat, X, conn, dofs, vals, res, off, ph, params,
             seed, load_factors=(1.0,), rve_size=1.0, f_ext=None, meta=None):
    n_dofs = X.shape[0] * dim
    return Problem(name=name, dim=dim, kinematics=kin, material=mat,
                   X=np.ascontiguousarray(X, dtype=np.float64),
                   conn=np.ascontiguousarray(conn, dtype=np.int32),
                   dir_dofs=np.ascontiguousarray(dofs, dtype=np.int32),
                   dir_vals=np.ascontiguousarray(vals, dtype=np.float64),
                   f_ext=(np.zeros(n_dofs) if f_ext is None else
                          np.ascontiguousarray(f_ext, dtype=np.float64)),
                   rve_res=np.ascontiguousarray(res, dtype=np.int32),
                   rve_off=np.ascontiguousarray(off, dtype=np.int64),
                   phase_id=np.ascontiguousarray(ph, dtype=np.uint8),
                   phase_params=np.ascontiguousarray(params, dtype=np.float64),
                   rve_size=float(rve_size), load_factors=tuple(load_factors),
                   seed=int(seed), meta=dict(meta or {}))


def cfg1(macro=(4, 4), rve=8, E=(1.0, 10.0), nu=0.3, disp=1e-3, order=1):
    """2D plane-strain linear laminate: 4x4 Q4 macro, 8x8 RVE, E 1 / 10
    (order=2: Q9 macro elements, 3x3 Gauss points)."""
    X, conn = macro_q4_grid(*macro) if order == 1 else macro_q9_grid(*macro)
    n_rve = conn.shape[0] * (order + 1) ** 2
    ph1 = phases_laminate(rve, rve)
    off, ph = _pack_phases([ph1] * n_rve)
    lam, mu = lame_from_young(np.array(E), nu)
    params = np.broadcast_to(np.stack([lam, mu], axis=1), (n_rve, 2, 2)).copy()
    dofs, vals = rollers_2d(X, 1.0, disp)
    res = np.full((n_rve, 2), rve, dtype=np.int32)
    return dataclasses.replace(
        _problem("cfg1", 2, "small", "linear", X, conn, dofs, vals, res, off,
                 ph, params, SEED_BASE + 1,
                 meta=dict(E=E, nu=nu, disp=disp, macro=macro, rve=rve)), macro_order=order)


def cfg2(macro=(64, 64), rve=32, vf=0.3, nu=0.3, disp=1e-3, seed=None, order=1):
    """2D linear: 64x64 Q4 macro, 32x32 RVE with a centred circle of volume
    fraction 0.3; inclusion/matrix E ratio lognormal(ln 10, 0.5) drawn per
    macro element (order=2: Q9 macro elements, 3x3 Gauss points)."""
    seed = SEED_BASE + 2 if seed is None else seed
    rng = np.random.default_rng(seed)
    X, conn = macro_q4_grid(*macro) if order == 1 else macro_q9_grid(*macro)
    ne = conn.shape[0]
    ngp = (order + 1) ** 2
    n_rve = ne * ngp
    ratio = np.exp(rng.normal(np.log(10.0), 0.5, size=ne))
    r = np.sqrt(vf / np.pi)
    ph1 = phases_circle(rve, rve, r)
    off, ph = _pack_phases([ph1] * n_rve)
    lam0, mu0 = lame_from_young(1.0, nu)
    lam1, mu1 = lame_from_young(ratio, nu)
    params = np.zeros((n_rve, 2, 2))
    params[:, 0, 0] = lam0
    params[:, 0, 1] = mu0
    params[:, 1, 0] = np.repeat(lam1, ngp)
    params[:, 1, 1] = np.repeat(mu1, ngp)
    dofs, vals = rollers_2d(X, 1.0, disp)
    res = np.full((n_rve, 2), rve, dtype=np.int32)
    return dataclasses.replace(
        _problem("cfg2", 2, "small", "linear", X, conn, dofs, vals, res, off,
                 ph, params, seed,
                 meta=dict(nu=nu, disp=disp, macro=macro, rve=rve, radius=r,
                           ratio=ratio)), macro_order=order)


def cfg3(macro=(128, 128), resolutions=(16, 32, 48), nu=0.3, disp=1e-3,
         seed=None):
    """2D uneven batch: RVE resolution per macro element from a 3-region
    Voronoi partition; radius U[0.1, 0.35] and E ratio U[5, 50] per element."""
    seed = SEED_BASE + 3 if seed is None else seed
    rng = np.random.default_rng(seed)
    X, conn = macro_q4_grid(*macro)
    ne = conn.shape[0]
    seeds = rng.uniform(0.0, 1.0, size=(3, 2))
    cent = X[conn].mean(axis=1)
    d2 = ((cent[:, None, :] - seeds[None, :, :]) ** 2).sum(axis=2)
    region = np.argmin(d2, axis=1)
    radius = rng.uniform(0.1, 0.35, size=ne)
    ratio = rng.uniform(5.0, 50.0, size=ne)
    per = []
    res = []
    for e in range(ne):
        n = resolutions[region[e]]
        p = phases_circle(n, n, radius[e])
        for _ in range(4):
            per.append(p)
            res.append((n, n))
    off, ph = _pack_phases(per)
    lam0, mu0 = lame_from_young(1.0, nu)
    lam1, mu1 = lame_from_young(ratio, nu)
    n_rve = ne * 4
    params = np.zeros((n_rve, 2, 2))
    params[:, 0, 0] = lam0
    params[:, 0, 1] = mu0
    params[:, 1, 0] = np.repeat(lam1, 4)
    params[:, 1, 1] = np.repeat(mu1, 4)
    dofs, vals = rollers_2d(X, 1.0, disp)
    return _problem("cfg3", 2, "small", "linear", X, conn, dofs, vals,
                    np.array(res, dtype=np.int32), off, ph, params, seed,
                    meta=dict(nu=nu, disp=disp, macro=macro, region=region,
                              voronoi_seeds=seeds, radius=radius, ratio=ratio,
                              resolutions=resolutions))


def cfg4(macro=(8, 8, 8), rve=10, vf=0.2, ratio=10.0, nu=0.3, disp=1e-3):
    """3D linear: 8^3 hex8 macro (2x2x2 Gauss), 10^3 hex8 RVE with a centred
    sphere of volume fraction 0.2, E ratio 10."""
    X, conn = macro_hex8_grid(*macro)
    n_rve = conn.shape[0] * 8
    r = (3.0 * vf / (4.0 * np.pi)) ** (1.0 / 3.0)
    ph1 = phases_sphere(rve, r)
    off, ph = _pack_phases([ph1] * n_rve)
    lam, mu = lame_from_young(np.array([1.0, ratio]), nu)
    params = np.broadcast_to(np.stack([lam, mu], axis=1), (n_rve, 2, 2)).copy()
    dofs, vals = rollers_3d(X, 1.0, disp)
    res = np.full((n_rve, 3), rve, dtype=np.int32)
    return _problem("cfg4", 3, "small", "linear", X, conn, dofs, vals, res, off,
                    ph, params, SEED_BASE + 4,
                    meta=dict(nu=nu, disp=disp, macro=macro, rve=rve, radius=r,
                              ratio=ratio))


def cfg5(macro=(64, 64), rve=32, mu=(1.0, 20.0), stretch=0.1, n_steps=10,
         seed=None):
    """2D finite-strain compressible Neo-Hookean: 64x64 Q4 macro, 32x32 RVE
    with a centred circle of radius U[0.15, 0.35] per macro element, shear
    moduli 1 and 20, lambda = 2 mu; 10 increments to 10 % stretch."""
    seed = SEED_BASE + 5 if seed is None else seed
    rng = np.random.default_rng(seed)
    X, conn = macro_q4_grid(*macro)
    ne = conn.shape[0]
    radius = rng.uniform(0.15, 0.35, size=ne)
    per = []
    for e in range(ne):
        p = phases_circle(rve, rve, radius[e])
        per.extend([p] * 4)
    off, ph = _pack_phases(per)
    n_rve = ne * 4
    params = np.zeros((n_rve, 2, 2))
    params[:, 0, 0] = 2.0 * mu[0]
    params[:, 0, 1] = mu[0]
    params[:, 1, 0] = 2.0 * mu[1]
    params[:, 1, 1] = mu[1]
    dofs, vals = rollers_2d(X, 1.0, stretch)
    res = np.full((n_rve, 2), rve, dtype=np.int32)
    lf = tuple((k + 1) / n_steps for k in range(n_steps))
    return _problem("cfg5", 2, "finite", "neohooke", X, conn, dofs, vals, res,
                    off, ph, params, seed, load_factors=lf,
                    meta=dict(mu=mu, stretch=stretch, macro=macro, rve=rve,
                              radius=np.repeat(radius, 4)))


def cook(n_macro=20, n_rve=30, n_steps=22, traction=(-5.0, 10.0)):
    """Cook's membrane of the paper's Sec. 5.2: mapped Q4 macro mesh, left edge
    clamped, uniform traction on the right edge, 30x30 RVE of side 6 with a
    centred cross of width 2 (phase 1) and the two Mooney-Rivlin parameter
    sets (alpha, beta, kappa) = (27, 18, 60) and (13.5, 6.5, 30)."""
    X, conn = macro_q4_cook(n_macro)
    n_nodes = X.shape[0]
    left = np.where(np.abs(X[:, 0]) < 1e-9)[0]
    dofs = np.sort(np.concatenate([2 * left, 2 * left + 1])).astype(np.int32)
    vals = np.zeros(len(dofs))
    # consistent nodal forces of a uniform traction on the right edge
    right = np.where(np.abs(X[:, 0] - 480.0) < 1e-9)[0]
    right = right[np.argsort(X[right, 1])]
    f = np.zeros(2 * n_nodes)
    t = np.asarray(traction, dtype=np.float64)
    for a, b in zip(right[:-1], right[1:]):
        L = np.linalg.norm(X[b] - X[a])
        f[2 * a:2 * a + 2] += 0.5 * L * t
        f[2 * b:2 * b + 2] += 0.5 * L * t
    n_r = conn.shape[0] * 4
    ph1 = phases_cross(n_rve, 1.0 / 6.0)
    off, ph = _pack_phases([ph1] * n_r)
    params = np.zeros((n_r, 2, 3))
    params[:, 0] = (27.0, 18.0, 60.0)
    params[:, 1] = (13.5, 6.5, 30.0)
    res = np.full((n_r, 2), n_rve, dtype=np.int32)
    lf = tuple((k + 1) / n_steps for k in range(n_steps))
    return _problem("cook", 2, "finite", "mooney_rivlin", X, conn, dofs, vals,
                    res, off, ph, params, 0, load_factors=lf, rve_size=6.0,
                    f_ext=f, meta=dict(n_macro=n_macro, n_rve=n_rve,
                                       traction=traction))


# Strain box of the surrogate's training set: Green-Lagrange strains met along
# the Neo-Hookean configuration's uniaxial path to 10 % stretch (E11 up to
# 0.105, lateral contraction, small shear) with a margin, and the phase-1
# volume fractions of its inclusions (radius 0.15 to 0.35).
SURROGATE_BOX = dict(E11=(-0.005, 0.115), E22=(-0.05, 0.005), E12=(-0.02, 0.02))


def cfg5_material_points(n: int, rve: int = 32, mu=(1.0, 20.0), seed: int = SEED_BASE + 50) -> Problem:
    """n RVEs of the Neo-Hookean configuration's kind (circle of radius
    U[0.15, 0.35] drawn per RVE, shear moduli 1 / 20, lambda = 2 mu), hung on
    a dummy strip of n/4 macro elements (numbered along the strip, so the
    macro band stays narrow): the batch of a material-point
    driver (training data of the surrogate)."""
    if n % 4:
        raise ValueError("n must be a multiple of 4")
    rng = np.random.default_rng(seed)
    X, conn = macro_q4_grid(1, n // 4, 1.0, float(n // 4))
    radius = rng.uniform(0.15, 0.35, size=n)
    off, ph = _pack_phases([phases_circle(rve, rve, r) for r in radius])
    params = np.zeros((n, 2, 2))
    params[:, 0] = (2.0 * mu[0], mu[0])
    params[:, 1] = (2.0 * mu[1], mu[1])
    res = np.full((n, 2), rve, dtype=np.int32)
    return _problem("cfg5_points", 2, "finite", "neohooke", X, conn, np.zeros(0, dtype=np.int32), np.zeros(0),
                    res, off, ph, params, seed, meta=dict(radius=radius))


def surrogate_samples(n: int, seed: int, box=None):
    """n Green-Lagrange strains uniform in ``box`` and the matching
    symmetric right stretch tensors U = sqrt(I + 2E) (row-major 2x2), the
    macro gradients at which training RVE responses are computed."""
    box = SURROGATE_BOX if box is None else box
    rng = np.random.default_rng(seed)
    E = np.stack([rng.uniform(*box["E11"], n), rng.uniform(*box["E22"], n), rng.uniform(*box["E12"], n)], axis=1)
    Cm = np.zeros((n, 2, 2))
    Cm[:, 0, 0] = 1 + 2 * E[:, 0]
    Cm[:, 1, 1] = 1 + 2 * E[:, 1]
    Cm[:, 0, 1] = Cm[:, 1, 0] = 2 * E[:, 2]
    lam, V = np.linalg.eigh(Cm)
    U = np.einsum("nij,nj,nkj->nik", V, np.sqrt(lam), V)
    return E, U.reshape(n, 4)


def mlp_init(sizes: Sequence[int], seed: int = SEED_BASE) -> np.ndarray:
    """Initial parameters of a multilayer perceptron in the flat layout
    W_0, b_0, W_1, b_1, ... (W_l of shape (sizes[l+1], sizes[l]), row-major):
    weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        a = np.sqrt(6.0 / (sizes[i] + sizes[i + 1]))
        parts.append(rng.uniform(-a, a, size=sizes[i + 1] * sizes[i]))
        parts.append(np.zeros(sizes[i + 1]))
    return np.concatenate(parts)


_CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4,
            "cfg5": cfg5, "cook": cook}


def config_names():
    return list(_CONFIGS)


def config(name: str, **kw) -> Problem:
    return _CONFIGS[name](**kw)


def subset_problem(p: Problem, rves: Optional[np.ndarray] = None) -> Problem:
    """The same problem with the RVE batch restricted to the RVEs of the first
    macro elements (used to time or check a bounded sample)."""
    if rves is None:
        return p
    rves = np.asarray(rves)
    per = [p.phase_id[p.rve_off[b]:p.rve_off[b + 1]] for b in rves]
    off, ph = _pack_phases(per)
    return dataclasses.replace(p, rve_res=p.rve_res[rves].copy(), rve_off=off,
                               phase_id=ph,
                               phase_params=p.phase_params[rves].copy())


def element_basis(p: Problem) -> Problem:
    """The same problem with the piecewise-constant macro basis of the
    fluctuation: one RVE per macro element, the one the generators placed at
    the element's Gauss points (all Gauss points of an element carry the same
    RVE in every generator; anything else is rejected)."""
    if p.macro_basis != "dirac":
        raise ValueError("expected a problem with one RVE per Gauss point")
    ng = p.n_gp
    for e in range(p.n_elems):
        b0 = e * ng
        ph0 = p.phase_id[p.rve_off[b0]:p.rve_off[b0 + 1]]
        for b in range(b0 + 1, b0 + ng):
            if (not np.array_equal(p.rve_res[b], p.rve_res[b0])
                    or not np.array_equal(p.phase_params[b], p.phase_params[b0])
                    or not np.array_equal(p.phase_id[p.rve_off[b]:p.rve_off[b + 1]], ph0)):
                raise ValueError(f"the Gauss points of element {e} carry different RVEs")
    q = subset_problem(p, np.arange(p.n_elems) * ng)
    return dataclasses.replace(q, macro_basis="element", name=p.name + "_element")


# ---------------------------------------------------------------------------
# 1+1D benchmark of Sec. 5.1 (material data and boundary data only)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class OneDProblem:
    order: int                 # Lagrange order q of both scales
    n_macro: int
    n_micro: int
    basis: str                 # "dirac" | "element"
    macro_length: float
    body_load: float
    phi_left: float
    phi_right: float
    lambda_gp: np.ndarray      # (n_micro, 5): lambda at the 5 Gauss-Legendre points of each RVE element


def oned_problem(k: int, order: int, basis: str = "dirac") -> OneDProblem:
    """Sec. 5.1 with 2^k macro and 2^k RVE elements: bar (0, 1000), RVE
    (0, 1), lambda(X~) = 20 / cos(2 pi X~ / 3 - pi / 3) sampled at the RVE
    quadrature points, B = 1, phi(0) = 0, phi(1000) = 37575 sqrt(3) / (2 pi)."""
    n = 2 ** k
    xg, _ = np.polynomial.legendre.leggauss(5)
    h = 1.0 / n
    xt = h * np.arange(n)[:, None] + (xg[None, :] + 1.0) * h / 2.0
    lam = 20.0 / np.cos(2.0 * np.pi / 3.0 * xt - np.pi / 3.0)
    return OneDProblem(order=order, n_macro=n, n_micro=n, basis=basis, macro_length=1000.0,
                       body_load=1.0, phi_left=0.0, phi_right=37575.0 * np.sqrt(3.0) / (2.0 * np.pi),
                       lambda_gp=np.ascontiguousarray(lam))
