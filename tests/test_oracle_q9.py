"""Pins of the oracle's biquadratic (Q9) macro elements, the [delta, 2]
setting of Sec. 5.1 carried to 2D (3x3 Gauss points, one RVE each).

* Shape functions: Kronecker property at the nodes, partition of unity,
  exact reproduction of every quadratic polynomial, derivatives against
  central differences.
* The 3x3 Gauss rule integrates xi^a eta^b exactly up to degree 5.
* Patch tests with a homogeneous RVE (C-bar equals the constituent tensor):
  a uniform strain on a distorted mesh and a quadratic displacement field in
  equilibrium (div sigma = 0) are reproduced exactly at every node when the
  boundary nodes carry the exact values.  Bilinear Q4 elements on the same
  field are nodally exact too on a uniform mesh, but their interpolant misses
  it inside the elements, where the Q9 centre nodes carry the exact value.
"""
import dataclasses

import numpy as np

import workloads as W
from oracle import macro as M


def test_q9_shape_functions():
    for a, xa in enumerate(M.Q9_NODES):
        N, _ = M.q9_shape(xa)
        e = np.zeros(9)
        e[a] = 1.0
        np.testing.assert_allclose(N, e, atol=1e-15)
    rng = np.random.default_rng(3)
    for _ in range(20):
        xi = rng.uniform(-1, 1, 2)
        N, dN = M.q9_shape(xi)
        assert abs(N.sum() - 1.0) < 1e-14
        for (p, q) in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (2, 1), (1, 2), (2, 2)]:
            f = M.Q9_NODES[:, 0] ** p * M.Q9_NODES[:, 1] ** q
            assert abs(N @ f - xi[0] ** p * xi[1] ** q) < 1e-14
        h = 1e-6
        for J in range(2):
            d = np.zeros(2)
            d[J] = h
            fd = (M.q9_shape(xi + d)[0] - M.q9_shape(xi - d)[0]) / (2 * h)
            np.testing.assert_allclose(dN[:, J], fd, atol=1e-9)


def test_three_point_gauss_rule_is_exact_to_degree_five():
    x, w = M.GAUSS3
    for p in range(6):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.sum(w * x ** p) - exact) < 1e-14


def _homogeneous(p):
    pp = p.phase_params.copy()
    pp[:, 1] = pp[:, 0]
    return dataclasses.replace(p, phase_params=pp)


def _with_boundary_values(p, field):
    """All boundary nodes prescribed with field(X), no other loads."""
    X = p.X
    bnd = np.where((np.abs(X[:, 0]) < 1e-12) | (np.abs(X[:, 0] - 1) < 1e-12)
                   | (np.abs(X[:, 1]) < 1e-12) | (np.abs(X[:, 1] - 1) < 1e-12))[0]
    dofs = np.sort(np.concatenate([2 * bnd, 2 * bnd + 1])).astype(np.int32)
    u = field(X)
    return dataclasses.replace(p, dir_dofs=dofs, dir_vals=u.ravel()[dofs].copy(),
                               f_ext=np.zeros(p.n_dofs))


def _distort(p, amp=0.08, seed=4):
    """Move interior corner nodes; mid-side and centre nodes follow (straight
    edges), so the map stays affine on no element."""
    rng = np.random.default_rng(seed)
    X = p.X.copy()
    m = int(round(np.sqrt(X.shape[0])))
    grid = X.reshape(m, m, 2)
    for j in range(2, m - 1, 2):
        for i in range(2, m - 1, 2):
            grid[j, i] += amp * (rng.uniform(-1, 1, 2)) / (m - 1)
    for j in range(0, m, 2):          # mid-edge nodes on horizontal edges
        for i in range(1, m, 2):
            grid[j, i] = 0.5 * (grid[j, i - 1] + grid[j, i + 1])
    for j in range(1, m, 2):
        for i in range(0, m, 2):       # mid-edge nodes on vertical edges
            grid[j, i] = 0.5 * (grid[j - 1, i] + grid[j + 1, i])
        for i in range(1, m, 2):       # centres
            grid[j, i] = 0.25 * (grid[j - 1, i - 1] + grid[j - 1, i + 1] + grid[j + 1, i - 1] + grid[j + 1, i + 1])
    return dataclasses.replace(p, X=grid.reshape(-1, 2))


def test_q9_patch_test_uniform_strain_on_a_distorted_mesh():
    p = _homogeneous(W.config("cfg2", macro=(3, 3), rve=6, order=2))
    p = _distort(p)
    eps = np.array([1e-3, -4e-4, 6e-4])
    field = lambda X: np.stack([eps[0] * X[:, 0] + 0.5 * eps[2] * X[:, 1],
                                0.5 * eps[2] * X[:, 0] + eps[1] * X[:, 1]], axis=1)
    p = _with_boundary_values(p, field)
    st, _ = M.solve(p, tol=1e-13)
    ex = field(p.X).ravel()
    assert np.abs(st.u - ex).max() <= 1e-12 * np.abs(ex).max()


def _equilibrium_quadratic(lam, mu, s=1e-3):
    """u_x = s (x^2 + a2 x y), u_y = s (b2 x y + y^2) with
    (lam + 2mu) u_x,xx + mu u_x,yy + (lam + mu) u_y,xy = 0 and
    mu u_y,xx + (lam + 2mu) u_y,yy + (lam + mu) u_x,xy = 0."""
    b2 = -2.0 * (lam + 2.0 * mu) / (lam + mu)
    a2 = -2.0 * (lam + 2.0 * mu) / (lam + mu)
    return lambda X: s * np.stack([X[:, 0] ** 2 + a2 * X[:, 0] * X[:, 1],
                                   b2 * X[:, 0] * X[:, 1] + X[:, 1] ** 2], axis=1)


def test_q9_reproduces_a_quadratic_equilibrium_field_and_q4_does_not():
    base = _homogeneous(W.config("cfg2", macro=(3, 3), rve=6, order=2))
    lam, mu = base.phase_params[0, 0]
    field = _equilibrium_quadratic(lam, mu)
    p = _with_boundary_values(base, field)
    st, _ = M.solve(p, tol=1e-13)
    ex = field(p.X).ravel()
    assert np.abs(st.u - ex).max() <= 1e-11 * np.abs(ex).max()
    p4 = _with_boundary_values(_homogeneous(W.config("cfg2", macro=(6, 6), rve=6)), field)
    st4, _ = M.solve(p4, tol=1e-13)
    u4 = st4.u.reshape(-1, 2)
    centres = p4.X[p4.conn].mean(axis=1)
    u4c = u4[p4.conn].mean(axis=1)          # the Q4 interpolant at element centres
    assert np.abs(u4c - field(centres)).max() > 1e-3 * np.abs(ex).max()
