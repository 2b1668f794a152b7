"""The 1+1-dimensional benchmark of Sec. 5.1 (FP64), oracle side.

Macro body (0, 1000), RVE (0, 1), micro energy Psi~ = lambda(X~) (F~^2 - 1)
with lambda(X~) = 20 / cos(2 pi X~ / 3 - pi / 3), body load B = 1, phi(0) = 0,
phi(1000) = 37575 sqrt(3) / (2 pi) and zero fluctuation at both RVE ends
(condition (ii) of Eq. (15)).  F~ = dphi/dX + dw~/dX~ and P~ = 2 lambda F~, so
the problem is linear and its discrete solution is the minimiser of the
quadratic discrete energy.

Six discretisations p = [p_X, p_X~] of the fluctuation: Lagrange order q in
X~ (1 or 2) and, in X, either the same order q (continuous tensor-product
basis, "full"), piecewise constant per macro element ("const", the basis of
Eqs. (constSolution1)-(constSolution2)), or Dirac pulses at the macro Gauss
points ("dirac", Eqs. (31)-(35)).  The macro deformation uses order q.  Both
meshes are uniform with 2^k elements.

Quadrature: q + 1 Gauss points per macro element (the Dirac RVEs sit at these
points), 5 per micro element (lambda is not a polynomial; its quadrature error
stays far below the discretisation error).

Because lambda depends on X~ only and the micro mesh is the same everywhere,
every block of the Hessian is a Kronecker product of a macro matrix (taken
with the macro quadrature) and a micro matrix:
    K_pp = S_X * K_FF,  K_pw = G_X (x) K_Fw,  K_ww = M_X (x) K_ww~,
with S_X = int N_A' N_B', G_X = int N_A' c_B, M_X = int c_A c_B over the macro
rule (c_B the X-basis of the fluctuation), K_FF = int 2 lambda,
K_Fw = int 2 lambda R_b', K_ww~ = int 2 lambda R_a' R_b' over the RVE.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

L_MACRO = 1000.0
PHI_END = 37575.0 * np.sqrt(3.0) / (2.0 * np.pi)
B_LOAD = 1.0
N_GAUSS_MICRO = 5


def lam(xt):
    """Material parameter lambda(X~) of Sec. 5.1 (J/mm)."""
    return 20.0 / np.cos(2.0 * np.pi / 3.0 * np.asarray(xt) - np.pi / 3.0)


def phi_exact(X):
    """Closed-form macro deformation of Sec. 5.1."""
    X = np.asarray(X)
    s = np.sqrt(3.0) / np.pi
    return -3.0 * s / 160.0 * X ** 2 + 3003.0 * s / 80.0 * X


def F_exact(X):
    X = np.asarray(X)
    s = np.sqrt(3.0) / np.pi
    return -3.0 * s / 80.0 * X + 3003.0 * s / 80.0


def w_exact(X, xt):
    """Closed-form fluctuation of Sec. 5.1 (broadcasts X against X~)."""
    xt = np.asarray(xt)
    return F_exact(X) * (np.sin(2.0 * np.pi / 3.0 * xt - np.pi / 3.0) / np.sqrt(3.0) - xt + 0.5)


def lagrange(q, xi):
    """Shape functions of order q on [-1, 1] with equally spaced nodes
    (-1, 1 for q = 1; -1, 0, 1 for q = 2) and their xi-derivatives."""
    xi = np.asarray(xi, dtype=np.float64)
    if q == 1:
        N = np.stack([(1 - xi) / 2, (1 + xi) / 2], axis=-1)
        dN = np.stack([-0.5 + 0 * xi, 0.5 + 0 * xi], axis=-1)
    elif q == 2:
        N = np.stack([xi * (xi - 1) / 2, 1 - xi ** 2, xi * (xi + 1) / 2], axis=-1)
        dN = np.stack([xi - 0.5, -2 * xi, xi + 0.5], axis=-1)
    else:
        raise ValueError(q)
    return N, dN


def gauss(n):
    return np.polynomial.legendre.leggauss(n)


@dataclasses.dataclass
class Mesh:
    n_el: int
    q: int
    length: float

    @property
    def n_nodes(self):
        return self.q * self.n_el + 1

    @property
    def h(self):
        return self.length / self.n_el

    def conn(self, e):
        return self.q * e + np.arange(self.q + 1)


def micro_matrices(k: int, q: int):
    """K_FF (scalar), K_Fw (n_int,) and K_ww~ (n_int, n_int) of the RVE with
    2^k elements of order q; interior nodes only (zero fluctuation at both
    ends)."""
    m = Mesh(2 ** k, q, 1.0)
    xg, wg = gauss(N_GAUSS_MICRO)
    N, dN = lagrange(q, xg)
    j = m.h / 2.0
    nn = m.n_nodes
    KFF = 0.0
    KFw = np.zeros(nn)
    rows, cols, vals = [], [], []
    for e in range(m.n_el):
        c = m.conn(e)
        xt = m.h * e + (xg + 1.0) * j
        w2l = 2.0 * lam(xt) * wg * j                  # 2 lambda times the weight
        dR = dN / j                                   # (n_g, q+1) dR/dX~
        KFF += w2l.sum()
        KFw[c] += dR.T @ w2l
        ke = (dR * w2l[:, None]).T @ dR
        rows.append(np.repeat(c, q + 1))
        cols.append(np.tile(c, q + 1))
        vals.append(ke.ravel())
    Kww = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nn, nn))
    inner = np.arange(1, nn - 1)
    return KFF, KFw[inner], Kww[inner][:, inner].tocsr()


def macro_matrices(k: int, q: int, setting: str):
    """S_X (n_phi x n_phi), G_X (n_phi x n_c), M_X (n_c x n_c), the load
    vector and the fluctuation's X-basis size n_c, over q + 1 Gauss points per
    macro element."""
    m = Mesh(2 ** k, q, L_MACRO)
    xg, wg = gauss(q + 1)
    N, dN = lagrange(q, xg)
    J = m.h / 2.0
    dNX = dN / J
    ng = q + 1
    n_phi = m.n_nodes
    n_c = {"full": m.n_nodes, "const": m.n_el, "dirac": m.n_el * ng}[setting]
    S = sp.lil_matrix((n_phi, n_phi))
    G = sp.lil_matrix((n_phi, n_c))
    Mx = sp.lil_matrix((n_c, n_c))
    f = np.zeros(n_phi)
    for e in range(m.n_el):
        c = m.conn(e)
        for g in range(ng):
            wJ = wg[g] * J
            if setting == "full":
                cid, cval = c, N[g]
            elif setting == "const":
                cid, cval = np.array([e]), np.array([1.0])
            else:
                cid, cval = np.array([e * ng + g]), np.array([1.0])
            S[np.ix_(c, c)] += wJ * np.outer(dNX[g], dNX[g])
            G[np.ix_(c, cid)] += wJ * np.outer(dNX[g], cval)
            Mx[np.ix_(cid, cid)] += wJ * np.outer(cval, cval)
            f[c] += wJ * B_LOAD * N[g]
    return S.tocsr(), G.tocsr(), Mx.tocsr(), f, n_c


@dataclasses.dataclass
class Solution:
    k: int
    q: int
    setting: str
    phi: np.ndarray        # macro nodal values (n_phi,)
    w: np.ndarray          # (n_c, n_int) fluctuation coefficients per X-basis function
    macro: Mesh
    micro: Mesh


def solve(k: int, q: int, setting: str) -> Solution:
    """Discrete solution of setting p = [setting, q] with 2^k macro and 2^k
    micro elements: the minimiser of the discrete energy under the Dirichlet
    data (direct sparse solve of the whole coupled system)."""
    KFF, KFw, Kww = micro_matrices(k, q)
    S, G, Mx, f, n_c = macro_matrices(k, q, setting)
    n_phi = S.shape[0]
    n_int = Kww.shape[0]
    A = sp.bmat([[S * KFF, sp.kron(G, KFw[None, :])],
                 [sp.kron(G.T, KFw[:, None]), sp.kron(Mx, Kww)]]).tocsr()
    rhs = np.concatenate([f, np.zeros(n_c * n_int)])
    dirv = np.zeros(A.shape[0])
    dirv[n_phi - 1] = PHI_END
    fixed = np.array([0, n_phi - 1])
    free = np.setdiff1d(np.arange(A.shape[0]), fixed)
    x = dirv.copy()
    x[free] = spla.spsolve(A[free][:, free].tocsc(), rhs[free] - A[free] @ dirv)
    return Solution(k=k, q=q, setting=setting, phi=x[:n_phi], w=x[n_phi:].reshape(n_c, n_int),
                    macro=Mesh(2 ** k, q, L_MACRO), micro=Mesh(2 ** k, q, 1.0))


def _micro_eval(sol: Solution, coef, n_pts=6):
    """Values of micro fields (rows of coef, interior coefficients) at n_pts
    Gauss points per micro element; returns (points, weights, values)."""
    m = sol.micro
    xg, wg = gauss(n_pts)
    N, _ = lagrange(m.q, xg)
    full = np.zeros((coef.shape[0], m.n_nodes))
    full[:, 1:-1] = coef
    pts, wts, vals = [], [], []
    for e in range(m.n_el):
        c = m.conn(e)
        pts.append(m.h * e + (xg + 1.0) * m.h / 2.0)
        wts.append(wg * m.h / 2.0)
        vals.append(full[:, c] @ N.T)
    return np.concatenate(pts), np.concatenate(wts), np.concatenate(vals, axis=1)


def errors(sol: Solution, n_pts=6):
    """Relative L2 errors err_phi and err_w of Sec. 5.1 against the closed
    form.  Full/const: both integrals by n_pts x n_pts Gauss points per
    element pair.  Dirac: the fluctuation exists at the macro Gauss points
    only, so the macro integral of the error uses the macro rule there; the
    norm of the closed form uses the tensor rule."""
    M = sol.macro
    xg, wg = gauss(n_pts)
    N, _ = lagrange(M.q, xg)
    num = den = 0.0
    Xs, Ws, cvals = [], [], []
    for e in range(M.n_el):
        c = M.conn(e)
        X = M.h * e + (xg + 1.0) * M.h / 2.0
        W = wg * M.h / 2.0
        ph = N @ sol.phi[c]
        pa = phi_exact(X)
        num += float(np.sum(W * (ph - pa) ** 2))
        den += float(np.sum(W * pa ** 2))
        Xs.append(X)
        Ws.append(W)
        if sol.setting == "full":
            cvals.append(N @ sol.w[c])                # (n_pts, n_int)
        elif sol.setting == "const":
            cvals.append(np.repeat(sol.w[e][None, :], n_pts, axis=0))
    err_phi = np.sqrt(num / den)
    Xs, Ws = np.concatenate(Xs), np.concatenate(Ws)
    xt, wt, _ = _micro_eval(sol, np.zeros((1, sol.w.shape[1])), n_pts)
    wa = w_exact(Xs[:, None], xt[None, :])
    den_w = float(Ws @ (wa ** 2) @ wt)
    if sol.setting == "dirac":
        ng = M.q + 1
        xq, wq = gauss(ng)
        Xq = (M.h * np.arange(M.n_el)[:, None] + (xq[None, :] + 1.0) * M.h / 2.0).ravel()
        Wq = np.tile(wq * M.h / 2.0, M.n_el)
        _, _, wh = _micro_eval(sol, sol.w, n_pts)     # (n_gp, n_micro_pts)
        num_w = float(Wq @ ((wh - w_exact(Xq[:, None], xt[None, :])) ** 2) @ wt)
    else:
        _, _, wh = _micro_eval(sol, np.concatenate(cvals, axis=0), n_pts)
        num_w = float(Ws @ ((wh - wa) ** 2) @ wt)
    return float(err_phi), float(np.sqrt(num_w / den_w))


def lambda_eff():
    """Harmonic mean of lambda over the RVE: 40 pi / (3 sqrt 3)."""
    return 40.0 * np.pi / (3.0 * np.sqrt(3.0))
