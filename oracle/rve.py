"""RVE element integration, periodic null-space reduction and condensation
(FP64, SciPy sparse direct), oracle side.

What one macro Gauss point b needs (Sec. 3, Eqs. (34)-(35); Sec. 4,
Eqs. (39)-(49)):

* micro gradient: F~ = F_b + grad w~ (Eq. (11)); small strain uses
  eps~ = eps_b + sym grad w~ with the Voigt order of ``tensors``;
* micro residual r_b = sum_l eta_l G^T P~ (Eq. (35) with the periodic
  test space (iii) of Eq. (15));
* tangent blocks K_ww = int G^T A G (the RVE block of L, Eq. (41)),
  K_wF = int G^T A (its coupling to F, Eq. (40)) and K_FF = int A (Eq. (39));
* integral of the micro stress, int P~ (so that P = <P~>, Eq. (17)).

Discretisation choices (the paper leaves them open; see the readings listed
in the design notes): an n1 x n2 (x n3) grid of Q4 (hex8) box elements on a
cube cell of side L (edge L/n_i along direction i), full 2-point Gauss-Legendre quadrature per
direction, periodic images identified by (i mod n1, j mod n2, k mod n3) and
the fluctuation of the corner node fixed to zero (periodicity then fixes all
corners).

Condensation (Sec. 4.2, Eqs. (46)-(49)): with K_ww [X_F | x_r] =
[K_wF | r_b]
    C_b   = (K_FF - K_wF^T X_F) / |Omega|       (Schur complement, D L^-1 E)
    Phat_b = (int P~ - K_wF^T x_r) / |Omega|    (the -D L^-1 R_micro term)
and after the macro update dF_b the fluctuation moves by
    dw_b = -(x_r + X_F dF_b)                     (Eq. (49)).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import tensors

GP1 = np.array([-1.0, 1.0]) / np.sqrt(3.0)


# --------------------------------------------------------------------------
# reference element
# --------------------------------------------------------------------------

def ref_nodes(dim):
    if dim == 2:
        return np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    return np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]],
                    dtype=np.float64)


def gauss_points(dim):
    """2-point Gauss-Legendre points, xi fastest; all weights equal 1."""
    if dim == 2:
        return np.array([[GP1[i], GP1[j]] for j in range(2) for i in range(2)])
    return np.array([[GP1[i], GP1[j], GP1[k]]
                     for k in range(2) for j in range(2) for i in range(2)])


def dshape_ref(xi):
    """Derivatives dN_a/dxi_J of the (bi/tri)linear shape functions."""
    nodes = ref_nodes(len(xi))
    dim = len(xi)
    d = np.ones((nodes.shape[0], dim))
    for a, na in enumerate(nodes):
        for J in range(dim):
            v = 0.5 ** dim
            for K in range(dim):
                v *= na[K] if K == J else (1.0 + na[K] * xi[K])
            d[a, J] = v
    return d


def shape_ref(xi):
    nodes = ref_nodes(len(xi))
    return np.prod(0.5 * (1.0 + nodes * xi[None, :]), axis=1)


def micro_gradients(dim, h):
    """dN_a/dX~_J at each Gauss point of a box element with edge lengths h
    (scalar or per direction), shape (n_gp, n_nodes, dim), and the
    quadrature weight prod(h/2)."""
    gps = gauss_points(dim)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (dim,))
    return np.stack([dshape_ref(g) * (2.0 / h)[None, :] for g in gps]), float(np.prod(0.5 * h))


def strain_B(dN):
    """Small-strain B (Voigt, engineering shear) from dN (n_nodes, dim)."""
    nn, dim = dN.shape
    if dim == 2:
        B = np.zeros((3, 2 * nn))
        B[0, 0::2] = dN[:, 0]
        B[1, 1::2] = dN[:, 1]
        B[2, 0::2] = dN[:, 1]
        B[2, 1::2] = dN[:, 0]
        return B
    B = np.zeros((6, 3 * nn))
    B[0, 0::3] = dN[:, 0]
    B[1, 1::3] = dN[:, 1]
    B[2, 2::3] = dN[:, 2]
    B[3, 1::3] = dN[:, 2]
    B[3, 2::3] = dN[:, 1]
    B[4, 0::3] = dN[:, 2]
    B[4, 2::3] = dN[:, 0]
    B[5, 0::3] = dN[:, 1]
    B[5, 1::3] = dN[:, 0]
    return B


def grad_G(dN):
    """Finite-strain G with (grad w)_iJ = sum_a dN_a/dX_J w_ai, rows in the
    row-major order (i, J) -> dim*i + J, columns (a, i) -> dim*a + i."""
    nn, dim = dN.shape
    G = np.zeros((dim * dim, dim * nn))
    for i in range(dim):
        for J in range(dim):
            G[dim * i + J, i::dim] = dN[:, J]
    return G


# --------------------------------------------------------------------------
# periodic grid bookkeeping
# --------------------------------------------------------------------------

def element_nodes(res):
    """Periodic node ids (lexicographic, x fastest) of every element, shape
    (n_elems, 2**dim), elements in lexicographic order."""
    res = [int(r) for r in res]
    dim = len(res)
    offs = ref_nodes(dim) > 0
    if dim == 2:
        n1, n2 = res
        j, i = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
        i, j = i.ravel(), j.ravel()
        cols = [((i + o[0]) % n1) + n1 * ((j + o[1]) % n2) for o in offs]
    else:
        n1, n2, n3 = res
        k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
        i, j, k = i.ravel(), j.ravel(), k.ravel()
        cols = [((i + o[0]) % n1) + n1 * (((j + o[1]) % n2) + n2 * ((k + o[2]) % n3))
                for o in offs]
    return np.stack(cols, axis=1)


def element_dofs(res):
    dim = len(res)
    en = element_nodes(res)
    return (en[:, :, None] * dim + np.arange(dim)[None, None, :]).reshape(en.shape[0], -1)


# --------------------------------------------------------------------------
# RVE assembly
# --------------------------------------------------------------------------

@dataclasses.dataclass
class RVESystem:
    K_ww: sp.csr_matrix      # (N, N) reduced (corner pinned)
    K_wF: np.ndarray         # (N, nF)
    K_FF: np.ndarray         # (nF, nF)
    r: np.ndarray            # (N,)
    P_int: np.ndarray        # (nF,)  integral of the micro stress
    energy: float            # integral of the micro energy
    free: np.ndarray         # indices of the reduced DOFs in the periodic numbering
    n_full: int              # DOFs of the periodic field before the pin
    volume: float            # |Omega|
    r_round: float = 0.0     # finite strain: size of a rounding bound of the element residual terms


def n_macro_components(dim, kinematics):
    if kinematics == "small":
        return 3 if dim == 2 else 6
    return dim * dim


def assemble_rve(res, phases, params, kinematics, material, macro, w_full=None,
                 L=1.0) -> RVESystem:
    """Element integration and periodic reduction of one RVE.

    res: (n1, n2[, n3]); phases: phase id per element (lexicographic);
    params: (2, n_params) per-phase parameters; macro: eps_b (Voigt) for
    small strain or F_b (row-major, dim*dim) for finite strain; w_full:
    periodic nodal fluctuation (n_nodes*dim,), corner entry zero.
    """
    res = [int(r) for r in res]
    dim = len(res)
    nF = n_macro_components(dim, kinematics)
    n_nodes = int(np.prod(res))
    n_full = n_nodes * dim
    h = np.array([L / r for r in res])
    phases = np.asarray(phases).ravel().astype(np.int64)
    ne = phases.size
    edofs = element_dofs(res)
    w = np.zeros(n_full) if w_full is None else np.asarray(w_full, dtype=np.float64)
    we = w[edofs]                                   # (ne, nd)
    dNs, wt = micro_gradients(dim, h)
    nd = edofs.shape[1]
    ke = np.zeros((ne, nd, nd))
    kwF = np.zeros((ne, nd, nF))
    re = np.zeros((ne, nd))
    re_abs = np.zeros((ne, nd))   # finite strain: rounding bound of re
    K_FF = np.zeros((nF, nF))
    P_int = np.zeros(nF)
    energy = 0.0
    macro = np.asarray(macro, dtype=np.float64)
    for dN in dNs:
        if kinematics == "small":
            B = strain_B(dN)
            eps = macro[None, :] + we @ B.T                      # (ne, nF)
            Cs = np.stack([tensors.voigt_C(params[p, 0], params[p, 1], dim)
                           for p in range(params.shape[0])])
            C = Cs[phases]                                      # (ne, nF, nF)
            sig = np.einsum("eij,ej->ei", C, eps)
            re += wt * sig @ B
            ke += wt * np.einsum("ai,eij,jb->eab", B.T, C, B)
            kwF += wt * np.einsum("ai,eij->eaj", B.T, C)
            K_FF += wt * C.sum(axis=0)
            P_int += wt * sig.sum(axis=0)
            energy += wt * 0.5 * np.einsum("ei,ei->", eps, sig)
        else:
            G = grad_G(dN)
            Fv = macro[None, :] + we @ G.T                      # (ne, 4)
            F2 = Fv.reshape(ne, dim, dim)
            if material == "neohooke":
                lam, mu = params[phases, 0], params[phases, 1]
                P, A = tensors.nh_stress_tangent(F2, lam, mu)
                psi = tensors.nh_energy(F2, lam, mu)
                al, be, ka = mu / 2.0, np.zeros_like(mu), lam   # the beta = 0 member of Eq. (59)
            elif material == "mooney_rivlin":
                a, b, k = params[phases, 0], params[phases, 1], params[phases, 2]
                P, A = tensors.mr_stress_tangent(F2, a, b, k)
                psi = tensors.mr_energy(F2, a, b, k)
                al, be, ka = a, b, k
            else:
                raise ValueError(material)
            re += wt * P @ G
            # P = 2(a+b) F + (2bJ + k(J-1) - 2(a+2b)/J) cof F: its FP64 value
            # is the difference of terms of the size below, which bounds the
            # rounding of the residual (relevant near F = I, where they cancel)
            J = np.linalg.det(F2)
            H = np.stack([F2[:, 1, 1], -F2[:, 1, 0], -F2[:, 0, 1], F2[:, 0, 0]], axis=1)
            c1a = np.abs(2 * be * J) + np.abs(ka * (J - 1.0)) + np.abs(2 * (al + 2 * be) / J)
            Pa = np.abs(2 * (al + be))[:, None] * np.abs(Fv) + c1a[:, None] * np.abs(H)
            re_abs += wt * Pa @ np.abs(G)
            ke += wt * np.einsum("ai,eij,jb->eab", G.T, A, G)
            kwF += wt * np.einsum("ai,eij->eaj", G.T, A)
            K_FF += wt * A.sum(axis=0)
            P_int += wt * P.sum(axis=0)
            energy += wt * float(psi.sum())
    rows = np.repeat(edofs, nd, axis=1).ravel()
    cols = np.tile(edofs, (1, nd)).ravel()
    K = sp.csr_matrix((ke.ravel(), (rows, cols)), shape=(n_full, n_full))
    r_full = np.zeros(n_full)
    np.add.at(r_full, edofs.ravel(), re.ravel())
    KwF_full = np.zeros((n_full, nF))
    np.add.at(KwF_full, edofs.ravel(), kwF.reshape(-1, nF))
    free = np.arange(dim, n_full)                      # corner node pinned
    K_ww = K[free][:, free].tocsr()
    return RVESystem(K_ww=K_ww, K_wF=KwF_full[free], K_FF=K_FF, r=r_full[free],
                     P_int=P_int, energy=energy, free=free, n_full=n_full,
                     volume=L ** dim, r_round=float(np.sqrt(np.sum(re_abs ** 2))))


@dataclasses.dataclass
class Condensed:
    C: np.ndarray         # (nF, nF) homogenized tangent
    P_hat: np.ndarray     # (nF,) condensed stress (Eq. (48) right-hand side)
    P_bar: np.ndarray     # (nF,) volume-averaged micro stress, Eq. (17)
    X_F: np.ndarray       # (N, nF)
    x_r: np.ndarray       # (N,)
    system: RVESystem


def condense(sysm: RVESystem) -> Condensed:
    """Solve K_ww [X_F | x_r] = [K_wF | r] by sparse LU and condense."""
    lu = spla.splu(sysm.K_ww.tocsc())
    rhs = np.concatenate([sysm.K_wF, sysm.r[:, None]], axis=1)
    sol = lu.solve(rhs)
    X_F, x_r = sol[:, :-1], sol[:, -1]
    V = sysm.volume
    C = (sysm.K_FF - sysm.K_wF.T @ X_F) / V
    P_hat = (sysm.P_int - sysm.K_wF.T @ x_r) / V
    return Condensed(C=C, P_hat=P_hat, P_bar=sysm.P_int / V, X_F=X_F, x_r=x_r,
                     system=sysm)


def expand(sysm: RVESystem, v_reduced):
    """Reduced fluctuation vector -> periodic nodal field (corner zero)."""
    out = np.zeros(sysm.n_full)
    out[sysm.free] = v_reduced
    return out


def rve_problem_args(prob, b):
    """(res, phases, params, L) of RVE b of a workloads.Problem."""
    return (prob.rve_res[b], prob.phase_id[prob.rve_off[b]:prob.rve_off[b + 1]],
            prob.phase_params[b], prob.rve_size)


def homogenize_rve(prob, b, macro, w_full: Optional[np.ndarray] = None) -> Condensed:
    res, ph, par, L = rve_problem_args(prob, b)
    return condense(assemble_rve(res, ph, par, prob.kinematics, prob.material,
                                 macro, w_full, L))


def equilibrate_rve(prob, b, macro, w_full=None, tol=1e-13, max_it=30, norm="absolute"):
    """Classical inner Newton of Sec. 4.1 at fixed macro gradient: iterate
    w <- w - K_ww^-1 r until ||r|| < tol * max(1, ||r_0||), or until ||r|| is
    at the FP64 rounding level 1e-14 * r_round of its evaluation (finite
    strain; the paper's tolerance can lie below that level).  Returns the
    final periodic field and the residual history.

    norm="per_volume" is the other reading of the criterion of Sec. 5.2: the
    residual of the volume-averaged weak form, ||r|| / |Omega|, against tol
    with no relative factor and no rounding escape (the inner residuals of
    Table 2 end near 2e-15, below the rounding level of ||r|| itself)."""
    res, ph, par, L = rve_problem_args(prob, b)
    w = np.zeros(int(np.prod(res)) * len(res)) if w_full is None else np.array(w_full, dtype=np.float64)
    vol = float(L) ** len(res)   # |Omega| of the cubic cell of side L
    hist = []
    r0 = None
    for _ in range(max_it + 1):
        s = assemble_rve(res, ph, par, prob.kinematics, prob.material, macro, w, L)
        nr = float(np.linalg.norm(s.r))
        if norm == "per_volume":
            hist.append(nr / vol)
            if nr / vol < tol:
                break
        else:
            hist.append(nr)
            if r0 is None:
                r0 = nr
            if nr < tol * max(1.0, r0) or nr <= 1e-14 * s.r_round:
                break
        dw = spla.spsolve(s.K_ww.tocsc(), s.r)
        w[s.free] -= dw
    return w, hist
