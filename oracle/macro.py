"""Macro finite elements and the two Newton schemes of Sec. 4 (FP64), oracle
side.

* Macro discretisation (Sec. 3, Eqs. (25)-(28)): isoparametric Q4 / hex8,
  2-point Gauss-Legendre rule per direction, or biquadratic Q9 (2D) with 3
  points per direction (the [delta, 2] setting of Sec. 5.1 carried to 2D);
  one RVE per Gauss point
  (Dirac macro basis of the fluctuation, Eqs. (31)-(35)), b = e*n_gp + g.
* Macro residual R = sum_b eta_b J_b G_b^T P_b - lambda f_ext (Eq. (35)),
  tangent K = sum_b eta_b J_b G_b^T C_b G_b with the condensed C_b.
* Micro residual rows carry the factor eta_b J_b / |Omega| that makes the
  global Hessian symmetric (E = D^T, Eqs. (39)-(41)).
* Generalized scheme (Sec. 4.2, Eqs. (46)-(49)): one condensation per macro
  iteration at the current (q, w~), right-hand side with the -D L^-1 R_micro
  term, then dw_b = -(x_r + X_F dF_b).
* Classical scheme (Sec. 4.1, Eqs. (43)-(45)): every RVE first equilibrated
  at fixed q, then the Schur complement step and the predictor
  dw_b = -X_F dF_b.
* Full block solve of Eq. (42) for tiny meshes.
* Piecewise-constant macro basis of the fluctuation (Sec. 3, Eqs.
  (constSolution1)-(constSolution2)): one fluctuation field per macro element,
  shared by the element's Gauss points; its micro residual, Hessian blocks and
  macro residual are the Gauss sums of the RVE quantities at (F_g, w~_e), and
  both Newton schemes condense element by element.

Prescribed displacements: the whole increment (lambda_new - lambda_old) g is
applied through the linear system in the first iteration of a load step;
later iterations carry zero increments.  Convergence: the norm
||[R_macro(free); R_micro]|| of a state, tested against tol * ||F_int||
(the internal nodal forces over all DOFs) from the second iteration of a
load step on.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import rve as R


# --------------------------------------------------------------------------
# macro geometry
# --------------------------------------------------------------------------

@dataclasses.dataclass
class MacroGeometry:
    dNdX: np.ndarray    # (n_rve, n_en, dim)
    wdet: np.ndarray    # (n_rve,) Gauss weight times Jacobian determinant
    edofs: np.ndarray   # (n_elems, n_en*dim)
    Bs: np.ndarray      # (n_rve, nF, n_en*dim)  strain-B or gradient-G
    n_gp: int


# Biquadratic (Q9) macro element: reference coordinates of the nodes in the
# generators' order (corners counter-clockwise, mid-sides bottom, right, top,
# left, centre); shape functions are products of the 1D quadratic Lagrange
# polynomials on the nodes -1, 0, 1; 3-point Gauss-Legendre per direction.
Q9_NODES = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1], [0, -1], [1, 0], [0, 1], [-1, 0], [0, 0]], dtype=np.float64)
GAUSS3 = (np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]), np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0]))


def _lagrange2(x, node):
    """1D quadratic Lagrange polynomial of node -1, 0 or 1 and its derivative."""
    if node < 0:
        return 0.5 * x * (x - 1.0), x - 0.5
    if node > 0:
        return 0.5 * x * (x + 1.0), x + 0.5
    return 1.0 - x * x, -2.0 * x


def q9_shape(xi):
    """N_a(xi, eta) and dN_a/dxi_J of the Q9 element, shapes (9,), (9, 2)."""
    N = np.zeros(9)
    d = np.zeros((9, 2))
    for a, (na, nb) in enumerate(Q9_NODES):
        lx, dlx = _lagrange2(xi[0], na)
        ly, dly = _lagrange2(xi[1], nb)
        N[a] = lx * ly
        d[a] = (dlx * ly, lx * dly)
    return N, d


def macro_rule(prob):
    """Gauss points, weights and the reference shape-derivative function of
    the macro element (order 1: Q4 / hex8 with 2 points per direction, weight
    1; order 2: Q9 with 3 points per direction, xi fastest)."""
    if getattr(prob, "macro_order", 1) == 2:
        if prob.dim != 2:
            raise ValueError("quadratic macro elements are 2D")
        x, w = GAUSS3
        gps = np.array([[x[i], x[j]] for j in range(3) for i in range(3)])
        wts = np.array([w[i] * w[j] for j in range(3) for i in range(3)])
        return gps, wts, lambda xi: q9_shape(xi)[1]
    gps = R.gauss_points(prob.dim)
    return gps, np.ones(len(gps)), R.dshape_ref


def macro_geometry(prob) -> MacroGeometry:
    dim = prob.dim
    gps, wts, dshape = macro_rule(prob)
    ne = prob.n_elems
    n_gp = len(gps)
    nen = prob.conn.shape[1]
    dNdX = np.zeros((ne * n_gp, nen, dim))
    wdet = np.zeros(ne * n_gp)
    for e in range(ne):
        Xe = prob.X[prob.conn[e]]
        for g, xi in enumerate(gps):
            dxi = dshape(xi)
            J = Xe.T @ dxi
            dNdX[e * n_gp + g] = dxi @ np.linalg.inv(J)
            wdet[e * n_gp + g] = wts[g] * np.linalg.det(J)
    edofs = (prob.conn[:, :, None] * dim + np.arange(dim)).reshape(ne, -1)
    if prob.kinematics == "small":
        Bs = np.stack([R.strain_B(d) for d in dNdX])
    else:
        Bs = np.stack([R.grad_G(d) for d in dNdX])
    return MacroGeometry(dNdX=dNdX, wdet=wdet, edofs=edofs, Bs=Bs, n_gp=n_gp)


def macro_gradient(prob, geo: MacroGeometry, u, q):
    """eps (small strain) or F = I + grad u (finite strain), Eq. (11), at
    macro Gauss point q = e * n_gp + g."""
    e = q // geo.n_gp
    g = geo.Bs[q] @ u[geo.edofs[e]]
    if prob.kinematics == "small":
        return g
    return g + np.eye(prob.dim).ravel()


# --------------------------------------------------------------------------
# state and linearisation
# --------------------------------------------------------------------------

@dataclasses.dataclass
class State:
    u: np.ndarray                  # macro displacement q - X
    w: List[np.ndarray]            # periodic fluctuation per RVE (corner 0)
    lam: float = 0.0               # load factor the prescribed values are at


def initial_state(prob) -> State:
    w = [np.zeros(int(np.prod(prob.rve_res[b])) * prob.dim) for b in range(prob.n_rve)]
    return State(u=np.zeros(prob.n_dofs), w=w, lam=0.0)


def linearize(prob, geo, state) -> List[R.Condensed]:
    """Condensed RVE of every Gauss point (Dirac macro basis)."""
    if prob.macro_basis != "dirac":
        raise ValueError("linearize covers the Dirac macro basis")
    return [R.homogenize_rve(prob, b, macro_gradient(prob, geo, state.u, b), state.w[b])
            for b in range(prob.n_rve)]


@dataclasses.dataclass
class Norms:
    total: float
    macro: float
    micro: float
    scale: float


def macro_system(prob, geo, conds, lam, use_phat=True):
    """Assembled macro tangent (CSR), condensed right-hand side and the true
    residual (with P_bar), both including -lam f_ext, plus F_int."""
    nd = prob.n_dofs
    rows, cols, vals = [], [], []
    R_hat = np.zeros(nd)
    F_int = np.zeros(nd)
    for b, c in enumerate(conds):
        e = b // geo.n_gp
        B = geo.Bs[b]
        w = geo.wdet[b]
        ke = w * B.T @ c.C @ B
        d = geo.edofs[e]
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(ke.ravel())
        np.add.at(R_hat, d, w * B.T @ (c.P_hat if use_phat else c.P_bar))
        np.add.at(F_int, d, w * B.T @ c.P_bar)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nd, nd))
    R_hat -= lam * prob.f_ext
    R_true = F_int - lam * prob.f_ext
    return K, R_hat, R_true, F_int


def free_dofs(prob):
    mask = np.ones(prob.n_dofs, dtype=bool)
    mask[prob.dir_dofs] = False
    return np.where(mask)[0]


def norms_of(prob, geo, conds, R_true, F_int):
    fr = free_dofs(prob)
    rm = float(np.linalg.norm(R_true[fr]))
    mic2 = 0.0
    for b, c in enumerate(conds):
        mic2 += float(np.sum((geo.wdet[b] / c.system.volume * c.system.r) ** 2))
    mic = float(np.sqrt(mic2))
    return Norms(total=float(np.hypot(rm, mic)), macro=rm, micro=mic,
                 scale=float(np.linalg.norm(F_int)))


def solve_macro(prob, K, rhs_full, du_D):
    """Solve K du = rhs with du = du_D on the Dirichlet DOFs (elimination)."""
    fr = free_dofs(prob)
    dd = prob.dir_dofs
    Kc = K.tocsc()
    du = np.zeros(prob.n_dofs)
    du[dd] = du_D
    rhs = rhs_full[fr] - Kc[fr][:, dd] @ du_D
    du[fr] = spla.spsolve(Kc[fr][:, fr].tocsc(), rhs)
    return du


# --------------------------------------------------------------------------
# Newton schemes
# --------------------------------------------------------------------------

def generalized_step(prob, geo, state: State, lam_target: float):
    """One iteration of the generalized (null-space) scheme, Eqs. (46)-(49).
    Returns the norms of the state it linearised at and the increments."""
    conds = linearize(prob, geo, state)
    K, R_hat, R_true, F_int = macro_system(prob, geo, conds, lam_target)
    nrm = norms_of(prob, geo, conds, R_true, F_int)
    du_D = (lam_target - state.lam) * prob.dir_vals
    du = solve_macro(prob, K, -R_hat, du_D)
    dws = []
    for b, c in enumerate(conds):
        e = b // geo.n_gp
        dF = geo.Bs[b] @ du[geo.edofs[e]]
        dw = -(c.x_r + c.X_F @ dF)
        state.w[b] = state.w[b] + R.expand(c.system, dw)
        dws.append(dw)
    state.u = state.u + du
    state.lam = lam_target
    return nrm, du, dws, conds


def classical_step(prob, geo, state: State, lam_target: float, tol_micro=1e-13,
                   max_micro=30, micro_hist=None, predictor=True, micro_norm="absolute"):
    """One macro iteration of the classical staggered scheme, Eqs. (43)-(45):
    equilibrate every RVE at the current q, condense, solve the macro Schur
    system, update q and predict w with dw_b = -X_F dF_b (predictor=False:
    the fluctuations go unchanged into the next inner loop, the plain
    staggered reading).  micro_norm selects the inner criterion (see
    R.equilibrate_rve)."""
    for b in range(prob.n_rve):
        Fb = macro_gradient(prob, geo, state.u, b)
        state.w[b], h = R.equilibrate_rve(prob, b, Fb, state.w[b], tol=tol_micro,
                                          max_it=max_micro, norm=micro_norm)
        if micro_hist is not None:
            micro_hist.append(h)
    conds = linearize(prob, geo, state)
    K, R_hat, R_true, F_int = macro_system(prob, geo, conds, lam_target, use_phat=False)
    nrm = norms_of(prob, geo, conds, R_true, F_int)
    du_D = (lam_target - state.lam) * prob.dir_vals
    du = solve_macro(prob, K, -R_true, du_D)
    if predictor:
        for b, c in enumerate(conds):
            e = b // geo.n_gp
            dF = geo.Bs[b] @ du[geo.edofs[e]]
            state.w[b] = state.w[b] + R.expand(c.system, -(c.X_F @ dF))
    state.u = state.u + du
    state.lam = lam_target
    return nrm, du, conds


def solve(prob, scheme="generalized", tol=1e-10, max_it=20, load_factors=None,
          state: Optional[State] = None, diverge_at=1e10, classical_opts=None):
    """Load stepping with either Newton scheme.  Returns (state, history)
    where history[k] lists the norms per iteration of load step k; raises
    RuntimeError when ||R_macro|| exceeds ``diverge_at`` (the failure
    definition of Sec. 5.2) or a step does not converge."""
    geo = macro_geometry(prob)
    state = initial_state(prob) if state is None else state
    hist = []
    for lam in (prob.load_factors if load_factors is None else load_factors):
        h = []
        for it in range(max_it):
            element = prob.macro_basis == "element"
            if scheme == "generalized":
                step = element_generalized_step if element else generalized_step
            else:
                step = element_classical_step if element else classical_step
            if scheme != "generalized" and not element and classical_opts:
                nrm = step(prob, geo, state, lam, **classical_opts)[0]
            else:
                nrm = step(prob, geo, state, lam)[0]
            h.append(nrm)
            if not np.isfinite(nrm.macro) or nrm.macro > diverge_at:
                raise RuntimeError(f"diverged at load {lam}, iteration {it}")
            if it >= 1 and nrm.total <= tol * nrm.scale:
                break
        else:
            raise RuntimeError(f"no convergence at load {lam}")
        hist.append(h)
    return state, hist


# --------------------------------------------------------------------------
# full block system, Eq. (42)
# --------------------------------------------------------------------------

def full_block_system(prob, state: State, lam_target: float):
    """Assemble [K D; E L] and -[R_macro; R_micro] of Eq. (42) for the whole
    problem (Dirac macro basis; tiny meshes only).  K, D, L follow
    Eqs. (39)-(41); E = D^T.  Returns (A, rhs, offs) with the fluctuation of
    RVE b at rows offs[b]:offs[b+1] (reduced numbering)."""
    geo = macro_geometry(prob)
    conds = linearize(prob, geo, state)
    nd = prob.n_dofs
    sizes = [c.system.K_ww.shape[0] for c in conds]
    offs = nd + np.concatenate([[0], np.cumsum(sizes)])
    ntot = int(offs[-1])
    A = sp.lil_matrix((ntot, ntot))
    rhs = np.zeros(ntot)
    for b, c in enumerate(conds):
        e = b // geo.n_gp
        B = geo.Bs[b]
        s = geo.wdet[b] / c.system.volume
        d = geo.edofs[e]
        A[np.ix_(d, d)] = A[np.ix_(d, d)].toarray() + s * B.T @ c.system.K_FF @ B
        Dblk = s * B.T @ c.system.K_wF.T
        sl = slice(offs[b], offs[b + 1])
        A[d, sl] = A[d, sl].toarray() + Dblk
        A[sl, d] = A[sl, d].toarray() + Dblk.T
        A[sl, sl] = s * c.system.K_ww.toarray()
        rhs[d] -= geo.wdet[b] * B.T @ c.P_bar
        rhs[sl] = -s * c.system.r
    rhs[:nd] += lam_target * prob.f_ext
    return A.tocsr(), rhs, offs


def solve_full_block(prob, A, rhs, state: State, lam_target: float):
    """Solve the assembled block system with the prescribed increment on the
    Dirichlet DOFs (elimination)."""
    ntot = A.shape[0]
    mask = np.ones(ntot, dtype=bool)
    mask[prob.dir_dofs] = False
    fr = np.where(mask)[0]
    x = np.zeros(ntot)
    x[prob.dir_dofs] = (lam_target - state.lam) * prob.dir_vals
    r = rhs[fr] - A[fr][:, prob.dir_dofs] @ x[prob.dir_dofs]
    x[fr] = spla.spsolve(A[fr][:, fr].tocsc(), r)
    return x


def full_block_step(prob, state: State, lam_target: float):
    """One Newton step on the full block system of Eq. (42) (tiny meshes)."""
    A, rhs, offs = full_block_system(prob, state, lam_target)
    x = solve_full_block(prob, A, rhs, state, lam_target)
    du = x[:prob.n_dofs]
    dws = [x[offs[b]:offs[b + 1]] for b in range(prob.n_rve)]
    return du, dws


# --------------------------------------------------------------------------
# piecewise-constant macro basis, Eqs. (constSolution1)-(constSolution2)
# --------------------------------------------------------------------------
#
# The basis function of micro DOF c of element e is the indicator of e times
# the RVE shape function R~^c (discontinuous across macro elements, so the
# micro-micro Hessian block stays block diagonal).  With the element's Gauss
# rule the micro residual of element e is sum_g (wdet_g/|Omega|) r(F_g, w~_e)
# and the macro residual sum_g wdet_g B_g^T P_bar(F_g, w~_e); the Hessian
# blocks are the Gauss sums of the RVE blocks of Eqs. (39)-(41).

@dataclasses.dataclass
class ElementBlocks:
    K: np.ndarray          # (nd, nd)  sum_g s_g B_g^T K_FF,g B_g
    D: np.ndarray          # (nd, N)   sum_g s_g B_g^T K_Fw,g   (E = D^T)
    L: sp.csr_matrix       # (N, N)    sum_g s_g K_ww,g
    f: np.ndarray          # (nd,)     sum_g wdet_g B_g^T P_bar,g
    r: np.ndarray          # (N,)      sum_g s_g r_g
    r_round: float         # sum_g s_g r_round,g (rounding size of r)
    energy: float          # sum_g wdet_g psi_bar,g
    system: R.RVESystem    # RVE system at the first Gauss point (numbering)


def element_blocks(prob, geo: MacroGeometry, state: State, e: int) -> ElementBlocks:
    """Blocks of macro element e at the current (q, w~_e); s_g = wdet_g/|Omega|."""
    if prob.macro_basis != "element":
        raise ValueError("element blocks need the piecewise-constant macro basis")
    res, ph, par, Lc = R.rve_problem_args(prob, e)
    K = D = Lm = f = r = None
    r_round = energy = 0.0
    first = None
    for g in range(geo.n_gp):
        q = e * geo.n_gp + g
        F = macro_gradient(prob, geo, state.u, q)
        sy = R.assemble_rve(res, ph, par, prob.kinematics, prob.material, F, state.w[e], Lc)
        s = geo.wdet[q] / sy.volume
        B = geo.Bs[q]
        terms = (s * B.T @ sy.K_FF @ B, s * B.T @ sy.K_wF.T, s * sy.K_ww,
                 geo.wdet[q] * B.T @ (sy.P_int / sy.volume), s * sy.r)
        if first is None:
            first = sy
            K, D, Lm, f, r = terms
        else:
            K, D, Lm, f, r = K + terms[0], D + terms[1], Lm + terms[2], f + terms[3], r + terms[4]
        r_round += s * sy.r_round
        energy += s * sy.energy
    return ElementBlocks(K=K, D=D, L=Lm.tocsr(), f=f, r=r, r_round=r_round,
                         energy=energy, system=first)


@dataclasses.dataclass
class ElementCondensed:
    S: np.ndarray          # (nd, nd) K - D L^-1 E
    f_hat: np.ndarray      # (nd,)    f - D L^-1 r
    Y: np.ndarray          # (N, nd)  L^-1 E
    y_r: np.ndarray        # (N,)     L^-1 r
    blocks: ElementBlocks


def element_condense(blk: ElementBlocks) -> ElementCondensed:
    """Schur complement of the element's micro block (Eqs. (46)-(48) with the
    element basis): sparse LU of L, then S, the condensed force, and the two
    solves the update needs."""
    lu = spla.splu(blk.L.tocsc())
    sol = lu.solve(np.concatenate([blk.D.T, blk.r[:, None]], axis=1))
    Y, y_r = sol[:, :-1], sol[:, -1]
    return ElementCondensed(S=blk.K - blk.D @ Y, f_hat=blk.f - blk.D @ y_r,
                            Y=Y, y_r=y_r, blocks=blk)


def element_macro_system(prob, geo, conds: List[ElementCondensed], lam, use_fhat=True):
    """Assembled condensed tangent, right-hand side (with f_hat, or with the
    true internal force for the classical scheme), true residual and F_int."""
    nd = prob.n_dofs
    rows, cols, vals = [], [], []
    R_hat = np.zeros(nd)
    F_int = np.zeros(nd)
    for e, c in enumerate(conds):
        d = geo.edofs[e]
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(c.S.ravel())
        np.add.at(R_hat, d, c.f_hat if use_fhat else c.blocks.f)
        np.add.at(F_int, d, c.blocks.f)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nd, nd))
    R_hat -= lam * prob.f_ext
    return K, R_hat, F_int - lam * prob.f_ext, F_int


def element_norms(prob, conds: List[ElementCondensed], R_true, F_int) -> Norms:
    fr = free_dofs(prob)
    rm = float(np.linalg.norm(R_true[fr]))
    mic = float(np.sqrt(sum(float(np.sum(c.blocks.r ** 2)) for c in conds)))
    return Norms(total=float(np.hypot(rm, mic)), macro=rm, micro=mic,
                 scale=float(np.linalg.norm(F_int)))


def element_generalized_step(prob, geo, state: State, lam_target: float):
    """Generalized scheme (Sec. 4.2) with the element basis: condense every
    element at the current (q, w~), solve the macro system, then
    dw~_e = -(L_e^-1 r_e + L_e^-1 E_e dq_e)."""
    conds = [element_condense(element_blocks(prob, geo, state, e)) for e in range(prob.n_elems)]
    K, R_hat, R_true, F_int = element_macro_system(prob, geo, conds, lam_target)
    nrm = element_norms(prob, conds, R_true, F_int)
    du_D = (lam_target - state.lam) * prob.dir_vals
    du = solve_macro(prob, K, -R_hat, du_D)
    dws = []
    for e, c in enumerate(conds):
        dw = -(c.y_r + c.Y @ du[geo.edofs[e]])
        state.w[e] = state.w[e] + R.expand(c.blocks.system, dw)
        dws.append(dw)
    state.u = state.u + du
    state.lam = lam_target
    return nrm, du, dws, conds


def element_classical_step(prob, geo, state: State, lam_target: float, tol_micro=1e-13,
                           max_micro=30):
    """Classical scheme (Sec. 4.1) with the element basis: Newton on every
    element's micro residual at fixed q (stop as equilibrate_rve), then the
    Schur complement step with the true residual and dw~_e = -L_e^-1 E_e dq_e."""
    for e in range(prob.n_elems):
        r0 = None
        for _ in range(max_micro + 1):
            blk = element_blocks(prob, geo, state, e)
            nr = float(np.linalg.norm(blk.r))
            r0 = nr if r0 is None else r0
            if nr < tol_micro * max(1.0, r0) or nr <= 1e-14 * blk.r_round:
                break
            dw = spla.spsolve(blk.L.tocsc(), blk.r)
            state.w[e] = state.w[e] - R.expand(blk.system, dw)
    conds = [element_condense(element_blocks(prob, geo, state, e)) for e in range(prob.n_elems)]
    K, _, R_true, F_int = element_macro_system(prob, geo, conds, lam_target, use_fhat=False)
    nrm = element_norms(prob, conds, R_true, F_int)
    du_D = (lam_target - state.lam) * prob.dir_vals
    du = solve_macro(prob, K, -R_true, du_D)
    for e, c in enumerate(conds):
        state.w[e] = state.w[e] + R.expand(c.blocks.system, -(c.Y @ du[geo.edofs[e]]))
    state.u = state.u + du
    state.lam = lam_target
    return nrm, du, conds


def potential_energy(prob, geo: MacroGeometry, state: State) -> float:
    """Pi = sum_q wdet_q psi_bar(F_q, w~ of the RVE at q) - lambda f_ext . u
    (the functional whose variations are Eqs. (35) and (constSolution1/2))."""
    tot = 0.0
    for q in range(prob.n_qp):
        b = q // geo.n_gp if prob.macro_basis == "element" else q
        res, ph, par, Lc = R.rve_problem_args(prob, b)
        sy = R.assemble_rve(res, ph, par, prob.kinematics, prob.material,
                            macro_gradient(prob, geo, state.u, q), state.w[b], Lc)
        tot += geo.wdet[q] * sy.energy / sy.volume
    return tot - state.lam * float(prob.f_ext @ state.u)
