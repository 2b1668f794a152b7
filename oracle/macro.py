"""Macro finite elements and the two Newton schemes of Sec. 4 (FP64), oracle
side.

* Macro discretisation (Sec. 3, Eqs. (25)-(28)): isoparametric Q4 / hex8,
  2-point Gauss-Legendre rule per direction; one RVE per Gauss point
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


def macro_geometry(prob) -> MacroGeometry:
    dim = prob.dim
    gps = R.gauss_points(dim)
    ne = prob.n_elems
    n_gp = len(gps)
    nen = prob.conn.shape[1]
    dNdX = np.zeros((ne * n_gp, nen, dim))
    wdet = np.zeros(ne * n_gp)
    for e in range(ne):
        Xe = prob.X[prob.conn[e]]
        for g, xi in enumerate(gps):
            dxi = R.dshape_ref(xi)
            J = Xe.T @ dxi
            dNdX[e * n_gp + g] = dxi @ np.linalg.inv(J)
            wdet[e * n_gp + g] = np.linalg.det(J)
    edofs = (prob.conn[:, :, None] * dim + np.arange(dim)).reshape(ne, -1)
    if prob.kinematics == "small":
        Bs = np.stack([R.strain_B(d) for d in dNdX])
    else:
        Bs = np.stack([R.grad_G(d) for d in dNdX])
    return MacroGeometry(dNdX=dNdX, wdet=wdet, edofs=edofs, Bs=Bs, n_gp=n_gp)


def macro_gradient(prob, geo: MacroGeometry, u, b):
    """eps_b (small strain) or F_b = I + grad u (finite strain), Eq. (11)."""
    e = b // geo.n_gp
    g = geo.Bs[b] @ u[geo.edofs[e]]
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
                   max_micro=30, micro_hist=None):
    """One macro iteration of the classical staggered scheme, Eqs. (43)-(45):
    equilibrate every RVE at the current q, condense, solve the macro Schur
    system, update q and predict w with dw_b = -X_F dF_b."""
    for b in range(prob.n_rve):
        Fb = macro_gradient(prob, geo, state.u, b)
        state.w[b], h = R.equilibrate_rve(prob, b, Fb, state.w[b], tol=tol_micro,
                                          max_it=max_micro)
        if micro_hist is not None:
            micro_hist.append(h)
    conds = linearize(prob, geo, state)
    K, R_hat, R_true, F_int = macro_system(prob, geo, conds, lam_target, use_phat=False)
    nrm = norms_of(prob, geo, conds, R_true, F_int)
    du_D = (lam_target - state.lam) * prob.dir_vals
    du = solve_macro(prob, K, -R_true, du_D)
    for b, c in enumerate(conds):
        e = b // geo.n_gp
        dF = geo.Bs[b] @ du[geo.edofs[e]]
        state.w[b] = state.w[b] + R.expand(c.system, -(c.X_F @ dF))
    state.u = state.u + du
    state.lam = lam_target
    return nrm, du, conds


def solve(prob, scheme="generalized", tol=1e-10, max_it=20, load_factors=None,
          state: Optional[State] = None, diverge_at=1e10):
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
            if scheme == "generalized":
                nrm = generalized_step(prob, geo, state, lam)[0]
            else:
                nrm = classical_step(prob, geo, state, lam)[0]
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

def full_block_step(prob, state: State, lam_target: float):
    """Assemble [K D; E L] [dq; dw] = -[R_macro; R_micro] for the whole
    problem and solve it directly (tiny meshes only).  K, D, L follow
    Eqs. (39)-(41) with the Dirac macro basis; E = D^T."""
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
    A = A.tocsr()
    mask = np.ones(ntot, dtype=bool)
    mask[prob.dir_dofs] = False
    fr = np.where(mask)[0]
    x = np.zeros(ntot)
    x[prob.dir_dofs] = (lam_target - state.lam) * prob.dir_vals
    r = rhs[fr] - A[fr][:, prob.dir_dofs] @ x[prob.dir_dofs]
    x[fr] = spla.spsolve(A[fr][:, fr].tocsc(), r)
    du = x[:nd]
    dws = [x[offs[b]:offs[b + 1]] for b in range(prob.n_rve)]
    return du, dws
