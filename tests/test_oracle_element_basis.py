"""Pins of the oracle's piecewise-constant macro basis (Sec. 3, Eqs.
(constSolution1)-(constSolution2)): one fluctuation field per macro element.

* Restriction identity: the element basis is the Dirac basis constrained to
  w~_g = w~_e at the Gauss points of each element, so its Newton step equals
  the step of the Dirac full block system of Eq. (42) restricted by that
  constraint (Z^T A Z, Z^T rhs), for small and finite strain.  The restricted
  system is assembled by the Dirac code, not by the element code.
* Energy bounds: with prescribed displacements and a linear law, the minimum
  of the potential over the element basis lies between the Dirac-basis
  minimum (a larger space) and the Taylor (w~ = 0) minimum (a smaller one).
* Patch test: under a uniform macro strain both bases give the same state.
* A linear problem is solved by one Newton step, by both schemes.
"""
import copy

import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import macro as M


def _perturbed_states(pd, pe, rng, su, sw):
    se = M.initial_state(pe)
    se.u = su * rng.standard_normal(pe.n_dofs)
    for e in range(pe.n_elems):
        se.w[e] = sw * rng.standard_normal(se.w[e].size)
        se.w[e][:pe.dim] = 0.0              # pinned corner
    sd = M.initial_state(pd)
    sd.u = se.u.copy()
    sd.w = [se.w[b // pd.n_gp].copy() for b in range(pd.n_rve)]
    return se, sd


def _restriction(pd, offs, n_elem_dofs):
    nd = pd.n_dofs
    Z = sp.lil_matrix((int(offs[-1]), nd + pd.n_elems * n_elem_dofs))
    Z[np.arange(nd), np.arange(nd)] = 1.0
    for b in range(pd.n_rve):
        e = b // pd.n_gp
        Z[offs[b] + np.arange(n_elem_dofs), nd + e * n_elem_dofs + np.arange(n_elem_dofs)] = 1.0
    return Z.tocsr()


def _check_restriction(pd, lam, su, sw, seed):
    pe = W.element_basis(pd)
    geo = M.macro_geometry(pe)
    se, sd = _perturbed_states(pd, pe, np.random.default_rng(seed), su, sw)
    A, rhs, offs = M.full_block_system(pd, sd, lam)
    N = int(offs[1] - offs[0])
    Z = _restriction(pd, offs, N)
    x = M.solve_full_block(pe, (Z.T @ A @ Z).tocsr(), Z.T @ rhs, se, lam)
    s1 = copy.deepcopy(se)
    _, du, dws, _ = M.element_generalized_step(pe, geo, s1, lam)
    nd = pd.n_dofs
    assert np.abs(du - x[:nd]).max() <= 1e-12 * np.abs(du).max()
    dw_ref = [x[nd + e * N: nd + (e + 1) * N] for e in range(pe.n_elems)]
    scale = max(np.abs(d).max() for d in dw_ref)
    assert max(np.abs(dws[e] - dw_ref[e]).max() for e in range(pe.n_elems)) <= 1e-11 * scale


def test_element_step_is_restricted_full_block_small_strain():
    _check_restriction(W.config("cfg2", macro=(2, 2), rve=6), 1.0, 1e-3, 1e-3, 11)


def test_element_step_is_restricted_full_block_finite_strain():
    _check_restriction(W.config("cfg5", macro=(2, 2), rve=6, n_steps=1), 0.5, 2e-2, 1e-2, 12)


def _taylor_energy(pd, geo):
    """Minimum of the potential with w~ = 0: macro FE with the Voigt average
    K_FF / |Omega| of every RVE (assembled here, not by the method's code)."""
    conds = M.linearize(pd, geo, M.initial_state(pd))
    rows, cols, vals = [], [], []
    for b, c in enumerate(conds):
        d = geo.edofs[b // geo.n_gp]
        B = geo.Bs[b]
        ke = geo.wdet[b] * B.T @ (c.system.K_FF / c.system.volume) @ B
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(ke.ravel())
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(pd.n_dofs, pd.n_dofs))
    st = M.initial_state(pd)
    st.u = M.solve_macro(pd, K, np.zeros(pd.n_dofs), pd.dir_vals)
    st.lam = 1.0
    return M.potential_energy(pd, geo, st)


def test_element_basis_energy_between_dirac_and_taylor():
    pd = W.config("cfg2", macro=(3, 3), rve=8)
    pe = W.element_basis(pd)
    geo = M.macro_geometry(pd)
    std, _ = M.solve(pd, tol=1e-12)
    ste, _ = M.solve(pe, tol=1e-12)
    e_d = M.potential_energy(pd, geo, std)
    e_e = M.potential_energy(pe, geo, ste)
    e_t = _taylor_energy(pd, geo)
    assert e_d < e_e < e_t
    # the macro field varies, so the element constraint costs energy
    assert e_e - e_d > 1e-6 * e_d


def test_element_basis_patch_test_matches_dirac():
    """Uniaxial loading on rollers of a mesh whose RVEs are all the same
    square-symmetric inclusion cell: the macro strain is uniform, w~ (nonzero)
    is the same at every Gauss point, and both bases reach the same state."""
    pd = W.config("cfg2", macro=(2, 2), rve=8)
    pd.phase_params[:] = pd.phase_params[0]
    pe = W.element_basis(pd)
    std, _ = M.solve(pd, tol=1e-12)
    ste, _ = M.solve(pe, tol=1e-12)
    assert np.abs(std.u - ste.u).max() <= 1e-14 * np.abs(std.u).max()
    for b in range(pd.n_rve):
        wd, we = std.w[b], ste.w[b // pd.n_gp]
        assert np.abs(wd - we).max() <= 1e-12 * np.abs(wd).max()


def test_element_basis_linear_one_step_both_schemes():
    pe = W.element_basis(W.config("cfg2", macro=(3, 3), rve=6))
    for scheme in ("generalized", "classical"):
        st, hist = M.solve(pe, scheme=scheme, tol=1e-12)
        assert len(hist[0]) == 2                  # update, then the converged check
        assert hist[0][1].total <= 1e-12 * hist[0][1].scale
    sg, _ = M.solve(pe, tol=1e-12)
    sc, _ = M.solve(pe, scheme="classical", tol=1e-12)
    assert np.abs(sg.u - sc.u).max() <= 1e-12 * np.abs(sg.u).max()


def test_element_basis_rejects_unequal_gauss_point_rves():
    pd = W.config("cfg2", macro=(2, 2), rve=6)
    pd.phase_params[1, 1, 1] *= 2.0
    try:
        W.element_basis(pd)
    except ValueError:
        return
    raise AssertionError("element_basis accepted different RVEs within one element")
