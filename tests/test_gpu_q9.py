"""GPU parity of biquadratic (Q9) macro elements with 3x3 Gauss points (one
RVE each, Dirac basis), the order-2 setting of Sec. 5.1 carried to 2D.

* One generalized Newton step from a random state on a curved
  (isoparametric) Q9 mesh: macro strains at the 9 Gauss points, the dense
  macro tangent, the increment, the updated state and the norms against the
  oracle step.
* Whole linear solves (cfg2-type circle inclusions, the cfg1 laminate) in
  both precisions against the oracle's converged state.
* The quadratic equilibrium field of a homogeneous body is reproduced at
  every node (a property of the discretisation, independent of the oracle).
* The classical scheme on Q9 against the oracle's classical scheme.
* Q9 with the element basis is rejected with FE2_ENOTSUP.

Tolerances as for the Q4 tests: 1e-13 on strains, 1e-10 on the tangent and
converged displacement, 1e-9 on increments and fluctuations.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import macro as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def dz(n):
    return torch.zeros(int(n), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def get(fe2, h, which, n):
    t = dz(n)
    fe2.fe2_get_data(h, which, t)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def curved(p, amp=0.15, seed=8):
    """Move every interior node (mid-side and centre nodes included) by up to
    amp of the node spacing: curved element edges, a non-affine map."""
    rng = np.random.default_rng(seed)
    X = p.X.copy()
    inner = (X[:, 0] > 1e-12) & (X[:, 0] < 1 - 1e-12) & (X[:, 1] > 1e-12) & (X[:, 1] < 1 - 1e-12)
    hx = 1.0 / (2 * p.meta["macro"][0])
    X[inner] += amp * hx * rng.uniform(-1, 1, (int(inner.sum()), 2))
    return dataclasses.replace(p, X=X)


def random_state(p, seed, amp):
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal(p.n_dofs)
    ws = []
    for b in range(p.n_rve):
        w = amp * rng.standard_normal(int(np.prod(p.rve_res[b])) * p.dim)
        w[:p.dim] = 0.0
        ws.append(w)
    return u, ws


def state_of(fe2, h, p):
    u, w = dz(p.n_dofs), dz(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN))
    fe2.fe2_get_state(h, u, w)
    torch.cuda.synchronize()
    return u.cpu().numpy(), w.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_q9_newton_step_on_a_curved_mesh(fe2, prec):
    p = curved(W.config("cfg2", macro=(3, 2), rve=16, order=2))
    assert p.n_rve == 54
    u, ws = random_state(p, 31, 2e-4)
    print("Q9 newton step", prec, flush=True)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-12)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"),
                      w=torch.tensor(np.concatenate(ws), device="cuda"), load_factor=0.25)
    st, norms = fe2.fe2_newton_step(h, 0.5)
    assert st == fe2.FE2_OK
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    mg = get(fe2, h, fe2.FE2_D_MACRO_GRAD, p.n_rve * nF).reshape(p.n_rve, nF)
    K = get(fe2, h, fe2.FE2_D_MACRO_KDENSE, p.n_dofs ** 2).reshape(p.n_dofs, p.n_dofs)
    du = get(fe2, h, fe2.FE2_D_MACRO_DU, p.n_dofs)
    u_gpu, w_gpu = state_of(fe2, h, p)
    h.close()

    geo = M.macro_geometry(p)
    assert geo.n_gp == 9
    for b in range(p.n_rve):
        assert rel(mg[b], M.macro_gradient(p, geo, u, b)) < 1e-13, b
    state = M.State(u=u.copy(), w=[w.copy() for w in ws], lam=0.25)
    Ko, _, _, _ = M.macro_system(p, geo, M.linearize(p, geo, state), 0.5)
    nrm, du_o, _, _ = M.generalized_step(p, geo, state, 0.5)
    assert rel(K, Ko.toarray()) < 1e-10
    assert rel(du, du_o) < 1e-9
    assert rel(u_gpu, state.u) < 1e-12
    assert rel(w_gpu, np.concatenate(state.w)) < 1e-9
    for a, b in zip(norms, [nrm.total, nrm.macro, nrm.micro, nrm.scale]):
        assert abs(a - b) <= 1e-9 * max(abs(b), 1e-300)


_ORACLE = {}


def oracle_solution(name, kw, scheme="generalized"):
    key = (name, tuple(sorted(kw.items())), scheme)
    if key not in _ORACLE:
        _ORACLE[key] = M.solve(W.config(name, **kw), scheme=scheme)[0]
    return _ORACLE[key]


CASES = [
    ("cfg2", dict(macro=(4, 4), rve=16, order=2)),
    ("cfg2", dict(macro=(3, 3), rve=15, order=2)),     # odd RVE size: node-centric operator
    ("cfg1", dict(macro=(4, 2), rve=8, order=2)),      # laminate
]


@pytest.mark.parametrize("name,kw", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_q9_end_to_end(fe2, name, kw, prec):
    p = W.config(name, **kw)
    print("Q9 solve", name, kw, prec, flush=True)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-11)
    hist = []
    fe2.solve(h, p.load_factors, history=hist)
    assert len(hist[0]) == 2          # linear: one update, then converged
    u, w = state_of(fe2, h, p)
    h.close()
    st = oracle_solution(name, kw)
    assert rel(u, st.u) < 1e-10
    wo = np.concatenate(st.w)
    # the laminate under its load has no fluctuation (w~ is rounding noise):
    # an absolute floor of 1e-11 of the displacement scale
    assert np.abs(w - wo).max() <= 1e-8 * np.abs(wo).max() + 1e-11 * np.abs(st.u).max()


def _equilibrium_quadratic(lam, mu, s=1e-3):
    """A quadratic displacement with div(C : eps) = 0 for the isotropic
    tensor (lam, mu): u_x = s (x^2 + a x y), u_y = s (a x y + y^2) with
    a = -2 (lam + 2 mu) / (lam + mu)."""
    a = -2.0 * (lam + 2.0 * mu) / (lam + mu)
    return lambda X: s * np.stack([X[:, 0] ** 2 + a * X[:, 0] * X[:, 1], a * X[:, 0] * X[:, 1] + X[:, 1] ** 2], axis=1)


def test_q9_reproduces_a_quadratic_equilibrium_field(fe2):
    p = W.config("cfg2", macro=(4, 3), rve=8, order=2)
    pp = p.phase_params.copy()
    pp[:, 1] = pp[:, 0]                                 # homogeneous RVEs
    lam, mu = pp[0, 0]
    field = _equilibrium_quadratic(lam, mu)
    X = p.X
    bnd = np.where((np.abs(X[:, 0]) < 1e-12) | (np.abs(X[:, 0] - 1) < 1e-12)
                   | (np.abs(X[:, 1]) < 1e-12) | (np.abs(X[:, 1] - 1) < 1e-12))[0]
    dofs = np.sort(np.concatenate([2 * bnd, 2 * bnd + 1])).astype(np.int32)
    ex = field(X).ravel()
    p = dataclasses.replace(p, phase_params=pp, dir_dofs=dofs, dir_vals=ex[dofs].copy(), f_ext=np.zeros(p.n_dofs))
    print("Q9 quadratic patch", flush=True)
    h = fe2.fe2_setup(p, precision="fp64", rve_tol=1e-13)
    fe2.solve(h, [1.0])
    u, _ = state_of(fe2, h, p)
    h.close()
    assert rel(u, ex) < 1e-11


def test_q9_classical_scheme(fe2):
    kw = dict(macro=(3, 3), rve=16, order=2)
    p = W.config("cfg2", **kw)
    print("Q9 classical", flush=True)
    h = fe2.fe2_setup(p, precision="fp64", scheme="classical", rve_tol=1e-12)
    fe2.solve(h, p.load_factors)
    u, w = state_of(fe2, h, p)
    h.close()
    st = oracle_solution("cfg2", kw, scheme="classical")
    assert rel(u, st.u) < 1e-10
    assert rel(w, np.concatenate(st.w)) < 1e-8


def test_q9_with_element_basis_not_supported(fe2):
    p = W.element_basis(W.config("cfg2", macro=(2, 2), rve=8, order=2))
    with pytest.raises(fe2.FE2Error) as ei:
        fe2.fe2_setup(p)
    assert ei.value.status == fe2.FE2_ENOTSUP
