"""GPU parity of the piecewise-constant macro basis of the fluctuation (one RVE
per macro element, Eqs. (constSolution1)-(constSolution2)) against the
oracle's element-by-element Schur complements.

The HIP path never forms the element's micro blocks: it drives each RVE with
the element-average strain and adds the in-element strain variation through
the volume-averaged elasticity.  The oracle assembles the Gauss sums of the
RVE blocks literally and condenses them, so agreement checks that reduction.
Tolerances: 1e-10 relative on the macro tangent and displacement (FP64
path), 1e-9 on the step increment and fluctuations at rve_tol 1e-11 to 1e-13.
"""
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


def random_state(p, seed, amp):
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal(p.n_dofs)
    ws = []
    for b in range(p.n_rve):
        w = amp * rng.standard_normal(int(np.prod(p.rve_res[b])) * p.dim)
        w[:p.dim] = 0.0
        ws.append(w)
    return u, ws


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_element_newton_step_at_nonzero_state(fe2, prec):
    """One generalized step from a random (u, w~) with a pending load
    increment: element-average strains, the assembled macro tangent, the
    increment, the updated state and the norms."""
    p = W.element_basis(W.config("cfg2", macro=(3, 2), rve=16))
    u, ws = random_state(p, 21, 2e-4)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-12)
    print("element basis step", prec, flush=True)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"),
                      w=torch.tensor(np.concatenate(ws), device="cuda"), load_factor=0.25)
    st, norms = fe2.fe2_newton_step(h, 0.5)
    assert st == fe2.FE2_OK
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    mg = get(fe2, h, fe2.FE2_D_MACRO_GRAD, p.n_rve * nF).reshape(p.n_rve, nF)
    K = get(fe2, h, fe2.FE2_D_MACRO_KDENSE, p.n_dofs ** 2).reshape(p.n_dofs, p.n_dofs)
    du = get(fe2, h, fe2.FE2_D_MACRO_DU, p.n_dofs)
    u_gpu, w_gpu = dz(p.n_dofs), dz(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN))
    fe2.fe2_get_state(h, u_gpu, w_gpu)
    torch.cuda.synchronize()
    h.close()

    geo = M.macro_geometry(p)
    for e in range(p.n_elems):
        q = e * geo.n_gp + np.arange(geo.n_gp)
        ebar = sum(geo.wdet[k] * M.macro_gradient(p, geo, u, k) for k in q) / geo.wdet[q].sum()
        assert rel(mg[e], ebar) < 1e-13
    state = M.State(u=u.copy(), w=[w.copy() for w in ws], lam=0.25)
    nrm, du_o, _, conds = M.element_generalized_step(p, geo, state, 0.5)
    Ko, _, _, _ = M.element_macro_system(p, geo, conds, 0.5)
    assert rel(K, Ko.toarray()) < 1e-10
    assert rel(du, du_o) < 1e-9
    assert rel(u_gpu.cpu().numpy(), state.u) < 1e-12
    assert rel(w_gpu.cpu().numpy(), np.concatenate(state.w)) < 1e-9
    for a, b in zip(norms, [nrm.total, nrm.macro, nrm.micro, nrm.scale]):
        assert abs(a - b) <= 1e-9 * max(abs(b), 1e-300)


_ORACLE = {}


def oracle_solution(name, kw):
    """Converged oracle state of a case (cached: both precisions compare
    against it)."""
    key = (name, tuple(sorted(kw.items())))
    if key not in _ORACLE:
        _ORACLE[key] = M.solve(W.element_basis(W.config(name, **kw)))[0]
    return _ORACLE[key]


CASES = [
    ("cfg2", dict(macro=(4, 4), rve=32)),              # the benchmark RVE size
    ("cfg2", dict(macro=(3, 3), rve=15)),              # odd size: ragged 2x2 blocks
    ("cfg3", dict(macro=(3, 3), resolutions=(16, 32, 48))),  # uneven batch
    ("cfg4", dict(macro=(2, 2, 2), rve=6)),            # 3D, 8 RVEs of 6^3
]


@pytest.mark.parametrize("name,kw", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_element_end_to_end(fe2, name, kw, prec):
    """Whole linear solve with the element basis: converged macro
    displacement and fluctuations against the oracle."""
    p = W.element_basis(W.config(name, **kw))
    print("element basis solve", name, kw, prec, flush=True)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-11)
    hist = []
    fe2.solve(h, p.load_factors, history=hist)
    assert len(hist[0]) == 2          # linear: one update, then converged
    u, w = dz(p.n_dofs), dz(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN))
    fe2.fe2_get_state(h, u, w)
    torch.cuda.synchronize()
    h.close()
    st = oracle_solution(name, kw)
    assert rel(u.cpu().numpy(), st.u) < 1e-10
    assert rel(w.cpu().numpy(), np.concatenate(st.w)) < 1e-8


def test_element_classical_scheme(fe2):
    """Classical scheme with the element basis: the inner loop equilibrates
    every element's RVE, then the Schur complement step; same converged
    state as the oracle's classical scheme."""
    p = W.element_basis(W.config("cfg2", macro=(3, 3), rve=16))
    print("element basis classical", flush=True)
    h = fe2.fe2_setup(p, precision="fp64", scheme="classical", rve_tol=1e-12)
    fe2.solve(h, p.load_factors)
    u, w = dz(p.n_dofs), dz(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN))
    fe2.fe2_get_state(h, u, w)
    torch.cuda.synchronize()
    h.close()
    st, _ = M.solve(p, scheme="classical")
    assert rel(u.cpu().numpy(), st.u) < 1e-10
    assert rel(w.cpu().numpy(), np.concatenate(st.w)) < 1e-8


def test_element_basis_finite_strain_not_supported(fe2):
    p = W.element_basis(W.config("cfg5", macro=(2, 2), rve=8, n_steps=1))
    with pytest.raises(fe2.FE2Error) as ei:
        fe2.fe2_setup(p)
    assert ei.value.status == fe2.FE2_ENOTSUP
