"""GPU parity of the 3D small-strain path (hex8 macro and RVEs, Voigt
[11, 22, 33, 23, 13, 12] with engineering shear) against the FP64 oracle,
through the C ABI.

Rows a2-a6 are compared RVE by RVE at a nonzero state (random macro
displacement and periodic fluctuations) for the 4^3 and 10^3 sphere RVEs of
the 3D configuration; rows a7-a10 through one generalized Newton iteration;
the whole linear solve through the converged macro displacement.  The
centred sphere gives a cubic-symmetric tangent at any size, and a
homogeneous RVE returns the phase stiffness with no iteration.
"""
import numpy as np
import pytest

import workloads as W
from oracle import macro as M
from oracle import rve as R
from oracle import tensors as T

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


def random_state(p, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal(p.n_dofs)
    ws = []
    for b in range(p.n_rve):
        w = amp * rng.standard_normal(int(np.prod(p.rve_res[b])) * 3)
        w[:3] = 0.0
        ws.append(w)
    return u, ws


@pytest.mark.parametrize("rve", [4, 10])
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_3d_rows_a2_to_a6_at_nonzero_state(fe2, rve, prec):
    p = W.config("cfg4", macro=(1, 1, 1), rve=rve)
    u, ws = random_state(p, 9)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-13)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"), w=torch.tensor(np.concatenate(ws), device="cuda"))
    fe2.fe2_assemble_rve(h)
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    assert nF == 6
    flen = fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN)
    off = fe2.fe2_query(h, fe2.FE2_Q_FIELD_OFFSETS)
    mg = get(fe2, h, fe2.FE2_D_MACRO_GRAD, p.n_rve * nF).reshape(p.n_rve, nF)
    res = get(fe2, h, fe2.FE2_D_RESIDUAL, flen)
    pbar = get(fe2, h, fe2.FE2_D_PBAR, p.n_rve * nF).reshape(p.n_rve, nF)
    Cb, Ph = dz(p.n_rve * nF * nF), dz(p.n_rve * nF)
    fe2.fe2_condense(h, Cb, Ph)
    torch.cuda.synchronize()
    Cb = Cb.cpu().numpy().reshape(p.n_rve, nF, nF)
    Ph = Ph.cpu().numpy().reshape(p.n_rve, nF)
    sol = get(fe2, h, fe2.FE2_D_SOLUTION, flen * (nF + 1))
    geo = M.macro_geometry(p)
    for b in range(p.n_rve):
        macro = M.macro_gradient(p, geo, u, b)
        assert rel(mg[b], macro) < 1e-13
        c = R.homogenize_rve(p, b, macro, ws[b])
        s = c.system
        fl = off[b + 1] - off[b]
        assert rel(res[off[b]:off[b + 1]], R.expand(s, s.r)) < 1e-11
        assert rel(pbar[b], c.P_bar) < 1e-12
        assert rel(Cb[b], c.C) < 1e-10, (b, Cb[b], c.C)
        assert rel(Ph[b], c.P_hat) < 1e-10
        Xb = sol[off[b] * (nF + 1):off[b + 1] * (nF + 1)].reshape(nF + 1, fl)
        for j in range(nF):
            assert rel(Xb[j], R.expand(s, c.X_F[:, j])) < 1e-9
        assert rel(Xb[nF], R.expand(s, c.x_r)) < 1e-9
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_3d_rows_a7_to_a10_one_newton_step(fe2, prec):
    p = W.config("cfg4", macro=(2, 1, 1), rve=4)
    u, ws = random_state(p, 4, amp=2e-4)
    h = fe2.fe2_setup(p, precision=prec, rve_tol=1e-11)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"), w=torch.tensor(np.concatenate(ws), device="cuda"),
                      load_factor=0.5)
    st, norms = fe2.fe2_newton_step(h, 1.0)
    assert st == fe2.FE2_OK
    du = get(fe2, h, fe2.FE2_D_MACRO_DU, p.n_dofs)
    u_gpu, w_gpu = dz(p.n_dofs), dz(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN))
    fe2.fe2_get_state(h, u_gpu, w_gpu)
    torch.cuda.synchronize()
    geo = M.macro_geometry(p)
    state = M.State(u=u.copy(), w=[w.copy() for w in ws], lam=0.5)
    nrm, du_o, _, _ = M.generalized_step(p, geo, state, 1.0)
    assert rel(du, du_o) < 1e-9
    assert rel(u_gpu.cpu().numpy(), state.u) < 1e-12
    assert rel(w_gpu.cpu().numpy(), np.concatenate(state.w)) < 1e-9
    for a, b in zip(norms, [nrm.total, nrm.macro, nrm.micro, nrm.scale]):
        assert abs(a - b) <= 1e-10 * max(abs(b), 1e-300)
    h.close()


def test_3d_reduced_linear_solve(fe2):
    """The 3D recipe on a 2x2x2 macro mesh with 6^3 sphere RVEs: one update,
    then converged; the macro displacement equals the oracle's."""
    p = W.config("cfg4", macro=(2, 2, 2), rve=6)
    h = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=1e-11)
    hist = []
    fe2.solve(h, p.load_factors, history=hist)
    assert len(hist[0]) == 2
    u = dz(p.n_dofs)
    fe2.fe2_get_state(h, u=u)
    torch.cuda.synchronize()
    st, _ = M.solve(p)
    assert rel(u.cpu().numpy(), st.u) < 1e-10
    h.close()


def test_sphere_tangent_is_cubic_at_full_size(fe2):
    """Centred sphere in a 10^3 cube: C11 = C22 = C33, C12 = C13 = C23,
    C44 = C55 = C66, no normal-shear or shear-shear coupling; symmetric."""
    p = W.config("cfg4", macro=(1, 1, 1), rve=10)
    h = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=1e-10)
    fe2.fe2_assemble_rve(h)
    Cb = dz(p.n_rve * 36)
    fe2.fe2_condense(h, Cb)
    C = Cb.cpu().numpy().reshape(p.n_rve, 6, 6)[0]
    s = np.abs(C).max()
    assert np.abs(C - C.T).max() < 1e-9 * s
    assert abs(C[0, 0] - C[1, 1]) < 1e-9 * s and abs(C[0, 0] - C[2, 2]) < 1e-9 * s
    assert abs(C[0, 1] - C[0, 2]) < 1e-9 * s and abs(C[0, 1] - C[1, 2]) < 1e-9 * s
    assert abs(C[3, 3] - C[4, 4]) < 1e-9 * s and abs(C[3, 3] - C[5, 5]) < 1e-9 * s
    assert np.abs(C[:3, 3:]).max() < 1e-9 * s
    assert np.abs(C[3:, 3:] - np.diag(np.diag(C[3:, 3:]))).max() < 1e-9 * s
    assert np.all(np.linalg.eigvalsh(C) > 0)
    h.close()


def test_3d_homogeneous_rve_exact(fe2):
    p = W.config("cfg4", macro=(1, 1, 1), rve=6)
    p.phase_params[:, 1, :] = p.phase_params[:, 0, :]
    h = fe2.fe2_setup(p, precision="fp64", rve_tol=1e-12)
    fe2.fe2_assemble_rve(h)
    Cb = dz(p.n_rve * 36)
    fe2.fe2_condense(h, Cb)
    lam, mu = p.phase_params[0, 0]
    C = T.voigt_C(lam, mu, 3)
    for b in range(p.n_rve):
        assert rel(Cb.cpu().numpy().reshape(p.n_rve, 6, 6)[b], C) < 1e-13
    assert np.all(get(fe2, h, fe2.FE2_D_RVE_ITERS, p.n_rve) == 0)
    h.close()
