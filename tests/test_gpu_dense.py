"""The dense direct RVE solve (2D small strain) against the oracle.

K_ww is assembled densely in LDS, factored once per RVE by an FP32
Cholesky whose panel and trailing products run on the matrix cores, and
applied inside the FP64 residual refinement.  Checked at every compiled
size it covers (4^2, 6x10, 8^2) at a nonzero state (rows a2-a6): C-bar and
P-hat at 1e-10, every solution column by its FP64 residual and the
cond(K_ww) perturbation bound; the configuration-1 closed form end to end;
the same C-bar as the PCG path; and the refusals (sizes beyond the LDS
factor, FP64, finite strain, BF16 refinement).
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import macro as M
from oracle import rve as R

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


def kappa(K):
    lmax = spla.eigsh(K, k=1, which="LA", return_eigenvectors=False, tol=1e-8)[0]
    lmin = spla.eigsh(K.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-10)[0]
    return lmax / lmin


def with_resolution(p, n1, n2, radius=0.3):
    ph = W.phases_circle(n1, n2, radius)
    off = np.arange(p.n_rve + 1, dtype=np.int64) * ph.size
    return dataclasses.replace(p, rve_res=np.tile(np.array([n1, n2], np.int32), (p.n_rve, 1)), rve_off=off,
                               phase_id=np.tile(ph.astype(np.uint8), p.n_rve))


def random_state(p, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal(p.n_dofs)
    ws = []
    for b in range(p.n_rve):
        w = amp * rng.standard_normal(int(np.prod(p.rve_res[b])) * p.dim)
        w[:p.dim] = 0.0
        ws.append(w)
    return u, ws


def solve_state(fe2, p, u, ws, solver, rve_tol=1e-13):
    h = fe2.fe2_setup(p, precision="fp32_ir", solver=solver, rve_tol=rve_tol)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"), w=torch.tensor(np.concatenate(ws), device="cuda"),
                      load_factor=0.0)
    fe2.fe2_assemble_rve(h)
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    flen = fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN)
    off = fe2.fe2_query(h, fe2.FE2_Q_FIELD_OFFSETS)
    Cb, Ph = dz(p.n_rve * nF * nF), dz(p.n_rve * nF)
    fe2.fe2_condense(h, Cb, Ph)
    torch.cuda.synchronize()
    out = dict(nF=nF, off=off, flen=flen,
               C=Cb.cpu().numpy().reshape(p.n_rve, nF, nF), Ph=Ph.cpu().numpy().reshape(p.n_rve, nF),
               X=get(fe2, h, fe2.FE2_D_SOLUTION, flen * (nF + 1)),
               iters=get(fe2, h, fe2.FE2_D_RVE_ITERS, p.n_rve),
               relres=get(fe2, h, fe2.FE2_D_RVE_RELRES, p.n_rve))
    h.close()
    return out


@pytest.mark.parametrize("n1,n2", [(4, 4), (6, 10), (8, 8)])
def test_dense_rows_a2_to_a6_every_size(fe2, n1, n2):
    print("dense", n1, n2, flush=True)
    p = with_resolution(W.config("cfg2", macro=(1, 1), rve=8), n1, n2)
    u, ws = random_state(p, 5)
    g = solve_state(fe2, p, u, ws, "dense")
    geo = M.macro_geometry(p)
    nF, off = g["nF"], g["off"]
    assert np.all(g["relres"] <= 1e-13)
    for b in range(p.n_rve):
        c = R.homogenize_rve(p, b, M.macro_gradient(p, geo, u, b), ws[b])
        s = c.system
        assert rel(g["C"][b], c.C) < 1e-10, (b, rel(g["C"][b], c.C))
        assert rel(g["Ph"][b], c.P_hat) < 1e-10
        fl = off[b + 1] - off[b]
        Xb = g["X"][off[b] * (nF + 1):off[b + 1] * (nF + 1)].reshape(nF + 1, fl)
        kap = kappa(s.K_ww)
        eps = np.finfo(np.float64).eps
        for j in range(nF + 1):
            bvec = s.K_wF[:, j] if j < nF else s.r
            xref = c.X_F[:, j] if j < nF else c.x_r
            x = Xb[j][s.free]
            nb = np.linalg.norm(bvec)
            floor = 32 * eps * np.linalg.norm(abs(s.K_ww) @ np.abs(x)) / nb
            rg = np.linalg.norm(bvec - s.K_ww @ x) / nb
            assert rg <= 2e-13 + floor, (j, rg, floor)
            assert np.linalg.norm(x - xref) / np.linalg.norm(xref) <= kap * (2e-13 + floor) + 1e-14
            assert np.abs(Xb[j][:2]).max() == 0.0   # pinned corner
        # a direct solve with the FP32 factor contracts the error by about
        # cond(K_ww) * 2^-24 (< 1e-3 at these sizes) per refinement sweep:
        # at most five sweeps per column reach 1e-13
        assert kap * 2.0 ** -24 < 1e-3
        assert g["iters"][b] <= 5 * (nF + 1)


def test_dense_cfg1_end_to_end_closed_form(fe2):
    """Configuration 1 (8x8 laminate RVEs, E ratio 10) through the dense
    solve: macro displacement is the closed-form uniaxial field and every
    RVE carries the laminate tangent."""
    p = W.config("cfg1")
    h = fe2.fe2_setup(p, precision="fp32_ir", solver="dense", rve_tol=1e-11)
    hist = []
    fe2.solve(h, p.load_factors, history=hist)
    assert len(hist[0]) == 2
    u = dz(p.n_dofs)
    fe2.fe2_get_state(h, u=u)
    Cb = get(fe2, h, fe2.FE2_D_CBAR, p.n_rve * 9).reshape(p.n_rve, 3, 3)
    u = u.cpu().numpy()
    h.close()
    ex = np.zeros_like(u)
    ex[0::2] = 1e-3 * p.X[:, 0]
    ex[1::2] = -3.0 / 7.0 * 1e-3 * p.X[:, 1]
    assert rel(u, ex) < 1e-10
    Cex = np.array([[500 / 77, 150 / 143, 0], [150 / 143, 350 / 143, 0], [0, 0, 100 / 143]])
    for b in range(p.n_rve):
        assert rel(Cb[b], Cex) < 1e-10


def test_dense_agrees_with_pcg(fe2):
    """The 8x8 circle RVEs of configuration 2 (lognormal stiffness ratios)
    at a nonzero state: the dense and PCG solves give the same C-bar and
    P-hat (both refined to 1e-13); the dense path needs a few sweeps per
    RVE where the PCG path runs tens of inner iterations."""
    p = W.config("cfg2", macro=(4, 2), rve=8)
    u, ws = random_state(p, 9)
    gd = solve_state(fe2, p, u, ws, "dense")
    gp = solve_state(fe2, p, u, ws, "jacobi")
    assert rel(gd["C"], gp["C"]) < 1e-11
    assert rel(gd["Ph"], gp["Ph"]) < 1e-11
    print(f"sweeps (dense) mean {gd['iters'].mean():.1f}; inner iterations (PCG) mean {gp['iters'].mean():.1f}")
    assert gd["iters"].mean() < gp["iters"].mean()


def test_dense_and_bf16_refusals(fe2):
    p16 = W.config("cfg2", macro=(1, 1), rve=16)     # 510 unknowns: beyond the LDS factor
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_setup(p16, precision="fp32_ir", solver="dense")
    assert e.value.status == fe2.FE2_ENOTSUP
    p8 = W.config("cfg2", macro=(1, 1), rve=8)
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_setup(p8, precision="fp64", solver="dense")
    assert e.value.status == fe2.FE2_ENOTSUP
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_setup(p8, precision="bf16_ir")
    assert e.value.status == fe2.FE2_ENOTSUP
    pf = W.config("cfg5", macro=(1, 1), rve=8)
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_setup(pf, precision="fp32_ir", solver="dense")
    assert e.value.status == fe2.FE2_ENOTSUP
