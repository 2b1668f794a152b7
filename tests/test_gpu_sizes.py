"""Every compiled RVE resolution against the oracle (rows a2-a6 at a nonzero
state): 2D small strain 4^2, 6x10, 8^2, 10^2, 15^2, 16^2, 17^2, 30^2, 32^2,
48^2 (even sizes run the element-wise operator, odd and non-square sizes the
node-centric one), 2D finite strain 4^2, 6x10, 8^2, 15^2, 16^2, 30^2, 32^2 and
3D 4^3, 6^3, 8^3, 10^3, and the square 2D sizes 8, 16, 32, 48 once more with
each preconditioner (spectral, Jacobi) in each precision.  One macro element (one RVE per Gauss point) with a
centred circular / spherical inclusion at each size, in the mixed form with
the residual driven to 1e-13 so that C-bar and P-hat compare at 1e-10.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import macro as M
from oracle import rve as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES_2D = [(4, 4), (6, 10), (8, 8), (10, 10), (15, 15), (16, 16), (17, 17), (30, 30), (32, 32), (48, 48)]
SIZES_FIN = [(4, 4), (6, 10), (8, 8), (15, 15), (16, 16), (30, 30), (32, 32)]
SIZES_3D = [4, 6, 8, 10]


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def with_resolution(p, n1, n2, radius=0.3):
    """The same problem with every RVE an n1 x n2 grid with a centred circle."""
    ph = W.phases_circle(n1, n2, radius)
    off = np.arange(p.n_rve + 1, dtype=np.int64) * ph.size
    return dataclasses.replace(p, rve_res=np.tile(np.array([n1, n2], np.int32), (p.n_rve, 1)), rve_off=off,
                               phase_id=np.tile(ph.astype(np.uint8), p.n_rve))


def random_state(p, seed, u_amp, w_amp):
    rng = np.random.default_rng(seed)
    u = u_amp * rng.standard_normal(p.n_dofs)
    ws = []
    for b in range(p.n_rve):
        w = w_amp * rng.standard_normal(int(np.prod(p.rve_res[b])) * p.dim)
        w[:p.dim] = 0.0
        ws.append(w)
    return u, ws


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def check_a2_to_a6(fe2, p, u, ws, tol_c, precision="fp32_ir", solver="auto"):
    h = fe2.fe2_setup(p, precision=precision, solver=solver, rve_tol=1e-13)
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"), w=torch.tensor(np.concatenate(ws), device="cuda"),
                      load_factor=0.0)
    fe2.fe2_assemble_rve(h)
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    Cb = torch.zeros(p.n_rve * nF * nF, dtype=torch.float64, device="cuda")
    Ph = torch.zeros(p.n_rve * nF, dtype=torch.float64, device="cuda")
    fe2.fe2_condense(h, Cb, Ph)
    torch.cuda.synchronize()
    h.close()
    Cb = Cb.cpu().numpy().reshape(p.n_rve, nF, nF)
    Ph = Ph.cpu().numpy().reshape(p.n_rve, nF)
    geo = M.macro_geometry(p)
    for b in range(p.n_rve):
        c = R.homogenize_rve(p, b, M.macro_gradient(p, geo, u, b), ws[b])
        assert rel(Cb[b], c.C) < tol_c, (b, rel(Cb[b], c.C))
        assert rel(Ph[b], c.P_hat) < tol_c, (b, rel(Ph[b], c.P_hat))


@pytest.mark.parametrize("n1,n2", SIZES_2D)
def test_small_strain_2d_every_size(fe2, n1, n2):
    print("2D small strain", n1, n2, flush=True)
    p = with_resolution(W.config("cfg2", macro=(1, 1), rve=8), n1, n2)
    u, ws = random_state(p, n1 * 100 + n2, 1e-3, 1e-3)
    check_a2_to_a6(fe2, p, u, ws, 1e-10)


@pytest.mark.parametrize("n1,n2", SIZES_FIN)
def test_finite_strain_2d_every_size(fe2, n1, n2):
    print("2D finite strain", n1, n2, flush=True)
    p = with_resolution(W.config("cfg5", macro=(1, 1), rve=8, n_steps=1), n1, n2)
    u, ws = random_state(p, n1 * 100 + n2 + 7, 5e-3, 1e-4)
    check_a2_to_a6(fe2, p, u, ws, 1e-10)


@pytest.mark.parametrize("n", SIZES_3D)
def test_small_strain_3d_every_size(fe2, n):
    print("3D small strain", n, flush=True)
    p = W.config("cfg4", macro=(1, 1, 1), rve=n)
    u, ws = random_state(p, n + 3, 1e-3, 1e-3)
    check_a2_to_a6(fe2, p, u, ws, 1e-10)


@pytest.mark.parametrize("n", [8, 16, 32, 48])
@pytest.mark.parametrize("prec,solver", [("fp32_ir", "jacobi"), ("fp64", "auto"), ("fp64", "jacobi")])
def test_small_strain_2d_both_preconditioners(fe2, n, prec, solver):
    """The square sizes 8, 16, 32 and 48 run the spectral preconditioner by
    default; the Jacobi one is selectable in both precisions and reaches the
    same C-bar."""
    print("2D small strain", n, prec, solver, flush=True)
    p = with_resolution(W.config("cfg2", macro=(1, 1), rve=8), n, n)
    u, ws = random_state(p, n * 101, 1e-3, 1e-3)
    check_a2_to_a6(fe2, p, u, ws, 1e-10, precision=prec, solver=solver)


def test_spectral_preconditioner_selection(fe2):
    """FE2_SOLVER_AUTO picks the spectral preconditioner on square 8/16/32/48
    RVEs only (both precisions); Jacobi is selectable; an explicit spectral
    request elsewhere is rejected."""
    p = W.config("cfg3", macro=(2, 2), resolutions=(16, 32, 48))
    res = p.rve_res[:, 0]
    h = fe2.fe2_setup(p, precision="fp32_ir")
    assert fe2.fe2_query(h, fe2.FE2_Q_SPECTRAL_RVES) == int(np.isin(res, (16, 32, 48)).sum())
    h.close()
    h = fe2.fe2_setup(p, precision="fp64")
    assert fe2.fe2_query(h, fe2.FE2_Q_SPECTRAL_RVES) == int(np.isin(res, (16, 32, 48)).sum())
    h.close()
    h = fe2.fe2_setup(p, precision="fp32_ir", solver="jacobi")
    assert fe2.fe2_query(h, fe2.FE2_Q_SPECTRAL_RVES) == 0
    h.close()
    with pytest.raises(fe2.FE2Error) as ei:
        fe2.fe2_setup(with_resolution(W.config("cfg2", macro=(1, 1), rve=8), 30, 30), solver="fft")
    assert ei.value.status == fe2.FE2_ENOTSUP
    with pytest.raises(fe2.FE2Error) as ei:
        fe2.fe2_setup(W.config("cfg4", macro=(1, 1, 1), rve=4), solver="fft")
    assert ei.value.status == fe2.FE2_ENOTSUP
