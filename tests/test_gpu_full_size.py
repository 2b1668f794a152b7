"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (mixed form: FP32 PCG with FP64 refinement at the bench's rve_tol),
on sampled outputs the oracle computes one by one, plus properties that hold
for every RVE of the batch.

* 2D linear, 64x64 macro, 16 384 RVEs of 32x32;
* 2D uneven batch, 128x128 macro, 65 536 RVEs of 16^2 / 32^2 / 48^2 (samples
  from every resolution class);
* 2D finite strain, 64x64 macro, 16 384 RVEs of 32x32, first iteration of
  the first increment (condensation at F = I), and the second iteration
  (a nonlinear state: macro gradient and fluctuation of the first update,
  five right-hand sides per RVE);
* 3D linear, 8x8x8 hex8 macro, 4 096 RVEs of 10^3.

Bar: the sampled C-bar within 1e-6 (Frobenius-relative) of the oracle, the
accuracy target of the mixed form; every C-bar symmetric to 1e-6 and
positive definite.
"""
import numpy as np
import pytest

import workloads as W
from oracle import rve as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def one_step_cbar(fe2, p, rve_tol, lam):
    h = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=rve_tol, inner_tol=1e-5)
    st, _ = fe2.fe2_newton_step(h, lam)
    assert st == fe2.FE2_OK
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    cb = torch.zeros(p.n_rve * nF * nF, dtype=torch.float64, device="cuda")
    fe2.fe2_get_data(h, fe2.FE2_D_CBAR, cb)
    torch.cuda.synchronize()
    assert fe2.fe2_query(h, fe2.FE2_Q_FAILED_RVES) == 0
    h.close()
    return cb.cpu().numpy().reshape(p.n_rve, nF, nF)


def check_batch_properties(C, semidefinite=False):
    """Symmetry of every C-bar; positive definite (small strain) or positive
    semidefinite up to rounding (finite strain at F = I, where the
    infinitesimal rotation is a zero-energy mode of the first elasticity
    tensor)."""
    sym = np.abs(C - C.transpose(0, 2, 1)).max(axis=(1, 2)) / np.abs(C).max(axis=(1, 2))
    assert sym.max() <= 1e-6, sym.max()
    ev = np.linalg.eigvalsh(0.5 * (C + C.transpose(0, 2, 1)))
    if semidefinite:
        assert (ev[:, 0] >= -1e-6 * ev[:, -1]).all(), ev[:, 0].min()
        assert (ev[:, 1] > 0.0).all()
    else:
        assert ev.min() > 0.0


def frob(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sample(n, k, seed):
    rng = np.random.default_rng(seed)
    return sorted({0, n - 1, *rng.choice(n, size=k, replace=False).tolist()})


def test_linear_2d_full_batch(fe2):
    p = W.config("cfg2")
    print("full size: 2D linear, 16384 RVEs of 32x32, mixed form", flush=True)
    C = one_step_cbar(fe2, p, 5e-4, 1.0)
    check_batch_properties(C)
    nF = 3
    for b in sample(p.n_rve, 20, 1):
        ref = R.homogenize_rve(p, b, np.zeros(nF)).C
        assert frob(C[b], ref) <= 1e-6, (b, frob(C[b], ref))


def test_uneven_batch_full_size(fe2):
    p = W.config("cfg3")
    print("full size: uneven batch, 65536 RVEs of 16/32/48, mixed form", flush=True)
    C = one_step_cbar(fe2, p, 5e-4, 1.0)
    check_batch_properties(C)
    res = p.rve_res[:, 0]
    for n in (16, 32, 48):
        ids = np.where(res == n)[0]
        assert ids.size > 0
        for b in ids[sample(ids.size, 5, n)]:
            ref = R.homogenize_rve(p, int(b), np.zeros(3)).C
            assert frob(C[b], ref) <= 1e-6, (int(b), n, frob(C[b], ref))


def test_finite_strain_full_batch(fe2):
    p = W.config("cfg5")
    print("full size: 2D finite strain, 16384 RVEs of 32x32, mixed form", flush=True)
    C = one_step_cbar(fe2, p, 1e-4, p.load_factors[0])
    check_batch_properties(C, semidefinite=True)
    F = np.eye(2).ravel()
    for b in sample(p.n_rve, 12, 5):
        ref = R.homogenize_rve(p, b, F).C
        assert frob(C[b], ref) <= 1e-6, (b, frob(C[b], ref))


def test_finite_strain_full_batch_nonlinear_state(fe2):
    """Second Newton iteration of the first increment at full size: the RVEs
    are linearised at the macro gradient and fluctuation of the first update
    (r_b != 0, the residual column solved too); sampled C-bar and P-hat
    against the oracle at that state."""
    p = W.config("cfg5")
    print("full size: 2D finite strain, 16384 RVEs of 32x32, second iteration", flush=True)
    h = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=1e-4, inner_tol=1e-5)
    lam = p.load_factors[0]
    st, _ = fe2.fe2_newton_step(h, lam)
    assert st == fe2.FE2_OK
    flen = fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN)
    off = fe2.fe2_query(h, fe2.FE2_Q_FIELD_OFFSETS)
    w1 = torch.zeros(flen, dtype=torch.float64, device="cuda")
    fe2.fe2_get_state(h, w=w1)
    st, norms = fe2.fe2_newton_step(h, lam)
    assert st == fe2.FE2_OK and norms[2] > 0.0   # the RVE residuals are nonzero
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    mg = torch.zeros(p.n_rve * nF, dtype=torch.float64, device="cuda")
    cb = torch.zeros(p.n_rve * nF * nF, dtype=torch.float64, device="cuda")
    ph = torch.zeros(p.n_rve * nF, dtype=torch.float64, device="cuda")
    fe2.fe2_get_data(h, fe2.FE2_D_MACRO_GRAD, mg)
    fe2.fe2_get_data(h, fe2.FE2_D_CBAR, cb)
    fe2.fe2_get_data(h, fe2.FE2_D_PHAT, ph)
    torch.cuda.synchronize()
    assert fe2.fe2_query(h, fe2.FE2_Q_FAILED_RVES) == 0
    h.close()
    mg = mg.cpu().numpy().reshape(p.n_rve, nF)
    C = cb.cpu().numpy().reshape(p.n_rve, nF, nF)
    Ph = ph.cpu().numpy().reshape(p.n_rve, nF)
    w1 = w1.cpu().numpy()
    sym = np.abs(C - C.transpose(0, 2, 1)).max(axis=(1, 2)) / np.abs(C).max(axis=(1, 2))
    assert sym.max() <= 1e-6, sym.max()
    for b in sample(p.n_rve, 8, 7):
        c = R.homogenize_rve(p, b, mg[b], w1[off[b]:off[b + 1]])
        assert frob(C[b], c.C) <= 1e-6, (b, frob(C[b], c.C))
        assert frob(Ph[b], c.P_hat) <= 1e-6, (b, frob(Ph[b], c.P_hat))


def test_linear_3d_full_batch(fe2):
    p = W.config("cfg4")
    print("full size: 3D linear, 4096 RVEs of 10^3, mixed form", flush=True)
    C = one_step_cbar(fe2, p, 5e-4, 1.0)
    check_batch_properties(C)
    for b in sample(p.n_rve, 6, 4):
        ref = R.homogenize_rve(p, b, np.zeros(6)).C
        assert frob(C[b], ref) <= 1e-6, (b, frob(C[b], ref))
