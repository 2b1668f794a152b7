"""GPU parity of the 1+1D problem of Sec. 5.1 (FE^2 settings [delta, q] and
[0, q]) against the oracle's direct solve of the whole coupled system, and
the convergence of the GPU solutions to the closed form at the orders the
paper reports.

The problem is linear: one generalized Newton step from the initial state
reaches the discrete solution; the second step reports its residual.
Tolerances: 1e-11 relative on phi, 1e-9 on the fluctuations (FP64
throughout; the oracle solves the monolithic system, the GPU condenses).
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import oned as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_sec5.json")))["one_d_benchmark"]


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def gpu_solve(fe2, k, q, basis):
    p = W.oned_problem(k, q, basis)
    print("1d", k, q, basis, flush=True)
    h = fe2.fe2_1d_setup(p)
    n0 = fe2.fe2_1d_newton_step(h)
    n1 = fe2.fe2_1d_newton_step(h)
    nphi = fe2.fe2_1d_query(h, fe2.FE2_1D_Q_N_PHI)
    nr = fe2.fe2_1d_query(h, fe2.FE2_1D_Q_N_RVE)
    ni = fe2.fe2_1d_query(h, fe2.FE2_1D_Q_N_INT)
    phi = torch.zeros(nphi, dtype=torch.float64, device="cuda")
    w = torch.zeros(nr * ni, dtype=torch.float64, device="cuda")
    fe2.fe2_1d_get_state(h, phi, w)
    torch.cuda.synchronize()
    h.close()
    return phi.cpu().numpy(), w.cpu().numpy().reshape(nr, ni), n0, n1


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


SETTING = {"dirac": "dirac", "element": "const"}


@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("basis", ["dirac", "element"])
@pytest.mark.parametrize("k", [3, 6])
def test_oned_matches_oracle(fe2, k, q, basis):
    phi, w, n0, n1 = gpu_solve(fe2, k, q, basis)
    ref = O.solve(k, q, SETTING[basis])
    assert rel(phi, ref.phi) < 1e-11
    assert rel(w, ref.w) < 1e-9
    # the second step starts from the discrete solution
    assert n1[1] <= 1e-10 * n1[3] and n1[2] <= 1e-10 * n1[3]
    assert n0[1] > 1e-3 * n0[3]


def _orders(errs):
    return [np.log2(a / b) for a, b in zip(errs[:-1], errs[1:])]


@pytest.mark.parametrize("q,basis,key", [(1, "dirac", "[delta,1]"), (1, "element", "[0,1]"),
                                         (2, "dirac", "[delta,2]"), (2, "element", "[0,2]")])
def test_oned_convergence_orders_on_gpu(fe2, q, basis, key):
    """GPU solutions for k = 4..9 (up to 512 macro elements and 512 RVE
    elements): relative L2 errors against the closed form fall at the paper's
    reported orders (discussion of Fig. 2)."""
    ks = range(4, 10)
    e_phi, e_w = [], []
    for k in ks:
        phi, w, _, _ = gpu_solve(fe2, k, q, basis)
        sol = O.Solution(k=k, q=q, setting=SETTING[basis], phi=phi, w=w,
                         macro=O.Mesh(2 ** k, q, O.L_MACRO), micro=O.Mesh(2 ** k, q, 1.0))
        ep, ew = O.errors(sol)
        e_phi.append(ep)
        e_w.append(ew)
    print(key, "err_phi", e_phi, "err_w", e_w, flush=True)
    rep_p = GOLD["reported_orders"]["err_phi"][key]
    rep_w = GOLD["reported_orders"]["err_w"][key]
    op, ow = _orders(e_phi), _orders(e_w)
    # orders over the first levels (later err_phi levels of q = 2 reach rounding)
    if rep_p == ">2":
        assert min(op) > 1.95
    elif rep_p == 3.5:
        assert min(op[:3]) >= 3.5
    else:
        assert all(abs(o - rep_p) < 0.15 for o in op)
    assert all(abs(o - rep_w) < 0.15 for o in ow)
