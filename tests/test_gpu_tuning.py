"""Per-class solver overrides and the autotuner, through the C ABI.

* Overrides: on an uneven batch (16^2, 32^2, 48^2 classes) each class is
  switched to another solver variant (three columns per PCG pass, Jacobi,
  one column at a time); C-bar and P-hat still match the oracle at 1e-10
  with the residual driven to 1e-13, and the spectral-RVE count follows
  the choices.  Refusals: a variant the class cannot run, a resolution with
  no class, an unknown solver.
* Tuner: on a small uneven batch it times every variant of every class and
  keeps the fastest (the default unless another is faster by over 1 %);
  its table applied to a fresh handle gives the same C-bar (within the
  solve tolerance) as the default choice.
"""
import numpy as np
import pytest

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


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def condense_at(fe2, h, p, u):
    fe2.fe2_set_state(h, u=torch.tensor(u, device="cuda"), load_factor=0.0)
    fe2.fe2_assemble_rve(h)
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    Cb = torch.zeros(p.n_rve * nF * nF, dtype=torch.float64, device="cuda")
    Ph = torch.zeros(p.n_rve * nF, dtype=torch.float64, device="cuda")
    fe2.fe2_condense(h, Cb, Ph)
    torch.cuda.synchronize()
    return Cb.cpu().numpy().reshape(p.n_rve, nF, nF), Ph.cpu().numpy().reshape(p.n_rve, nF)


def test_class_overrides_match_oracle(fe2):
    p = W.config("cfg3", macro=(3, 3), resolutions=(16, 32, 48))
    u = 1e-3 * np.random.default_rng(4).standard_normal(p.n_dofs)
    h = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=1e-13)
    assert fe2.fe2_query(h, fe2.FE2_Q_SPECTRAL_RVES) == p.n_rve
    fe2.fe2_set_class_solver(h, (16, 16), "fft_mc")
    fe2.fe2_set_class_solver(h, (32, 32), "jacobi")
    fe2.fe2_set_class_solver(h, (48, 48), "fft")
    n32 = int(np.all(p.rve_res == 32, axis=1).sum())
    assert fe2.fe2_query(h, fe2.FE2_Q_SPECTRAL_RVES) == p.n_rve - n32
    C, Ph = condense_at(fe2, h, p, u)
    geo = M.macro_geometry(p)
    for b in range(p.n_rve):
        c = R.homogenize_rve(p, b, M.macro_gradient(p, geo, u, b))
        assert rel(C[b], c.C) < 1e-10, (b, p.rve_res[b], rel(C[b], c.C))
        assert rel(Ph[b], c.P_hat) < 1e-10
    # refusals
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_set_class_solver(h, (16, 16), "dense")       # 510 unknowns
    assert e.value.status == fe2.FE2_ENOTSUP
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_set_class_solver(h, (24, 24), "fft")         # no such class
    assert e.value.status == fe2.FE2_EINVAL
    h.close()
    hj = fe2.fe2_setup(p, precision="fp32_ir", solver="jacobi", rve_tol=1e-8)
    with pytest.raises(fe2.FE2Error) as e:
        fe2.fe2_set_class_solver(hj, (32, 32), "fft")        # no spectral tables built
    assert e.value.status == fe2.FE2_ENOTSUP
    hj.close()


def test_tuner_table_applies(fe2):
    from paper_2312_12771_amd import tune
    p = W.config("cfg3", macro=(8, 8), resolutions=(16, 32, 48))
    table = tune.tune(p, "test", "fp32_ir", 5e-4, 1.0, reps=2)
    print({("x".join(map(str, c["res"]))): (c["choice"], c["ms"]) for c in table["classes"]},
          table["rve_solve_ms_default"], table["rve_solve_ms_tuned"])
    assert {tuple(c["res"]) for c in table["classes"]} == {(16, 16), (32, 32), (48, 48)}
    for c in table["classes"]:
        best = min(c["ms"].values())
        assert c["choice"] in c["ms"]
        # the fastest, or the default when the fastest is within the margin
        assert c["ms"][c["choice"]] == best or (c["choice"] == tune.default_of(c["ms"]) and
                                               best > (1.0 - tune.MARGIN) * c["ms"][c["choice"]])
        assert "dense" not in c["ms"]                         # none of these sizes runs it
        assert "fft_mc" in c["ms"] and "jacobi" in c["ms"]
    u = 1e-3 * np.random.default_rng(5).standard_normal(p.n_dofs)
    h0 = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=5e-4)
    C0, _ = condense_at(fe2, h0, p, u)
    h0.close()
    h1 = fe2.fe2_setup(p, precision="fp32_ir", rve_tol=5e-4)
    tune.apply(h1, table, precision="fp32_ir", rve_tol=5e-4)
    C1, _ = condense_at(fe2, h1, p, u)
    h1.close()
    err = [np.linalg.norm(C1[b] - C0[b]) / np.linalg.norm(C0[b]) for b in range(p.n_rve)]
    assert max(err) < 1e-6
    with pytest.raises(ValueError):
        tune.apply(h1, table, precision="fp64")
