"""Newton steps replayed from HIP graphs (fe2_set_graph) against the same
steps launched individually, on two handles of the same problem.

Each graph is captured once per launch configuration and replayed several
times with the program's own eager work (assembly, state copies, syncs) in
between; every replay must give the eager handle's state exactly (the same
kernels run in the same order on the same data).  Covered: the bench
pattern (state reset, one step at the same load factor, repeated: one
graph replayed), load stepping (the load factor changes: a new graph per
increment, then replays for the later iterations), an uneven batch with
three resolution classes, the element basis and Q9 macro elements.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def state(fe2, h, p):
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device="cuda")
    w = torch.zeros(fe2.fe2_query(h, fe2.FE2_Q_FIELD_LEN), dtype=torch.float64, device="cuda")
    fe2.fe2_get_state(h, u, w)
    torch.cuda.synchronize()
    return u.cpu().numpy(), w.cpu().numpy()


def eager_work(fe2, h, p):
    """Unrelated eager launches between replays."""
    fe2.fe2_assemble_rve(h)
    nF = fe2.fe2_query(h, fe2.FE2_Q_NF)
    t = torch.zeros(p.n_rve * nF, dtype=torch.float64, device="cuda")
    fe2.fe2_get_data(h, fe2.FE2_D_PBAR, t)
    torch.cuda.synchronize()


CASES = [
    ("cfg2", dict(macro=(3, 3), rve=16), False),
    ("cfg3", dict(macro=(3, 3), resolutions=(16, 32, 48)), False),
    ("cfg2", dict(macro=(3, 3), rve=16), True),
    ("cfg2", dict(macro=(2, 2), rve=16, order=2), False),
]


@pytest.mark.parametrize("name,kw,element", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_graph_replays_match_individual_launches(fe2, name, kw, element, prec):
    p = W.config(name, **kw)
    if element:
        p = W.element_basis(p)
    print("graph replay", name, kw, element, prec, flush=True)
    he = fe2.fe2_setup(p, precision=prec, rve_tol=1e-10)
    hg = fe2.fe2_setup(p, precision=prec, rve_tol=1e-10)
    fe2.fe2_set_graph(hg, True)
    zu = torch.zeros(p.n_dofs, dtype=torch.float64, device="cuda")
    zw = torch.zeros(fe2.fe2_query(he, fe2.FE2_Q_FIELD_LEN), dtype=torch.float64, device="cuda")
    # bench pattern: reset, one step at load factor 1, four times
    for rep in range(4):
        for h in (he, hg):
            fe2.fe2_set_state(h, zu, zw, 0.0)
            st, _ = fe2.fe2_newton_step(h, 1.0)
            assert st == fe2.FE2_OK
        ue, we = state(fe2, he, p)
        ug, wg = state(fe2, hg, p)
        assert np.array_equal(ue, ug), (rep, np.abs(ue - ug).max())
        assert np.array_equal(we, wg), (rep, np.abs(we - wg).max())
        eager_work(fe2, hg, p)
    # load stepping: new configurations, then replays of the later iterations
    for h in (he, hg):
        fe2.fe2_set_state(h, zu, zw, 0.0)
    for lam in (0.5, 1.0):
        for it in range(3):
            for h in (he, hg):
                fe2.fe2_newton_step(h, lam)
            ue, we = state(fe2, he, p)
            ug, wg = state(fe2, hg, p)
            assert np.array_equal(ue, ug), (lam, it, np.abs(ue - ug).max())
            assert np.array_equal(we, wg), (lam, it, np.abs(we - wg).max())
            eager_work(fe2, hg, p)
    he.close()
    hg.close()
