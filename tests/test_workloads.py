"""Seeded input generators: determinism, shapes and the stated recipes."""
import numpy as np

import workloads as W


def test_generators_are_deterministic_and_consistent():
    for name, kw in [("cfg1", {}), ("cfg2", dict(macro=(4, 4))), ("cfg3", dict(macro=(6, 6))),
                     ("cfg4", dict(macro=(2, 2, 2))), ("cfg5", dict(macro=(4, 4))), ("cook", dict(n_macro=4))]:
        a = W.config(name, **kw)
        b = W.config(name, **kw)
        assert np.array_equal(a.phase_id, b.phase_id)
        assert np.array_equal(a.phase_params, b.phase_params)
        assert a.n_rve == a.n_elems * a.n_gp
        assert a.rve_off[-1] == a.phase_id.size
        sizes = np.prod(a.rve_res, axis=1)
        assert np.array_equal(np.diff(a.rve_off), sizes)
        assert a.dir_dofs.dtype == np.int32 and np.all(np.diff(a.dir_dofs) > 0)


def test_recipes():
    p = W.config("cfg2")
    assert p.n_rve == 16384 and tuple(p.rve_res[0]) == (32, 32)
    vf = p.rve_phases(0).mean()
    assert abs(vf - 0.3) < 0.02                      # voxelised circle
    ratio = p.phase_params[::4, 1, 1] / p.phase_params[::4, 0, 1]
    assert abs(np.median(np.log(ratio)) - np.log(10)) < 0.05
    q = W.config("cfg3")
    assert q.n_rve == 65536 and set(np.unique(q.rve_res[:, 0])) == {16, 32, 48}
    c4 = W.config("cfg4")
    assert c4.n_rve == 4096 and abs(c4.rve_phases(0).mean() - 0.2) < 0.03
    c5 = W.config("cfg5")
    assert len(c5.load_factors) == 10 and abs(c5.dir_vals.max() - 0.1) < 1e-15
    ck = W.config("cook")
    assert abs(ck.f_ext[0::2].sum() + 5 * 160) < 1e-9 and abs(ck.f_ext[1::2].sum() - 10 * 160) < 1e-9
