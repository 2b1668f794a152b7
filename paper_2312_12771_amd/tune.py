"""Autotuner of the RVE solve: for every resolution class of a problem, the
solver variant (preconditioner, right-hand sides per PCG pass, or the dense
form) that solves the class fastest at the handle's precision and rve_tol.

The RVE blocks of the monolithic system are independent (Sec. 4.1), and the
resolution classes of a batch are solved by separate launches one after
another, so the time of a Newton step's RVE solve is the sum of the classes'
times and the choice separates: each class is timed with every variant it
can run while the others keep their current choice, and the fastest is kept.
Timings are those of the library's own launches (the RVE-solve phase of
fe2_newton_step from the reference state, HIP events on the stream); a
variant replaces the default only when it is faster by more than MARGIN.  Host
orchestration only: the result is a table of per-class choices that
fe2_set_class_solver applies.

Tables live in ``tuning/<name>.json`` next to this file, written by
``bench.py --tune`` on the GPU they are used on.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import numpy as np

from . import fe2

CANDIDATES = ("fft", "fft_mc", "jacobi", "dense")
TABLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")
# A variant replaces the class's default only when it is faster by more than
# the run-to-run spread of the timed phase (about 1 %); closer timings are
# noise, and picking by them only reshuffles the classes.
MARGIN = 0.01


def default_of(ms: dict) -> str:
    """The variant the library uses for a class without an override: the
    spectral preconditioner with one column per pass where the class has it,
    else Jacobi."""
    return "fft" if "fft" in ms else "jacobi"


def pick(ms: dict) -> str:
    """The fastest variant, or the default when the fastest is not faster by
    more than MARGIN."""
    best = min(ms, key=ms.get)
    d = default_of(ms)
    if d in ms and ms[best] > (1.0 - MARGIN) * ms[d]:
        return d
    return best


def classes_of(problem):
    """Resolutions of the problem's RVEs with their counts, most RVEs first."""
    res, cnt = np.unique(np.asarray(problem.rve_res), axis=0, return_counts=True)
    order = np.argsort(-cnt, kind="stable")
    return [(tuple(int(x) for x in res[k]), int(cnt[k])) for k in order]


def _rve_phase_ms(h, torch, lam, reps):
    """GPU time of the RVE solve phase of one Newton step from the reference
    state (fastest of reps)."""
    fe2.fe2_reset_state(h, 0.0)
    fe2.fe2_newton_step(h, lam)   # warm-up: kernels loaded
    best = float("inf")
    for _ in range(reps):
        fe2.fe2_reset_state(h, 0.0)
        fe2.fe2_set_profiling(h, True)
        fe2.fe2_newton_step(h, lam)
        prof = fe2.fe2_get_profile(h)
        fe2.fe2_set_profiling(h, False)
        best = min(best, float(prof[1]))
    return best


def tune(problem, name: str, precision: str = "fp32_ir", rve_tol: float = 5e-4, lam: float = 1.0,
         reps: int = 3, candidates=CANDIDATES) -> dict:
    """Time every class with every variant it can run; return the table."""
    import torch
    h = fe2.fe2_setup(problem, precision=precision, rve_tol=rve_tol, inner_tol=1e-5)
    try:
        base = _rve_phase_ms(h, torch, lam, reps)
        classes = []
        for res, n in classes_of(problem):
            ms = {}
            for cand in candidates:
                try:
                    fe2.fe2_set_class_solver(h, res, cand)
                except fe2.FE2Error as e:
                    if e.status not in (fe2.FE2_ENOTSUP,):
                        raise
                    continue
                ms[cand] = round(_rve_phase_ms(h, torch, lam, reps), 4)
            choice = pick(ms)
            fe2.fe2_set_class_solver(h, res, choice)
            classes.append(dict(res=list(res), n_rve=n, ms=ms, choice=choice))
        tuned = _rve_phase_ms(h, torch, lam, reps)
    finally:
        h.close()
    return dict(name=name, device=torch.cuda.get_device_name(0), precision=precision, rve_tol=rve_tol,
                load_factor=lam,
                note="ms: RVE-solve phase of a Newton step from the reference state with this class's variant "
                     "and the other classes at their choice so far (fastest of several runs)",
                classes=classes, rve_solve_ms_default=round(base, 4), rve_solve_ms_tuned=round(tuned, 4))


def path(name: str) -> str:
    return os.path.join(TABLE_DIR, f"{name}.json")


def save(table: dict) -> str:
    os.makedirs(TABLE_DIR, exist_ok=True)
    p = path(table["name"])
    with open(p, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    return p


def load(name: str) -> Optional[dict]:
    try:
        with open(path(name)) as f:
            return json.load(f)
    except OSError:
        return None


def apply(h, table: dict, precision: Optional[str] = None, rve_tol: Optional[float] = None) -> dict:
    """Apply a table's choices to a handle; returns {resolution: choice}.  A
    table tuned for another precision or tolerance is refused."""
    if precision is not None and table["precision"] != precision:
        raise ValueError(f"table tuned for {table['precision']}, handle runs {precision}")
    if rve_tol is not None and table["rve_tol"] != rve_tol:
        raise ValueError(f"table tuned for rve_tol {table['rve_tol']}, handle runs {rve_tol}")
    out = {}
    for c in table["classes"]:
        fe2.fe2_set_class_solver(h, c["res"], c["choice"])
        out["x".join(map(str, c["res"]))] = c["choice"]
    return out
