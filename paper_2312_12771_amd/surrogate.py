"""RVE-response surrogate: training-data generation, training and use in the
macro Newton loop.

Host-side orchestration only: every numeric step (RVE equilibration and
condensation, feature and target extraction, statistics, normalisation,
network forward/backward/Adam, decoding inside the Newton step, the error
judge) runs in libfe2's kernels through the C ABI; PyTorch provides device
buffers and index gathers.

Representation: input (E11, E22, E12, phi) -- Green-Lagrange strain of the
macro gradient and the phase-1 volume fraction; output the second
Piola-Kirchhoff stress and the Voigt matrix of dS/dE (see include/fe2.h).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import fe2

SIZES = (4, 128, 128, 128, 9)


def _torch():
    import torch
    return torch


def _dz(n, dtype=None):
    torch = _torch()
    return torch.zeros(int(n), dtype=dtype or torch.float64, device="cuda")


def rve_responses(problem, F: np.ndarray, precision: str = "fp32_ir", rve_tol: float = 1e-8,
                  micro_tol: float = 1e-10):
    """Equilibrated responses of the problem's RVEs at the macro gradients F
    [n_rve, 4] and the training pairs built from them.  Returns device
    tensors X [n,4], T [n,9], ok [n] (1 where the RVE solve succeeded) and
    the raw P [n,4], A [n,16]."""
    torch = _torch()
    h = fe2.fe2_setup(problem, precision=precision, rve_tol=rve_tol, micro_tol=micro_tol, scheme="classical")
    try:
        n = problem.n_rve
        Fd = torch.tensor(np.ascontiguousarray(F, dtype=np.float64).reshape(-1), device="cuda")
        P, A, ok = _dz(4 * n), _dz(16 * n), _dz(n)
        fe2.fe2_rve_response(h, Fd, P, A, ok, allow_noconv=True)
        X, T = _dz(4 * n), _dz(9 * n)
        fe2.fe2_surrogate_dataset(h, Fd, P, A, X, T)
        torch.cuda.synchronize()
    finally:
        h.close()
    return X, T, ok, P, A


@dataclass
class Surrogate:
    net: "fe2.MLP"
    norm: object                     # device float64 [26]
    train_log: dict = field(default_factory=dict)

    @classmethod
    def train(cls, X, T, ok, steps: int = 3000, lr: float = 3e-3, lr_min: float = 3e-5,
              max_batch: int = 16384, seed: int = 0, init_seed: int = 12771, log=None):
        """Fit the network to the rows of (X, T) with ok != 0: inputs scaled to
        [-1, 1] by their range, outputs standardised; full-batch Adam with a
        cosine learning-rate decay."""
        torch = _torch()
        import workloads as W
        n = ok.numel()
        si = fe2.fe2_surrogate_stats(X, 4, ok)
        so = fe2.fe2_surrogate_stats(T, 9, ok)
        norm = torch.cat([si[0:4], si[4:8], so[18:27], so[27:36]]).contiguous()
        if not bool(torch.all(norm[17:26] > 0)):
            raise RuntimeError("degenerate training targets")
        Xn = _dz(4 * n, torch.float32)
        Tn = _dz(9 * n, torch.float32)
        fe2.fe2_surrogate_normalize(X, 4, norm[0:4].contiguous(), norm[4:8].contiguous(), 1, Xn)
        fe2.fe2_surrogate_normalize(T, 9, norm[8:17].contiguous(), norm[17:26].contiguous(), 0, Tn)
        keep = torch.nonzero(ok > 0.5).flatten()
        Xn = Xn.view(n, 4).index_select(0, keep).contiguous()
        Tn = Tn.view(n, 9).index_select(0, keep).contiguous()
        nfit = Xn.shape[0]
        net = fe2.MLP(SIZES, max_batch=max(max_batch, nfit))
        net.set_params(torch.tensor(W.mlp_init(SIZES, init_seed), dtype=torch.float32, device="cuda"))
        w = torch.ones(9, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []
        for s in range(steps):
            a = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / steps))
            want = (s % 500 == 0) or s == steps - 1
            L = net.loss_grad(Xn, Tn, w, want_loss=want)
            if want:
                hist.append((s, L))
                if log:
                    log(f"surrogate step {s}: loss {L:.3e}")
            net.adam_step(a)
        torch.cuda.synchronize()
        L = net.loss_grad(Xn, Tn, w)
        info = dict(samples=int(nfit), rejected_samples=int(n - nfit), steps=steps,
                    seconds=time.perf_counter() - t0, final_loss=L, history=hist)
        return cls(net=net, norm=norm, train_log=info)

    def validation_rms(self, X, T, ok) -> float:
        """Root-mean-square error per output in standardised units on a
        held-out set."""
        torch = _torch()
        n = ok.numel()
        Xn = _dz(4 * n, torch.float32)
        Tn = _dz(9 * n, torch.float32)
        fe2.fe2_surrogate_normalize(X, 4, self.norm[0:4].contiguous(), self.norm[4:8].contiguous(), 1, Xn)
        fe2.fe2_surrogate_normalize(T, 9, self.norm[8:17].contiguous(), self.norm[17:26].contiguous(), 0, Tn)
        keep = torch.nonzero(ok > 0.5).flatten()
        Xn = Xn.view(n, 4).index_select(0, keep).contiguous()
        Tn = Tn.view(n, 9).index_select(0, keep).contiguous()
        w = torch.ones(9, dtype=torch.float32, device="cuda")
        L = self.net.loss_grad(Xn, Tn, w)
        return math.sqrt(L / 9.0)

    def close(self):
        self.net.close()


def solve_with_surrogate(h, sur: Surrogate, load_factors, judge_tol: float = 2e-2, judge: str = "last",
                         max_it: int = 20, history: Optional[list] = None):
    """Load stepping with the surrogate attached: accepted Gauss points take
    stress and tangent from the network, the others run the classical RVE
    path.  The full RVE solve judges the surrogate after the last load step
    (judge="last") or after every step ("every"); rejected points switch to
    the RVE path and the step is re-converged.  Returns statistics.

    The network evaluates the stress in FP32 (about 1e-7 relative), so the
    handle's newton_tol should be about 1e-6 or looser."""
    fe2.fe2_surrogate_attach(h, sur.net, sur.norm)
    stats = dict(judge_calls=0, rejected=0, max_err=[], newton=[])
    try:
        lams = list(load_factors)
        for k, lam in enumerate(lams):
            for _attempt in range(4):
                n_it = 0
                for it in range(max_it + 1):
                    st, norms = fe2.fe2_newton_step(h, lam)
                    n_it += 1
                    if history is not None:
                        history.append(norms)
                    if not np.isfinite(norms[1]) or norms[1] > 1e10:
                        raise RuntimeError(f"diverged at load factor {lam}")
                    if st == fe2.FE2_CONVERGED:
                        break
                else:
                    raise RuntimeError(f"no convergence at load factor {lam}")
                stats["newton"].append(n_it)
                if judge == "every" or (judge == "last" and k == len(lams) - 1):
                    _, err, nrej = fe2.fe2_surrogate_judge(h, judge_tol)
                    stats["judge_calls"] += 1
                    stats["max_err"].append(err)
                    stats["rejected"] += nrej
                    if nrej:
                        continue          # re-converge with the rejected points on the RVE path
                break
    finally:
        fe2.fe2_surrogate_detach(h)
    return stats
