"""Python binding of libfe2 (argument marshalling only).

Every function here forwards to the C ABI declared in include/fe2.h with the
same name; all arithmetic of the hot path runs in the library's HIP kernels.
Device buffers are torch tensors (float64, contiguous, on the current HIP
device) and streams are torch streams.  Importing this module fails loudly
when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe2.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run paper_2312_12771_amd/build.py "
                      "(or __graft_entry__.build()) first")
# torch (the provider of device buffers and streams) ships a HIP runtime
# with the same soname as the system one: load it first, so that libfe2
# binds to that runtime instead of torch then resolving to the system copy
# (a process whose torch runs on another runtime than it was built with
# finds no device)
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)
FE2_ABI_VERSION = 4

# status codes and enums (include/fe2.h)
FE2_OK, FE2_CONVERGED = 0, 1
FE2_EINVAL, FE2_ENOMEM, FE2_EHIP, FE2_ENOCONV, FE2_ESTATE, FE2_ENOTSUP = -1, -2, -3, -4, -5, -6
FE2_SMALL_STRAIN, FE2_FINITE_STRAIN = 0, 1
FE2_LINEAR_ISO, FE2_NEO_HOOKE, FE2_MOONEY_RIVLIN = 0, 1, 2
FE2_PREC_FP64, FE2_PREC_FP32_IR, FE2_PREC_BF16_IR = 0, 1, 2
FE2_SOLVER_AUTO, FE2_SOLVER_PCG_JACOBI, FE2_SOLVER_PCG_FFT, FE2_SOLVER_DENSE, FE2_SOLVER_PCG_FFT_MC = 0, 1, 2, 3, 4
FE2_SCHEME_GENERALIZED, FE2_SCHEME_CLASSICAL, FE2_SCHEME_CLASSICAL_PLAIN = 0, 1, 2
FE2_BASIS_DIRAC, FE2_BASIS_ELEMENT = 0, 1
(FE2_D_MACRO_GRAD, FE2_D_RESIDUAL, FE2_D_PBAR, FE2_D_SOLUTION, FE2_D_RVE_ITERS,
 FE2_D_RVE_RELRES, FE2_D_MACRO_RHS, FE2_D_MACRO_RTRUE, FE2_D_MACRO_DU,
 FE2_D_MACRO_KDENSE, FE2_D_CBAR, FE2_D_PHAT, FE2_D_RVE_MV64, FE2_D_PHASE_FRACTION,
 FE2_D_SURR_ERR) = range(15)
(FE2_Q_NF, FE2_Q_FIELD_LEN, FE2_Q_NDOF, FE2_Q_BANDWIDTH, FE2_Q_FAILED_RVES,
 FE2_Q_N_RVE, FE2_Q_FIELD_OFFSETS, FE2_Q_MICRO_ITERS, FE2_Q_SPECTRAL_RVES) = range(9)

_KIN = {"small": FE2_SMALL_STRAIN, "finite": FE2_FINITE_STRAIN}
_MAT = {"linear": FE2_LINEAR_ISO, "neohooke": FE2_NEO_HOOKE,
        "mooney_rivlin": FE2_MOONEY_RIVLIN}
_PREC = {"fp64": FE2_PREC_FP64, "fp32_ir": FE2_PREC_FP32_IR, "bf16_ir": FE2_PREC_BF16_IR}


class fe2_problem_desc(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("dim", C.c_int32), ("kinematics", C.c_int32), ("material", C.c_int32),
        ("n_nodes", C.c_int32), ("X", C.POINTER(C.c_double)),
        ("n_elems", C.c_int32), ("conn", C.POINTER(C.c_int32)),
        ("n_dir", C.c_int32), ("dir_dofs", C.POINTER(C.c_int32)),
        ("dir_vals", C.POINTER(C.c_double)),
        ("f_ext", C.POINTER(C.c_double)),
        ("n_rve", C.c_int32), ("rve_res", C.POINTER(C.c_int32)),
        ("rve_off", C.POINTER(C.c_int64)), ("phase_id", C.POINTER(C.c_uint8)),
        ("n_phase_params", C.c_int32), ("phase_params", C.POINTER(C.c_double)),
        ("rve_size", C.c_double),
        ("precision", C.c_int32), ("solver", C.c_int32), ("scheme", C.c_int32),
        ("rve_tol", C.c_double), ("inner_tol", C.c_double),
        ("newton_tol", C.c_double), ("micro_tol", C.c_double),
        ("max_pcg_it", C.c_int32), ("max_ir", C.c_int32), ("max_micro_it", C.c_int32),
        ("macro_basis", C.c_int32),
        ("macro_order", C.c_int32),
    ]


class fe2_1d_desc(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("order", C.c_int32), ("n_macro", C.c_int32), ("n_micro", C.c_int32), ("basis", C.c_int32),
        ("macro_length", C.c_double), ("body_load", C.c_double),
        ("phi_left", C.c_double), ("phi_right", C.c_double),
        ("lambda_gp", C.POINTER(C.c_double)),
    ]


FE2_1D_Q_N_PHI, FE2_1D_Q_N_RVE, FE2_1D_Q_N_INT = 0, 1, 2

_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_sig = {
    "fe2_setup": (C.c_int, [C.POINTER(fe2_problem_desc), _vp, C.POINTER(_vp)]),
    "fe2_assemble_rve": (C.c_int, [_vp, _vp]),
    "fe2_condense": (C.c_int, [_vp, _vp, _vp, _vp]),
    "fe2_newton_step": (C.c_int, [_vp, C.c_double, _dp, _vp]),
    "fe2_equilibrate_rve": (C.c_int, [_vp, C.POINTER(C.c_int), _vp]),
    "fe2_get_state": (C.c_int, [_vp, _vp, _vp, _vp]),
    "fe2_set_state": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp]),
    "fe2_reset_state": (C.c_int, [_vp, C.c_double, _vp]),
    "fe2_get_data": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "fe2_query": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int64)]),
    "fe2_destroy": (C.c_int, [_vp]),
    "fe2_set_profiling": (C.c_int, [_vp, C.c_int]),
    "fe2_get_profile": (C.c_int, [_vp, _dp]),
    "fe2_mlp_create": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.c_int, _vp, C.POINTER(_vp)]),
    "fe2_mlp_destroy": (C.c_int, [_vp]),
    "fe2_mlp_n_params": (C.c_int, [_vp, C.POINTER(C.c_int64)]),
    "fe2_mlp_set_params": (C.c_int, [_vp, _vp, _vp]),
    "fe2_mlp_get_params": (C.c_int, [_vp, _vp, _vp]),
    "fe2_mlp_forward": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "fe2_mlp_loss_grad": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp, _dp, _vp]),
    "fe2_mlp_adam_step": (C.c_int, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "fe2_mlp_reset_optimizer": (C.c_int, [_vp, _vp]),
    "fe2_rve_response": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fe2_surrogate_dataset": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fe2_surrogate_stats": (C.c_int, [C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "fe2_surrogate_normalize": (C.c_int, [C.c_int, C.c_int, _vp, _vp, _vp, C.c_int, _vp, _vp]),
    "fe2_surrogate_attach": (C.c_int, [_vp, _vp, _vp, _vp]),
    "fe2_surrogate_detach": (C.c_int, [_vp]),
    "fe2_surrogate_judge": (C.c_int, [_vp, C.c_double, _dp, C.POINTER(C.c_int), _vp]),
    "fe2_set_graph": (C.c_int, [_vp, C.c_int]),
    "fe2_set_class_solver": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    "fe2_band_solve": (C.c_int, [C.c_int, C.c_int, _vp, _vp, C.POINTER(C.c_int), _vp]),
    "fe2_band_solve_noalloc": (C.c_int, [C.c_int, C.c_int, _vp, _vp, C.POINTER(C.c_int), _vp]),
    "fe2_spectral_table": (C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "fe2_1d_setup": (C.c_int, [C.POINTER(fe2_1d_desc), _vp, C.POINTER(_vp)]),
    "fe2_1d_newton_step": (C.c_int, [_vp, _dp, _vp]),
    "fe2_1d_get_state": (C.c_int, [_vp, _vp, _vp, _vp]),
    "fe2_1d_query": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int64)]),
    "fe2_1d_destroy": (C.c_int, [_vp]),
    "fe2_strerror": (C.c_char_p, [C.c_int]),
    "fe2_last_error": (C.c_char_p, []),
    "fe2_abi_version": (C.c_int, []),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a
if _lib.fe2_abi_version() != FE2_ABI_VERSION:
    raise ImportError(f"{LIB_PATH} has ABI version {_lib.fe2_abi_version()}, this binding expects "
                      f"{FE2_ABI_VERSION}: rebuild the library")


class FE2Error(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.fe2_last_error().decode()
        super().__init__(f"{where}: {_lib.fe2_strerror(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status: int, where: str, allow=(FE2_OK,)):
    if status not in allow:
        raise FE2Error(status, where)
    return status


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def _dev_ptr(t):
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("device buffers must be contiguous float64 tensors on the GPU")
    return _vp(t.data_ptr())


def _dev_ptr32(t):
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("network buffers must be contiguous float32 tensors on the GPU")
    return _vp(t.data_ptr())


class Handle:
    """Owns an fe2_handle; ``close()`` (or garbage collection) destroys it."""

    def __init__(self, ptr: _vp):
        self._ptr = ptr

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("handle is closed")
        return self._ptr

    def close(self):
        if self._ptr is not None:
            _lib.fe2_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def make_desc(problem, precision: str = "fp64", solver: str = "auto",
              scheme: str = "generalized", rve_tol: float = 1e-10, inner_tol: float = 1e-5,
              newton_tol: float = 1e-10, micro_tol: float = 1e-13, max_pcg_it: int = 4000,
              max_ir: int = 8, max_micro_it: int = 30):
    """fe2_problem_desc of a problem description (any object with the
    attributes of workloads.Problem).  Returns (desc, keep): ``keep`` holds
    the arrays the descriptor points into and must outlive its use."""
    keep = dict(
        X=_arr(problem.X, np.float64), conn=_arr(problem.conn, np.int32),
        dd=_arr(problem.dir_dofs, np.int32), dv=_arr(problem.dir_vals, np.float64),
        fe=_arr(problem.f_ext, np.float64), res=_arr(problem.rve_res, np.int32),
        off=_arr(problem.rve_off, np.int64), ph=_arr(problem.phase_id, np.uint8),
        pp=_arr(problem.phase_params, np.float64))
    d = fe2_problem_desc()
    d.struct_size = C.sizeof(fe2_problem_desc)
    d.dim = int(problem.dim)
    d.kinematics = _KIN[problem.kinematics]
    d.material = _MAT[problem.material]
    d.n_nodes = keep["X"].shape[0]
    d.X = keep["X"].ctypes.data_as(_dp)
    d.n_elems = keep["conn"].shape[0]
    d.conn = keep["conn"].ctypes.data_as(C.POINTER(C.c_int32))
    d.n_dir = keep["dd"].size
    d.dir_dofs = keep["dd"].ctypes.data_as(C.POINTER(C.c_int32))
    d.dir_vals = keep["dv"].ctypes.data_as(_dp)
    d.f_ext = keep["fe"].ctypes.data_as(_dp) if np.any(keep["fe"]) else C.cast(None, _dp)
    d.n_rve = keep["res"].shape[0]
    d.rve_res = keep["res"].ctypes.data_as(C.POINTER(C.c_int32))
    d.rve_off = keep["off"].ctypes.data_as(C.POINTER(C.c_int64))
    d.phase_id = keep["ph"].ctypes.data_as(C.POINTER(C.c_uint8))
    d.n_phase_params = keep["pp"].shape[2]
    d.phase_params = keep["pp"].ctypes.data_as(_dp)
    d.rve_size = float(problem.rve_size)
    d.precision = _PREC[precision]
    d.solver = SOLVERS[solver]
    d.scheme = {"generalized": FE2_SCHEME_GENERALIZED, "classical": FE2_SCHEME_CLASSICAL,
                "classical_plain": FE2_SCHEME_CLASSICAL_PLAIN}[scheme]
    d.rve_tol, d.inner_tol, d.newton_tol, d.micro_tol = rve_tol, inner_tol, newton_tol, micro_tol
    d.max_pcg_it, d.max_ir, d.max_micro_it = max_pcg_it, max_ir, max_micro_it
    d.macro_basis = {"dirac": FE2_BASIS_DIRAC, "element": FE2_BASIS_ELEMENT}[
        getattr(problem, "macro_basis", "dirac")]
    d.macro_order = int(getattr(problem, "macro_order", 1))
    return d, keep


def fe2_setup(problem, precision: str = "fp64", solver: str = "auto",
              scheme: str = "generalized", rve_tol: float = 1e-10, inner_tol: float = 1e-5,
              newton_tol: float = 1e-10, micro_tol: float = 1e-13, max_pcg_it: int = 4000,
              max_ir: int = 8, max_micro_it: int = 30, stream=None) -> Handle:
    """Create a handle from a problem description (any object with the
    attributes of workloads.Problem)."""
    d, keep = make_desc(problem, precision, solver, scheme, rve_tol, inner_tol, newton_tol,
                        micro_tol, max_pcg_it, max_ir, max_micro_it)
    out = _vp()
    _check(_lib.fe2_setup(C.byref(d), _stream_ptr(stream), C.byref(out)), "fe2_setup")
    del keep
    return Handle(out)


def fe2_assemble_rve(h: Handle, stream=None):
    return _check(_lib.fe2_assemble_rve(h.ptr, _stream_ptr(stream)), "fe2_assemble_rve")


def fe2_condense(h: Handle, Cbar=None, Phat=None, stream=None, allow_noconv=False):
    allow = (FE2_OK, FE2_ENOCONV) if allow_noconv else (FE2_OK,)
    return _check(_lib.fe2_condense(h.ptr, _dev_ptr(Cbar), _dev_ptr(Phat), _stream_ptr(stream)),
                  "fe2_condense", allow)


def fe2_newton_step(h: Handle, load_factor: float, stream=None):
    """Returns (status, norms[4]) with status FE2_OK or FE2_CONVERGED."""
    norms = np.zeros(4)
    st = _lib.fe2_newton_step(h.ptr, float(load_factor), norms.ctypes.data_as(_dp),
                              _stream_ptr(stream))
    _check(st, "fe2_newton_step", (FE2_OK, FE2_CONVERGED))
    return st, norms


def fe2_equilibrate_rve(h: Handle, stream=None, allow_noconv=False):
    """Classical inner loop at the current state; returns (status, rounds)."""
    its = C.c_int(0)
    st = _lib.fe2_equilibrate_rve(h.ptr, C.byref(its), _stream_ptr(stream))
    _check(st, "fe2_equilibrate_rve", (FE2_OK, FE2_ENOCONV) if allow_noconv else (FE2_OK,))
    return st, int(its.value)


def fe2_spectral_table(n: int, rho: float) -> np.ndarray:
    """The RVE solver's spectral preconditioner table (host, no GPU work)."""
    ln = C.c_int()
    _check(_lib.fe2_spectral_table(int(n), float(rho), None, C.byref(ln)), "fe2_spectral_table")
    out = np.zeros(ln.value, dtype=np.float64)
    _check(_lib.fe2_spectral_table(int(n), float(rho), out.ctypes.data_as(C.POINTER(C.c_double)), None),
           "fe2_spectral_table")
    return out


def fe2_band_solve(n: int, bw: int, band, rhs, stream=None, allow_notspd=False):
    """Solve the SPD band system (lower band storage band [n*(bw+1)]) in place
    in rhs [n].  Returns (status, pivot): pivot is 0, or the 1-based index of
    a non-positive pivot (status FE2_ENOCONV, raised unless allow_notspd)."""
    piv = C.c_int(0)
    st = _lib.fe2_band_solve(int(n), int(bw), _dev_ptr(band), _dev_ptr(rhs), C.byref(piv), _stream_ptr(stream))
    _check(st, "fe2_band_solve", (FE2_OK, FE2_ENOCONV) if allow_notspd else (FE2_OK,))
    return st, piv.value


def fe2_band_solve_noalloc(n: int, bw: int, band, rhs, stream=None, allow_notspd=False):
    """fe2_band_solve with its workspace in the library's static device
    scratch (no allocation); same arguments and result."""
    piv = C.c_int(0)
    st = _lib.fe2_band_solve_noalloc(int(n), int(bw), _dev_ptr(band), _dev_ptr(rhs), C.byref(piv),
                                     _stream_ptr(stream))
    _check(st, "fe2_band_solve_noalloc", (FE2_OK, FE2_ENOCONV) if allow_notspd else (FE2_OK,))
    return st, piv.value


def fe2_rve_response(h: Handle, F, P=None, Cm=None, ok=None, stream=None, allow_noconv=False):
    """Equilibrated RVE response at the macro gradients F [n_rve*nF]."""
    st = _lib.fe2_rve_response(h.ptr, _dev_ptr(F), _dev_ptr(P), _dev_ptr(Cm), _dev_ptr(ok), _stream_ptr(stream))
    return _check(st, "fe2_rve_response", (FE2_OK, FE2_ENOCONV) if allow_noconv else (FE2_OK,))


def fe2_surrogate_dataset(h: Handle, F, P, Cm, X, T, stream=None):
    return _check(_lib.fe2_surrogate_dataset(h.ptr, _dev_ptr(F), _dev_ptr(P), _dev_ptr(Cm), _dev_ptr(X),
                                             _dev_ptr(T), _stream_ptr(stream)), "fe2_surrogate_dataset")


def fe2_surrogate_stats(V, m: int, ok=None, out=None, stream=None):
    """Column statistics of V [n*m] -> out [4*m] (min, max, mean, std)."""
    import torch
    n = V.numel() // m
    if out is None:
        out = torch.zeros(4 * m, dtype=torch.float64, device=V.device)
    _check(_lib.fe2_surrogate_stats(int(n), int(m), _dev_ptr(V), _dev_ptr(ok), _dev_ptr(out), _stream_ptr(stream)),
           "fe2_surrogate_stats")
    return out


def fe2_surrogate_normalize(V, m: int, a, b, mode: int, out, stream=None):
    n = V.numel() // m
    return _check(_lib.fe2_surrogate_normalize(int(n), int(m), _dev_ptr(V), _dev_ptr(a), _dev_ptr(b), int(mode),
                                               _dev_ptr32(out), _stream_ptr(stream)), "fe2_surrogate_normalize")


def fe2_surrogate_attach(h: Handle, net, norm, stream=None):
    return _check(_lib.fe2_surrogate_attach(h.ptr, net.ptr, _dev_ptr(norm), _stream_ptr(stream)),
                  "fe2_surrogate_attach")


def fe2_surrogate_detach(h: Handle):
    return _check(_lib.fe2_surrogate_detach(h.ptr), "fe2_surrogate_detach")


def fe2_surrogate_judge(h: Handle, tol: float, stream=None):
    """Returns (status, max error, rejected points)."""
    err = C.c_double(0.0)
    nrej = C.c_int(0)
    st = _lib.fe2_surrogate_judge(h.ptr, float(tol), C.byref(err), C.byref(nrej), _stream_ptr(stream))
    _check(st, "fe2_surrogate_judge", (FE2_OK, FE2_ENOCONV))
    return st, float(err.value), int(nrej.value)


def fe2_get_state(h: Handle, u=None, w=None, stream=None):
    return _check(_lib.fe2_get_state(h.ptr, _dev_ptr(u), _dev_ptr(w), _stream_ptr(stream)),
                  "fe2_get_state")


def fe2_set_state(h: Handle, u=None, w=None, load_factor: float = 0.0, stream=None):
    return _check(_lib.fe2_set_state(h.ptr, _dev_ptr(u), _dev_ptr(w), float(load_factor),
                                     _stream_ptr(stream)), "fe2_set_state")


def fe2_reset_state(h: Handle, load_factor: float = 0.0, stream=None):
    return _check(_lib.fe2_reset_state(h.ptr, float(load_factor), _stream_ptr(stream)), "fe2_reset_state")


def fe2_get_data(h: Handle, which: int, dst, stream=None):
    return _check(_lib.fe2_get_data(h.ptr, int(which), _dev_ptr(dst), _stream_ptr(stream)),
                  "fe2_get_data")


def fe2_query(h: Handle, which: int):
    if which == FE2_Q_FIELD_OFFSETS:
        n = fe2_query(h, FE2_Q_N_RVE)
        out = np.zeros(n + 1, dtype=np.int64)
        _check(_lib.fe2_query(h.ptr, which, out.ctypes.data_as(C.POINTER(C.c_int64))), "fe2_query")
        return out
    v = C.c_int64()
    _check(_lib.fe2_query(h.ptr, int(which), C.byref(v)), "fe2_query")
    return int(v.value)


def fe2_set_profiling(h: Handle, enable: bool = True):
    return _check(_lib.fe2_set_profiling(h.ptr, int(bool(enable))), "fe2_set_profiling")


def fe2_get_profile(h: Handle):
    """Accumulated ms of [assemble+norms, RVE solve, macro assemble+solve,
    update, whole step] and the number of timed solving steps (cleared)."""
    out = np.zeros(6)
    _check(_lib.fe2_get_profile(h.ptr, out.ctypes.data_as(_dp)), "fe2_get_profile")
    return out


def fe2_destroy(h: Handle):
    h.close()


def abi_version() -> int:
    return int(_lib.fe2_abi_version())


# --------------------------------------------------------------------------
# host-side driver: load stepping around fe2_newton_step
# --------------------------------------------------------------------------

def solve(h: Handle, load_factors, max_it: int = 20, stream=None, history: Optional[list] = None,
          diverge_at: float = 1e10):
    """Load stepping: for every load factor call fe2_newton_step until it
    reports convergence.  Raises RuntimeError when a step exceeds max_it or
    the macro residual norm exceeds ``diverge_at`` (or is not finite)."""
    for lam in load_factors:
        h_step = []
        for it in range(max_it + 1):
            st, norms = fe2_newton_step(h, lam, stream)
            h_step.append(norms)
            if not np.isfinite(norms[1]) or norms[1] > diverge_at:
                raise RuntimeError(f"diverged at load factor {lam}, iteration {it}")
            if st == FE2_CONVERGED:
                break
        else:
            raise RuntimeError(f"no convergence at load factor {lam}")
        if history is not None:
            history.append(h_step)
    return h


# --------------------------------------------------------------------------
# surrogate network
# --------------------------------------------------------------------------

class MLP:
    """Owns an fe2_mlp: tanh multilayer perceptron with FP32 forward,
    loss gradient and Adam on the GPU (argument marshalling only)."""

    def __init__(self, sizes, max_batch: int, stream=None):
        arr = (C.c_int * len(sizes))(*[int(x) for x in sizes])
        p = _vp()
        _check(_lib.fe2_mlp_create(len(sizes) - 1, arr, int(max_batch), _stream_ptr(stream), C.byref(p)),
               "fe2_mlp_create")
        self._ptr = p
        self.sizes = list(sizes)
        self.max_batch = int(max_batch)
        n = C.c_int64()
        _check(_lib.fe2_mlp_n_params(self._ptr, C.byref(n)), "fe2_mlp_n_params")
        self.n_params = int(n.value)

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("network is closed")
        return self._ptr

    def set_params(self, theta, stream=None):
        _check(_lib.fe2_mlp_set_params(self.ptr, _dev_ptr32(theta), _stream_ptr(stream)), "fe2_mlp_set_params")

    def get_params(self, out, stream=None):
        _check(_lib.fe2_mlp_get_params(self.ptr, _dev_ptr32(out), _stream_ptr(stream)), "fe2_mlp_get_params")
        return out

    def forward(self, X, Y, stream=None):
        _check(_lib.fe2_mlp_forward(self.ptr, int(X.shape[0]), _dev_ptr32(X), _dev_ptr32(Y),
                                    _stream_ptr(stream)), "fe2_mlp_forward")
        return Y

    def loss_grad(self, X, T, w_out, grad=None, want_loss=True, stream=None):
        loss = C.c_double(0.0)
        _check(_lib.fe2_mlp_loss_grad(self.ptr, int(X.shape[0]), _dev_ptr32(X), _dev_ptr32(T),
                                      _dev_ptr32(w_out), _dev_ptr32(grad),
                                      C.byref(loss) if want_loss else None, _stream_ptr(stream)),
               "fe2_mlp_loss_grad")
        return float(loss.value) if want_loss else None

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.fe2_mlp_adam_step(self.ptr, float(lr), float(beta1), float(beta2), float(eps),
                                      _stream_ptr(stream)), "fe2_mlp_adam_step")

    def reset_optimizer(self, stream=None):
        _check(_lib.fe2_mlp_reset_optimizer(self.ptr, _stream_ptr(stream)), "fe2_mlp_reset_optimizer")

    def close(self):
        if self._ptr is not None:
            _lib.fe2_mlp_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# 1+1D problem of Sec. 5.1
# ---------------------------------------------------------------------------

class Handle1D:
    """Owns an fe2_1d_handle."""

    def __init__(self, ptr):
        self._ptr = ptr

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("handle is closed")
        return self._ptr

    def close(self):
        if self._ptr is not None:
            _lib.fe2_1d_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc_1d(problem):
    """fe2_1d_desc of a workloads.OneDProblem; returns (desc, keep)."""
    lam = _arr(problem.lambda_gp, np.float64)
    d = fe2_1d_desc()
    d.struct_size = C.sizeof(fe2_1d_desc)
    d.order, d.n_macro, d.n_micro = int(problem.order), int(problem.n_macro), int(problem.n_micro)
    d.basis = {"dirac": FE2_BASIS_DIRAC, "element": FE2_BASIS_ELEMENT}[problem.basis]
    d.macro_length, d.body_load = float(problem.macro_length), float(problem.body_load)
    d.phi_left, d.phi_right = float(problem.phi_left), float(problem.phi_right)
    d.lambda_gp = lam.ctypes.data_as(_dp)
    return d, lam


def fe2_1d_setup(problem, stream=None) -> Handle1D:
    d, keep = make_desc_1d(problem)
    out = _vp()
    _check(_lib.fe2_1d_setup(C.byref(d), _stream_ptr(stream), C.byref(out)), "fe2_1d_setup")
    del keep
    return Handle1D(out)


def fe2_1d_newton_step(h: Handle1D, stream=None):
    norms = np.zeros(4)
    _check(_lib.fe2_1d_newton_step(h.ptr, norms.ctypes.data_as(_dp), _stream_ptr(stream)), "fe2_1d_newton_step")
    return norms


def fe2_1d_query(h: Handle1D, which: int) -> int:
    v = C.c_int64(0)
    _check(_lib.fe2_1d_query(h.ptr, which, C.byref(v)), "fe2_1d_query")
    return int(v.value)


def fe2_1d_get_state(h: Handle1D, phi=None, w=None, stream=None):
    _check(_lib.fe2_1d_get_state(h.ptr, _dev_ptr(phi), _dev_ptr(w), _stream_ptr(stream)), "fe2_1d_get_state")


SOLVERS = {"auto": FE2_SOLVER_AUTO, "jacobi": FE2_SOLVER_PCG_JACOBI, "fft": FE2_SOLVER_PCG_FFT,
           "fft_mc": FE2_SOLVER_PCG_FFT_MC, "dense": FE2_SOLVER_DENSE}


def fe2_set_class_solver(h: Handle, res, solver: str):
    """Per-class solver override for the RVEs of resolution `res` (see fe2.h)."""
    r = [int(x) for x in res] + [1, 1]
    return _check(_lib.fe2_set_class_solver(h.ptr, r[0], r[1], r[2], SOLVERS[solver]), "fe2_set_class_solver")


def fe2_set_graph(h: Handle, enable: bool):
    """Newton steps as one HIP graph launch per configuration (see fe2.h)."""
    return _check(_lib.fe2_set_graph(h.ptr, 1 if enable else 0), "fe2_set_graph")
