"""ctypes binding of ``libope.so`` (declared in ``include/ope.h``).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the C names; device buffers may be passed as torch CUDA tensors
(float64, contiguous) or as raw integer device addresses.  A missing or
unloadable library raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libope.so")

OPE_OK = 0
OPE_EINVAL = 1
OPE_ENOMEM = 2
OPE_EHIP = 3
OPE_ENONFINITE = 4
OPE_ECG_MAXIT = 5
OPE_EPIVOT = 6
OPE_EUNSUPPORTED = 7
OPE_ENOTSPD = 8
OPE_FP64 = 0
OPE_MIXED = 1
MK_F64, MK_F32, MK_BF16 = 0, 1, 2

STATUS_NAMES = {
    OPE_OK: "OPE_OK", OPE_EINVAL: "OPE_EINVAL", OPE_ENOMEM: "OPE_ENOMEM", OPE_EHIP: "OPE_EHIP",
    OPE_ENONFINITE: "OPE_ENONFINITE", OPE_ECG_MAXIT: "OPE_ECG_MAXIT", OPE_EPIVOT: "OPE_EPIVOT",
    OPE_EUNSUPPORTED: "OPE_EUNSUPPORTED", OPE_ENOTSPD: "OPE_ENOTSPD",
}


class OpeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({ope_status_string(status)})")


class ope_op_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("m", ctypes.c_int64 * 3),
        ("h", ctypes.c_double * 3),
        ("kinetic", ctypes.c_double),
        ("shift", ctypes.c_double),
        ("V", ctypes.POINTER(ctypes.c_double)),
    ]


class ope_step_info(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double),
        ("residual", ctypes.c_double),
        ("drift", ctypes.c_double),
        ("inner_iterations", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


class ope_solve_info(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("residual", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("drift", ctypes.c_double),
        ("inner_iterations", ctypes.c_int64),
        ("stalled", ctypes.c_int32),
        ("learned_steps", ctypes.c_int32),
        ("rejected", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("tau", ctypes.c_double),
    ]


class ope_solve_opts(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("tau_min", ctypes.c_double),
        ("tau_max", ctypes.c_double),
        ("grow", ctypes.c_double),
        ("shrink", ctypes.c_double),
        ("res_tol", ctypes.c_double),
        ("energy_tol", ctypes.c_double),
        ("energy_ref", ctypes.c_double),
        ("max_steps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ope_kernel_time(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


OPE_KERNEL_STENCIL = 0
OPE_KERNEL_CG_SWEEP_A = 1
OPE_KERNEL_CG_SWEEP_B = 2
OPE_KERNEL_GRAM = 3
OPE_KERNEL_ROWMM = 4
OPE_KERNEL_SMALL = 5
OPE_KERNEL_CG_SWEEP_B_Y = 6
OPE_KERNEL_CG_REDUCE = 7
OPE_KERNEL_MG = 8
OPE_KERNEL_MG_POST = 9

_lib = None

_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

SIGNATURES = {
    "ope_create": ([ctypes.POINTER(_P), ctypes.POINTER(ope_op_desc), _I64, _I32, _P], _I32),
    "ope_destroy": ([_P], _I32),
    "ope_status_string": ([_I32], ctypes.c_char_p),
    "ope_set_inner": ([_P, _D, _D, _I32], _I32),
    "ope_apply_h": ([_P, _P, _P], _I32),
    "ope_source_solve": ([_P, _P, _P, _P, _D, _I32, ctypes.POINTER(_I32)], _I32),
    "ope_gram": ([_P, _P, _I64, _I64, _P, _I64, _I64, _I64, _P], _I32),
    "ope_small_solve": ([_P, _P, _P, _D, _P, _P, _P], _I32),
    "ope_update": ([_P, _P, _P, _P], _I32),
    "ope_energy": ([_P, _P, ctypes.POINTER(_D)], _I32),
    "ope_residual": ([_P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)], _I32),
    "ope_step": ([_P, _P, _D, ctypes.POINTER(ope_step_info)], _I32),
    "ope_solve": ([_P, _P, _D, _D, _I32, ctypes.POINTER(ope_solve_info)], _I32),
    "ope_set_sweep_shape": ([_P, _I32, _I32, _I32], _I32),
    "ope_set_graphs": ([_P, _I32], _I32),
    "ope_set_multigrid": ([_P, _I32], _I32),
    "ope_mg_info": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_I64)], _I32),
    "ope_mg_vcycle": ([_P, _P, _P], _I32),
    "ope_autotune": ([_P], _I32),
    "ope_batch_create": ([ctypes.POINTER(_P), ctypes.POINTER(ope_op_desc), ctypes.POINTER(_I64), _I32, _I32, _P],
                         _I32),
    "ope_batch_destroy": ([_P], _I32),
    "ope_batch_context": ([_P, _I32, ctypes.POINTER(_P)], _I32),
    "ope_batch_step": ([_P, ctypes.POINTER(_P), _D, ctypes.POINTER(ope_step_info)], _I32),
    "ope_batch_solve": ([_P, ctypes.POINTER(_P), _D, _D, _I32, ctypes.POINTER(ope_solve_info)], _I32),
    "ope_batch_autotune": ([_P, ctypes.POINTER(_I32)], _I32),
    "ope_batch_set_shared": ([_P, _I32], _I32),
    "ope_batch_capture": ([_P, ctypes.POINTER(_P), ctypes.c_double, _I32], _I32),
    "ope_batch_replay": ([_P, _P], _I32),
    "ope_get_sweep_shape": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)], _I32),
    "ope_profile_begin": ([_P, _I32], _I32),
    "ope_convert": ([_P, _P, _P, _I64, _I32], _I32),
    "ope_gram_f32": ([_P, _I32, _P, _I64, _I64, _P, _I64, _I64, _I64, _P], _I32),
    "ope_rowmm_f32": ([_P, _I32, _P, _P, _P, _P, _P, _D, _D, _P], _I32),
    "ope_profile_end": ([_P, ctypes.POINTER(ope_kernel_time)], _I32),
    "ope_set_recycle": ([_P, _I32], _I32),
    "ope_profile_end_launches": ([_P, ctypes.POINTER(ope_kernel_time), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_int64], _I32),
    "ope_net_create": ([_P, _I64, ctypes.POINTER(_P)], _I32),
    "ope_net_destroy": ([_P], _I32),
    "ope_net_set_weights": ([_P, _P], _I32),
    "ope_net_get_weights": ([_P, _P], _I32),
    "ope_net_potential": ([_P, _P], _I32),
    "ope_net_set_loss": ([_P, _I32], _I32),
    "ope_net_forward": ([_P, _P, _P, _I64, _P], _I32),
    "ope_net_grad": ([_P, _P, _P, _P, _I64, ctypes.POINTER(_D), _P], _I32),
    "ope_net_train_step": ([_P, _P, _P, _P, _I64, _D, ctypes.POINTER(_D)], _I32),
    "ope_net_samples": ([_P, _P, _P, _I64, _I64, _P, _P], _I32),
    "ope_set_preconditioner": ([_P, _P, _I32], _I32),
    "ope_step_learned": ([_P, _P, _D, ctypes.POINTER(ope_step_info), ctypes.POINTER(_I32)], _I32),
    "ope_gram_noalloc": ([_P, _I64, _I64, _P, _I64, _I64, _I64, _P, _P], _I32),
    "ope_solve_ex": ([_P, _P, ctypes.POINTER(ope_solve_opts), ctypes.POINTER(ope_solve_info)], _I32),
    "ope_net_apply_grad": ([_P, _P, _D], _I32),
    "ope_spectrum_bounds": ([_P, ctypes.POINTER(_D), ctypes.POINTER(_D)], _I32),
    "ope_set_mass": ([_P, _P, _P], _I32),
    "ope_apply_mass": ([_P, _P, _P], _I32),
    "ope_orthonormalize": ([_P, _P], _I32),
    "ope_workspace_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I32),
    "ope_set_workspace": ([_P, _P, ctypes.c_size_t], _I32),
    "ope_energy_d": ([_P, _P, _P], _I32),
    "ope_residual_d": ([_P, _P, _P, _P], _I32),
    "ope_step_ld": ([_P, _P, _I64, _D, ctypes.POINTER(ope_step_info)], _I32),
    "ope_energy_ld": ([_P, _P, _I64, ctypes.POINTER(_D)], _I32),
    "ope_residual_ld": ([_P, _P, _I64, ctypes.POINTER(_D), _P, ctypes.POINTER(_D)], _I32),
}

OPE_NET_PARAMS = 15120
OPE_NET_LOSS_ENERGY = 0
OPE_NET_LOSS_RESIDUAL = 1
OPE_NET_LOSS_BOTH = 2


def lib() -> ctypes.CDLL:
    """Load ``libope.so`` once; raise if it is missing (build it first).

    torch is imported first when it is installed: its ROCm build ships its own
    HIP runtime under the same soname, and loading torch first makes this
    library bind to that one runtime, so torch's streams and allocations are
    valid here.  Loading the system runtime first would leave two runtimes in
    the process."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2511_06788_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    # torch tensor: must live on the GPU and be contiguous
    if not x.is_cuda:
        raise ValueError("device buffer expected (torch CUDA tensor)")
    if not x.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return x.data_ptr()


def _check(status: int, where: str, allow=()):
    if status != OPE_OK and status not in allow:
        raise OpeError(status, where)
    return status


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def ope_status_string(status: int) -> str:
    return lib().ope_status_string(status).decode()


def ope_create(dim: int, m: Sequence[int], h: Sequence[float], V: np.ndarray, N: int, kinetic: float = 1.0,
               shift: float = 0.0, precision: int = OPE_FP64, stream=None) -> int:
    """Create a context; returns the opaque handle (an int)."""
    Vh = np.ascontiguousarray(V, dtype=np.float64)
    d = ope_op_desc()
    d.dim = dim
    for a in range(3):
        d.m[a] = int(m[a]) if a < len(m) else 1
        d.h[a] = float(h[a]) if a < len(h) else 1.0
    d.kinetic = kinetic
    d.shift = shift
    d.V = Vh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = _P()
    _check(lib().ope_create(ctypes.byref(out), ctypes.byref(d), int(N), int(precision), _stream_ptr(stream)),
           "ope_create")
    return out.value


def ope_destroy(ctx: int) -> None:
    _check(lib().ope_destroy(ctx), "ope_destroy")


def ope_set_inner(ctx: int, eta_rel: float = 0.1, eta_floor: float = 1e-12, max_iter: int = 2000) -> None:
    _check(lib().ope_set_inner(ctx, eta_rel, eta_floor, max_iter), "ope_set_inner")


def ope_apply_h(ctx: int, X, Y) -> None:
    _check(lib().ope_apply_h(ctx, _ptr(X), _ptr(Y)), "ope_apply_h")


def ope_source_solve(ctx: int, U, Y, Y0=None, tol: float = 1e-12, max_iter: int = 10000, allow_maxit=False) -> int:
    it = _I32(0)
    st = lib().ope_source_solve(ctx, _ptr(U), _ptr(Y), _ptr(Y0), tol, max_iter, ctypes.byref(it))
    _check(st, "ope_source_solve", allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
    return it.value


def ope_gram(ctx: int, A, lda: int, na: int, B, ldb: int, nb: int, rows: int, out) -> None:
    _check(lib().ope_gram(ctx, _ptr(A), lda, na, _ptr(B), ldb, nb, rows, _ptr(out)), "ope_gram")


def ope_gram_noalloc(A, lda: int, na: int, B, ldb: int, nb: int, rows: int, out, stream=None) -> None:
    _check(lib().ope_gram_noalloc(_ptr(A), lda, na, _ptr(B), ldb, nb, rows, _ptr(out), _stream_ptr(stream)),
           "ope_gram_noalloc")


def ope_small_solve(ctx: int, Sb, T, tau: float, Z, A=None, B=None) -> None:
    _check(lib().ope_small_solve(ctx, _ptr(Sb), _ptr(T), tau, _ptr(Z), _ptr(A), _ptr(B)), "ope_small_solve")


def ope_update(ctx: int, U, Y, Z) -> None:
    _check(lib().ope_update(ctx, _ptr(U), _ptr(Y), _ptr(Z)), "ope_update")


def ope_energy(ctx: int, U) -> float:
    e = _D(0.0)
    _check(lib().ope_energy(ctx, _ptr(U), ctypes.byref(e)), "ope_energy")
    return e.value


def ope_residual(ctx: int, U, N: int, want_ritz: bool = True):
    """Returns ``(residual, ritz values (N,) or None, drift)``."""
    res = _D(0.0)
    drift = _D(0.0)
    ritz = (ctypes.c_double * N)() if want_ritz else None
    _check(lib().ope_residual(ctx, _ptr(U), ctypes.byref(res), ritz, ctypes.byref(drift)), "ope_residual")
    return res.value, (np.array(ritz[:], dtype=np.float64) if want_ritz else None), drift.value


def ope_step(ctx: int, U, tau: float, allow_maxit: bool = True) -> ope_step_info:
    info = ope_step_info()
    st = lib().ope_step(ctx, _ptr(U), tau, ctypes.byref(info))
    _check(st, "ope_step", allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
    return info


def ope_step_raw(ctx: int, U, tau: float) -> int:
    """``ope_step`` without diagnostics (NULL info); returns the status."""
    return lib().ope_step(ctx, _ptr(U), tau, None)


def ope_solve(ctx: int, U, tau: float, res_tol: float, max_steps: int) -> ope_solve_info:
    info = ope_solve_info()
    _check(lib().ope_solve(ctx, _ptr(U), tau, res_tol, max_steps, ctypes.byref(info)), "ope_solve",
           allow=(OPE_ECG_MAXIT,))
    return info


def ope_solve_ex(ctx: int, U, tau: float, tau_min: Optional[float] = None, tau_max: Optional[float] = None,
                 grow: float = 1.5, shrink: float = 0.5, res_tol: float = -1.0, energy_tol: float = -1.0,
                 energy_ref: Optional[float] = None, max_steps: int = 10000) -> ope_solve_info:
    """Algorithm 1 with the step chosen in [tau_min, tau_max] (fixed when equal)."""
    o = ope_solve_opts()
    o.tau = tau
    o.tau_min = tau if tau_min is None else tau_min
    o.tau_max = tau if tau_max is None else tau_max
    o.grow, o.shrink = grow, shrink
    o.res_tol, o.energy_tol = res_tol, energy_tol
    o.energy_ref = float("nan") if energy_ref is None else energy_ref
    o.max_steps = int(max_steps)
    o.reserved = 0
    info = ope_solve_info()
    _check(lib().ope_solve_ex(ctx, _ptr(U), ctypes.byref(o), ctypes.byref(info)), "ope_solve_ex",
           allow=(OPE_ECG_MAXIT,))
    return info


def ope_spectrum_bounds(ctx: int):
    """Returns the Lanczos estimates ``(lambda_min, lambda_max)`` of H."""
    lo, hi = _D(0.0), _D(0.0)
    _check(lib().ope_spectrum_bounds(ctx, ctypes.byref(lo), ctypes.byref(hi)), "ope_spectrum_bounds")
    return lo.value, hi.value


def ope_set_mass(ctx: int, d: Optional[np.ndarray], mu: Sequence[float] = (0.0, 0.0, 0.0)) -> None:
    if d is None:
        _check(lib().ope_set_mass(ctx, None, None), "ope_set_mass")
        return
    dh = np.ascontiguousarray(d, dtype=np.float64)
    muh = np.ascontiguousarray(list(mu) + [0.0] * (3 - len(mu)), dtype=np.float64)
    _check(lib().ope_set_mass(ctx, dh.ctypes.data, muh.ctypes.data), "ope_set_mass")


def ope_apply_mass(ctx: int, X, Y) -> None:
    _check(lib().ope_apply_mass(ctx, _ptr(X), _ptr(Y)), "ope_apply_mass")


def ope_orthonormalize(ctx: int, U) -> None:
    _check(lib().ope_orthonormalize(ctx, _ptr(U)), "ope_orthonormalize")


def ope_workspace_size(ctx: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().ope_workspace_size(ctx, ctypes.byref(b)), "ope_workspace_size")
    return b.value


def ope_set_workspace(ctx: int, buf, nbytes: int) -> None:
    _check(lib().ope_set_workspace(ctx, _ptr(buf), int(nbytes)), "ope_set_workspace")


def ope_energy_d(ctx: int, U, d_energy) -> None:
    _check(lib().ope_energy_d(ctx, _ptr(U), _ptr(d_energy)), "ope_energy_d")


def ope_residual_d(ctx: int, U, d_residual, d_drift) -> None:
    _check(lib().ope_residual_d(ctx, _ptr(U), _ptr(d_residual), _ptr(d_drift)), "ope_residual_d")


def ope_step_ld(ctx: int, U, ldu: int, tau: float, allow_maxit: bool = True) -> ope_step_info:
    info = ope_step_info()
    st = lib().ope_step_ld(ctx, _ptr(U), int(ldu), tau, ctypes.byref(info))
    _check(st, "ope_step_ld", allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
    return info


def ope_energy_ld(ctx: int, U, ldu: int) -> float:
    e = _D(0.0)
    _check(lib().ope_energy_ld(ctx, _ptr(U), int(ldu), ctypes.byref(e)), "ope_energy_ld")
    return e.value


def ope_residual_ld(ctx: int, U, ldu: int, N: int, want_ritz: bool = True):
    res = _D(0.0)
    drift = _D(0.0)
    ritz = (ctypes.c_double * N)() if want_ritz else None
    _check(lib().ope_residual_ld(ctx, _ptr(U), int(ldu), ctypes.byref(res), ritz, ctypes.byref(drift)),
           "ope_residual_ld")
    return res.value, (np.array(ritz[:], dtype=np.float64) if want_ritz else None), drift.value


OPE_SWEEP_CHUNK_MAJOR = 1
OPE_SWEEP_NONTEMPORAL = 2
OPE_SWEEP_NARROW = 4
OPE_SWEEP_LINES = 8
OPE_SWEEP_LINES4 = 16
OPE_SWEEP_LINES8 = 32


def ope_autotune(ctx: int) -> None:
    _check(lib().ope_autotune(ctx), "ope_autotune")


def ope_set_graphs(ctx: int, enable: bool) -> None:
    _check(lib().ope_set_graphs(ctx, 1 if enable else 0), "ope_set_graphs")


def ope_set_multigrid(ctx: int, enable: bool) -> None:
    _check(lib().ope_set_multigrid(ctx, 1 if enable else 0), "ope_set_multigrid")


def ope_mg_info(ctx: int):
    """(levels, nodes of the coarsest level); (0, 0) when the preconditioner is off."""
    lv, nc = _I32(0), _I64(0)
    _check(lib().ope_mg_info(ctx, ctypes.byref(lv), ctypes.byref(nc)), "ope_mg_info")
    return lv.value, nc.value


def ope_mg_vcycle(ctx: int, R, Z) -> None:
    _check(lib().ope_mg_vcycle(ctx, _ptr(R), _ptr(Z)), "ope_mg_vcycle")


def ope_set_sweep_shape(ctx: int, q_max: int, march_chunks: int, flags: int = 0) -> None:
    _check(lib().ope_set_sweep_shape(ctx, q_max, march_chunks, flags), "ope_set_sweep_shape")


def ope_get_sweep_shape(ctx: int):
    """Returns ``(q, march_chunks, workgroups)`` of the stencil / CG sweeps."""
    q, mc, wg = _I32(0), _I32(0), _I32(0)
    _check(lib().ope_get_sweep_shape(ctx, ctypes.byref(q), ctypes.byref(mc), ctypes.byref(wg)), "ope_get_sweep_shape")
    return q.value, mc.value, wg.value


def ope_convert(ctx: int, src, dst, count: int, to_double: bool) -> None:
    _check(lib().ope_convert(ctx, _ptr(src), _ptr(dst), int(count), 1 if to_double else 0), "ope_convert")


def ope_gram_f32(ctx: int, kind: int, A, lda: int, na: int, B, ldb: int, nb: int, rows: int, out) -> None:
    _check(lib().ope_gram_f32(ctx, kind, _ptr(A), lda, na, _ptr(B), ldb, nb, rows, _ptr(out)), "ope_gram_f32")


def ope_rowmm_f32(ctx: int, kind: int, X0, M0, X1, M1, Cm, cbeta: float, ascale: float, Out) -> None:
    _check(lib().ope_rowmm_f32(ctx, kind, _ptr(X0), _ptr(M0), _ptr(X1), _ptr(M1), _ptr(Cm), cbeta, ascale, _ptr(Out)),
           "ope_rowmm_f32")


def ope_profile_begin(ctx: int, kernel: int) -> None:
    _check(lib().ope_profile_begin(ctx, kernel), "ope_profile_begin")


def ope_profile_end(ctx: int):
    """Returns ``(launches, total_ms)`` of the kernel timed since ope_profile_begin."""
    t = ope_kernel_time()
    _check(lib().ope_profile_end(ctx, ctypes.byref(t)), "ope_profile_end")
    return t.launches, t.total_ms


def ope_set_recycle(ctx: int, enable: bool) -> None:
    _check(lib().ope_set_recycle(ctx, 1 if enable else 0), "ope_set_recycle")


def ope_profile_end_launches(ctx: int, cap: int):
    """Returns ``(launches, total_ms, tags, ms)``: the totals and, for the first
    ``cap`` timed launches, each launch's CG iteration tag and device time."""
    t = ope_kernel_time()
    tags = (ctypes.c_int32 * max(cap, 1))()
    ms = (ctypes.c_double * max(cap, 1))()
    _check(lib().ope_profile_end_launches(ctx, ctypes.byref(t), tags, ms, cap), "ope_profile_end_launches")
    k = min(cap, t.launches)
    return t.launches, t.total_ms, list(tags[:k]), list(ms[:k])


def ope_net_create(ctx: int, max_batch: int) -> int:
    h = _P()
    _check(lib().ope_net_create(ctx, int(max_batch), ctypes.byref(h)), "ope_net_create")
    return h.value


def ope_net_destroy(net: int) -> None:
    _check(lib().ope_net_destroy(net), "ope_net_destroy")


def ope_net_set_weights(net: int, w: np.ndarray) -> None:
    w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    if w.size != OPE_NET_PARAMS:
        raise ValueError(f"{OPE_NET_PARAMS} weights expected")
    _check(lib().ope_net_set_weights(net, w.ctypes.data), "ope_net_set_weights")


def ope_net_get_weights(net: int) -> np.ndarray:
    w = np.empty(OPE_NET_PARAMS, dtype=np.float32)
    _check(lib().ope_net_get_weights(net, w.ctypes.data), "ope_net_get_weights")
    return w


def ope_net_set_loss(net: int, kind: int) -> None:
    _check(lib().ope_net_set_loss(net, int(kind)), "ope_net_set_loss")


def ope_net_potential(net: int, V2) -> None:
    _check(lib().ope_net_potential(net, _ptr(V2)), "ope_net_potential")


def ope_net_forward(net: int, X, V2, B: int, F) -> None:
    _check(lib().ope_net_forward(net, _ptr(X), _ptr(V2), int(B), _ptr(F)), "ope_net_forward")


def ope_net_grad(net: int, X, V2, T, B: int, want_grad: bool = True):
    """Returns ``(loss, grad)`` (grad a host FP32 array, or None)."""
    loss = _D(0.0)
    g = np.empty(OPE_NET_PARAMS, dtype=np.float32) if want_grad else None
    _check(lib().ope_net_grad(net, _ptr(X), _ptr(V2), _ptr(T), int(B), ctypes.byref(loss),
                              g.ctypes.data if g is not None else None), "ope_net_grad")
    return loss.value, g


def ope_net_train_step(net: int, X, V2, T, B: int, lr: float) -> float:
    loss = _D(0.0)
    _check(lib().ope_net_train_step(net, _ptr(X), _ptr(V2), _ptr(T), int(B), float(lr), ctypes.byref(loss)),
           "ope_net_train_step")
    return loss.value


def ope_net_apply_grad(net: int, grad: np.ndarray, lr: float) -> None:
    g = np.ascontiguousarray(grad, dtype=np.float32).reshape(-1)
    if g.size != OPE_NET_PARAMS:
        raise ValueError(f"{OPE_NET_PARAMS} gradient values expected")
    _check(lib().ope_net_apply_grad(net, g.ctypes.data, float(lr)), "ope_net_apply_grad")


def ope_net_samples(net: int, R, S, ld: int, B: int, X, T) -> None:
    _check(lib().ope_net_samples(net, _ptr(R), _ptr(S), int(ld), int(B), _ptr(X), _ptr(T)), "ope_net_samples")


def ope_set_preconditioner(ctx: int, net: Optional[int], judge: bool = True) -> None:
    _check(lib().ope_set_preconditioner(ctx, net, 1 if judge else 0), "ope_set_preconditioner")


def ope_step_learned(ctx: int, U, tau: float, allow_maxit: bool = True):
    """Returns ``(info, accepted)``."""
    info = ope_step_info()
    acc = _I32(0)
    st = lib().ope_step_learned(ctx, _ptr(U), tau, ctypes.byref(info), ctypes.byref(acc))
    _check(st, "ope_step_learned", allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
    return info, bool(acc.value)


def net_weights_to_layers(w: np.ndarray):
    """Split a flat parameter vector into W1 (27,2,16), W2, W3 (27,16,16), W4 (27,16,1)."""
    w = np.asarray(w).reshape(-1)
    out, off = [], 0
    for ci, co in ((2, 16), (16, 16), (16, 16), (16, 1)):
        k = 27 * ci * co
        out.append(w[off:off + k].reshape(27, ci, co))
        off += k
    return out


def net_layers_to_weights(Ws) -> np.ndarray:
    return np.concatenate([np.asarray(W, dtype=np.float32).reshape(-1) for W in Ws])


NET_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "net_wells64.npy")


def load_net_weights(path: str = NET_WEIGHTS) -> np.ndarray:
    """Trained weights shipped with the package (FP32, OPE_NET_PARAMS values)."""
    w = np.load(path, allow_pickle=False).astype(np.float32).reshape(-1)
    if w.size != OPE_NET_PARAMS:
        raise ValueError(f"{path}: {w.size} values, {OPE_NET_PARAMS} expected")
    return w


class Net:
    """Owns one ``ope_net`` created on a Context."""

    def __init__(self, ctx, max_batch: int, weights: Optional[np.ndarray] = None):
        self.ctx = ctx
        self.handle = ope_net_create(ctx.handle, max_batch)
        if weights is not None:
            ope_net_set_weights(self.handle, weights)

    def close(self):
        if self.handle:
            ope_net_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns one ``ope_batch`` of independent problems (workloads.Problem list)."""

    def __init__(self, problems, precision=OPE_FP64, stream=None):
        self.count = len(problems)
        self.N = [int(p.N) for p in problems]
        self.n = [int(p.grid.n) for p in problems]
        descs = (ope_op_desc * self.count)()
        self._keep = []
        for i, p in enumerate(problems):
            Vc = np.ascontiguousarray(p.V, dtype=np.float64)
            self._keep.append(Vc)
            d = descs[i]
            d.dim = p.grid.dim
            for a in range(3):
                d.m[a] = p.grid.m[a] if a < p.grid.dim else 1
                d.h[a] = p.grid.h[a] if a < p.grid.dim else 1.0
            d.kinetic = p.kinetic
            d.shift = p.shift
            d.V = Vc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        Ns = (_I64 * self.count)(*self.N)
        h = _P()
        _check(lib().ope_batch_create(ctypes.byref(h), descs, Ns, self.count, precision, _stream_ptr(stream)),
               "ope_batch_create")
        self.handle = h.value

    def context(self, i: int) -> int:
        c = _P()
        _check(lib().ope_batch_context(self.handle, i, ctypes.byref(c)), "ope_batch_context")
        return c.value

    def _ptrs(self, Us):
        if len(Us) != self.count:
            raise ValueError("one block per problem expected")
        return (_P * self.count)(*[_ptr(U) for U in Us])

    def step(self, Us, tau: float, allow_maxit: bool = True):
        infos = (ope_step_info * self.count)()
        _check(lib().ope_batch_step(self.handle, self._ptrs(Us), tau, infos), "ope_batch_step",
               allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
        return list(infos)

    def solve(self, Us, tau: float, res_tol: float, max_steps: int):
        infos = (ope_solve_info * self.count)()
        _check(lib().ope_batch_solve(self.handle, self._ptrs(Us), tau, res_tol, max_steps, infos), "ope_batch_solve",
               allow=(OPE_ECG_MAXIT,))
        return list(infos)

    def capture(self, Us, tau: float, cg_iterations: int) -> None:
        """One batched step of the blocks Us as a HIP graph (ope_batch_capture)."""
        self._captured = list(Us)          # the graph steps these buffers: keep them alive
        _check(lib().ope_batch_capture(self.handle, self._ptrs(Us), tau, cg_iterations), "ope_batch_capture")

    def replay(self, wait: bool = True, allow_maxit: bool = True):
        """Replays the captured step; with wait, returns the per-problem infos."""
        if not wait:
            _check(lib().ope_batch_replay(self.handle, None), "ope_batch_replay")
            return None
        infos = (ope_step_info * self.count)()
        _check(lib().ope_batch_replay(self.handle, ctypes.cast(infos, _P)), "ope_batch_replay",
               allow=(OPE_ECG_MAXIT,) if allow_maxit else ())
        return list(infos)

    def set_shared(self, shared: bool) -> None:
        _check(lib().ope_batch_set_shared(self.handle, 1 if shared else 0), "ope_batch_set_shared")

    def autotune(self) -> int:
        k = _I32(0)
        _check(lib().ope_batch_autotune(self.handle, ctypes.byref(k)), "ope_batch_autotune")
        return k.value

    def close(self):
        if self.handle:
            lib().ope_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Owns one ``ope_ctx`` for a workload (grid, potential, N)."""

    def __init__(self, grid, V, N, kinetic=1.0, shift=0.0, stream=None, precision=OPE_FP64):
        self.N = int(N)
        self.n = int(np.prod(grid.m))
        self.precision = precision
        self.handle = ope_create(grid.dim, grid.m, grid.h, V, N, kinetic=kinetic, shift=shift, stream=stream,
                                 precision=precision)

    def close(self):
        if self.handle:
            ope_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
