"""pISTA for the graphical lasso on MI355X (gfx950): Python binding of libglasso.

Argument marshalling only: torch supplies device memory and the current HIP
stream, every step of the solver runs in the HIP kernels behind the C ABI
(include/glasso.h).  Importing this package loads libglasso.so and fails when it
is missing.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _native
from ._native import GlassoInfo, GlassoOptions

_lib = _native.load()

FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3}
CONVERGED, MAX_ITER, LS_FAILED = 0, 1, 2
STATUS_NAMES = {CONVERGED: "converged", MAX_ITER: "max_iter", LS_FAILED: "ls_failed"}


class GlassoError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.glasso_error_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise GlassoError(code, where)


def _dev(t: torch.Tensor, name: str, dtype=torch.float64) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _square(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square, got {tuple(t.shape)}")
    return t.shape[0]


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


@dataclass
class Result:
    A: torch.Tensor
    W: torch.Tensor | None
    objective: float
    iterations: int
    status: int
    kkt_rel1: float
    kkt_fro: float
    kkt_max: float
    nnz: int
    ls_trials: int
    fallback_steps: int
    time_ms: tuple

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


class Solver:
    """A libglasso handle: options plus a cached device workspace."""

    def __init__(self, precision: str | int = "fp64", max_iter: int = 500, t0: float = 1.0,
                 shrink: float = 0.5, t_floor: float = 1e-4, t_min: float = 1e-12,
                 warm_start: bool = False):
        opt = GlassoOptions()
        _check(_lib.glasso_default_options(ctypes.byref(opt)), "glasso_default_options")
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.max_iter = int(max_iter)
        opt.t0 = float(t0)
        opt.shrink = float(shrink)
        opt.t_floor = float(t_floor)
        opt.t_min = float(t_min)
        opt.warm_start = int(bool(warm_start))
        self.options = opt
        h = ctypes.c_void_p()
        _check(_lib.glasso_create(ctypes.byref(h), ctypes.byref(opt)), "glasso_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.glasso_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- full solve
    def solve(self, S: torch.Tensor, lam: float, tol: float, A: torch.Tensor | None = None,
              want_W: bool = True, stream=None) -> Result:
        n = _square(S, "S")
        pS = _dev(S, "S")
        if A is None:
            if self.options.warm_start:
                raise ValueError("warm_start solver needs A")
            A = torch.empty_like(S)
        else:
            if tuple(A.shape) != (n, n):
                raise ValueError("A must have the shape of S")
        pA = _dev(A, "A")
        W = torch.empty_like(S) if want_W else None
        info = GlassoInfo()
        _check(_lib.glasso_solve(self._h, pS, n, float(lam), float(tol), pA,
                                 W.data_ptr() if W is not None else None,
                                 ctypes.byref(info), _stream(stream)), "glasso_solve")
        return Result(A, W, info.objective, info.iterations, info.status, info.kkt_rel1,
                      info.kkt_fro, info.kkt_max, int(info.nnz), info.ls_trials,
                      info.fallback_steps, tuple(info.time_ms))

    # ---------------------------------------------------------------- single steps
    def cholesky(self, A: torch.Tensor, stream=None):
        n = _square(A, "A")
        L = torch.empty_like(A)
        info = ctypes.c_int64(0)
        logdet = ctypes.c_double(0.0)
        _check(_lib.glasso_cholesky(self._h, _dev(A, "A"), n, L.data_ptr(), ctypes.byref(info),
                                    ctypes.byref(logdet), _stream(stream)), "glasso_cholesky")
        return L, int(info.value), float(logdet.value)

    def inverse(self, A: torch.Tensor, stream=None) -> torch.Tensor:
        n = _square(A, "A")
        W = torch.empty_like(A)
        _check(_lib.glasso_inverse(self._h, _dev(A, "A"), n, W.data_ptr(), _stream(stream)),
               "glasso_inverse")
        return W

    def gradient_pass(self, S, W, A, lam: float, stream=None):
        n = _square(S, "S")
        Z = torch.empty_like(S)
        GM = torch.empty((n, n), dtype=torch.int8, device=S.device)
        kkt = (ctypes.c_double * 4)()
        _check(_lib.glasso_gradient_pass(self._h, _dev(S, "S"), _dev(W, "W"), _dev(A, "A"), n,
                                         float(lam), Z.data_ptr(), GM.data_ptr(), kkt,
                                         _stream(stream)), "glasso_gradient_pass")
        return Z, GM, {"sum_abs_z": kkt[0], "sum_abs_a": kkt[1], "kkt_fro": kkt[2], "kkt_max": kkt[3]}

    def precond_product(self, A, Z, precision: str | int = "fp64", stream=None) -> torch.Tensor:
        n = _square(A, "A")
        P = torch.empty_like(A)
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(_lib.glasso_precond_product(self._h, _dev(A, "A"), _dev(Z, "Z"), n, prec,
                                           P.data_ptr(), _stream(stream)), "glasso_precond_product")
        return P

    def trial_point(self, A, P, S, GM, lam: float, t: float, stream=None):
        n = _square(A, "A")
        At = torch.empty_like(A)
        sums = (ctypes.c_double * 2)()
        _check(_lib.glasso_trial_point(self._h, _dev(A, "A"), _dev(P, "P"), _dev(S, "S"),
                                       _dev(GM, "GM", torch.int8), n, float(lam), float(t),
                                       At.data_ptr(), sums, _stream(stream)), "glasso_trial_point")
        return At, {"dtr": sums[0], "dl1": sums[1]}


def workspace_bytes(n: int, precision: str | int = "fp64") -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = ctypes.c_size_t(0)
    _check(_lib.glasso_workspace_size(int(n), prec, ctypes.byref(out)), "glasso_workspace_size")
    return int(out.value)


def solve(S: torch.Tensor, lam: float, tol: float, **options) -> Result:
    """One-shot solve with a temporary handle."""
    s = Solver(**options)
    try:
        return s.solve(S, lam, tol)
    finally:
        s.close()
