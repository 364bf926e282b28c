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
PISTA, GISTA = 0, 1  # glasso_method
METHODS = {"pista": PISTA, "gista": GISTA}
TILES_AUTO = -1  # tile policy chosen by the autotuner (GLASSO_TILES_AUTO)
SMALL_MAX_N = 64  # largest n of glasso_solve_small (GLASSO_SMALL_MAX_N)
SMALL_STATIC_MAX_COUNT = 16384  # problems per glasso_solve_small_static call
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
    aza_gemm_products: int = 0
    aza_sparse_products: int = 0
    leaf_launches: int = 0
    leaf_ms: float = 0.0
    leaf_flops: float = 0.0
    components: int = 1
    largest_component: int = 0

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


class Solver:
    """A libglasso handle: options plus a cached device workspace."""

    def __init__(self, precision: str | int = "fp64", max_iter: int = 500, t0: float = 1.0,
                 shrink: float = 0.5, t_floor: float = 1e-4, t_min: float = 1e-12,
                 warm_start: bool = False, tile_policy: int = TILES_AUTO, graphs: bool = False,
                 w_mixed: int = -1, ls_width: int = 0, dense_product: bool = False, screen: bool = False,
                 sigma: float = 0.0, method: str | int = "pista"):
        opt = GlassoOptions()
        _check(_lib.glasso_default_options(ctypes.byref(opt)), "glasso_default_options")
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.max_iter = int(max_iter)
        opt.t0 = float(t0)
        opt.shrink = float(shrink)
        opt.t_floor = float(t_floor)
        opt.t_min = float(t_min)
        opt.warm_start = int(bool(warm_start))
        opt.tile_policy = int(tile_policy)
        opt.graphs = int(bool(graphs))
        opt.w_mixed = int(w_mixed)
        opt.ls_width = int(ls_width)
        opt.dense_product = int(bool(dense_product))
        opt.screen = int(bool(screen))
        opt.sigma = float(sigma)
        opt.method = METHODS[method] if isinstance(method, str) else int(method)
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

    def autotune(self, n: int, count: int = 1, stream=None) -> int:
        """Measure and record the GEMM tile policy for problems of size n solved
        `count` at a time (glasso_autotune); returns the chosen threshold."""
        pol = ctypes.c_int()
        _check(_lib.glasso_autotune(self._h, int(n), int(count), ctypes.byref(pol), _stream(stream)),
               "glasso_autotune")
        return pol.value

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
                      info.fallback_steps, tuple(info.time_ms), info.aza_gemm_products,
                      info.aza_sparse_products, info.leaf_launches, info.leaf_ms, info.leaf_flops,
                      info.components, info.largest_component)

    def solve_batched(self, S_list, lams, tol: float, A_list=None, want_W: bool = True, stream=None):
        """Solve len(lams) problems in batched launches (glasso_solve_batched).
        S_list: one tensor per problem (the same tensor may repeat) or a single
        tensor shared by all.  With a warm_start solver, A_list holds the starting
        iterates.  Returns one Result per problem."""
        return self._multi("glasso_solve_batched", S_list, lams, tol, A_list, want_W, stream)

    def solve_small(self, S_list, lams, tol: float, A_list=None, want_W: bool = True, stream=None):
        """Solve many problems of n <= SMALL_MAX_N in one persistent launch
        (glasso_solve_small; every step FP64, no host round trip).  Arguments and
        results as for solve_batched."""
        return self._multi("glasso_solve_small", S_list, lams, tol, A_list, want_W, stream)

    def solve_small_static(self, S_list, lams, tol: float, A_list=None, want_W: bool = True, stream=None):
        """solve_small through the entry point that allocates nothing
        (glasso_solve_small_static: scratch in the library's fixed device array,
        this solver's options, no handle).  Arguments and results as solve_small."""
        return self._multi("glasso_solve_small_static", S_list, lams, tol, A_list, want_W, stream)

    def _multi(self, entry, S_list, lams, tol, A_list, want_W, stream):
        lams = [float(x) for x in lams]
        count = len(lams)
        if isinstance(S_list, torch.Tensor):
            S_list = [S_list] * count
        if len(S_list) != count:
            raise ValueError("one S per lambda")
        ns = [_square(S, "S") for S in S_list]
        for S in S_list:
            _dev(S, "S")
        if A_list is None:
            if self.options.warm_start:
                raise ValueError("warm_start solver needs A_list")
            A_list = [torch.empty_like(S) for S in S_list]
        for A, n in zip(A_list, ns):
            if tuple(A.shape) != (n, n):
                raise ValueError("A_list entries must match S")
            _dev(A, "A")
        W_list = [torch.empty_like(S) for S in S_list] if want_W else None
        VP = ctypes.c_void_p
        Sp = (VP * count)(*[S.data_ptr() for S in S_list])
        Ap = (VP * count)(*[A.data_ptr() for A in A_list])
        Wp = (VP * count)(*[W.data_ptr() for W in W_list]) if want_W else None
        nn = (ctypes.c_int64 * count)(*ns)
        ll = (ctypes.c_double * count)(*lams)
        infos = (GlassoInfo * count)()
        first = ctypes.byref(self.options) if entry == "glasso_solve_small_static" else self._h
        _check(getattr(_lib, entry)(first, count, Sp, nn, ll, float(tol), Ap, Wp, infos, _stream(stream)), entry)
        out = []
        for i in range(count):
            inf = infos[i]
            out.append(Result(A_list[i], W_list[i] if want_W else None, inf.objective, inf.iterations,
                              inf.status, inf.kkt_rel1, inf.kkt_fro, inf.kkt_max, int(inf.nnz),
                              inf.ls_trials, inf.fallback_steps, tuple(inf.time_ms), inf.aza_gemm_products,
                              inf.aza_sparse_products, inf.leaf_launches, inf.leaf_ms, inf.leaf_flops,
                              inf.components, inf.largest_component))
        return out

    # ---------------------------------------------------------------- workloads
    def generate(self, kind: str, n: int, m: int = 0, seed: int = 0, want_A: bool = False, want_Y: bool = False,
                 want_S: bool = True, device=None, stream=None):
        """Seeded synthetic workload on the device (glasso_generate): kind "random"
        (random sparse precision) or "chain".  Returns (A_true, Y, S, lambda_max),
        the tensors not asked for as None; lambda_max = max_{i != j} |S_ij| when
        samples are drawn."""
        dev = device or torch.device("cuda", torch.cuda.current_device())
        k = {"random": 0, "chain": 1}[kind]
        A = torch.empty((n, n), dtype=torch.float64, device=dev) if want_A else None
        Y = torch.empty((m, n), dtype=torch.float64, device=dev) if want_Y else None
        S = torch.empty((n, n), dtype=torch.float64, device=dev) if want_S else None
        lm = ctypes.c_double(float("nan"))
        samples = want_Y or want_S or m > 0
        _check(_lib.glasso_generate(self._h, k, int(n), int(m), int(seed) & (2**64 - 1),
                                    A.data_ptr() if A is not None else None,
                                    Y.data_ptr() if Y is not None else None,
                                    S.data_ptr() if S is not None else None,
                                    ctypes.byref(lm) if samples else None, _stream(stream)), "glasso_generate")
        return A, Y, S, (lm.value if samples else None)

    # ---------------------------------------------------------------- single steps
    def covariance(self, Y: torch.Tensor, center: bool = True, stream=None) -> torch.Tensor:
        """Sample covariance of the rows of Y (m x n, device FP64), eq. empirical_cov."""
        if Y.dim() != 2:
            raise ValueError(f"Y must be m x n, got {tuple(Y.shape)}")
        m, n = Y.shape
        S = torch.empty((n, n), dtype=torch.float64, device=Y.device)
        _check(_lib.glasso_covariance(self._h, _dev(Y, "Y"), m, n, int(bool(center)), S.data_ptr(),
                                      _stream(stream)), "glasso_covariance")
        return S

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

    def sparse_product(self, A, Z, GM, stream=None):
        """(A Z A) on the free set (GM != 0), zero elsewhere, FP64 (glasso_sparse_product).
        Returns (P, used_sparse)."""
        n = _square(A, "A")
        P = torch.empty_like(A)
        used = ctypes.c_int(0)
        _check(_lib.glasso_sparse_product(self._h, _dev(A, "A"), _dev(Z, "Z"), _dev(GM, "GM", torch.int8), n,
                                          P.data_ptr(), ctypes.byref(used), _stream(stream)),
               "glasso_sparse_product")
        return P, bool(used.value)

    def gista_trial_point(self, A, S, W, GM, lam: float, t: float, stream=None):
        """G-ISTA trial point ST(A - t (S - W), t lam) on the free set
        (glasso_gista_trial_point); returns (At, sums[4])."""
        n = _square(A, "A")
        for name, x in (("S", S), ("W", W)):
            if tuple(x.shape) != (n, n):
                raise ValueError(f"{name} must be n x n")
        At = torch.empty_like(A)
        sums = (ctypes.c_double * 4)()
        _check(_lib.glasso_gista_trial_point(self._h, _dev(A, "A"), _dev(S, "S"), _dev(W, "W"),
                                             _dev(GM, "GM", torch.int8), n, float(lam), float(t), At.data_ptr(),
                                             sums, _stream(stream)), "glasso_gista_trial_point")
        return At, list(sums)

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


def lambda_path(S: torch.Tensor, lams, tol: float, mode: str = "waves", waves: int = 4,
                precision: str | int = "fp64", want_W: bool = False, **options):
    """Regularisation path: solutions for every lambda in `lams` (any order).

    mode "independent": all lambdas in one batched solve from the diagonal start;
    mode "sequential":  one solve per lambda in decreasing order, each warm-started
                        from the previous solution;
    mode "waves":       lambdas in decreasing order split into `waves` consecutive
                        groups; each group is one batched solve warm-started from the
                        solution of the smallest lambda of the previous group (the
                        first group starts from the diagonal).
    The minimiser of each problem is unique, so every mode returns the same
    solutions up to the stopping tolerance.  Returns Results in the order of `lams`."""
    lams = [float(x) for x in lams]
    order = sorted(range(len(lams)), key=lambda i: -lams[i])
    results = [None] * len(lams)
    cold = Solver(precision=precision, **options)
    warm = Solver(precision=precision, warm_start=True, **options)
    try:
        if mode == "independent":
            rs = cold.solve_batched(S, lams, tol, want_W=want_W)
            return rs
        if mode == "sequential":
            prev = None
            for i in order:
                if prev is None:
                    r = cold.solve(S, lams[i], tol, want_W=want_W)
                else:
                    r = warm.solve(S, lams[i], tol, A=prev.A.clone(), want_W=want_W)
                results[i] = r
                prev = r
            return results
        if mode == "waves":
            size = -(-len(order) // max(1, waves))
            groups = [order[k:k + size] for k in range(0, len(order), size)]
            prev = None
            for grp in groups:
                gl = [lams[i] for i in grp]
                if prev is None:
                    rs = cold.solve_batched(S, gl, tol, want_W=want_W)
                else:
                    rs = warm.solve_batched(S, gl, tol, A_list=[prev.A.clone() for _ in grp], want_W=want_W)
                for i, r in zip(grp, rs):
                    results[i] = r
                prev = rs[-1]  # smallest lambda of this wave
            return results
        raise ValueError(f"unknown mode {mode!r}")
    finally:
        cold.close()
        warm.close()
