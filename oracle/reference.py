"""Plain FP64 pISTA (graphical lasso) -- test infrastructure only.

Problem (Sec. 3.1, eqs. log_MLE and sparse_obj):
    minimise F(A) = -log det A + tr(S A) + lam * sum_{i,j} |A_ij|   over A > 0,
with the diagonal penalised.  The minimiser is unique (F is strictly convex on
the PD cone), so any correct solver reaches the same A*.

Each function follows one equation of the paper, written from the text with
full dense matrices and no blocking or fusion.  Readings of ambiguous passages
(applied identically by the GPU path):
  * eq. d_sol is elementwise: ST(A_ij - t B_ij, t C_ij), as in App. B.
  * Alg. 1 applies the masked update A + M (.) D (Sec. 4.1, eq. proximal_gen_free
    and Sec. 4.3.2); we evaluate it as M (.) ST(A - tB, tC), which is that value
    without the rounding of A + (-A + s).  Off the free set A_ij is already 0.
  * Line search: t = 1, halved until the trial is PD and F strictly decreases
    (Sec. 4.3.2).  Optionally (sigma > 0) the decrease must reach sigma times the
    decrease predicted by the linear model of f plus the l1 term,
    <g, At - A> + lam (||At||_1 - ||A||_1) (an Armijo rule); sigma = 0 is the
    paper's strict decrease.  Below t = 1e-4 the step becomes min(t, (0.9/cond(A))^2) and
    halving continues down to 1e-12, after which the search fails (Sec. 6).
  * The decrease is evaluated in difference form,
        F(At) - F(A) = 2 sum_i log(L_ii / Lt_ii) + sum S (.) (At - A)
                       + lam * sum (|At| - |A|),
    so that tiny decreases near convergence are resolved.
  * Stopping: ||Z||_1 <= tol * ||A||_1 with Z the minimum-norm subgradient (Sec. 6).
  * The two halves of each product are averaged, 1/2 (P + P^T), to keep every
    iterate exactly symmetric.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

CONVERGED = 0
MAX_ITER = 1
LS_FAILED = 2


# --------------------------------------------------------------------------- input
def empirical_covariance(Y: np.ndarray, center: bool = True) -> np.ndarray:
    """S = (1/m) sum_i (y_i - mu)(y_i - mu)^T with mu = (1/m) sum_i y_i, the samples
    y_i being the m rows of Y (Sec. 3.1, eq. empirical_cov).  center=False takes
    mu = 0, for samples whose mean is known to be zero."""
    Y = np.asarray(Y, dtype=np.float64)
    m = Y.shape[0]
    mu = Y.sum(axis=0) / m if center else np.zeros(Y.shape[1])
    Yc = Y - mu[None, :]
    return (Yc.T @ Yc) / m


# --------------------------------------------------------------------------- basics
def initial_iterate(S: np.ndarray, lam: float) -> np.ndarray:
    """A^(0) = diag(1 / (S_ii + lam)): the G-ISTA initialisation used in Sec. 6."""
    return np.diag(1.0 / (np.diag(S) + lam))


def cholesky_or_none(A: np.ndarray):
    """Lower Cholesky factor of A, or None when A is not (numerically) PD.
    The PD test of the line search (condition t_cond_pd, Sec. 4.3.2)."""
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return None
    d = np.diag(L)
    if not (np.all(np.isfinite(L)) and np.all(d > 0)):
        return None
    return L


def logdet_from_cholesky(L: np.ndarray) -> float:
    """log det A = 2 sum_i log L_ii for A = L L^T."""
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def objective(S: np.ndarray, A: np.ndarray, lam: float, L=None) -> float:
    """F(A) = -log det A + tr(SA) + lam ||A||_1 (eq. sparse_obj); +inf off the PD cone."""
    if L is None:
        L = cholesky_or_none(A)
        if L is None:
            return np.inf
    # tr(SA) = sum_ij S_ij A_ji = sum_ij S_ij A_ij for symmetric A
    return -logdet_from_cholesky(L) + float(np.sum(S * A)) + lam * float(np.sum(np.abs(A)))


def inverse_from_cholesky(L: np.ndarray) -> np.ndarray:
    """W = A^{-1} = L^{-T} L^{-1}, symmetrised."""
    n = L.shape[0]
    W = sla.cho_solve((L, True), np.eye(n))
    return 0.5 * (W + W.T)


# --------------------------------------------------------------------------- Sec. 4.1
def gradient(S: np.ndarray, W: np.ndarray) -> np.ndarray:
    """g = grad f(A) = S - A^{-1} (eq. grad_hessian)."""
    return S - W


def free_set_mask(A: np.ndarray, g: np.ndarray, lam: float) -> np.ndarray:
    """M: indicator of the free set {A_ij != 0} U {|g_ij| > lam} (eqs. free_set, M)."""
    return (A != 0) | (np.abs(g) > lam)


def sign_guess(A: np.ndarray, g: np.ndarray) -> np.ndarray:
    """G: sign(A_ij) where A_ij != 0, else -sign(g_ij) (eq. G+)."""
    return np.where(A != 0, np.sign(A), -np.sign(g))


def min_norm_subgradient(g: np.ndarray, G: np.ndarray, M: np.ndarray, lam: float) -> np.ndarray:
    """Z = (g + lam G) (.) M: G with the free-set mask gives the minimum-norm
    subgradient of F at A (closing remark of Sec. 4.3.1)."""
    return np.where(M, g + lam * G, 0.0)


def kkt_measures(Z: np.ndarray, A: np.ndarray) -> dict:
    """Stopping measure ||Z||_1 / ||A||_1 (Sec. 6) plus the Frobenius and max norms."""
    sz = float(np.sum(np.abs(Z)))
    sa = float(np.sum(np.abs(A)))
    return {"kkt_rel1": sz / sa, "kkt_fro": float(np.sqrt(np.sum(Z * Z))),
            "kkt_max": float(np.max(np.abs(Z))) if Z.size else 0.0,
            "sum_abs_z": sz, "sum_abs_a": sa}


# --------------------------------------------------------------------------- Sec. 4.3
def c_matrix(A: np.ndarray, lam: float) -> np.ndarray:
    """C_ii = lam A_ii A_ii, C_ij = lam (A_ii A_jj + A_ij A_ji) for i != j (eq. c):
    the diagonal of lam A (x) A belonging to entry (i, j)."""
    d = np.diag(A)
    C = lam * (np.outer(d, d) + A * A.T)
    idx = np.arange(A.shape[0])
    C[idx, idx] = lam * (d * d)
    return C


def preconditioned_products(A: np.ndarray, g: np.ndarray, G: np.ndarray,
                            M: np.ndarray, lam: float) -> np.ndarray:
    """A (g (.) M) A + lam A (G (.) M) A: the first two terms of eq. b, each
    product symmetrised."""
    gm = np.where(M, g, 0.0)
    Gm = np.where(M, G, 0.0)
    P1 = A @ gm @ A
    P2 = A @ Gm @ A
    return 0.5 * (P1 + P1.T) + lam * (0.5 * (P2 + P2.T))


def b_from_products(P: np.ndarray, C: np.ndarray, G: np.ndarray, M: np.ndarray) -> np.ndarray:
    """B = [A (g.M) A + lam A (G.M) A] - C (.) (G (.) M) (eq. b)."""
    Gm = np.where(M, G, 0.0)
    return P - C * Gm


def b_matrix(A, g, G, M, C, lam):
    """B of eq. b."""
    return b_from_products(preconditioned_products(A, g, G, M, lam), C, G, M)


def soft_threshold(x, tau):
    """SoftThreshold(x, tau) = sign(x) max(|x| - tau, 0): the solution operator of the
    scalar sign equation of App. A (Lemma A.1)."""
    return np.sign(x) * np.maximum(np.abs(x) - tau, 0.0)


def direction(A: np.ndarray, B: np.ndarray, C: np.ndarray, t: float) -> np.ndarray:
    """D = -A + SoftThreshold(A - t B, t C), elementwise (eq. d_sol; App. B)."""
    return -A + soft_threshold(A - t * B, t * C)


def trial_point(A: np.ndarray, M: np.ndarray, B: np.ndarray, C: np.ndarray, t: float) -> np.ndarray:
    """A + M (.) D(t), evaluated as M (.) SoftThreshold(A - tB, tC)."""
    return np.where(M, soft_threshold(A - t * B, t * C), 0.0)


def objective_change(S, A, At, L, Lt, lam) -> float:
    """F(At) - F(A) in difference form (each term differenced before summing)."""
    dlog = 2.0 * float(np.sum(np.log(np.diag(L) / np.diag(Lt))))
    dtr = float(np.sum(S * (At - A)))
    dl1 = lam * float(np.sum(np.abs(At) - np.abs(A)))
    return dlog + dtr + dl1


def predicted_change(g: np.ndarray, A: np.ndarray, At: np.ndarray, lam: float) -> float:
    """<g, At - A> + lam (||At||_1 - ||A||_1): the change of F that its linear model
    (gradient of f, exact l1 term) predicts for the step from A to At; negative for
    a descent step.  The Armijo rule accepts At when F(At) - F(A) < sigma times it."""
    return float(np.sum(g * (At - A))) + lam * float(np.sum(np.abs(At)) - np.sum(np.abs(A)))


def cond_fallback_step(A: np.ndarray, factor: float = 0.9) -> float:
    """t = (0.9 / cond(A))^2, the step assumed safe once t drops below 1e-4 (Sec. 6).
    cond(A) = lambda_max / lambda_min (2-norm condition number)."""
    ev = np.linalg.eigvalsh(A)
    return (factor / (ev[-1] / ev[0])) ** 2


# --------------------------------------------------------------------------- Alg. 1
@dataclass
class PistaResult:
    A: np.ndarray
    W: np.ndarray
    objective: float
    iterations: int
    status: int
    kkt_rel1: float
    kkt_fro: float
    kkt_max: float
    ls_trials: int
    history: list = field(default_factory=list)


def pista(S: np.ndarray, lam: float, tol: float, A0=None, max_iter: int = 500,
          t0: float = 1.0, shrink: float = 0.5, t_floor: float = 1e-4,
          t_min: float = 1e-12, sigma: float = 0.0) -> PistaResult:
    """pISTA(S, lam, A0) (Alg. 1) with the stopping rule and line search of Sec. 6;
    sigma > 0 asks each step for sigma times its predicted decrease (see
    predicted_change)."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    A = initial_iterate(S, lam) if A0 is None else np.array(A0, dtype=np.float64)
    L = cholesky_or_none(A)
    if L is None:
        raise ValueError("initial iterate is not positive definite")
    F = objective(S, A, lam, L)
    history = []
    total_trials = 0
    k = 0
    while True:
        W = inverse_from_cholesky(L)
        g = gradient(S, W)
        M = free_set_mask(A, g, lam)
        G = sign_guess(A, g)
        Z = min_norm_subgradient(g, G, M, lam)
        km = kkt_measures(Z, A)
        rec = {"F": F, "kkt_rel1": km["kkt_rel1"]}
        if km["kkt_rel1"] <= tol:
            history.append(rec)
            return PistaResult(A, W, F, k, CONVERGED, km["kkt_rel1"], km["kkt_fro"],
                               km["kkt_max"], total_trials, history)
        if k >= max_iter:
            history.append(rec)
            return PistaResult(A, W, F, k, MAX_ITER, km["kkt_rel1"], km["kkt_fro"],
                               km["kkt_max"], total_trials, history)
        C = c_matrix(A, lam)
        B = b_matrix(A, g, G, M, C, lam)
        # backtracking over t (Sec. 4.3.2, Sec. 6)
        t = t0
        fallback = False
        accepted = None
        trials = 0
        while True:
            if t < t_floor and not fallback:
                t = min(t, cond_fallback_step(A))
                fallback = True
            if t < t_min:
                break
            At = trial_point(A, M, B, C, t)
            Lt = cholesky_or_none(At)
            trials += 1
            if Lt is not None:
                dF = objective_change(S, A, At, L, Lt, lam)
                target = sigma * predicted_change(g, A, At, lam) if sigma > 0.0 else 0.0
                if dF < target:
                    accepted = (At, Lt, dF)
                    break
            t *= shrink
        total_trials += trials
        rec.update({"t": t, "trials": trials, "fallback": fallback})
        history.append(rec)
        if accepted is None:
            return PistaResult(A, W, F, k, LS_FAILED, km["kkt_rel1"], km["kkt_fro"],
                               km["kkt_max"], total_trials, history)
        rec["pred"] = predicted_change(g, A, accepted[0], lam)
        A, L, dF = accepted
        rec["dF"] = dF
        F = F + dF
        k += 1


# --------------------------------------------------------------------------- G-ISTA (Sec. 3.2)
def gista_trial_point(A: np.ndarray, g: np.ndarray, lam: float, t: float) -> np.ndarray:
    """A + D with D the minimiser of eq. proximal_gen for H = I scaled by 1/t (the
    proximal-gradient step): <g, D> + ||D||_F^2 / (2t) + lam ||A + D||_1 separates
    into scalar problems whose minimiser is SoftThreshold(A - t g, t lam)."""
    return soft_threshold(A - t * g, t * lam)


def quadratic_bound_excess(A, At, L, Lt, W, t) -> float:
    """f(At) - f(A) - <g, At - A> - ||At - A||_F^2 / (2t), f = -log det + tr(S .), in
    difference form: f(At) - f(A) - <S - W, At - A> = 2 sum_i log(L_ii / Lt_ii) +
    sum W (.) (At - A).  The proximal-gradient step is accepted when this is <= 0,
    i.e. when the quadratic model behind the step bounds f at the trial point."""
    dA = At - A
    dlog = 2.0 * float(np.sum(np.log(np.diag(L) / np.diag(Lt))))
    return dlog + float(np.sum(W * dA)) - float(np.sum(dA * dA)) / (2.0 * t)


def bb_step(dA: np.ndarray, W_old: np.ndarray, W_new: np.ndarray) -> float:
    """Barzilai-Borwein step <dA, dA> / <dA, grad f(A_new) - grad f(A_old)> with
    grad f = S - W, i.e. <dA, dA> / <dA, W_old - W_new>: the first step size G-ISTA
    tries in the next iteration.  The denominator is positive for dA != 0 (f is
    strictly convex); otherwise the caller keeps its previous step."""
    num = float(np.sum(dA * dA))
    den = float(np.sum(dA * (W_old - W_new)))
    return num / den if den > 0.0 and num > 0.0 else np.nan


def gista(S: np.ndarray, lam: float, tol: float, A0=None, max_iter: int = 5000,
          t0: float = 1.0, shrink: float = 0.5, t_min: float = 1e-12) -> PistaResult:
    """G-ISTA: proximal gradient descent on F, the H = I case of eq. proximal_gen
    (Sec. 3.2), the paper's first-order comparison method (Sec. 6).  Same start
    (Sec. 6), same stopping rule and measures as pista.  Step sizes follow the
    G-ISTA authors' recommendation: the first trial of an iteration takes the
    Barzilai-Borwein step of the previous accepted step (t0 in the first
    iteration), and backtracking multiplies t by `shrink` until the trial point is
    PD and quadratic_bound_excess <= 0; the search fails below t_min, or when the
    trial point no longer differs from A (rounding has swallowed the step)."""
    S = np.asarray(S, dtype=np.float64)
    A = initial_iterate(S, lam) if A0 is None else np.array(A0, dtype=np.float64)
    L = cholesky_or_none(A)
    if L is None:
        raise ValueError("initial iterate is not positive definite")
    F = objective(S, A, lam, L)
    history = []
    total_trials = 0
    k = 0
    t_next = t0
    W_prev = dA_prev = None
    while True:
        W = inverse_from_cholesky(L)
        if dA_prev is not None:
            bb = bb_step(dA_prev, W_prev, W)
            if np.isfinite(bb):
                t_next = bb
        g = gradient(S, W)
        M = free_set_mask(A, g, lam)
        G = sign_guess(A, g)
        Z = min_norm_subgradient(g, G, M, lam)
        km = kkt_measures(Z, A)
        rec = {"F": F, "kkt_rel1": km["kkt_rel1"]}
        if km["kkt_rel1"] <= tol or k >= max_iter:
            history.append(rec)
            status = CONVERGED if km["kkt_rel1"] <= tol else MAX_ITER
            return PistaResult(A, W, F, k, status, km["kkt_rel1"], km["kkt_fro"],
                               km["kkt_max"], total_trials, history)
        t = t_next
        accepted = None
        trials = 0
        while t >= t_min:
            At = gista_trial_point(A, g, lam, t)
            if np.array_equal(At, A):
                break  # the step has shrunk below the resolution of A: no progress left
            Lt = cholesky_or_none(At)
            trials += 1
            if Lt is not None and quadratic_bound_excess(A, At, L, Lt, W, t) <= 0.0:
                accepted = (At, Lt)
                break
            t *= shrink
        total_trials += trials
        rec.update({"t": t, "trials": trials})
        history.append(rec)
        if accepted is None:
            return PistaResult(A, W, F, k, LS_FAILED, km["kkt_rel1"], km["kkt_fro"],
                               km["kkt_max"], total_trials, history)
        At, Lt = accepted
        dF = objective_change(S, A, At, L, Lt, lam)
        rec["dF"] = dF
        W_prev, dA_prev = W, At - A
        A, L = At, Lt
        F = F + dF
        t_next = t
        k += 1


# --------------------------------------------------------------------------- certificate
def check_solution(S: np.ndarray, A: np.ndarray, lam: float) -> dict:
    """Optimality measures of any candidate A, independent of how it was found:
    PD test, F(A), and the KKT residual of its minimum-norm subgradient."""
    A = np.asarray(A, dtype=np.float64)
    L = cholesky_or_none(A)
    if L is None:
        return {"pd": False}
    W = inverse_from_cholesky(L)
    g = gradient(S, W)
    M = free_set_mask(A, g, lam)
    G = sign_guess(A, g)
    Z = min_norm_subgradient(g, G, M, lam)
    out = kkt_measures(Z, A)
    out.update({"pd": True, "objective": objective(S, A, lam, L), "W": W, "g": g,
                "nnz": int(np.count_nonzero(A))})
    return out
