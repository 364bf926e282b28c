"""Checks that pin the oracle to the mathematics, not to itself.

Each check is a function of an oracle module so the mutation tests can run the
same checks against deliberately broken copies of the oracle.  None of them
retypes the oracle's formulas: they use closed forms, optimality conditions
written directly on W = inv(A) (computed here with numpy.linalg.inv), an
independent proximal-gradient solver, and brute-force search.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- independent pieces
def st(x, tau):
    return np.sign(x) * np.maximum(np.abs(x) - tau, 0.0)


def f_direct(S, A, lam):
    """F(A) via slogdet (not the oracle's Cholesky path)."""
    sign, ld = np.linalg.slogdet(A)
    if sign <= 0:
        return np.inf
    return -ld + np.trace(S @ A) + lam * np.abs(A).sum()


def kkt_violation(S, A, lam):
    """Largest violation of the GLASSO optimality conditions, written on
    W = inv(A): W_ii = S_ii + lam; W_ij - S_ij = lam sign(A_ij) where A_ij != 0;
    |W_ij - S_ij| <= lam where A_ij == 0."""
    W = np.linalg.inv(A)
    W = 0.5 * (W + W.T)
    R = W - S
    n = A.shape[0]
    viol = 0.0
    for i in range(n):
        for j in range(n):
            if A[i, j] != 0:
                viol = max(viol, abs(R[i, j] - lam * np.sign(A[i, j])))
            else:
                viol = max(viol, max(0.0, abs(R[i, j]) - lam))
    return viol


def gista(S, lam, tol=1e-12, max_iter=20000):
    """Proximal gradient (G-ISTA, H = I in eq. proximal_gen) with the classical safe
    step t = 0.9 lambda_min(A)^2 (inverse Lipschitz constant of grad f near A),
    halved while the step leaves the PD cone or fails to decrease F.  Independent
    of the oracle's code."""
    A = np.diag(1.0 / (np.diag(S) + lam))
    F = f_direct(S, A, lam)
    for _ in range(max_iter):
        W = np.linalg.inv(A)
        g = S - W
        t = 0.9 * np.linalg.eigvalsh(A)[0] ** 2
        while True:
            An = st(A - t * g, t * lam)
            An = 0.5 * (An + An.T)
            Fn = f_direct(S, An, lam)
            if np.isfinite(Fn) and Fn <= F + 1e-14 * abs(F):
                break
            t *= 0.5
        D = An - A
        A, F = An, Fn
        if np.abs(D).max() < tol:
            break
    return A


def n2_closed_form(S, lam):
    """n = 2: W* = [[S11+lam, ST(S12, lam)], [ST(S12, lam), S22+lam]], A* = inv(W*)."""
    w12 = st(S[0, 1], lam)
    W = np.array([[S[0, 0] + lam, w12], [w12, S[1, 1] + lam]])
    return np.linalg.inv(W)


def random_psd(n, m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, m))
    S = X @ X.T / m
    return 0.5 * (S + S.T)


# ----------------------------------------------------------------- pin checks
def check_scalar_lemma(orc, trials=200, seed=0):
    """App. A lemma: D = -A + ST(A - tB, tC) solves x/t + B + C T(A + x) = 0 and
    minimises x^2/(2t) + Bx + C|A + x| (brute force on a fine grid)."""
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        a, b = rng.normal(scale=2.0, size=2)
        c = rng.uniform(0.01, 2.0)
        t = rng.uniform(0.05, 2.0)
        x = float(orc.direction(np.array([[a]]), np.array([[b]]), np.array([[c]]), t)[0, 0])
        grid = np.linspace(x - 3.0, x + 3.0, 60001)
        h = grid ** 2 / (2 * t) + b * grid + c * np.abs(a + grid)
        hx = x ** 2 / (2 * t) + b * x + c * abs(a + x)
        if hx > h.min() + 1e-9:
            return False
        if abs(grid[np.argmin(h)] - x) > 2e-4:
            return False
    return True


def check_n2_closed_form(orc, seeds=range(6), lams=(0.05, 0.2, 0.6)):
    for seed in seeds:
        S = random_psd(2, 3, seed)
        for lam in lams:
            r = orc.pista(S, lam, 1e-12, max_iter=2000)
            A_ref = n2_closed_form(S, lam)
            if not np.allclose(r.A, A_ref, rtol=1e-8, atol=1e-10):
                return False
    return True


def check_kkt_invariants(orc, n=20, seed=3, lam=0.15, tol=1e-9):
    S = random_psd(n, n // 2, seed)
    r = orc.pista(S, lam, tol, max_iter=3000)
    if r.status != orc.CONVERGED:
        return False
    if kkt_violation(S, r.A, lam) > 1e-6:
        return False
    gap = np.trace(S @ r.A) + lam * np.abs(r.A).sum() - n
    return abs(gap) < 1e-6 * n


def check_against_gista(orc, n=12, seed=5, lam=0.1):
    S = random_psd(n, n, seed)
    r = orc.pista(S, lam, 1e-10, max_iter=3000)
    A_g = gista(S, lam)
    return np.allclose(r.A, A_g, rtol=1e-6, atol=1e-8)


def check_diagonal_solution(orc, n=15, seed=7):
    S = random_psd(n, 3 * n, seed)
    lam = np.abs(S - np.diag(np.diag(S))).max() * 1.01
    r = orc.pista(S, lam, 1e-12)
    A_ref = np.diag(1.0 / (np.diag(S) + lam))
    return r.iterations == 0 and np.allclose(r.A, A_ref, rtol=1e-14, atol=0)


def check_cond_fallback(orc, seeds=range(4)):
    """The line-search fallback step of the Sec. 6 settings, t = (0.9 / cond A)^2,
    pinned to the mathematics rather than to its own formula:
      * closed forms: diag(1, 4) has cond 4, so t = (0.9/4)^2; any multiple of
        the identity has cond 1, so t = 0.81;
      * it lies below (beta/gamma)^2 with beta, gamma the extreme singular values of
        A from an SVD (the step bound of the decrease lemma, Sec. 5.2), by the factor
        0.81 exactly;
      * taken from a real iterate of a solve, the trial point at that t is PD and
        lowers F (the property the paper assumes of this step)."""
    t = orc.cond_fallback_step(np.diag([1.0, 4.0]))
    if abs(t - (0.9 / 4.0) ** 2) > 1e-15:
        return False
    if abs(orc.cond_fallback_step(3.0 * np.eye(5)) - 0.81) > 1e-14:
        return False
    for seed in seeds:
        rng = np.random.default_rng(100 + seed)
        X = rng.normal(size=(7, 7))
        A = X @ X.T + 0.05 * np.eye(7)
        sv = np.linalg.svd(A, compute_uv=False)
        bound = (sv[-1] / sv[0]) ** 2
        t = orc.cond_fallback_step(A)
        if not (0.0 < t < bound) or abs(t / bound - 0.81) > 1e-8:
            return False
    for seed in seeds:
        S = random_psd(12, 6, 40 + seed)
        lam = 0.1
        A = np.diag(1.0 / (np.diag(S) + lam))
        for _ in range(3):  # a few plain pISTA iterations give a non-diagonal iterate
            A = orc.pista(S, lam, 0.0, A0=A, max_iter=1).A
        g = orc.gradient(S, np.linalg.inv(A))
        M = orc.free_set_mask(A, g, lam)
        G = orc.sign_guess(A, g)
        C = orc.c_matrix(A, lam)
        B = orc.b_matrix(A, g, G, M, C, lam)
        t = orc.cond_fallback_step(A)
        At = orc.trial_point(A, M, B, C, t)
        if np.linalg.eigvalsh(At)[0] <= 0:
            return False
        if not f_direct(S, At, lam) < f_direct(S, A, lam):
            return False
    return True


def check_armijo(orc, seed=9):
    """The sufficient-decrease variant of the line search (sigma > 0):
      * predicted_change is the first-order change of F: for a step eps E that
        keeps every sign, F(A + eps E) - F(A) minus the prediction shrinks like
        eps^2 (F from slogdet, independent of the oracle);
      * an Armijo solve reaches the minimiser of the plain solve, and every step it
        accepts decreased F by at least sigma times its (negative) prediction."""
    rng = np.random.default_rng(seed)
    S = random_psd(10, 6, seed)
    lam = 0.1
    A = orc.pista(S, lam, 0.0, max_iter=3).A
    g = S - np.linalg.inv(A)
    E = rng.standard_normal(A.shape)
    E = 0.5 * (E + E.T) * (A != 0)
    errs = []
    for eps in (1e-3, 1e-4):
        At = A + eps * E
        if np.any(np.sign(At) != np.sign(A)):
            return False
        errs.append(abs(f_direct(S, At, lam) - f_direct(S, A, lam) - orc.predicted_change(g, A, At, lam)))
    if not errs[1] < 0.02 * errs[0] + 1e-13:
        return False
    ref = orc.pista(S, lam, 1e-7, max_iter=3000)
    r = orc.pista(S, lam, 1e-7, max_iter=3000, sigma=0.3)
    if r.status != orc.CONVERGED or abs(r.objective - ref.objective) > 1e-10 * abs(ref.objective):
        return False
    if not np.array_equal(r.A != 0, ref.A != 0):
        return False
    steps = [h for h in r.history if "dF" in h]
    return all(h["pred"] < 0 and h["dF"] < 0.3 * h["pred"] for h in steps)


def check_gista(orc, seed=11):
    """G-ISTA (H = I in eq. proximal_gen) pinned to the mathematics:
      * its step minimises <g, D> + D^2/(2t) + lam |A + D| entry by entry (brute
        force on a fine grid);
      * the minimiser is a fixed point of the step for any t (gradient from
        numpy.linalg.inv of an independently certified A*);
      * the Barzilai-Borwein step of two multiples of the identity, a I -> b I, is
        a b (closed form);
      * quadratic_bound_excess equals f(At) - f(A) - <grad f(A), At - A> -
        ||At - A||^2/(2t) with f from slogdet and the gradient from inv;
      * a solve reaches the minimiser of the independent proximal-gradient solver
        (KKT conditions checked on inv(A)), the n = 2 closed form and the
        closed-form diagonal solution (0 iterations), decreasing F at every step."""
    rng = np.random.default_rng(seed)
    for _ in range(40):
        a, g = rng.normal(scale=2.0, size=2)
        lam = rng.uniform(0.01, 1.5)
        t = rng.uniform(0.05, 2.0)
        x = float(orc.gista_trial_point(np.array([[a]]), np.array([[g]]), lam, t)[0, 0])
        grid = np.linspace(x - 3.0, x + 3.0, 60001)
        h = g * (grid - a) + (grid - a) ** 2 / (2 * t) + lam * np.abs(grid)
        hx = g * (x - a) + (x - a) ** 2 / (2 * t) + lam * abs(x)
        if hx > h.min() + 1e-9 or abs(grid[np.argmin(h)] - x) > 2e-4:
            return False
    S = random_psd(10, 6, seed)
    lam = 0.12
    A_ind = gista(S, lam)
    if kkt_violation(S, A_ind, lam) > 1e-7:
        return False
    W_ind = np.linalg.inv(A_ind)
    for t in (0.05, 0.4, 1.0):
        if np.abs(orc.gista_trial_point(A_ind, S - W_ind, lam, t) - A_ind).max() > 1e-7:
            return False
    for a, b in ((0.5, 0.8), (2.0, 1.25)):
        n = 4
        bb = orc.bb_step((b - a) * np.eye(n), np.eye(n) / a, np.eye(n) / b)
        if abs(bb - a * b) > 1e-12 * a * b:
            return False
    X = rng.normal(size=(6, 6))
    A = X @ X.T + 0.5 * np.eye(6)
    E = rng.normal(size=(6, 6))
    At = A + 0.05 * (E + E.T)
    S6 = random_psd(6, 9, seed + 1)
    for t in (0.01, 0.3):
        d = At - A
        direct = (f_direct(S6, At, 0.0) - f_direct(S6, A, 0.0) - np.sum((S6 - np.linalg.inv(A)) * d)
                  - np.sum(d * d) / (2 * t))
        got = orc.quadratic_bound_excess(A, At, np.linalg.cholesky(A), np.linalg.cholesky(At),
                                         np.linalg.inv(A), t)
        if abs(got - direct) > 1e-9 * (1.0 + abs(direct)):
            return False
    r = orc.gista(S, lam, 1e-8, max_iter=20000)
    if r.status != orc.CONVERGED or np.abs(r.A - A_ind).max() > 1e-6:
        return False
    if abs(f_direct(S, r.A, lam) - f_direct(S, A_ind, lam)) > 1e-9 * abs(f_direct(S, A_ind, lam)):
        return False
    if not all(h["dF"] < 0 for h in r.history if "dF" in h):
        return False
    S2 = random_psd(2, 3, seed)
    r2 = orc.gista(S2, 0.2, 1e-10, max_iter=20000)
    if not np.allclose(r2.A, n2_closed_form(S2, 0.2), rtol=1e-7, atol=1e-9):
        return False
    Sd = random_psd(8, 24, seed + 2)
    lam_d = np.abs(Sd - np.diag(np.diag(Sd))).max() * 1.01
    rd = orc.gista(Sd, lam_d, 1e-12)
    return rd.iterations == 0 and np.allclose(rd.A, np.diag(1.0 / (np.diag(Sd) + lam_d)), rtol=1e-14, atol=0)


def all_pins(orc):
    return {
        "armijo": check_armijo(orc),
        "cond_fallback": check_cond_fallback(orc),
        "scalar_lemma": check_scalar_lemma(orc, trials=40),
        "n2_closed_form": check_n2_closed_form(orc, seeds=range(3)),
        "kkt_invariants": check_kkt_invariants(orc),
        "against_gista": check_against_gista(orc),
        "diagonal": check_diagonal_solution(orc),
        "gista": check_gista(orc),
    }
