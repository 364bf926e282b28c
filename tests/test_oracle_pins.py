"""Pins for the CPU oracle: closed forms, optimality conditions, an independent
solver, brute force, equivariances and mutation tests (all CPU, no GPU)."""
import types

import numpy as np
import pytest

import oracle
import oracle.reference as opista
import synth
from tests import pins


# ------------------------------------------------------------------ App. A lemma
def test_scalar_lemma_bruteforce():
    assert pins.check_scalar_lemma(oracle, trials=200)


def test_soft_threshold_edges():
    x = np.array([-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0])
    out = oracle.soft_threshold(x, 1.0)
    np.testing.assert_array_equal(out, [-1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0])
    # the tie |x| = tau gives an exact zero (needed for exact support tests)
    assert oracle.soft_threshold(np.array([0.3]), 0.3)[0] == 0.0


# ------------------------------------------------------------------ eq. empirical_cov
def test_empirical_covariance_worked_example():
    """Three samples on a line: mu = (3, 6), centred rows (-2, -4), (0, 0), (2, 4),
    so S = (1/3) [[8, 16], [16, 32]]; without centring S = (1/3) Y^T Y by hand."""
    Y = np.array([[1.0, 2.0], [3.0, 6.0], [5.0, 10.0]])
    np.testing.assert_allclose(oracle.empirical_covariance(Y), np.array([[8.0, 16.0], [16.0, 32.0]]) / 3,
                               rtol=1e-15)
    np.testing.assert_allclose(oracle.empirical_covariance(Y, center=False),
                               np.array([[35.0, 70.0], [70.0, 140.0]]) / 3, rtol=1e-15)


def test_empirical_covariance_library_and_invariants():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((40, 7)) @ rng.standard_normal((7, 7)) + 3.0
    S = oracle.empirical_covariance(Y)
    # the library's biased (1/m) sample covariance
    np.testing.assert_allclose(S, np.cov(Y, rowvar=False, bias=True), rtol=1e-12, atol=1e-12)
    # centring removes any common shift of the samples; S is symmetric PSD
    np.testing.assert_allclose(oracle.empirical_covariance(Y + rng.standard_normal(7)[None, :]), S,
                               rtol=1e-10, atol=1e-10)
    assert np.array_equal(S, S.T) and np.linalg.eigvalsh(S).min() > -1e-12
    # samples of exactly zero mean (each with its negation): both forms agree
    Z = np.vstack([Y - Y.mean(axis=0), -(Y - Y.mean(axis=0))])
    np.testing.assert_allclose(oracle.empirical_covariance(Z), oracle.empirical_covariance(Z, center=False),
                               rtol=1e-12, atol=1e-12)
    # one sample: zero covariance once centred
    assert np.all(oracle.empirical_covariance(Y[:1]) == 0.0)


# ------------------------------------------------------------------ closed forms
def test_n1_closed_form():
    for s, lam in [(0.5, 0.1), (2.0, 0.7), (1e-3, 1.0)]:
        S = np.array([[s]])
        r = oracle.pista(S, lam, 1e-12)
        assert r.iterations == 0
        assert r.A[0, 0] == 1.0 / (s + lam)


def test_n2_closed_form():
    assert pins.check_n2_closed_form(oracle, seeds=range(8), lams=(0.02, 0.1, 0.3, 0.9))


def test_n2_grid_search():
    """Brute force over the three free entries (a, b, c) of a 2x2 PD matrix."""
    S = pins.random_psd(2, 4, 11)
    lam = 0.1
    r = oracle.pista(S, lam, 1e-12, max_iter=2000)
    a0, b0, c0 = r.A[0, 0], r.A[0, 1], r.A[1, 1]
    h = 0.02 * max(abs(a0), abs(c0))
    a = a0 + np.linspace(-10 * h, 10 * h, 41)
    b = b0 + np.linspace(-10 * h, 10 * h, 41)
    c = c0 + np.linspace(-10 * h, 10 * h, 41)
    AA, BB, CC = np.meshgrid(a, b, c, indexing="ij")
    det = AA * CC - BB * BB
    ok = (AA > 0) & (det > 0)
    F = np.full(AA.shape, np.inf)
    F[ok] = (-np.log(det[ok]) + S[0, 0] * AA[ok] + 2 * S[0, 1] * BB[ok] + S[1, 1] * CC[ok]
             + lam * (np.abs(AA[ok]) + 2 * np.abs(BB[ok]) + np.abs(CC[ok])))
    idx = np.unravel_index(np.argmin(F), F.shape)
    assert F.min() >= r.objective - 1e-12
    assert abs(AA[idx] - a0) <= h and abs(BB[idx] - b0) <= h and abs(CC[idx] - c0) <= h


def test_diagonal_closed_form():
    """lam >= max_{i!=j}|S_ij| => A* = diag(1/(S_ii + lam)), reached in 0 iterations."""
    assert pins.check_diagonal_solution(oracle)
    S, _ = synth.chain_problem(40, 20, 0)
    lam = synth.lambda_max(S)
    r = oracle.pista(S, lam, 1e-12)
    assert r.iterations == 0 and r.kkt_rel1 < 1e-14


# ------------------------------------------------------------------ optimality
def test_kkt_invariants_random():
    assert pins.check_kkt_invariants(oracle)


def test_kkt_invariants_chain_config0():
    S, _ = synth.chain_problem(100, 50, 0)
    lam = 0.2
    r = oracle.pista(S, lam, 1e-8)
    assert r.status == oracle.CONVERGED
    assert pins.kkt_violation(S, r.A, lam) < 1e-6
    W = np.linalg.inv(r.A)
    np.testing.assert_allclose(np.diag(W), np.diag(S) + lam, rtol=0, atol=1e-6)
    gap = np.trace(S @ r.A) + lam * np.abs(r.A).sum() - 100
    assert abs(gap) < 1e-5
    # F* = n - logdet A* at the optimum
    assert abs(r.objective - (100 - np.linalg.slogdet(r.A)[1])) < 1e-5


def test_against_independent_gista():
    assert pins.check_against_gista(oracle)
    S = pins.random_psd(10, 30, 2)
    r = oracle.pista(S, 0.1, 1e-10, max_iter=3000)
    np.testing.assert_allclose(r.A, pins.gista(S, 0.1), rtol=1e-6, atol=1e-8)


def test_min_norm_subgradient_bruteforce():
    """Z = (g + lam G) (.) M is the smallest element of the subdifferential of F."""
    rng = np.random.default_rng(1)
    n, lam = 6, 0.3
    A = rng.normal(size=(n, n))
    A[rng.random((n, n)) < 0.5] = 0.0
    g = rng.normal(scale=0.5, size=(n, n))
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    Z = oracle.min_norm_subgradient(g, G, M, lam)
    grid = np.linspace(-1, 1, 20001)
    for i in range(n):
        for j in range(n):
            if A[i, j] != 0:
                best = g[i, j] + lam * np.sign(A[i, j])
            else:
                vals = g[i, j] + lam * grid
                best = vals[np.argmin(np.abs(vals))]
            assert abs(Z[i, j] - best) < 1e-4 * lam


def test_c_matrix_is_coefficient_of_own_sign():
    """eq. c: C_ij is the coefficient that multiplies G_ij (and G_ji) in
    lam [A (G (.) M) A]_ij, i.e. removing entries (i,j),(j,i) of G (App. B,
    eq. G_comp) lowers lam [A G A]_ij by exactly C_ij G_ij."""
    rng = np.random.default_rng(4)
    n, lam = 7, 0.37
    X = rng.normal(size=(n, n))
    A = X @ X.T + n * np.eye(n)
    G = np.sign(rng.normal(size=(n, n)))
    G = np.triu(G) + np.triu(G, 1).T
    C = oracle.c_matrix(A, lam)
    full = lam * (A @ G @ A)
    for i in range(n):
        for j in range(n):
            Gm = G.copy()
            Gm[i, j] = 0.0
            Gm[j, i] = 0.0
            reduced = lam * (A @ Gm @ A)
            assert abs(full[i, j] - reduced[i, j] - C[i, j] * G[i, j]) < 1e-10


def test_b_matrix_via_kronecker():
    """vec(A X A) = (A (x) A) vec(X): the preconditioner of eq. D_hess applied to the
    masked gradient and sign terms of eq. b, computed through np.kron."""
    rng = np.random.default_rng(6)
    n, lam = 5, 0.2
    X = rng.normal(size=(n, n))
    A = X @ X.T + n * np.eye(n)
    A[np.abs(A) < 0.8] = 0.0
    A = np.triu(A) + np.triu(A, 1).T
    g = rng.normal(size=(n, n))
    g = 0.5 * (g + g.T)
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    C = oracle.c_matrix(A, lam)
    B = oracle.b_matrix(A, g, G, M, C, lam)
    K = np.kron(A, A)
    vec = lambda Y: Y.reshape(-1, order="F")
    unvec = lambda v: v.reshape(n, n, order="F")
    ref = unvec(K @ vec(g * M)) + lam * unvec(K @ vec(G * M)) - C * (G * M)
    np.testing.assert_allclose(B, ref, rtol=1e-12, atol=1e-12)


def test_trial_point_equals_masked_update():
    """M (.) ST(A - tB, tC) equals A + M (.) D of Alg. 1 up to rounding of A + (-A + s)."""
    rng = np.random.default_rng(8)
    n, lam, t = 8, 0.25, 0.5
    X = rng.normal(size=(n, n))
    A = X @ X.T + n * np.eye(n)
    A[np.abs(A) < 1.0] = 0.0
    A = np.triu(A) + np.triu(A, 1).T
    g = rng.normal(size=(n, n))
    g = 0.5 * (g + g.T)
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    C = oracle.c_matrix(A, lam)
    B = oracle.b_matrix(A, g, G, M, C, lam)
    At = oracle.trial_point(A, M, B, C, t)
    ref = A + M * oracle.direction(A, B, C, t)
    np.testing.assert_allclose(At, ref, rtol=0, atol=1e-12 * np.abs(A).max())


def test_objective_and_change_direct():
    S, _ = synth.chain_problem(30, 15, 1)
    lam = 0.2
    A = oracle.initial_iterate(S, lam)
    r = oracle.pista(S, lam, 1e-12, max_iter=3)
    assert abs(oracle.objective(S, A, lam) - pins.f_direct(S, A, lam)) < 1e-11
    assert abs(r.objective - pins.f_direct(S, r.A, lam)) < 1e-10
    L = oracle.cholesky_or_none(A)
    Lt = oracle.cholesky_or_none(r.A)
    dF = oracle.objective_change(S, A, r.A, L, Lt, lam)
    assert abs(dF - (pins.f_direct(S, r.A, lam) - pins.f_direct(S, A, lam))) < 1e-10


# ------------------------------------------------------------------ convergence (Sec. 5)
def test_monotone_decrease_and_pd():
    S, _ = synth.chain_problem(60, 30, 2)
    lam = 0.15
    prev = np.inf
    for k in range(0, 8):
        r = oracle.pista(S, lam, 0.0, max_iter=k)
        assert np.linalg.eigvalsh(r.A)[0] > 0
        F = pins.f_direct(S, r.A, lam)
        assert F < prev
        prev = F
    full = oracle.pista(S, lam, 1e-9)
    # every accepted step strictly decreases F (condition t_cond_min); the running
    # value F may stop changing in FP64 once |dF| < ulp(F)
    steps = [h for h in full.history if "dF" in h]
    assert len(steps) == full.iterations
    assert all(h["dF"] < 0 for h in steps)
    Fs = [h["F"] for h in full.history]
    assert all(b <= a for a, b in zip(Fs, Fs[1:]))


def test_fixed_point():
    """Lemma (fixed point): one more iteration from A* leaves it unchanged."""
    S = pins.random_psd(15, 10, 9)
    lam = 0.2
    r = oracle.pista(S, lam, 1e-10, max_iter=3000)
    r2 = oracle.pista(S, lam, 0.0, A0=r.A, max_iter=1)
    assert np.abs(r2.A - r.A).max() < 1e-8
    # support unchanged
    assert np.array_equal(r2.A != 0, r.A != 0)


def test_line_search_floor_fallback():
    """Below t = 1e-4 the step falls back to (0.9/cond A)^2 (Sec. 6): closed forms,
    the eigenvalue bound of the decrease lemma (Sec. 5.2) from an SVD, and a PD,
    decreasing trial point at that step."""
    assert pins.check_cond_fallback(oracle)


def test_fallback_solve_reaches_the_minimiser():
    """A solve that takes the fallback at every line search (t_floor above every
    step that succeeds) still converges to the same minimiser: same F and support
    as the plain solve, and the optimality conditions hold."""
    S = pins.random_psd(14, 7, 12)
    lam = 0.12
    ref = oracle.pista(S, lam, 1e-8, max_iter=3000)
    r = oracle.pista(S, lam, 1e-7, max_iter=20000, t_floor=0.99, t0=0.5)
    assert ref.status == r.status == oracle.CONVERGED
    assert sum(h.get("fallback", False) for h in r.history) == r.iterations
    assert abs(r.objective - ref.objective) <= 1e-11 * abs(ref.objective)
    assert np.array_equal(r.A != 0, ref.A != 0)
    assert pins.kkt_violation(S, r.A, lam) < 1e-6


def test_armijo_line_search():
    """sigma > 0: the first-order prediction against finite differences and an
    Armijo solve reaching the plain solve's minimiser (see pins.check_armijo)."""
    assert pins.check_armijo(oracle)


def test_gista_pins():
    """G-ISTA (H = I in eq. proximal_gen, Sec. 3.2): prox step by brute force, fixed
    point, Barzilai-Borwein closed form, quadratic-bound excess against slogdet, and
    solves against the independent solver and the closed forms."""
    assert pins.check_gista(oracle)


def test_gista_reaches_the_pista_minimiser_chain_config0():
    """Both methods minimise the same strictly convex F: on the chain workload at
    n = 100 G-ISTA's solution has pISTA's objective and support."""
    S, _ = synth.chain_problem(100, 50, seed=0)
    r = oracle.pista(S, 0.2, 1e-9)
    g = oracle.gista(S, 0.2, 1e-7)
    assert g.status == oracle.CONVERGED
    assert abs(g.objective - r.objective) <= 1e-9 * abs(r.objective)
    chk = oracle.check_solution(S, g.A, 0.2)
    assert chk["kkt_rel1"] <= 1e-7
    assert np.array_equal(g.A != 0, r.A != 0)


def test_iteration_cap_status():
    S, _ = synth.chain_problem(50, 25, 0)
    r = oracle.pista(S, 0.2, 1e-12, max_iter=2)
    assert r.status == oracle.MAX_ITER and r.iterations == 2


# ------------------------------------------------------------------ equivariances
def test_permutation_equivariance():
    S = pins.random_psd(12, 8, 21)
    lam = 0.2
    perm = np.random.default_rng(0).permutation(12)
    r = oracle.pista(S, lam, 1e-10, max_iter=3000)
    rp = oracle.pista(S[np.ix_(perm, perm)], lam, 1e-10, max_iter=3000)
    np.testing.assert_allclose(rp.A, r.A[np.ix_(perm, perm)], rtol=1e-7, atol=1e-9)


def test_scale_equivariance():
    S = pins.random_psd(10, 7, 22)
    lam, c = 0.15, 3.0
    r = oracle.pista(S, lam, 1e-10, max_iter=3000)
    rc = oracle.pista(c * S, c * lam, 1e-10, max_iter=3000)
    np.testing.assert_allclose(rc.A, r.A / c, rtol=1e-7, atol=1e-9)


def test_block_diagonal_decoupling():
    """If |S_ij| <= lam across blocks, A* is block diagonal and each block is its own
    solve (screening rule of Witten-Friedman-Simon and Mazumder-Hastie)."""
    S1 = pins.random_psd(6, 4, 31)
    S2 = pins.random_psd(5, 4, 32)
    lam = 0.2
    S = np.zeros((11, 11))
    S[:6, :6] = S1
    S[6:, 6:] = S2
    S[:6, 6:] = 0.5 * lam
    S[6:, :6] = 0.5 * lam
    r = oracle.pista(S, lam, 1e-10, max_iter=3000)
    r1 = oracle.pista(S1, lam, 1e-10, max_iter=3000)
    r2 = oracle.pista(S2, lam, 1e-10, max_iter=3000)
    assert np.all(r.A[:6, 6:] == 0)
    np.testing.assert_allclose(r.A[:6, :6], r1.A, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(r.A[6:, 6:], r2.A, rtol=1e-7, atol=1e-9)


# ------------------------------------------------------------------ mutation tests
def _mutant(**overrides):
    """A copy of the oracle module with some functions replaced by broken ones."""
    m = types.ModuleType("oracle_mutant")
    m.__dict__.update({k: v for k, v in opista.__dict__.items() if not k.startswith("__")})
    # rebind every function so it resolves the overridden helpers from the mutant
    for name, f in opista.__dict__.items():
        if isinstance(f, types.FunctionType) and f.__module__ == opista.__name__:
            m.__dict__[name] = types.FunctionType(f.__code__, m.__dict__, name, f.__defaults__, f.__closure__)
    m.__dict__.update(overrides)
    return m


MUTANTS = {
    "sign_guess_wrong_sign": dict(sign_guess=lambda A, g: np.where(A != 0, np.sign(A), np.sign(g))),
    "c_matrix_drops_offdiag_term": dict(c_matrix=lambda A, lam: lam * np.outer(np.diag(A), np.diag(A))),
    "gradient_wrong_sign": dict(gradient=lambda S, W: W - S),
    "soft_threshold_wrong": dict(soft_threshold=lambda x, tau: np.sign(x) * np.maximum(np.abs(x) + tau, 0.0)),
    "b_drops_c_term": dict(b_from_products=lambda P, C, G, M: P),
    "free_set_drops_gradient_part": dict(free_set_mask=lambda A, g, lam: A != 0),
    "diag_not_penalised_init": dict(initial_iterate=lambda S, lam: np.diag(1.0 / np.diag(S))),
    "objective_change_sign": dict(objective_change=lambda S, A, At, L, Lt, lam:
                                  -opista.objective_change(S, A, At, L, Lt, lam)),
    "cond_fallback_always_one": dict(cond_fallback_step=lambda A, factor=0.9: 1.0),
    "predicted_change_sign": dict(predicted_change=lambda g, A, At, lam: -opista.predicted_change(g, A, At, lam)),
    "predicted_change_drops_l1": dict(predicted_change=lambda g, A, At, lam: float(np.sum(g * (At - A)))),
    "cond_fallback_unsquared": dict(cond_fallback_step=lambda A, factor=0.9:
                                    factor * np.linalg.eigvalsh(A)[0] / np.linalg.eigvalsh(A)[-1]),
    "gista_step_wrong_sign": dict(gista_trial_point=lambda A, g, lam, t: opista.soft_threshold(A + t * g, t * lam)),
    "gista_threshold_unscaled": dict(gista_trial_point=lambda A, g, lam, t: opista.soft_threshold(A - t * g, lam)),
    "bb_step_reciprocal": dict(bb_step=lambda dA, Wo, Wn: 1.0 / opista.bb_step(dA, Wo, Wn)),
    "quadratic_bound_drops_quadratic": dict(quadratic_bound_excess=lambda A, At, L, Lt, W, t:
                                            opista.quadratic_bound_excess(A, At, L, Lt, W, t)
                                            + float(np.sum((At - A) ** 2)) / (2.0 * t)),
    "quadratic_bound_gradient_sign": dict(quadratic_bound_excess=lambda A, At, L, Lt, W, t:
                                          opista.quadratic_bound_excess(A, At, L, Lt, W, t)
                                          - 2.0 * float(np.sum(W * (At - A)))),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    m = _mutant(**MUTANTS[name])
    caught = False
    for check in (pins.check_scalar_lemma, pins.check_diagonal_solution, pins.check_n2_closed_form,
                  pins.check_kkt_invariants, pins.check_against_gista, pins.check_cond_fallback,
                  pins.check_armijo, pins.check_gista):
        try:
            ok = check(m) if check is not pins.check_scalar_lemma else check(m, trials=40)
        except Exception:
            ok = False
        if not ok:
            caught = True
            break
    assert caught, f"mutation {name} passed every pin"


def test_unmutated_copy_passes():
    m = _mutant()
    assert all(pins.all_pins(m).values())
