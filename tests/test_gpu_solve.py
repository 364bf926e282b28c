"""End-to-end parity of glasso_solve (FP64 path) with the CPU oracle.

Acceptance (FP64): |F_gpu - F_oracle| <= 1e-8 max(1, |F_oracle|); the KKT measure
recomputed by the oracle from the returned A is <= max(tol, 1e-5); the support
equals the oracle's except entries within 1e-8 of the threshold.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import device, support_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


def check_against_oracle(g, S, lam, tol, solver=None, ref=None, obj_rtol=1e-8):
    s = solver or g.Solver()
    res = s.solve(to_dev(S), lam, tol)
    A = to_host(res.A)
    W = to_host(res.W)
    ref = ref or oracle.pista(S, lam, tol)
    chk = oracle.check_solution(S, A, lam)
    assert res.status == g.CONVERGED, res.status_name
    assert chk["pd"]
    assert chk["kkt_rel1"] <= max(tol, 1e-5) * 1.0001, chk["kkt_rel1"]
    assert abs(res.objective - ref.objective) <= obj_rtol * max(1.0, abs(ref.objective))
    assert abs(res.objective - chk["objective"]) <= 1e-10 * max(1.0, abs(chk["objective"]))
    ref_chk = oracle.check_solution(S, ref.A, lam)
    assert support_mismatch(A, ref.A, ref_chk["g"], lam) == 0
    assert np.array_equal(A, A.T)
    # W is the inverse of the returned A
    assert np.max(np.abs(W @ A - np.eye(len(S)))) <= 1e-10 * np.linalg.cond(A)
    assert res.nnz == np.count_nonzero(A)
    # every accepted step followed one product (the GEMM pair or the sparse form);
    # the first of a diagonal start is D Z D, formed elementwise
    assert res.aza_gemm_products + res.aza_sparse_products == max(res.iterations - 1, 0)
    if solver is None:
        s.close()
    return res, ref


@pytest.mark.parametrize("seed", range(5))
def test_chain_n100(g, seed):
    """Chain precision (A_ii = 1.25, A_i,i+1 = -0.5), n=100, m=50, lambda=0.2, tol 1e-6."""
    S, _ = synth.chain_problem(100, 50, seed)
    res, ref = check_against_oracle(g, S, 0.2, 1e-6)
    # same algorithm, same readings: iteration counts agree closely
    assert abs(res.iterations - ref.iterations) <= max(2, ref.iterations // 10)


@pytest.mark.parametrize("n,seed,frac", [(30, 0, 0.3), (130, 1, 0.25), (300, 2, 0.2), (257, 3, 0.5)])
def test_random_sparse(g, n, seed, frac):
    S, _ = synth.random_sparse_problem(n, n // 2, seed)
    lam = frac * synth.lambda_max(S)
    check_against_oracle(g, S, lam, 1e-6)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,seed,frac", [(130, 1, 0.25), (300, 2, 0.2)])
def test_mixed_precision_meets_fp64_bar(g, precision, n, seed, frac):
    """Mixed forms: A Z A in reduced precision, everything that decides acceptance
    and stopping in FP64 -> the same FP64 acceptance bar as the plain path."""
    S, _ = synth.random_sparse_problem(n, n // 2, seed)
    lam = frac * synth.lambda_max(S)
    check_against_oracle(g, S, lam, 1e-6, solver=g.Solver(precision=precision))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_chain(g, precision):
    S, _ = synth.chain_problem(100, 50, 0)
    res, ref = check_against_oracle(g, S, 0.2, 1e-6, solver=g.Solver(precision=precision))


def test_n1_and_n2(g):
    S = np.array([[0.7]])
    res = g.Solver().solve(to_dev(S), 0.1, 1e-10)
    assert res.iterations == 0
    assert to_host(res.A)[0, 0] == 1.0 / 0.8
    from tests import pins

    for seed in range(3):
        S = pins.random_psd(2, 3, seed)
        for lam in (0.05, 0.3):
            res = g.Solver().solve(to_dev(S), lam, 1e-9)
            np.testing.assert_allclose(to_host(res.A), pins.n2_closed_form(S, lam), rtol=1e-7, atol=1e-9)


def test_diagonal_solution_zero_iterations(g):
    S, _ = synth.chain_problem(150, 300, 4)
    lam = synth.lambda_max(S)
    res = g.Solver().solve(to_dev(S), lam, 1e-10)
    assert res.iterations == 0 and res.status == g.CONVERGED
    A = to_host(res.A)
    np.testing.assert_array_equal(A, np.diag(1.0 / (np.diag(S) + lam)))


@pytest.fixture(scope="module")
def n2000():
    cfg = json.load(open(os.path.join(HERE, "golden", "workloads.json")))["random_sparse_n2000"]
    S, _ = synth.random_sparse_problem(cfg["n"], cfg["m"], cfg["seed"])
    return cfg, S, oracle.pista(S, cfg["lambda"], cfg["tol"])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_random_sparse_n2000_workload(g, n2000, precision):
    """The n=2000 random-sparse workload with its frozen lambda (nnz ~ 5n): the FP64
    path and both mixed forms (FP64 factor, line search and KKT) against the oracle."""
    cfg, S, ref = n2000
    res, _ = check_against_oracle(g, S, cfg["lambda"], cfg["tol"], solver=g.Solver(precision=precision), ref=ref)
    assert abs(res.nnz - cfg["oracle_nnz"]) <= 0.01 * cfg["oracle_nnz"]


def test_warm_start_resumes(g):
    S, _ = synth.chain_problem(200, 100, 1)
    cold = g.Solver().solve(to_dev(S), 0.15, 1e-7)
    first = g.Solver().solve(to_dev(S), 0.25, 1e-7)
    warm = g.Solver(warm_start=True).solve(to_dev(S), 0.15, 1e-7, A=first.A.clone())
    assert warm.status == g.CONVERGED
    assert warm.aza_gemm_products + warm.aza_sparse_products == warm.iterations  # no diagonal start
    assert abs(warm.objective - cold.objective) <= 1e-9 * abs(cold.objective)


def test_status_and_errors(g):
    S, _ = synth.chain_problem(64, 32, 2)
    res = g.Solver(max_iter=1).solve(to_dev(S), 0.2, 1e-12)
    assert res.status == g.MAX_ITER and res.iterations == 1
    with pytest.raises(g.GlassoError) as e:
        g.Solver().solve(to_dev(S), -1.0, 1e-6)
    assert e.value.code == 1
    Sbad = S.copy()
    Sbad[5, 3] = np.nan
    with pytest.raises(g.GlassoError) as e:
        g.Solver().solve(to_dev(Sbad), 0.2, 1e-6)
    assert e.value.code == 1
    with pytest.raises(g.GlassoError) as e:
        g.Solver(warm_start=True).solve(to_dev(S), 0.2, 1e-6, A=to_dev(-np.eye(64)))
    assert e.value.code == 2
    # the line search can be forced to fail from the host: t0 below t_min
    res = g.Solver(t0=1e-13, t_min=1e-12, t_floor=0.0).solve(to_dev(S), 0.2, 1e-9)
    assert res.status == g.LS_FAILED and res.iterations == 0


def test_deterministic(g):
    S, _ = synth.random_sparse_problem(300, 150, 9)
    lam = 0.3 * synth.lambda_max(S)
    s = g.Solver()
    a = to_host(s.solve(to_dev(S), lam, 1e-7).A)
    b = to_host(s.solve(to_dev(S), lam, 1e-7).A)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n,seed", [(130, 1), (300, 2)])
def test_armijo_line_search(g, n, seed):
    """sigma = 0.3: a trial point is accepted only when F falls by 0.3 times the
    decrease the linear model predicts (the trial pass sums W (.) (At - A) for it).
    The blocked engine, its batch and the persistent launch follow the oracle's
    Armijo search step for step, and reach the minimiser of the plain solve."""
    S, _ = synth.random_sparse_problem(n, n // 2, seed)
    lam, tol = 0.3 * synth.lambda_max(S), 1e-8
    ref = oracle.pista(S, lam, tol, sigma=0.3, max_iter=3000)
    plain = oracle.pista(S, lam, tol, max_iter=3000)
    assert ref.status == plain.status == oracle.CONVERGED
    runs = [g.Solver(sigma=0.3).solve(to_dev(S), lam, tol),
            g.Solver(sigma=0.3).solve_batched(to_dev(S), [lam, 0.9 * lam], tol)[0]]
    if n <= g.SMALL_MAX_N:
        runs.append(g.Solver(sigma=0.3).solve_small([to_dev(S)], [lam], tol)[0])
    for r in runs:
        assert r.status == g.CONVERGED
        assert abs(r.iterations - ref.iterations) <= 1 and abs(r.ls_trials - ref.ls_trials) <= 2
        A = to_host(r.A)
        assert oracle.check_solution(S, A, lam)["kkt_rel1"] <= tol * 1.0001
        assert abs(r.objective - plain.objective) <= 1e-8 * max(1.0, abs(plain.objective))
        assert support_mismatch(A, plain.A, oracle.check_solution(S, plain.A, lam)["g"], lam) == 0


def test_armijo_small_problems(g):
    """The persistent launch with sigma = 0.3 against the oracle's Armijo solves."""
    probs = []
    for n, seed in [(20, 3), (48, 4), (64, 5)]:
        S, _ = synth.random_sparse_problem(n, n // 2, seed)
        probs.append((S, 0.25 * synth.lambda_max(S)))
    res = g.Solver(sigma=0.3).solve_small([to_dev(S) for S, _ in probs], [lam for _, lam in probs], 1e-8)
    for (S, lam), r in zip(probs, res):
        ref = oracle.pista(S, lam, 1e-8, sigma=0.3, max_iter=3000)
        assert r.status == ref.status == g.CONVERGED
        assert abs(r.iterations - ref.iterations) <= 1
        assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
