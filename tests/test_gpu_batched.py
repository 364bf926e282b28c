"""Batched engine (glasso_solve_batched) and the regularisation path.

* every problem of a batch is bitwise identical to its own glasso_solve (the
  kernels treat the problems of a batch independently);
* every lambda-path mode meets the FP64 acceptance bar against the oracle for
  every lambda (the minimiser is unique, so the path mode cannot matter).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, support_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_batch_bitwise_equals_single(g, precision):
    S, _ = synth.random_sparse_problem(300, 150, 3)
    lm = synth.lambda_max(S)
    lams = [0.6 * lm, 0.35 * lm, 0.2 * lm, 0.12 * lm]
    St = to_dev(S)
    s = g.Solver(precision=precision)
    batch = s.solve_batched(St, lams, 1e-7)
    for lam, rb in zip(lams, batch):
        r1 = g.Solver(precision=precision).solve(St, lam, 1e-7)
        assert rb.status == r1.status == g.CONVERGED
        assert rb.iterations == r1.iterations and rb.ls_trials == r1.ls_trials
        assert np.array_equal(to_host(rb.A), to_host(r1.A))
        assert np.array_equal(to_host(rb.W), to_host(r1.W))
        assert rb.objective == r1.objective


def test_batch_of_different_sizes(g):
    probs = [synth.chain_problem(130, 60, 0)[0], synth.random_sparse_problem(70, 40, 1)[0],
             synth.chain_problem(130, 60, 2)[0], synth.random_sparse_problem(260, 100, 4)[0]]
    lams = [0.2, 0.3 * synth.lambda_max(probs[1]), 0.25, 0.3 * synth.lambda_max(probs[3])]
    Sts = [to_dev(S) for S in probs]
    batch = g.Solver().solve_batched(Sts, lams, 1e-6)
    for S, St, lam, rb in zip(probs, Sts, lams, batch):
        r1 = g.Solver().solve(St, lam, 1e-6)
        assert np.array_equal(to_host(rb.A), to_host(r1.A))
        chk = oracle.check_solution(S, to_host(rb.A), lam)
        assert chk["kkt_rel1"] <= 1e-6 * 1.0001


@pytest.mark.parametrize("mode", ["independent", "sequential", "waves"])
def test_lambda_path_modes(g, mode):
    """A scaled-down path: one S (random sparse, n=130, m=65), 6 lambdas geometric
    from lambda_max to lambda_max/10 (below that the oracle needs hundreds of
    iterations per lambda on this rank-deficient S).  Warm starts follow other
    trajectories than the oracle's cold solves, so each result is compared with the
    oracle's solution to 1e-8; at tol 1e-7 every support is the converged one (at
    1e-6 the last lambda's cold oracle solve is itself two entries short of it)."""
    S, _ = synth.random_sparse_problem(130, 65, 5)
    lams = list(synth.lambda_path(S, count=6, ratio=10.0))
    tol = 1e-7
    res = g.lambda_path(to_dev(S), lams, tol, mode=mode, waves=3)
    assert len(res) == len(lams)
    for lam, r in zip(lams, res):
        assert r.status == g.CONVERGED
        A = to_host(r.A)
        ref = oracle.pista(S, lam, 1e-8, max_iter=5000)
        chk = oracle.check_solution(S, A, lam)
        assert chk["kkt_rel1"] <= tol * 1.0001
        assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
        ref_chk = oracle.check_solution(S, ref.A, lam)
        assert support_mismatch(A, ref.A, ref_chk["g"], lam) == 0
    # the lambda_max end of the path is the diagonal solution, reached at once
    assert res[0].iterations == 0
    np.testing.assert_array_equal(to_host(res[0].A), np.diag(1.0 / (np.diag(S) + lams[0])))


def test_batch_warm_start_not_pd(g):
    S, _ = synth.chain_problem(64, 32, 1)
    St = to_dev(S)
    good = to_dev(np.eye(64))
    bad = to_dev(-np.eye(64))
    with pytest.raises(g.GlassoError) as e:
        g.Solver(warm_start=True).solve_batched(St, [0.2, 0.3], 1e-6, A_list=[good, bad])
    assert e.value.code == 2


@pytest.mark.parametrize("t_floor", [1e-4, 0.3])
def test_line_search_width_invariant(g, t_floor):
    """Several step sizes per line-search round (ls_width) give the same accepted
    steps as one at a time: bitwise the same A and W, iterations, trial and
    fallback counts, single and batched.  t_floor = 0.3 sends every search that
    reaches t = 0.25 through the cond-based fallback step (Sec. 6), which a round
    must not run ahead of.  Every converged result also meets the objective bar
    against the oracle (KKT of the returned A recomputed by the oracle, F within 1e-8
    of the oracle's solve to 1e-8); the support is checked on the fallback path in
    test_fallback_solves_meet_oracle_bar."""
    S, _ = synth.random_sparse_problem(300, 150, 5)
    lm = synth.lambda_max(S)
    lams = [0.5 * lm, 0.15 * lm, 0.08 * lm]
    St = to_dev(S)
    runs = {}
    for width in (1, 3, 0, 16):
        s = g.Solver(ls_width=width, t_floor=t_floor)
        runs[width] = (s.solve_batched(St, lams, 1e-7), [s.solve(St, lam, 1e-7) for lam in lams])
    ref_b, ref_s = runs[1]
    assert sum(r.ls_trials for r in ref_s) > sum(r.iterations for r in ref_s)  # the searches backtrack
    if t_floor > 0.25:
        assert sum(r.fallback_steps for r in ref_s) > 0
    for width, (rb, rs) in runs.items():
        for a, b in list(zip(ref_b, rb)) + list(zip(ref_s, rs)) + list(zip(ref_s, rb)):
            assert (a.status, a.iterations, a.ls_trials, a.fallback_steps) == \
                (b.status, b.iterations, b.ls_trials, b.fallback_steps), width
            assert np.array_equal(to_host(a.A), to_host(b.A)), width
            assert np.array_equal(to_host(a.W), to_host(b.W)), width
    converged = 0
    for lam, r in zip(lams, ref_s):
        if r.status != g.CONVERGED:
            continue  # at t_floor = 0.3 the smallest lambda crawls on fallback steps
        converged += 1
        chk = oracle.check_solution(S, to_host(r.A), lam)
        assert chk["kkt_rel1"] <= 1e-7 * 1.0001
        ref = oracle.pista(S, lam, 1e-8)
        assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    assert converged >= 2


@pytest.mark.parametrize("n,m,seed", [(64, 640, 3), (48, 480, 5)])
def test_fallback_solves_meet_oracle_bar(g, n, m, seed):
    """Every step through the cond-based fallback (Sec. 6): t0 = 0.2 below t_floor =
    0.3 sends each line search straight to t = min(t0, (0.9/cond A)^2).  The GPU
    estimates cond(A) by power iteration where the oracle takes eigenvalues, so the
    two trajectories differ, but both reach the unique minimiser.  On these
    well-conditioned problems (m = 10 n samples, cond A* about 3) the small steps
    still converge in a few hundred iterations; the result is compared with the
    oracle's plain solve to 1e-8: KKT recomputed by the oracle, F to 1e-8, the same
    support up to the threshold exemptions."""
    S, _ = synth.random_sparse_problem(n, m, seed)
    lm = synth.lambda_max(S)
    tol = 3e-8
    for frac in (0.5, 0.3):
        lam = frac * lm
        r = g.Solver(t0=0.2, t_floor=0.3, max_iter=5000).solve(to_dev(S), lam, tol)
        assert r.status == g.CONVERGED
        assert r.fallback_steps >= r.iterations > 10  # every line search took the fallback step
        A = to_host(r.A)
        chk = oracle.check_solution(S, A, lam)
        assert chk["kkt_rel1"] <= tol * 1.0001
        ref = oracle.pista(S, lam, 1e-8)
        assert ref.status == oracle.CONVERGED
        assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
        ref_chk = oracle.check_solution(S, ref.A, lam)
        assert support_mismatch(A, ref.A, ref_chk["g"], lam) == 0


def test_batch_of_many_backtracking_problems_bitwise(g):
    """Eight backtracking problems at n = 1100 (padded 1152, nine leaf steps, 32
    trial slots per round) solved as one batch and one by one: bitwise the same
    results, iteration and trial counts."""
    S, _ = synth.random_sparse_problem(1100, 550, 7)
    lm = synth.lambda_max(S)
    lams = [lm * f for f in (0.3, 0.2, 0.15, 0.1, 0.08, 0.06, 0.05, 0.04)]
    St = to_dev(S)
    batch = g.Solver().solve_batched(St, lams, 1e-6)
    for lam, rb in zip(lams, batch):
        r1 = g.Solver().solve(St, lam, 1e-6)
        assert rb.status == r1.status == g.CONVERGED
        assert (rb.iterations, rb.ls_trials) == (r1.iterations, r1.ls_trials)
        assert np.array_equal(to_host(rb.A), to_host(r1.A))
        assert np.array_equal(to_host(rb.W), to_host(r1.W))
    assert sum(r.ls_trials for r in batch) > sum(r.iterations for r in batch)


def test_wide_line_search_falls_back_when_memory_is_short(g):
    """A batch sized so that the automatic four trial slots per problem cannot fit
    in the free device memory but one slot can: the solve still runs (one step size
    per round) and gives the bits of the same problems solved one by one."""
    import torch

    n, np_ = 2048, 2048
    free, _ = torch.cuda.mem_get_info()
    per1 = (9 * 8 + 1) * np_ * np_ + 4 * np_ * 128 * 8 + 8 * n * n  # workspace at width 1 + the output A
    count = int(0.75 * free // per1)
    per4 = per1 + 6 * 8 * np_ * np_
    assert count * per4 > free  # width 4 does not fit
    S, _ = synth.random_sparse_problem(n, n // 2, 9)
    lam = 0.3 * synth.lambda_max(S)
    St = to_dev(S)
    s = g.Solver(max_iter=2)
    res = s.solve_batched(St, [lam] * count, 1e-5, want_W=False)
    assert len(res) == count
    one = g.Solver(max_iter=2).solve(St, lam, 1e-5, want_W=False)
    for r in (res[0], res[-1]):
        assert (r.status, r.iterations, r.ls_trials) == (one.status, one.iterations, one.ls_trials)
        assert np.array_equal(to_host(r.A), to_host(one.A))
    s.close()
    del res
    torch.cuda.empty_cache()
