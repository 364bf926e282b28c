"""glasso_solve_small_static: the persistent small-problem solve through the entry
point that allocates nothing (its scratch in the library's fixed device array).

Checked through the C ABI against glasso_solve_small (the handle-workspace entry
point, the same kernel): bitwise the same A, W, objective and counts on two calls
in a row, the second with fewer and smaller problems (the array keeps the first
call's contents), and the oracle's FP64 bar on the results.  Sizes beyond the
array's limit are rejected on the host before any launch.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


def batch(count, n_lo, n_hi, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        S, _ = synth.random_sparse_problem(n, max(2, n // 2), 1000 * seed + i)
        out.append((S, 0.3 * synth.lambda_max(S)))
    return out


def same_results(g, probs, tol):
    Sd = [to_dev(S) for S, _ in probs]
    lams = [lam for _, lam in probs]
    ref = g.Solver().solve_small(Sd, lams, tol)
    got = g.Solver().solve_small_static(Sd, lams, tol)
    assert len(got) == len(ref)
    for r, q in zip(ref, got):
        assert (q.status, q.iterations, q.ls_trials, q.fallback_steps) == \
            (r.status, r.iterations, r.ls_trials, r.fallback_steps)
        assert q.objective == r.objective and q.kkt_rel1 == r.kkt_rel1
        assert np.array_equal(to_host(q.A), to_host(r.A))
        assert np.array_equal(to_host(q.W), to_host(r.W))
    return got


def test_static_entry_point_matches_workspace_entry_point(g):
    tol = 1e-7
    first = batch(300, 16, 64, 1)   # more problems than the 256 workgroups
    got = same_results(g, first, tol)
    for (S, lam), r in list(zip(first, got))[:6]:
        assert r.status == g.CONVERGED
        chk = oracle.check_solution(S, to_host(r.A), lam)
        assert chk["kkt_rel1"] <= tol * 1.0001
        ref = oracle.pista(S, lam, tol)
        assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    second = batch(7, 3, 20, 2)    # fewer and smaller problems on the same array
    same_results(g, second, tol)


def test_static_entry_point_rejects_oversize_on_host(g):
    lib = g._lib
    count = g.SMALL_STATIC_MAX_COUNT + 1
    S = to_dev(np.eye(4))
    VP = ctypes.c_void_p
    ptrs = (VP * count)(*([S.data_ptr()] * count))
    nn = (ctypes.c_int64 * count)(*([4] * count))
    ll = (ctypes.c_double * count)(*([0.1] * count))
    rc = lib.glasso_solve_small_static(None, count, ptrs, nn, ll, 1e-6, ptrs, None, None, None)
    assert rc == 1  # GLASSO_ERR_INVALID_ARG, nothing launched
    one = (ctypes.c_int64 * 1)(g.SMALL_MAX_N + 1)
    rc = lib.glasso_solve_small_static(None, 1, ptrs, one, ll, 1e-6, ptrs, None, None, None)
    assert rc == 1
