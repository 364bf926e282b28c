"""Block-diagonal screening (glasso_options.screen): the problem is split into the
connected components of {|S_ij| > lambda} and each block solved on its own.

The minimiser is unique, so the screened solve must meet the same bar against the
oracle's unscreened solve of the whole problem (F to 1e-8, the same support up to
the threshold exemptions, zeros between the blocks, the KKT measure of the
assembled A recomputed by the oracle), and every block must equal the same block
solved alone (bitwise: the persistent launch and the batched engine treat their
problems independently).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import golden_ref, pins
from tests.gpu_util import device, support_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


def components(S, lam):
    """Number and largest size of the connected components of {|S_ij| > lam}
    (scipy's graph routine, independent of the device union-find)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    G = np.abs(S) > lam
    np.fill_diagonal(G, False)
    k, lab = connected_components(csr_matrix(G), directed=False)
    return k, int(np.bincount(lab).max())


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


def block_problem(lam):
    """Blocks of 70 (batched engine), 20 and 9 (persistent launch) and two single
    variables, coupled by entries of size 0.9 lambda, variables shuffled."""
    sizes = [70, 20, 9, 1, 1]
    n = sum(sizes)
    S = np.zeros((n, n))
    rng = np.random.default_rng(5)
    o = 0
    for q, k in enumerate(sizes):
        S[o:o + k, o:o + k] = pins.random_psd(k, max(2, k), 40 + q) + 0.5 * np.eye(k)
        o += k
    cross = np.ones((n, n), dtype=bool)
    o = 0
    for k in sizes:
        cross[o:o + k, o:o + k] = False
        o += k
    C = 0.9 * lam * np.sign(rng.standard_normal((n, n)))
    C = np.triu(C, 1) + np.triu(C, 1).T
    S = np.where(cross, C, S)
    perm = rng.permutation(n)
    return S[np.ix_(perm, perm)], perm, sizes


def test_block_problem_meets_oracle_bar(g):
    lam, tol = 0.1, 3e-8
    S, perm, sizes = block_problem(lam)
    res = g.Solver(screen=True).solve(to_dev(S), lam, tol)
    assert res.status == g.CONVERGED
    assert res.components == len(sizes) and res.largest_component == max(sizes)
    A, W = to_host(res.A), to_host(res.W)
    ref = oracle.pista(S, lam, 1e-8, max_iter=5000)
    chk = oracle.check_solution(S, A, lam)
    assert chk["kkt_rel1"] <= tol * 1.0001
    assert abs(res.kkt_rel1 - chk["kkt_rel1"]) <= 1e-6 * chk["kkt_rel1"] + 1e-15
    assert abs(res.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    assert abs(res.objective - chk["objective"]) <= 1e-10 * abs(chk["objective"])
    assert support_mismatch(A, ref.A, oracle.check_solution(S, ref.A, lam)["g"], lam) == 0
    assert res.nnz == np.count_nonzero(A)
    np.testing.assert_allclose(W @ A, np.eye(len(S)), rtol=0, atol=1e-9)
    # zeros between the blocks, and each block equals the block solved alone
    inv = np.argsort(perm)
    o = 0
    for k in sizes:
        blk = np.sort(inv[o:o + k])
        mask = np.zeros(len(S), dtype=bool)
        mask[blk] = True
        assert np.all(A[np.ix_(mask, ~mask)] == 0)
        Sb = np.ascontiguousarray(S[np.ix_(blk, blk)])
        alone = (g.Solver().solve_small([to_dev(Sb)], [lam], tol)[0] if k <= g.SMALL_MAX_N
                 else g.Solver().solve(to_dev(Sb), lam, tol))
        assert np.array_equal(to_host(alone.A), A[np.ix_(blk, blk)])
        o += k


def test_unscreened_problem_is_solved_in_place(g):
    """One component (the chain at lambda 0.2): the screened solve is the plain solve."""
    S, _ = synth.chain_problem(300, 150, 1)
    a = g.Solver(screen=True).solve(to_dev(S), 0.2, 1e-7)
    b = g.Solver().solve(to_dev(S), 0.2, 1e-7)
    assert a.components == 1 and a.largest_component == 300
    assert np.array_equal(to_host(a.A), to_host(b.A)) and a.iterations == b.iterations


@pytest.mark.parametrize("mode", ["independent", "waves"])
def test_path_large_lambda_end_against_oracle(g, mode):
    """The first 12 lambdas of the n = 1000 path (from lambda_max, where the problem
    falls apart into single variables, down to where one component holds 985 of
    them), screened, batched and, in waves, warm-started: F to 1e-8 of the oracle's
    stored solutions and the same support."""
    S, _ = synth.random_sparse_problem(1000, 500, 0)
    lams = list(synth.lambda_path(S, count=32, ratio=100.0))[:12]
    refs = golden_ref.load("path1000")[:12]
    res = g.lambda_path(to_dev(S), lams, 1e-8, mode=mode, waves=3, max_iter=5000, screen=True)
    assert res[0].components == 1000 and res[0].iterations == 0
    bad = []
    for k, (r, ref) in enumerate(zip(res, refs)):
        assert (r.components, r.largest_component) == components(S, lams[k])
        assert r.status == g.CONVERGED
        relF, mism, _ = golden_ref.compare(to_host(r.A), r.objective, ref)
        if relF > 1e-8 or mism:
            bad.append((k, relF, mism, r.components, r.largest_component, r.iterations, r.kkt_rel1))
    assert not bad, bad


def test_serving_request_screened_against_oracle(g):
    """A serving request (random sparse drawn on the device, n = 1000, m = 500,
    lambda = 0.3 lambda_max) falls apart into hundreds of small blocks: screened
    against the oracle's solve of the whole problem."""
    s = g.Solver(screen=True)
    _, _, S, lm = s.generate("random", 1000, 500, seed=77)
    lam, tol = 0.3 * lm, 1e-8
    res = s.solve(S, lam, tol)
    assert res.status == g.CONVERGED and res.components > 100 and res.largest_component <= 64
    Sh, A = to_host(S), to_host(res.A)
    assert (res.components, res.largest_component) == components(Sh, lam)
    ref = oracle.pista(Sh, lam, tol, max_iter=5000)
    assert abs(res.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    assert support_mismatch(A, ref.A, oracle.check_solution(Sh, ref.A, lam)["g"], lam) == 0
    assert oracle.check_solution(Sh, A, lam)["kkt_rel1"] <= tol * 1.0001
