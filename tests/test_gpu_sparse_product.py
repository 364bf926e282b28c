"""The sampled sparse form of the preconditioned product (glasso_sparse_product and
its use inside the solves).

The trial point (eq. d_sol) reads P = A Z A only on the free set, so a solve forms
those entries from the short rows of the iterate when it can (the paper forms the
product densely, Sec. 4.3.3).  Checks: the entry point against the plain definition
A @ Z @ A on the free set (FP64, bound 4 n eps |A||Z||A|), zero elsewhere, with
both the sparse form and the dense fallback; solves against the oracle; the
automatic choice against the dense pair alone; batched problems that take
different forms against their single solves (bitwise); graph replay against eager
launches (bitwise).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import EPS, device, sym, to_dev, to_host
from tests.test_gpu_solve import check_against_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


@pytest.fixture(scope="module")
def solver(g):
    s = g.Solver()
    yield s
    s.close()


def short_rows(n, seed, long_row=None):
    """Symmetric A with at most 9 nonzeros per row (bands 1, 2, 5 with dropout and one
    long-range partner per row); long_row: give that row 20 nonzeros."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for off in (1, 2, 5):
        if off >= n:
            continue
        i = np.arange(n - off)
        keep = rng.random(n - off) < 0.7
        A[i[keep], i[keep] + off] = rng.standard_normal(keep.sum())
    perm = rng.permutation(n)
    for a, b in zip(perm[0::2], perm[1::2]):
        A[min(a, b), max(a, b)] = rng.standard_normal()
    if long_row is not None and n > 40:
        for c in rng.choice(np.setdiff1d(np.arange(n), [long_row]), 20, replace=False):
            A[min(c, long_row), max(c, long_row)] = 0.1
    A = np.triu(A, 1)
    A = A + A.T
    A[np.arange(n), np.arange(n)] = 2.0 + rng.random(n)
    return A


def free_set(n, seed, density=0.05, dense_row=None):
    """Symmetric int8 mask of +-1 with a set diagonal; row 0 (n > 2) left empty."""
    rng = np.random.default_rng(seed + 100)
    GM = np.where(rng.random((n, n)) < density, np.where(rng.random((n, n)) < 0.5, 1, -1), 0)
    GM = np.tril(GM, -1)
    if dense_row is not None:
        GM[dense_row, :dense_row] = 1
    GM = GM + GM.T
    GM[np.arange(n), np.arange(n)] = 1
    if n > 2:
        GM[0, :] = 0
        GM[:, 0] = 0
    return GM.astype(np.int8)


def check_product(solver, A, Z, GM, want_sparse):
    import torch

    n = len(A)
    P, used = solver.sparse_product(to_dev(A), to_dev(Z), torch.from_numpy(GM).to("cuda:0"))
    P = to_host(P)
    assert used == want_sparse
    ref = np.where(GM != 0, A @ Z @ A, 0.0)
    bound = np.where(GM != 0, 4 * n * EPS * (np.abs(A) @ np.abs(Z) @ np.abs(A)), 0.0)
    assert np.all(np.abs(P - ref) <= bound), np.max(np.abs(P - ref) - bound)
    assert np.array_equal(P, P.T)


@pytest.mark.parametrize("n", [1, 5, 130, 300, 513])
def test_sparse_product_matches_definition(solver, n):
    A = short_rows(n, n)
    rng = np.random.default_rng(n + 7)
    Z = sym(rng.standard_normal((n, n)))
    check_product(solver, A, Z, free_set(n, n), want_sparse=True)


@pytest.mark.parametrize("n", [300, 513])
def test_sparse_product_falls_back_to_the_pair(solver, n):
    """A row of A with 20 nonzeros, or a free-set row with more than 64 entries left of
    the diagonal: the FP64 GEMM pair forms the same entries."""
    rng = np.random.default_rng(n)
    Z = sym(rng.standard_normal((n, n)))
    check_product(solver, short_rows(n, 3, long_row=n // 2), Z, free_set(n, 3), want_sparse=False)
    check_product(solver, short_rows(n, 4), Z, free_set(n, 4, dense_row=n - 1), want_sparse=False)


def test_sparse_product_repeated_calls(solver):
    """A sparse call after a dense one and a smaller one after a larger one: no stale rows."""
    rng = np.random.default_rng(9)
    for n, long_row in ((513, 200), (300, None), (130, None)):
        Z = sym(rng.standard_normal((n, n)))
        check_product(solver, short_rows(n, n + 1, long_row=long_row), Z, free_set(n, n + 1),
                      want_sparse=long_row is None)


@pytest.mark.parametrize("seed", range(3))
def test_solve_takes_the_sparse_product(g, seed):
    """Chain n=300 from m=1500 samples, lambda=0.2: the iterates keep short rows, every
    product after the diagonal start is the sparse one, and the solve matches the oracle."""
    S, _ = synth.chain_problem(300, 1500, seed)
    res, _ = check_against_oracle(g, S, 0.2, 1e-6)
    assert res.aza_sparse_products == max(res.iterations - 1, 0)
    assert res.aza_gemm_products == 0


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_automatic_choice_against_the_dense_pair(g, precision):
    """Chain n=300 from m=300 samples, lambda=0.2: early iterates have long rows (dense
    pair), later ones short (sparse form).  The objective agrees with the dense pair
    alone and with the oracle."""
    S, _ = synth.chain_problem(300, 300, 0)
    auto = g.Solver(precision=precision).solve(to_dev(S), 0.2, 1e-6)
    dense = g.Solver(precision=precision, dense_product=True).solve(to_dev(S), 0.2, 1e-6)
    assert auto.status == dense.status == g.CONVERGED
    assert dense.aza_sparse_products == 0
    assert auto.aza_sparse_products > 0 and auto.aza_gemm_products > 0
    assert abs(auto.iterations - dense.iterations) <= 2
    assert abs(auto.objective - dense.objective) <= 1e-9 * abs(dense.objective)
    ref = oracle.pista(S, 0.2, 1e-6)
    assert abs(auto.objective - ref.objective) <= 1e-8 * abs(ref.objective)


def test_batched_problems_take_their_own_form(g):
    """One batch: a problem whose products are all sparse and one that starts dense.
    Each result equals its single solve bitwise."""
    S1, _ = synth.chain_problem(300, 1500, 0)
    S2, _ = synth.chain_problem(300, 300, 0)
    s = g.Solver()
    batch = s.solve_batched([to_dev(S1), to_dev(S2)], [0.2, 0.2], 1e-6)
    for S, lam, rb in ((S1, 0.2, batch[0]), (S2, 0.2, batch[1])):
        r1 = g.Solver().solve(to_dev(S), lam, 1e-6)
        assert (rb.iterations, rb.aza_gemm_products, rb.aza_sparse_products) == \
               (r1.iterations, r1.aza_gemm_products, r1.aza_sparse_products)
        assert np.array_equal(to_host(rb.A), to_host(r1.A))
    assert batch[0].aza_gemm_products == 0 and batch[1].aza_gemm_products > 0
    s.close()


def test_graphs_replay_the_choice(g):
    """Captured graphs hold both forms; replays follow the device-side choice."""
    S, _ = synth.chain_problem(300, 300, 0)
    eager = g.Solver().solve(to_dev(S), 0.2, 1e-6)
    graph = g.Solver(graphs=True).solve(to_dev(S), 0.2, 1e-6)
    assert eager.aza_sparse_products > 0 and eager.aza_gemm_products > 0
    assert (graph.iterations, graph.aza_gemm_products, graph.aza_sparse_products) == \
           (eager.iterations, eager.aza_gemm_products, eager.aza_sparse_products)
    assert np.array_equal(to_host(graph.A), to_host(eager.A))


@pytest.mark.parametrize("n", [300, 1100])
def test_zero_block_inverse_is_exact(g, n):
    """A single problem with one trial slot (ls_width=1) skips the FP32-accurate inverse's
    products over zero blocks of the factor; with two slots it does not.  Skipped products
    are exact zeros, so both runs agree bit for bit (chain trial points are banded)."""
    S, _ = synth.chain_problem(n, 5 * n, 0)
    one = g.Solver(precision="bf16x3", ls_width=1).solve(to_dev(S), 0.2, 1e-6)
    two = g.Solver(precision="bf16x3", ls_width=2).solve(to_dev(S), 0.2, 1e-6)
    assert one.status == two.status == g.CONVERGED
    assert (one.iterations, one.ls_trials) == (two.iterations, two.ls_trials)
    assert np.array_equal(to_host(one.A), to_host(two.A))
    assert np.array_equal(to_host(one.W), to_host(two.W))
    assert one.objective == two.objective
