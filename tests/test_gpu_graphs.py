"""Graph-captured iterations (the `graphs` option).

Each launch sequence of an iteration is captured once per workspace shape and
replayed many times (every iteration and trial of every later solve on the
handle).  The replays must give bitwise the same results as eager launches:
checked on repeated solves, with eager work of another handle between them, after
shape changes that force re-capture, for batches, warm starts and every precision.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


def same(r0, r1):
    assert r0.status == r1.status
    assert r0.iterations == r1.iterations and r0.ls_trials == r1.ls_trials
    assert np.array_equal(to_host(r0.A), to_host(r1.A))
    if r0.W is not None:
        assert np.array_equal(to_host(r0.W), to_host(r1.W))
    assert r0.objective == r1.objective and r0.kkt_rel1 == r1.kkt_rel1


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_graph_replays_equal_eager(g, precision):
    eager = g.Solver(precision=precision)
    graph = g.Solver(precision=precision, graphs=True)
    probs = []
    for n, seed in [(200, 1), (333, 2)]:
        S, _ = synth.random_sparse_problem(n, n // 2, seed)
        probs.append((to_dev(S), 0.25 * synth.lambda_max(S)))
    # repeated solves on one handle (replays), a shape change (re-capture) and back
    for St, lam in probs + probs[:1] + probs[1:] + probs[:1]:
        r_graph = graph.solve(St, lam, 1e-7)
        r_eager = eager.solve(St, lam, 1e-7)  # eager work between the replays
        same(r_eager, r_graph)


def test_graph_batched_and_warm_start(g):
    S, _ = synth.chain_problem(256, 128, 4)
    St = to_dev(S)
    lams = [0.12, 0.2, 0.3, 0.45]
    for _ in range(2):
        b_eager = g.Solver().solve_batched(St, lams, 1e-7)
        b_graph = g.Solver(graphs=True).solve_batched(St, lams, 1e-7)
        for r0, r1 in zip(b_eager, b_graph):
            same(r0, r1)
    # warm start from a neighbouring solution
    A0 = b_eager[1].A.clone()
    w_eager = g.Solver(warm_start=True).solve(St, 0.15, 1e-7, A=A0.clone())
    w_graph = g.Solver(warm_start=True, graphs=True).solve(St, 0.15, 1e-7, A=A0.clone())
    same(w_eager, w_graph)


def test_graph_lambda_path(g):
    S, _ = synth.random_sparse_problem(130, 65, 5)
    lams = list(synth.lambda_path(S, count=6, ratio=10.0))
    St = to_dev(S)
    p0 = g.lambda_path(St, lams, 1e-6, mode="waves", waves=3)
    p1 = g.lambda_path(St, lams, 1e-6, mode="waves", waves=3, graphs=True)
    for r0, r1 in zip(p0, p1):
        same(r0, r1)
