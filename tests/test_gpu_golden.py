"""Parity of the GPU path with the stored oracle solutions of the benchmark workloads
(tests/golden/*.npz: the oracle run to KKT <= 1e-8 by tests/golden/make_references.py).

Bar (FP64 path, and the mixed forms, whose every decision is FP64):
  * |F - F*| <= 1e-8 max(1, |F*|);
  * the KKT measure of the returned A recomputed by the oracle <= tol;
  * the lower-triangle support equals the oracle's except the stored threshold
    exemptions (a nonzero within 1e-8 of zero, a zero whose gradient is within 1e-8
    of lambda).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests import golden_ref
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


def meets_bar(S, lam, tol, res, ref, g):
    assert res.status == g.CONVERGED, res.status_name
    A = to_host(res.A)
    chk = oracle.check_solution(S, A, lam)
    assert chk["pd"] and chk["kkt_rel1"] <= tol * 1.0001, chk.get("kkt_rel1")
    relF, mism, _ = golden_ref.compare(A, res.objective, ref)
    assert relF <= 1e-8, relF
    assert mism == 0, mism
    return relF


@pytest.mark.parametrize("seed", range(5))
def test_chain_n100_against_stored_oracle(g, seed):
    """Chain n = 100, m = 50, lambda 0.2, tol 1e-6 (the smallest workload), FP64."""
    ref = golden_ref.load("chain100")[seed]
    S, _ = synth.chain_problem(100, 50, seed)
    res = g.Solver().solve(to_dev(S), 0.2, 1e-6)
    meets_bar(S, 0.2, 1e-6, res, ref, g)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_random_n2000_against_stored_oracle(g, precision):
    """Random sparse n = 2000, m = 1000, the frozen lambda (nnz ~ 5n), tol 1e-5: the
    FP64 path and both mixed forms."""
    with open(os.path.join(HERE, "golden", "workloads.json")) as f:
        w = json.load(f)["random_sparse_n2000"]
    ref = golden_ref.load("random2000")[0]
    assert float(ref["lam"]) == w["lambda"]
    S, _ = synth.random_sparse_problem(w["n"], w["m"], w["seed"])
    res = g.Solver(precision=precision).solve(to_dev(S), w["lambda"], w["tol"])
    meets_bar(S, w["lambda"], w["tol"], res, ref, g)
    assert res.nnz == 2 * len(ref["rows"]) - w["n"]  # the oracle's support, counted in full
