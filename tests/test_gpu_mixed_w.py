"""The mixed-W ladder (glasso_options.w_mixed): W = V^T V with FP32 accuracy while a
problem iterates, FP64 W and measures before it stops.

* the FP32-accurate inverse itself: every product is formed from exact three-part
  bf16 splits of FP32 values, six partial products per pair, each exact in FP32,
  accumulated in FP32 (at most 6 roundings per inner index), with three dropped
  partial products below 2.1 u32 |x y|.  V = inv(L) by recursive doubling then
  carries the triangular-inverse bound |dV| <= c u32 |V||L||V|: the levels' products
  (inner dimensions s = 128, 256, ... summing to about 2n, six roundings each, plus
  3 per level) and the rounding of L and of the diagonal-block inverses to FP32 give
  c = 12n + 32.  W32 = V^T V differs from inv(A) by at most
  2 |V|^T |dV| + (6n + 3) u32 |V|^T |V|, checked elementwise with factor 2 slack
  (V and L computed on the CPU);
* solves in both mixed forms meet the FP64 bar against the oracle, and their
  reported KKT measure is the FP64 one (recomputed on the CPU from the returned A);
* the returned W is the FP64 inverse on every exit: converged, MAX_ITER and
  LS_FAILED (the last one forced from the host with t0 < t_min).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, random_spd, to_dev, to_host

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


@pytest.mark.parametrize("n", [64, 200, 513, 1100])
def test_fp32_w_product(g, n):
    A = random_spd(n, 6)
    W32 = to_host(g.Solver(w_mixed=1).inverse(to_dev(A)))
    L = np.linalg.cholesky(A)
    V = np.linalg.inv(L)
    ref = np.linalg.inv(A)
    aV = np.abs(V)
    dV = (12 * n + 32) * U32 * (aV @ np.abs(L) @ aV)
    bound = 2 * (2 * aV.T @ dV + (6 * n + 3) * U32 * (aV.T @ aV)) + 1e-300
    assert np.all(np.abs(W32 - ref) <= bound), np.max(np.abs(W32 - ref) / bound)
    assert np.max(np.abs(W32 - ref)) > 0  # really the FP32 product
    W64 = to_host(g.Solver(w_mixed=0).inverse(to_dev(A)))
    assert np.max(np.abs(W64 - ref)) <= 1e-10 * np.linalg.cond(A) * np.max(np.abs(ref))


def fp64_w(W, A):
    return np.max(np.abs(W @ A - np.eye(len(A)))) <= 1e-10 * np.linalg.cond(A)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,seed,frac", [(130, 1, 0.25), (300, 2, 0.2)])
def test_ladder_meets_fp64_bar(g, precision, n, seed, frac):
    S, _ = synth.random_sparse_problem(n, n // 2, seed)
    lam = frac * synth.lambda_max(S)
    tol = 1e-6
    r = g.Solver(precision=precision, w_mixed=1).solve(to_dev(S), lam, tol)
    assert r.status == g.CONVERGED
    A, W = to_host(r.A), to_host(r.W)
    ref = oracle.pista(S, lam, tol)
    chk = oracle.check_solution(S, A, lam)
    assert chk["kkt_rel1"] <= tol * 1.0001
    assert abs(r.kkt_rel1 - chk["kkt_rel1"]) <= 1e-6 * chk["kkt_rel1"]
    assert abs(r.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    assert fp64_w(W, A)


def test_ladder_exits_return_fp64_w(g):
    S, _ = synth.chain_problem(200, 100, 3)
    Sd = to_dev(S)
    r = g.Solver(precision="bf16x3", w_mixed=1, max_iter=2).solve(Sd, 0.15, 1e-12)
    assert r.status == g.MAX_ITER and r.iterations == 2
    A = to_host(r.A)
    assert fp64_w(to_host(r.W), A)
    assert abs(r.kkt_rel1 - oracle.check_solution(S, A, 0.15)["kkt_rel1"]) <= 1e-9
    r = g.Solver(precision="bf16x3", w_mixed=1, t0=1e-13, t_min=1e-12, t_floor=0.0).solve(Sd, 0.15, 1e-9)
    assert r.status == g.LS_FAILED and r.iterations == 0
    A = to_host(r.A)
    assert fp64_w(to_host(r.W), A)
    assert abs(r.kkt_rel1 - oracle.check_solution(S, A, 0.15)["kkt_rel1"]) <= 1e-9
