"""GEMM tile policy and the autotuner.

The FP64 GEMMs run 128x128 or 64x64 output tiles; both accumulate every output
over k in the same order through the same MFMA instruction, so every result
(factor, inverse, A Z A, whole solves, batches) must be bitwise identical under
every tile policy.  The autotuner must return one of its candidates and be used
by later solves (no change in results either).
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import device, random_spd, to_dev, to_host

pytestmark = pytest.mark.gpu

NEVER, ALWAYS = 0, 1 << 30
CANDIDATES = {0, 64, 256, 1024, 1 << 30}


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


@pytest.mark.parametrize("n", [64, 200, 513, 1100])
def test_factor_inverse_product_tile_independent(g, n):
    A = random_spd(n, 4)
    rng = np.random.default_rng(5)
    Z = rng.standard_normal((n, n))
    Z = Z + Z.T
    out = []
    for pol in (NEVER, ALWAYS, 256):
        s = g.Solver(tile_policy=pol)
        L, info, logdet = s.cholesky(to_dev(A))
        W = s.inverse(to_dev(A))
        P = s.precond_product(to_dev(A), to_dev(Z))
        out.append((to_host(L), info, logdet, to_host(W), to_host(P)))
        s.close()
    for o in out[1:]:
        assert np.array_equal(o[0], out[0][0])
        assert o[1] == out[0][1] and o[2] == out[0][2]
        assert np.array_equal(o[3], out[0][3])
        assert np.array_equal(o[4], out[0][4])


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_solve_tile_independent(g, precision):
    S, _ = synth.random_sparse_problem(300, 150, 7)
    lam = 0.25 * synth.lambda_max(S)
    St = to_dev(S)
    res = [g.Solver(precision=precision, tile_policy=p).solve(St, lam, 1e-7) for p in (NEVER, ALWAYS)]
    assert res[0].iterations == res[1].iterations and res[0].ls_trials == res[1].ls_trials
    assert np.array_equal(to_host(res[0].A), to_host(res[1].A))
    assert np.array_equal(to_host(res[0].W), to_host(res[1].W))


def test_batch_tile_independent(g):
    S, _ = synth.chain_problem(256, 128, 3)
    St = to_dev(S)
    lams = [0.15, 0.2, 0.3]
    b0 = g.Solver(tile_policy=NEVER).solve_batched(St, lams, 1e-7)
    b1 = g.Solver(tile_policy=ALWAYS).solve_batched(St, lams, 1e-7)
    for r0, r1 in zip(b0, b1):
        assert np.array_equal(to_host(r0.A), to_host(r1.A))


def test_autotune(g):
    S, _ = synth.chain_problem(700, 350, 1)
    St = to_dev(S)
    s = g.Solver()
    pol = s.autotune(700)
    assert pol in CANDIDATES
    assert s.autotune(700, count=3) in CANDIDATES
    # a solve under the tuned policy equals one under a fixed policy
    r_auto = s.solve(St, 0.2, 1e-7)
    r_fix = g.Solver(tile_policy=NEVER).solve(St, 0.2, 1e-7)
    assert np.array_equal(to_host(r_auto.A), to_host(r_fix.A))
