"""Device workload generator (glasso_generate) against its host implementation
(synth/philox.py: the same Philox4x32-10 counters), and solves of generated
problems against the oracle.

Bars: structure and off-diagonal values bit-exact (integer decisions and exact
FP64 operations on both sides); the diagonal (a sum of |A_ij| in another order)
to 1e-14 relative; the samples (device log/cos against the host library's, then
a triangular solve) to 1e-11 of max |Y|; S against the oracle's covariance of the
returned samples to 1e-13 of max |S|; lambda_max exactly the largest off-diagonal
|S_ij| of the returned S.
"""
import ctypes

import numpy as np
import pytest

import oracle
from synth import philox
from tests.gpu_util import device, support_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    device()
    import paper_2205_10027_amd as g

    return g


@pytest.mark.parametrize("n", [1, 6, 130, 300, 1000])
def test_precision_matches_host(g, n):
    s = g.Solver()
    A, _, _, _ = s.generate("random", n, seed=11, want_A=True, want_S=False)
    A = to_host(A)
    H = philox.device_precision("random", n, seed=11)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(A[off], H[off])
    np.testing.assert_allclose(np.diag(A), np.diag(H), rtol=1e-14, atol=0)
    C, _, _, _ = s.generate("chain", n, want_A=True, want_S=False)
    assert np.array_equal(to_host(C), philox.device_precision("chain", n))
    s.close()


@pytest.mark.parametrize("kind,n,m,seed", [("random", 130, 65, 3), ("random", 300, 150, 2**40 + 5),
                                           ("chain", 257, 7, 9), ("random", 5, 1, 1)])
def test_samples_and_covariance_match_host(g, kind, n, m, seed):
    s = g.Solver()
    A, Y, S, lm = s.generate(kind, n, m, seed=seed, want_A=True, want_Y=True, want_S=True)
    Y, S = to_host(Y), to_host(S)
    Yh, _ = philox.device_samples(kind, n, m, seed=seed)
    assert np.abs(Y - Yh).max() <= 1e-11 * np.abs(Yh).max()
    Sref = oracle.empirical_covariance(Y, center=False)
    assert np.abs(S - Sref).max() <= 1e-13 * np.abs(Sref).max()
    assert np.array_equal(S, S.T)
    off = S[~np.eye(n, dtype=bool)]
    assert lm == (np.abs(off).max() if off.size else 0.0)
    s.close()


def test_generated_problem_solves_to_oracle_bar(g):
    """A random sparse problem drawn on the device (n = 300, m = 150), solved from
    the device S: F to 1e-8 of the oracle, its KKT measure and support."""
    s = g.Solver()
    _, _, S, lm = s.generate("random", 300, 150, seed=21)
    lam = 0.3 * lm
    Sh = to_host(S)
    res = s.solve(S, lam, 1e-7)
    assert res.status == g.CONVERGED
    A = to_host(res.A)
    ref = oracle.pista(Sh, lam, 1e-7)
    chk = oracle.check_solution(Sh, A, lam)
    assert chk["kkt_rel1"] <= 1e-7 * 1.0001
    assert abs(res.objective - ref.objective) <= 1e-8 * max(1.0, abs(ref.objective))
    assert support_mismatch(A, ref.A, oracle.check_solution(Sh, ref.A, lam)["g"], lam) == 0
    s.close()


def test_generate_rejects_bad_arguments(g):
    s = g.Solver()
    lib = g._lib
    out = to_dev(np.zeros((4, 4)))
    p = out.data_ptr()
    assert lib.glasso_generate(s._h, 2, 4, 2, 0, p, None, None, None, None) == 1   # unknown kind
    assert lib.glasso_generate(s._h, 0, 0, 2, 0, p, None, None, None, None) == 1   # n < 1
    assert lib.glasso_generate(s._h, 0, 4, 2, 0, None, None, None, None, None) == 1  # no output
    assert lib.glasso_generate(s._h, 0, 4, 0, 0, None, None, p, None, None) == 1   # samples without m
    lm = ctypes.c_double()
    assert lib.glasso_generate(None, 0, 4, 2, 0, None, None, None, ctypes.byref(lm), None) == 1
    s.close()
