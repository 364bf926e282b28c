"""Support recovery (the experiment of Sec. 6.3, Fig. 2): Matthews correlation
coefficient of the estimated sparsity pattern against the ground truth, over a
lambda grid, for the chain, random and planar ground truths.

CPU: the ground-truth generators and the MCC formula on worked cases.
GPU: the device path (sample covariance + one batched solve over the lambda grid)
against the oracle path (empirical covariance + one oracle solve per lambda) on
the same samples: the same support up to entries that either solution puts
within 1e-6 of zero, and the same MCC to 1e-2."""
import numpy as np
import pytest

import oracle
import synth


def mcc(A_est, A_true, zero=0.0):
    """MCC over the pairs i < j: positive = nonzero entry."""
    iu = np.triu_indices(A_true.shape[0], 1)
    e = np.abs(A_est[iu]) > zero
    t = A_true[iu] != 0
    tp, tn = float(np.sum(e & t)), float(np.sum(~e & ~t))
    fp, fn = float(np.sum(e & ~t)), float(np.sum(~e & t))
    den = np.sqrt((tp + fp) * (tp + fn) * (tn + fp) * (tn + fn))
    return (tp * tn - fp * fn) / den if den > 0 else 0.0


def test_mcc_worked_cases():
    T = np.array([[2.0, 1, 0, 0], [1, 2, 1, 0], [0, 1, 2, 1], [0, 0, 1, 2]])  # 3 edges of 6 pairs
    assert mcc(T, T) == 1.0
    assert mcc(np.where(T != 0, 0.0, 1.0) + np.eye(4), T) == -1.0
    E = T.copy()
    E[0, 2] = E[2, 0] = 0.5  # one false positive: TP 3, TN 2, FP 1, FN 0
    assert abs(mcc(E, T) - (3 * 2 - 0) / np.sqrt(4 * 3 * 3 * 2)) < 1e-15


def test_ground_truths():
    P = synth.planar_precision(300, 3)
    assert np.array_equal(P, P.T)
    np.testing.assert_allclose(P.sum(axis=1), 0.1, atol=1e-12)  # Laplacian rows + shift
    edges = (np.count_nonzero(P) - 300) // 2
    assert 300 <= edges <= 3 * 300 - 6  # a triangulation of points in general position
    assert np.linalg.eigvalsh(P).min() > 0.099
    for kind in ("chain", "random", "planar"):
        X, A = synth.support_samples(kind, 120, 60, 5)
        assert X.shape == (120, 60) and np.linalg.eigvalsh(A).min() > 0


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["chain", "random", "planar"])
def test_device_path_matches_oracle(kind):
    from tests.gpu_util import device, to_dev, to_host

    device()
    import paper_2205_10027_amd as g

    n, m = 120, 60
    X, A_true = synth.support_samples(kind, n, m, 7)
    Y = np.ascontiguousarray(X.T)
    s = g.Solver()
    S_dev = s.covariance(to_dev(Y), center=True)
    S_ref = oracle.empirical_covariance(Y, center=True)
    lm = float(np.max(np.abs(S_ref - np.diag(np.diag(S_ref)))))
    lams = [lm * 2.0 ** (-k / 2) for k in range(1, 7)]
    res = s.solve_batched(S_dev, lams, 1e-6)
    for lam, r in zip(lams, res):
        assert r.status == g.CONVERGED
        A_gpu = to_host(r.A)
        A_ref = oracle.pista(S_ref, lam, 1e-6).A
        clear = (np.abs(A_gpu) > 1e-6) | (np.abs(A_ref) > 1e-6)
        near = (np.abs(A_gpu) <= 1e-6) | (np.abs(A_ref) <= 1e-6)
        differ = (A_gpu != 0) != (A_ref != 0)
        assert not np.any(differ & clear & ~near)
        assert abs(mcc(A_gpu, A_true) - mcc(A_ref, A_true)) <= 1e-2
    s.close()
