"""Sample covariance on the device (glasso_covariance, eq. empirical_cov) against
the oracle's empirical_covariance, element by element within a rounding bound.

Bound: the device sums each column mean over m/4 + 3 terms (four interleaved
partial sums) and each entry of S over the padded sample count in FP64, so with
u = 2^-53, e_j = (m/4 + 4) u mean_i |Y_ij| (centring only) and C = |Yc|^T |Yc| / m:
    |S - S_ref| <= 2 (m + 4) u C_jk + 2 (e_j mean|Yc_k| + mean|Yc_j| e_k) + e_j e_k,
doubled for slack (the oracle's own rounding is of the same order)."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def solver():
    device()
    import paper_2205_10027_amd as g

    s = g.Solver()
    yield s
    s.close()


def bound(Y, center):
    m = Y.shape[0]
    mu = Y.mean(axis=0) if center else np.zeros(Y.shape[1])
    Yc = np.abs(Y - mu)
    C = Yc.T @ Yc / m
    e = (m / 4 + 4) * U * np.abs(Y).mean(axis=0) if center else np.zeros(Y.shape[1])
    a = Yc.mean(axis=0)
    return 2 * (2 * (m + 4) * U * C + 2 * (np.outer(e, a) + np.outer(a, e)) + np.outer(e, e)) + 1e-300


def samples(m, n, offset, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * rng.uniform(0.5, 2.0, size=n) + offset


@pytest.mark.parametrize("m,n,center,offset", [(1, 5, True, 0.0), (1, 5, False, 0.0), (37, 5, True, 3.0),
                                               (300, 130, True, -2.0), (1000, 1100, False, 0.0),
                                               (250, 2100, True, 1.5), (2, 1, True, 4.0)])
def test_covariance_matches_oracle(solver, m, n, center, offset):
    Y = samples(m, n, offset, seed=m + n)
    S = to_host(solver.covariance(to_dev(Y), center=center))
    ref = oracle.empirical_covariance(Y, center=center)
    err = np.abs(S - ref)
    b = bound(Y, center)
    assert np.all(err <= b), float(np.max(err / b))
    assert np.array_equal(S, S.T)
    if m == 1 and center:
        assert np.all(S == 0.0)


def test_covariance_deterministic_and_reuses_workspace(solver):
    Y = to_dev(samples(400, 300, 1.0, 3))
    S1 = solver.covariance(Y)
    solver.covariance(to_dev(samples(900, 700, 0.0, 4)))  # a larger call in between
    S2 = solver.covariance(Y)
    assert torch.equal(S1, S2)


def test_covariance_full_size_sampled(solver):
    """The config-2 sample shape, m = 5000 samples of n = 10000 variables (not
    centred, and centred with a mean offset): 400 sampled entries against the
    definition evaluated for those entries alone."""
    m, n = 5000, 10000
    Y = samples(m, n, 0.0, 11)
    Yd = to_dev(Y)
    rng = np.random.default_rng(5)
    j = rng.integers(0, n, 400)
    k = rng.integers(0, n, 400)
    j[:4], k[:4] = [0, n - 1, n - 1, 5000], [0, n - 1, 0, 4999]
    for center, off in ((False, 0.0), (True, 2.5)):
        Yo = Y + off
        S = solver.covariance(to_dev(Yo) if off else Yd, center=center)
        got = to_host(S[torch.as_tensor(j, device=S.device), torch.as_tensor(k, device=S.device)])
        cols = np.unique(np.concatenate([j, k]))
        Ys = Yo[:, cols]
        mu = Ys.mean(axis=0) if center else np.zeros(len(cols))
        Yc = Ys - mu
        pos = {c: i for i, c in enumerate(cols)}
        ji = np.array([pos[x] for x in j])
        ki = np.array([pos[x] for x in k])
        ref = np.einsum("ij,ij->j", Yc[:, ji], Yc[:, ki]) / m
        b = bound(Ys, center)[ji, ki]
        err = np.abs(got - ref)
        assert np.all(err <= b), float(np.max(err / b))
        del S
