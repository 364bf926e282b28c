"""The host side of the workload generator (synth/philox.py), pinned on the CPU:
the counter-based generator against its published known-answer vectors, and the
recipes' defining properties."""
import numpy as np

from synth import philox


def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors published with the generator's reference
    implementation (Random123): zero counter and key, all-ones counter and key, and
    the digits of pi."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = philox.philox4x32_10(*ctr, *key)
        assert tuple(int(x) for x in got) == want


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2**32, size=(4, 50), dtype=np.uint64)
    k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
    vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1])
    for t in (0, 17, 49):
        one = philox.philox4x32_10(c[0, t], c[1, t], c[2, t], c[3, t], k[0], k[1])
        assert all(int(v[t]) == int(o) for v, o in zip(vec, one))


def test_random_precision_recipe():
    n = 2000
    A = philox.device_precision("random", n, seed=7)
    assert np.array_equal(A, A.T)
    off = A - np.diag(np.diag(A))
    vals = np.abs(off[off != 0])
    assert vals.min() >= 0.5 and vals.max() < 1.0
    per_row = np.count_nonzero(off, axis=1)
    assert abs(per_row.mean() - 10.0) < 0.3  # about ten off-diagonal nonzeros per row
    # strictly diagonally dominant by 0.1, hence positive definite
    np.testing.assert_allclose(np.diag(A) - np.abs(off).sum(axis=1), 0.1, rtol=0, atol=1e-12)
    assert np.linalg.eigvalsh(A[:300, :300]).min() > 0
    # both signs, about equally often; another seed draws another matrix
    assert 0.45 < np.mean(off[off != 0] > 0) < 0.55
    assert not np.array_equal(A, philox.device_precision("random", n, seed=8))
    # small n: every pair is an edge (p = min(1, 10 / (n - 1)))
    B = philox.device_precision("random", 6, seed=1)
    assert np.count_nonzero(B) == 36
    assert np.array_equal(philox.device_precision("random", 1, seed=1), np.array([[0.1]]))


def test_chain_recipe_and_samples():
    A = philox.device_precision("chain", 5)
    assert A[0, 0] == 1.25 and A[1, 0] == -0.5 and A[2, 0] == 0.0 and np.array_equal(A, A.T)
    Z = philox.device_normals(4000, 30, seed=3)
    assert abs(Z.mean()) < 0.01 and abs(Z.var() - 1.0) < 0.02
    assert abs(np.corrcoef(Z[:, 0], Z[:, 1])[0, 1]) < 0.05
    # samples: the empirical covariance approaches A_true^{-1}
    Y, Atrue = philox.device_samples("random", 30, 20000, seed=5)
    C = Y.T @ Y / Y.shape[0]
    W = np.linalg.inv(Atrue)
    assert np.abs(C - W).max() < 0.08 * np.abs(W).max()
