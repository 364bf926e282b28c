"""Seeded precision matrices and sample covariances (FP64, NumPy PCG64).

Workloads follow the paper's synthetic experiments (Sec. 6.1.1): a true sparse
precision matrix, m < n Gaussian samples drawn from N(0, A_true^{-1}), and the
empirical covariance S of eq. (empirical_cov).  The recipes fixed here:

* chain: A_ii = 1.25, A_{i,i+1} = A_{i+1,i} = -0.5 (a chain graph as in Sec.
  5.1.1, with the diagonal raised so the matrix is strictly diagonally dominant
  instead of adding the paper's eigenvalue shift).
* random sparse: 5n distinct pairs i<j drawn uniformly (about 10 off-diagonal
  nonzeros per row), values +-U(0.5, 1) with a random sign, and
  A_ii = sum_j |A_ij| + 0.1 (strictly diagonally dominant, hence PD).

Samples: x = L^{-T} z with A_true = L L^T and z ~ N(0, I), so Cov(x) = A_true^{-1}.
S = X^T X / m, uncentred: the mean is known to be zero.  The solver consumes S
as given.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def chain_precision(n: int, diag: float = 1.25, off: float = -0.5) -> np.ndarray:
    """Tridiagonal chain precision matrix (dense, FP64)."""
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = diag
    if n > 1:
        A[idx[:-1], idx[1:]] = off
        A[idx[1:], idx[:-1]] = off
    return A


def random_sparse_precision(n: int, seed: int, pairs_per_node: int = 5,
                            lo: float = 0.5, hi: float = 1.0,
                            shift: float = 0.1) -> np.ndarray:
    """Random sparse symmetric precision matrix, diagonally dominant (dense FP64)."""
    rng = _rng(seed)
    A = np.zeros((n, n))
    npairs = n * (n - 1) // 2
    k = min(pairs_per_node * n, npairs)
    if k > 0:
        lin = rng.choice(npairs, size=k, replace=False)
        # map a linear index over the strict upper triangle (row-major) to (i, j)
        iu, ju = np.triu_indices(n, 1)
        i, j = iu[lin], ju[lin]
        mag = rng.uniform(lo, hi, size=k)
        sgn = np.where(rng.integers(0, 2, size=k) == 0, -1.0, 1.0)
        v = sgn * mag
        A[i, j] = v
        A[j, i] = v
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + shift
    return A


def _samples_dense(A_true: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    n = A_true.shape[0]
    L = np.linalg.cholesky(A_true)
    Z = rng.standard_normal((n, m))
    X = sla.solve_triangular(L.T, Z, lower=False)  # n x m, columns are samples
    return X


def _samples_chain(n: int, m: int, rng: np.random.Generator, diag: float, off: float) -> np.ndarray:
    # banded Cholesky of the tridiagonal matrix, then solve L^T x = z (upper bidiagonal)
    ab = np.zeros((2, n))
    ab[0, :] = diag
    ab[1, :-1] = off
    cb = sla.cholesky_banded(ab, lower=True)  # cb[0] = diag(L), cb[1][:-1] = subdiag(L)
    up = np.zeros((2, n))                      # L^T in upper banded storage
    up[1, :] = cb[0]
    up[0, 1:] = cb[1, :-1]
    Z = rng.standard_normal((n, m))
    return sla.solve_banded((0, 1), up, Z)


def sample_covariance(X: np.ndarray) -> np.ndarray:
    """S = X X^T / m for X of shape n x m (columns are zero-mean samples)."""
    m = X.shape[1]
    S = (X @ X.T) / m
    # exact symmetry (BLAS may round the two triangles differently)
    S = np.tril(S) + np.tril(S, -1).T
    return S


def chain_problem(n: int, m: int, seed: int, diag: float = 1.25, off: float = -0.5):
    """(S, A_true) for the chain recipe."""
    rng = _rng(seed)
    X = _samples_chain(n, m, rng, diag, off)
    return sample_covariance(X), chain_precision(n, diag, off)


def planar_precision(n: int, seed: int, shift: float = 0.1) -> np.ndarray:
    """Planar-graph precision (Sec. 6.1.1): the graph Laplacian of a Delaunay
    triangulation of n uniform points in the unit square (A_ij = -1 on edges,
    A_ii = degree) plus shift * I.  The Laplacian's smallest eigenvalue is 0, so
    the paper's diagonal term max(-1.2 lambda_min, 0.1) is 0.1."""
    from scipy.spatial import Delaunay

    rng = _rng(seed)
    pts = rng.uniform(size=(n, 2))
    A = np.zeros((n, n))
    for a, b, c in Delaunay(pts).simplices:
        for i, j in ((a, b), (b, c), (a, c)):
            A[i, j] = A[j, i] = -1.0
    A[np.arange(n), np.arange(n)] = -A.sum(axis=1) + shift
    return A


def support_samples(kind: str, n: int, m: int, seed: int):
    """(X, A_true) with X (n x m) the m samples as columns, for the ground truths
    of the support-recovery sweep: "chain" (chain_precision), "random"
    (random_sparse_precision) and "planar" (planar_precision)."""
    if kind == "chain":
        return _samples_chain(n, m, _rng(seed + 1_000_003), 1.25, -0.5), chain_precision(n)
    A_true = random_sparse_precision(n, seed) if kind == "random" else planar_precision(n, seed)
    return _samples_dense(A_true, m, _rng(seed + 1_000_003)), A_true


def random_sparse_samples(n: int, m: int, seed: int):
    """(X, A_true) for the random-sparse recipe: X (n x m) holds the m samples as
    columns.  The precision structure and the samples come from two streams
    derived from the same seed."""
    A_true = random_sparse_precision(n, seed)
    rng = _rng(seed + 1_000_003)
    return _samples_dense(A_true, m, rng), A_true


def random_sparse_problem(n: int, m: int, seed: int):
    """(S, A_true) for the random-sparse recipe (S from random_sparse_samples)."""
    X, A_true = random_sparse_samples(n, m, seed)
    return sample_covariance(X), A_true


def lambda_max(S: np.ndarray) -> float:
    """max_{i != j} |S_ij|: for lambda at or above it the solution is diagonal."""
    n = S.shape[0]
    if n < 2:
        return 0.0
    off = np.abs(S - np.diag(np.diag(S)))
    return float(off.max())


def lambda_path(S: np.ndarray, count: int = 32, ratio: float = 100.0) -> np.ndarray:
    """Geometric regularisation path from lambda_max down to lambda_max / ratio."""
    lm = lambda_max(S)
    k = np.arange(count)
    return lm * ratio ** (-k / (count - 1))


def serving_requests(count: int, seed: int, n_lo: int = 64, n_hi: int = 4096,
                     rate: float = 1.0):
    """Poisson arrival stream: list of (arrival_time_s, n, request_seed).
    n is log-uniform in [n_lo, n_hi]; arrival gaps are exponential with mean 1/rate."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    n = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(int)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [(float(t[i]), int(n[i]), int(seeds[i])) for i in range(count)]
