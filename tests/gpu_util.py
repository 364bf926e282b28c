"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import numpy as np
import pytest
import torch

EPS = np.finfo(np.float64).eps


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device(), dtype=dtype)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sym(X):
    return np.tril(X) + np.tril(X, -1).T


def random_spd(n, seed, shift=1.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, max(2, n // 2)))
    return sym(X @ X.T / X.shape[1] + shift * np.eye(n))


def sparse_sym(n, seed, density=0.1, diag=2.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    A = sym(A)
    A[np.arange(n), np.arange(n)] = diag + rng.random(n)
    return A


def support_mismatch(A_gpu, A_ref, g_ref, lam, eps=1e-8):
    """Entries whose zero/nonzero status differs, except those within eps of the
    threshold in the reference solution: a nonzero with |A*_ij| <= eps, or a zero
    with ||g*_ij| - lam| <= eps."""
    diff = (A_gpu != 0) != (A_ref != 0)
    nz = A_ref != 0
    exempt = (nz & (np.abs(A_ref) <= eps)) | (~nz & (np.abs(np.abs(g_ref) - lam) <= eps))
    return int(np.sum(diff & ~exempt))
