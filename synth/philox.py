"""Host implementation of the device workload generator (glasso_generate).

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011): a counter of four 32-bit words is enciphered with a
64-bit key in ten rounds; each round multiplies words 0 and 2 by the constants
0xD2511F53 and 0xCD9E8D57 (full 64-bit products), recombines the high and low
halves with words 1 and 3 and the key, and bumps the key by the Weyl constants
0x9E3779B9 and 0xBB67AE85.  The same words come out on the device, so the two
sides draw identical inputs.

Recipes (key = (seed mod 2^32, seed // 2^32)):
* random sparse precision: pair (i, j), i < j, counter (j, i, 0, 0); an edge when
  word 0 < floor(p 2^32), p = min(1, 10 / (n - 1)); value +-(0.5 + 0.5 (w2 + 0.5) 2^-32)
  with the sign from the low bit of word 1; A_ii = sum_j |A_ij| + 0.1;
* chain precision: A_ii = 1.25, A_{i,i+1} = -0.5;
* samples: z[r][c] from counter (c, r, 1, 0), Box-Muller of two 53-bit uniforms;
  sample r is L^{-T} z_r for A_true = L L^T.

Only input generation lives here: none of the solver's arithmetic.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10: counters and keys as arrays (or scalars) of
    32-bit values; returns the four output words as uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def _key(seed: int):
    seed = int(seed) & (2**64 - 1)
    return seed & 0xFFFFFFFF, seed >> 32


def edge_threshold(n: int) -> int:
    """floor(min(1, 10 / (n - 1)) 2^32), computed as the device computes it."""
    if n <= 11:
        return 1 << 32
    return int(np.floor(10.0 / float(n - 1) * 4294967296.0))


def device_precision(kind: str, n: int, seed: int = 0) -> np.ndarray:
    """The precision matrix glasso_generate draws ("random" or "chain"), dense FP64."""
    if kind == "chain":
        A = np.zeros((n, n))
        i = np.arange(n)
        A[i, i] = 1.25
        A[i[1:], i[:-1]] = -0.5
        A[i[:-1], i[1:]] = -0.5
        return A
    k0, k1 = _key(seed)
    i, j = np.triu_indices(n, 1)  # i < j
    w0, w1, w2, _ = philox4x32_10(j, i, 0, 0, k0, k1)
    edge = w0.astype(np.uint64) < np.uint64(edge_threshold(n))
    mag = 0.5 + 0.5 * ((w2.astype(np.float64) + 0.5) * 2.0 ** -32)
    val = np.where((w1 & 1) == 1, mag, -mag)
    A = np.zeros((n, n))
    A[i[edge], j[edge]] = val[edge]
    A[j[edge], i[edge]] = val[edge]
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + 0.1
    return A


def device_normals(m: int, n: int, seed: int = 0) -> np.ndarray:
    """The m x n standard normals glasso_generate draws for its samples."""
    k0, k1 = _key(seed)
    r, c = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    w0, w1, w2, w3 = philox4x32_10(c.ravel(), r.ravel(), 1, 0, k0, k1)
    u1 = ((w0 >> 5).astype(np.float64) * 67108864.0 + (w1 >> 6).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = ((w2 >> 5).astype(np.float64) * 67108864.0 + (w3 >> 6).astype(np.float64) + 0.5) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
    return z.reshape(m, n)


def device_samples(kind: str, n: int, m: int, seed: int = 0):
    """(Y, A_true): the m samples (rows of Y, x_r = L^{-T} z_r) and the precision
    matrix, as glasso_generate forms them."""
    A = device_precision(kind, n, seed)
    L = np.linalg.cholesky(A)
    Z = device_normals(m, n, seed)
    X = sla.solve_triangular(L.T, Z.T, lower=False)
    return np.ascontiguousarray(X.T), A
