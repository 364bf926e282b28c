"""Step-level parity of the HIP kernels against the CPU oracle (through the C ABI).

Tolerances:
  * elementwise passes (gradient/sign/Z, trial point): identical IEEE operations
    in both implementations -> bit-exact outputs for identical inputs;
  * sums over n^2 terms: summation order differs -> relative 1e-12;
  * A Z A: each entry is two length-n dot products; the textbook bound is
    |fl(AZA) - AZA| <= 2 n eps (|A||Z||A|) (elementwise), checked with factor 2 slack;
  * Cholesky: backward error |L L^T - A| <= 2 n eps |L||L^T| (factor 2 slack);
  * inverse: |W - inv(A)| <= c n eps cond(A) |inv(A)|_max with c = 4.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import EPS, device, random_spd, sparse_sym, sym, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [1, 5, 64, 128, 130, 300, 513]


@pytest.fixture(scope="module")
def solver():
    device()
    import paper_2205_10027_amd as g

    s = g.Solver()
    yield s
    s.close()


# ------------------------------------------------------------------ A Z A (MFMA GEMMs)
@pytest.mark.parametrize("n", SIZES + [1024])
def test_precond_product_fp64(solver, n):
    A = sparse_sym(n, 1, density=0.3)
    rng = np.random.default_rng(2)
    Z = sym(rng.standard_normal((n, n)))
    P = to_host(solver.precond_product(to_dev(A), to_dev(Z)))
    ref = A @ Z @ A
    bound = 4 * n * EPS * (np.abs(A) @ np.abs(Z) @ np.abs(A)) + 1e-300
    assert np.all(np.abs(P - ref) <= bound), np.max(np.abs(P - ref) / bound)
    assert np.array_equal(P, P.T)


@pytest.mark.parametrize("n", [5, 300, 1024, 8320])
def test_precond_product_fp64_diagonal_A(solver, n):
    """For a diagonal A every entry of the FP64 GEMM pair is one rounded product per
    GEMM, (A_ii Z_ij) A_jj, the other terms being exact zeros: the elementwise D Z D
    the solver uses for the first product of a diagonal start rounds the same way."""
    rng = np.random.default_rng(5)
    d = rng.uniform(0.1, 3.0, n)
    Z = sym(rng.standard_normal((n, n)))
    P = to_host(solver.precond_product(to_dev(np.diag(d)), to_dev(Z)))
    ref = (d[:, None] * Z) * d[None, :]
    assert np.array_equal(np.tril(P), np.tril(ref))


@pytest.mark.parametrize("n", [5, 128, 300, 1024])
def test_precond_product_fp32(solver, n):
    """FP32 MFMA product: inputs rounded to FP32 (relative 2^-24) and FP32
    accumulation over two length-n dot products -> 4 n u32 (|A||Z||A|)."""
    A = sparse_sym(n, 1, density=0.3)
    rng = np.random.default_rng(2)
    Z = sym(rng.standard_normal((n, n)))
    P = to_host(solver.precond_product(to_dev(A), to_dev(Z), precision="fp32"))
    ref = A @ Z @ A
    u32 = 2.0 ** -24
    bound = 4 * (n + 2) * u32 * (np.abs(A) @ np.abs(Z) @ np.abs(A)) + 1e-300
    assert np.all(np.abs(P - ref) <= bound), np.max(np.abs(P - ref) / bound)
    assert np.array_equal(P, P.T)
    # and it is not secretly the FP64 product
    assert np.max(np.abs(P - ref)) > 0


@pytest.mark.parametrize("n", [5, 128, 300, 1024, 2048, 2100])
def test_precond_product_bf16x3(solver, n):
    """BF16x3 product.  Splitting x = hi + lo leaves |x - hi - lo| <= 2^-16 |x|
    (two bf16 roundings, unit roundoff 2^-8 each); the dropped lo*lo term is
    <= 2^-16 |a b|; so one product carries 3 * 2^-16 relative to |a||b| plus the
    FP32 accumulation n u32.  X = A Z is split again (2^-16) before X A, so
    |P - A Z A| <= (7 * 2^-16 + 2 (n + 2) u32) (|A||Z||A|), checked with factor 2 slack."""
    A = sparse_sym(n, 1, density=0.3)
    rng = np.random.default_rng(2)
    Z = sym(rng.standard_normal((n, n)))
    P = to_host(solver.precond_product(to_dev(A), to_dev(Z), precision="bf16x3"))
    ref = A @ Z @ A
    u32 = 2.0 ** -24
    bound = 2 * (7 * 2.0 ** -16 + 2 * (n + 2) * u32) * (np.abs(A) @ np.abs(Z) @ np.abs(A)) + 1e-300
    assert np.all(np.abs(P - ref) <= bound), np.max(np.abs(P - ref) / bound)
    assert np.array_equal(P, P.T)
    assert np.max(np.abs(P - ref)) > 0


@pytest.mark.parametrize("precision,n", [("fp64", 256), ("fp32", 256), ("bf16x3", 256), ("bf16x3", 2100)])
def test_precond_product_structure(solver, precision, n):
    """Identity and permutation cases pin the MFMA lane layout exactly (small
    integers are exact in every form; n = 2100 pads to 17 tiles of 128, an odd
    count, with 52 rows of padding in the last)."""
    rng = np.random.default_rng(3)
    Z = sym(rng.integers(-3, 4, size=(n, n)).astype(np.float64))
    P = to_host(solver.precond_product(to_dev(np.eye(n)), to_dev(Z), precision=precision))
    assert np.array_equal(P, Z)
    perm = rng.permutation(n)
    Pm = np.eye(n)[perm]
    Pm = sym(Pm + Pm.T)  # symmetric 0/1/2 matrix
    P = to_host(solver.precond_product(to_dev(Pm), to_dev(Z), precision=precision))
    assert np.array_equal(P, Pm @ Z @ Pm)


# ------------------------------------------------------------------ Cholesky / inverse
@pytest.mark.parametrize("n", SIZES + [1100, 2100])
def test_cholesky(solver, n):
    A = random_spd(n, n)
    L, info, logdet = solver.cholesky(to_dev(A))
    L = to_host(L)
    assert info == 0
    assert np.all(np.triu(L, 1) == 0)
    back = np.abs(L @ L.T - A)
    bound = 4 * n * EPS * (np.abs(L) @ np.abs(L.T)) + 1e-300
    assert np.all(back <= bound), np.max(back / bound)
    sign, ld = np.linalg.slogdet(A)
    assert abs(logdet - ld) <= 1e-12 * max(1.0, abs(ld)) * n


@pytest.mark.parametrize("n", [2300, 3000])
def test_cholesky_left_looking_dense(solver, n):
    """Dense SPD above a padded size of 2048: the blocks of each 512-wide middle
    panel update each other inside the leaf steps (left-looking, K up to 384);
    backward error bound as for test_cholesky."""
    A = random_spd(n, n)
    L, info, logdet = solver.cholesky(to_dev(A))
    L = to_host(L)
    assert info == 0
    assert np.all(np.triu(L, 1) == 0)
    back = np.abs(L @ L.T - A)
    bound = 4 * n * EPS * (np.abs(L) @ np.abs(L.T)) + 1e-300
    assert np.all(back <= bound), np.max(back / bound)
    sign, ld = np.linalg.slogdet(A)
    assert abs(logdet - ld) <= 1e-12 * max(1.0, abs(ld)) * n


def banded_spd(n, seed, band):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for off in range(1, band + 1):
        A[np.arange(n - off), np.arange(off, n)] = rng.uniform(-0.5, 0.5, n - off) / band
    A = A + A.T
    A[np.arange(n), np.arange(n)] = 2.0 + rng.random(n)
    return A


def block_sparse_spd(n, seed):
    """SPD with most 128x128 blocks zero: dense diagonal blocks plus a few far
    off-diagonal ones (their fill-in creates more nonzero blocks below)."""
    rng = np.random.default_rng(seed)
    nb = (n + 127) // 128
    X = np.zeros((n, n))
    for i in range(nb):
        for j in [i] + list(rng.choice(nb, 2)):
            r, c = slice(128 * i, min(n, 128 * i + 128)), slice(128 * j, min(n, 128 * j + 128))
            X[r, c] = rng.standard_normal((X[r, c].shape)) * (rng.random(X[r, c].shape) < 0.2)
    return sym(X @ X.T / 64.0 + np.eye(n))


@pytest.mark.parametrize("n", [300, 1100, 2100])
@pytest.mark.parametrize("kind", ["band1", "band40", "blocks"])
def test_cholesky_zero_blocks(solver, n, kind):
    """Banded and block-sparse matrices: the updates skip tiles whose operand blocks
    are zero; the factor still matches A to the dense bound and keeps L's zero blocks."""
    A = block_sparse_spd(n, n) if kind == "blocks" else banded_spd(n, n, int(kind[4:]))
    L, info, logdet = solver.cholesky(to_dev(A))
    L = to_host(L)
    assert info == 0
    assert np.all(np.triu(L, 1) == 0)
    back = np.abs(L @ L.T - A)
    bound = 4 * n * EPS * (np.abs(L) @ np.abs(L.T)) + 1e-300
    assert np.all(back <= bound), np.max(back / bound)
    ref = np.linalg.cholesky(A)
    assert np.max(np.abs(L - ref)) <= 1e-12 * np.max(np.abs(ref))
    if kind.startswith("band"):
        assert np.all(np.tril(L, -int(kind[4:]) - 1) == 0)  # no fill outside the band
    sign, ld = np.linalg.slogdet(A)
    assert abs(logdet - ld) <= 1e-12 * max(1.0, abs(ld)) * n


@pytest.mark.parametrize("n", [300, 520, 1100, 2300, 4500])
def test_cholesky_scattered_sparse(solver, n):
    """A scattered sparse SPD matrix (random off-diagonal pattern, diagonally
    dominant, like the solver's iterates): the update tiles and, above a padded size
    of 2048 (n = 2300, 4500), the leaf steps' left-looking updates skip the 16x16
    blocks that are zero and keep the others, wherever in a block the nonzeros sit.
    Factor against numpy."""
    rng = np.random.default_rng(n + 3)
    A = np.zeros((n, n))
    i, j = rng.integers(0, n, 6 * n), rng.integers(0, n, 6 * n)
    A[i, j] = rng.uniform(-1.0, 1.0, 6 * n)
    A = sym(np.tril(A, -1))
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + 0.1
    L, info, logdet = solver.cholesky(to_dev(A))
    L = to_host(L)
    assert info == 0
    ref = np.linalg.cholesky(A)
    assert np.max(np.abs(L - ref)) <= 1e-12 * np.max(np.abs(ref))
    sign, ld = np.linalg.slogdet(A)
    assert abs(logdet - ld) <= 1e-12 * max(1.0, abs(ld)) * n


@pytest.mark.parametrize("n,bad", [(5, 3), (300, 200), (1100, 1030), (130, 129)])
def test_cholesky_reports_first_bad_pivot(solver, n, bad):
    A = np.eye(n)
    A[bad - 1, bad - 1] = -1.0
    _, info, _ = solver.cholesky(to_dev(A))
    assert info == bad
    A = random_spd(n, 7)
    A[bad - 1, bad - 1] = np.nan
    _, info, _ = solver.cholesky(to_dev(A))
    assert info == bad


@pytest.mark.parametrize("n", SIZES + [1100])
def test_inverse(solver, n):
    A = random_spd(n, n + 11)
    W = to_host(solver.inverse(to_dev(A)))
    ref = np.linalg.inv(A)
    cond = np.linalg.cond(A)
    assert np.array_equal(W, W.T)
    assert np.max(np.abs(W - ref)) <= 4 * n * EPS * cond * np.max(np.abs(ref))


def test_inverse_not_pd(solver):
    import paper_2205_10027_amd as g

    A = -np.eye(10)
    with pytest.raises(g.GlassoError) as e:
        solver.inverse(to_dev(A))
    assert e.value.code == 2


# ------------------------------------------------------------------ gradient pass
def _grad_inputs(n, seed, lam):
    rng = np.random.default_rng(seed)
    A = sparse_sym(n, seed, density=0.2)
    S = sym(rng.standard_normal((n, n)) * 0.5)
    W = sym(rng.standard_normal((n, n)) * 0.5)
    # plant exact ties |g| = lam and g = 0 off the support
    if n >= 4:
        S[2, 0] = S[0, 2] = W[2, 0] + lam
        S[3, 1] = S[1, 3] = W[3, 1]
        A[2, 0] = A[0, 2] = 0.0
        A[3, 1] = A[1, 3] = 0.0
    return S, W, A


@pytest.mark.parametrize("n", SIZES)
def test_gradient_pass_bit_exact(solver, n):
    lam = 0.3
    S, W, A = _grad_inputs(n, n, lam)
    Z, GM, k = solver.gradient_pass(to_dev(S), to_dev(W), to_dev(A), lam)
    Z, GM = to_host(Z), to_host(GM)
    g = oracle.gradient(S, W)
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    Zr = oracle.min_norm_subgradient(g, G, M, lam)
    assert np.array_equal(Z, Zr)
    assert np.array_equal(GM.astype(np.float64), np.where(M, G, 0.0))
    km = oracle.kkt_measures(Zr, A)
    assert abs(k["sum_abs_z"] - km["sum_abs_z"]) <= 1e-12 * km["sum_abs_z"]
    assert abs(k["sum_abs_a"] - km["sum_abs_a"]) <= 1e-12 * km["sum_abs_a"]
    assert abs(k["kkt_fro"] - km["kkt_fro"]) <= 1e-12 * km["kkt_fro"]
    assert k["kkt_max"] == km["kkt_max"]


# ------------------------------------------------------------------ trial point
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("t", [1.0, 0.25, 1e-3])
def test_trial_point_bit_exact(solver, n, t):
    lam = 0.2
    rng = np.random.default_rng(n + 5)
    A = sparse_sym(n, n + 3, density=0.2)
    g = sym(rng.standard_normal((n, n)) * 0.4)
    P = sym(rng.standard_normal((n, n)))
    S = sym(rng.standard_normal((n, n)))
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    GM = np.where(M, G, 0.0).astype(np.int8)
    At, sums = solver.trial_point(to_dev(A), to_dev(P), to_dev(S), to_dev(GM, torch.int8), lam, t)
    At = to_host(At)
    C = oracle.c_matrix(A, lam)
    B = oracle.b_from_products(P, C, G, M)
    ref = oracle.trial_point(A, M, B, C, t)
    assert np.array_equal(At, ref)
    dtr = float(np.sum(S * (ref - A)))
    dl1 = float(np.sum(np.abs(ref) - np.abs(A)))
    assert abs(sums["dtr"] - dtr) <= 1e-12 * max(1.0, np.sum(np.abs(S * (ref - A))))
    assert abs(sums["dl1"] - dl1) <= 1e-12 * max(1.0, np.sum(np.abs(ref)) + np.sum(np.abs(A)))


# ------------------------------------------------------------------ G-ISTA trial point
@pytest.mark.parametrize("n", [1, 5, 64, 130, 300])
@pytest.mark.parametrize("t", [1.0, 0.37, 1e-3])
def test_gista_trial_point_bit_exact(solver, n, t):
    """The proximal-gradient step ST(A - t (S - W), t lam) (eq. proximal_gen, H = I):
    the same IEEE operations as the oracle -> bit-exact on the free set and exact
    zeros off it (there |g| <= lam, so the step is exactly zero); sums in another
    order -> relative 1e-12."""
    lam = 0.2
    rng = np.random.default_rng(n + 11)
    A = sparse_sym(n, n + 4, density=0.2)
    S = sym(rng.standard_normal((n, n)))
    W = sym(S - 0.4 * rng.standard_normal((n, n)))
    # planted ties |g| = lam off the support
    g = oracle.gradient(S, W)
    if n >= 5:
        W[3, 1] = W[1, 3] = S[3, 1] - lam
        W[4, 0] = W[0, 4] = S[4, 0] + lam
        A[3, 1] = A[1, 3] = A[4, 0] = A[0, 4] = 0.0
        g = oracle.gradient(S, W)
    M = oracle.free_set_mask(A, g, lam)
    G = oracle.sign_guess(A, g)
    GM = np.where(M, G, 0.0).astype(np.int8)
    At, sums = solver.gista_trial_point(to_dev(A), to_dev(S), to_dev(W), to_dev(GM, torch.int8), lam, t)
    At = to_host(At)
    ref = oracle.gista_trial_point(A, g, lam, t)
    assert np.array_equal(At, ref)
    d = ref - A
    for got, want, scale in ((sums[0], np.sum(S * d), np.sum(np.abs(S * d))),
                             (sums[1], np.sum(np.abs(ref) - np.abs(A)), np.sum(np.abs(ref)) + np.sum(np.abs(A))),
                             (sums[2], np.sum(W * d), np.sum(np.abs(W * d))),
                             (sums[3], np.sum(d * d), np.sum(d * d))):
        assert abs(got - want) <= 1e-12 * max(1.0, scale)


def test_inverse_fp64_beyond_64_k_chunks(solver):
    """n = 8320: the products of the FP64 triangular inverse and LAUUM run K ranges
    longer than 64 chunks of 128; W A = I on 64 sampled rows (banded SPD A, whose
    inverse is dense), within the inverse's bound."""
    n = 8320
    rng = np.random.default_rng(12)
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = 2.5
    off = -0.5 + 0.2 * rng.random(n - 1)
    A[idx[1:], idx[:-1]] = off
    A[idx[:-1], idx[1:]] = off
    W = to_host(solver.inverse(to_dev(A)))
    rows = rng.choice(n, 64, replace=False)
    R = W[rows] @ A
    E = np.zeros_like(R)
    E[np.arange(64), rows] = 1.0
    # residual bound 4 n eps cond(A) max|W| |A|_inf; cond(A) <= 3.5 / 1.5 (Gershgorin)
    bound = 4 * n * EPS * (3.5 / 1.5) * np.max(np.abs(W)) * 3.5
    assert np.max(np.abs(R - E)) <= bound, (np.max(np.abs(R - E)), bound)
    assert np.array_equal(W, W.T)
