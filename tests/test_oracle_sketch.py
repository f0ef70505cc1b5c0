"""Pins of the oracle's randomized sketch (Alg. 2; Sec. 5.4 lemmas)."""
import numpy as np
import pytest

from oracle import precond, ridge, sketch
from paper_1602_02350_amd import inputs


def _eig_desc(C):
    ev, V = np.linalg.eigh(C)
    o = np.argsort(ev)[::-1]
    return ev[o], V[:, o]


def test_full_width_sketch_is_exact():
    """With k + p >= d the range finder spans R^d, so Rayleigh-Ritz returns the exact eigenpairs."""
    P = inputs.make_ridge(300, 12, 2.0, 1e-3, seed=31, dtype=np.float64)
    C = ridge.correlation(P.X)
    ev, V = _eig_desc(C)
    k = 7
    Om = inputs.gaussian((12, 12), seed=1).astype(np.float64)
    U, lt, Q = sketch.sketch(P.X, Om, k)
    assert np.allclose(lt, ev[:k], rtol=1e-10)
    assert np.allclose(U @ U.T, V[:, :k] @ V[:, :k].T, atol=1e-9)
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-12)


def test_low_rank_data_is_recovered_exactly():
    """If rank(X) <= k + p, range(X^T X Omega) = range(C) and the sketch is exact."""
    rng = np.random.default_rng(2)
    n, d, r = 200, 40, 6
    X = rng.standard_normal((n, r)) @ (rng.standard_normal((r, d)) * np.linspace(2, 0.5, r)[:, None])
    C = ridge.correlation(X)
    ev, V = _eig_desc(C)
    Om = inputs.gaussian((d, 9), seed=2).astype(np.float64)
    U, lt, _ = sketch.sketch(X, Om, 4)
    assert np.allclose(lt, ev[:4], rtol=1e-9)
    assert np.allclose(U @ U.T, V[:, :4] @ V[:, :4].T, atol=1e-8)


def test_ritz_values_interlace_and_basis_is_orthonormal():
    """Ritz values from any subspace are bounded by the true eigenvalues: lam~_i <= lam_i (Cauchy)."""
    P = inputs.make_ridge(500, 60, 1.5, 1e-4, seed=32, dtype=np.float64)
    ev, _ = _eig_desc(ridge.correlation(P.X))
    for seed in range(5):
        Om = inputs.gaussian((60, 15), seed=seed).astype(np.float64)
        U, lt, _ = sketch.sketch(P.X, Om, 10)
        assert np.all(lt <= ev[:10] * (1 + 1e-12))
        assert np.all(np.diff(lt) <= 0)
        assert np.allclose(U.T @ U, np.eye(10), atol=1e-12)


def test_one_block_equals_block_lanczos_started_from_the_same_block():
    """X^T X Omega is the first Krylov block of Alg. 2 started from Pi = X Omega / sqrt(n)."""
    P = inputs.make_ridge(400, 50, 2.0, 1e-4, seed=33, dtype=np.float64)
    Om = inputs.gaussian((50, 13), seed=3).astype(np.float64)
    U1, l1, _ = sketch.sketch(P.X, Om, 8)
    U2, l2, _ = sketch.block_lanczos(P.X, P.X @ Om / np.sqrt(400), 8, q=1)
    assert np.allclose(l1, l2, rtol=1e-10)
    assert np.allclose(U1 @ U1.T, U2 @ U2.T, atol=1e-9)


def test_deeper_krylov_space_is_at_least_as_accurate():
    """Adding blocks (q > 1) can only enlarge the subspace, so Ritz values do not decrease."""
    P = inputs.make_ridge(800, 80, 1.5, 1e-4, seed=34, dtype=np.float64)
    Pi = np.random.default_rng(4).standard_normal((800, 10))
    _, l1, _ = sketch.block_lanczos(P.X, Pi, 10, q=1)
    _, l3, _ = sketch.block_lanczos(P.X, Pi, 10, q=3)
    assert np.all(l3 >= l1 * (1 - 1e-12))


@pytest.mark.parametrize("alpha,lam,k", [(2.0, 1e-4, 10), (1.5, 1e-5, 20)])
def test_sketch_quality_bounds_hold_in_most_seeds(alpha, lam, k):
    """Per-vector bound |lam~_i - lam_i| <= eps' lam_{k+1} (Eq. (perVec), eps' = 1/2) and the three
    eigenvalue bounds of Sec. 5.4 (lambda_1 <= 17; lambda_i <= 2(lam_i+lam)/(lam_k+lam) for i > k;
    lambda_d >= lam/(19(lam_k+lam))) hold with probability >= 9/10; checked over 20 seeds."""
    P = inputs.make_ridge(1500, 100, alpha, lam, seed=35, dtype=np.float64)
    C = ridge.correlation(P.X)
    ev, _ = _eig_desc(C)
    H = C + lam * np.eye(100)
    ok = 0
    for seed in range(20):
        Om = inputs.gaussian((100, k + 5), seed=100 + seed).astype(np.float64)
        U, lt, _ = sketch.sketch(P.X, Om, k)
        Pm = precond.sketched_preconditioner(U, lt, lam)
        Ht = np.sort(np.linalg.eigvalsh(Pm @ H @ Pm))[::-1]
        good = np.all(np.abs(lt - ev[:k]) <= 0.5 * ev[k])
        good &= Ht[0] <= 17
        good &= np.all(Ht[k:] <= 2 * (ev[k:] + lam) / (ev[k - 1] + lam))
        good &= Ht[-1] >= lam / (19 * (ev[k - 1] + lam))
        ok += bool(good)
    assert ok >= 18
