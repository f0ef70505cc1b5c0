"""Randomized sketch of the data matrix in FP64 (Sec. 4.3, Alg. 2; Sec. 5.4).

Test infrastructure only (see oracle/__init__.py).

The paper runs Block Lanczos on Xbar = n^{-1/2} X (instances as columns,
Sec. 5.3), so Xbar Xbar^T = C and the squared singular values it returns
approximate the eigenvalues of C. In this package's row layout (X is n x d)
that operator is A = n^{-1/2} X^T (d x n).
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def rayleigh_ritz(X, Q, k):
    """Truncated SVD of Q^T A with A = n^{-1/2} X^T; returns (U_k, lam_k).  [Alg. 2, last two steps]

    (Q^T A)_k = W_k Sigma_k V_k^T and U_k = Q W_k; the eigenvalue estimates
    are lam_i = sigma_i^2 (sorted descending, hence non-negative).
    """
    X, Q = _f64(X), _f64(Q)
    n = X.shape[0]
    M = Q.T @ X.T / np.sqrt(n)                  # l x n
    W, sig, _ = np.linalg.svd(M, full_matrices=False)
    return Q @ W[:, :k], sig[:k] ** 2


def range_finder(X, Omega):
    """Y = X^T (X Omega) = n C Omega: one block of the Krylov space started from Omega (d x l)."""
    X = _f64(X)
    return X.T @ (X @ _f64(Omega))


def orthonormalize(Y):
    """Orthonormal basis of range(Y) by Householder QR (LAPACK geqrf/orgqr)."""
    Q, _ = np.linalg.qr(_f64(Y))
    return Q


def sketch(X, Omega, k):
    """One-block sketch: Y = X^T X Omega, Q = orth(Y), Rayleigh-Ritz on Q.  [Alg. 2 with one block]

    Omega is d x l with l = k + p (oversampling p). Returns (U_k d x k, lam_k, Q).
    """
    Q = orthonormalize(range_finder(X, Omega))
    U, lam = rayleigh_ritz(X, Q, k)
    return U, lam, Q


def block_lanczos(X, Pi, k, q):
    """Randomized Block Lanczos (Musco & Musco) on A = n^{-1/2} X^T.  [Alg. 2]

    Pi is n x b Gaussian (the paper takes b = k); the Krylov matrix is
    K = [A Pi, (A A^T) A Pi, ..., (A A^T)^{q-1} A Pi] (d x q b). Its columns are
    orthonormalized and Rayleigh-Ritz gives (U_k, lam_k, Q).
    """
    X = _f64(X)
    n = X.shape[0]
    blk = X.T @ _f64(Pi) / np.sqrt(n)          # A Pi
    blocks = [blk]
    for _ in range(q - 1):
        blk = X.T @ (X @ blk) / n               # (A A^T) = C
        blocks.append(blk)
    Q = orthonormalize(np.concatenate(blocks, axis=1))
    U, lam = rayleigh_ritz(X, Q, k)
    return U, lam, Q
