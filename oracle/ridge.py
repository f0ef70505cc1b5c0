"""Ridge regression in FP64: objective, gradient, closed form, condition numbers.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def objective(X, y, lam, w):
    """L(w) = (1/n) sum_i 1/2 (w^T x_i - y_i)^2 + (lam/2)||w||^2.  [Sec. 1, Eq. (ridge)]"""
    X, y, w = _f64(X), _f64(y), _f64(w)
    r = X @ w - y
    return 0.5 * float(r @ r) / X.shape[0] + 0.5 * lam * float(w @ w)


def gradient(X, y, lam, w):
    """grad L(w) = X^T (X w - y)/n + lam w.  [derivative of Eq. (ridge)]"""
    X, y, w = _f64(X), _f64(y), _f64(w)
    return X.T @ (X @ w - y) / X.shape[0] + lam * w


def correlation(X):
    """C = (1/n) sum_i x_i x_i^T.  [Sec. 1, Eq. (covSpec)]"""
    X = _f64(X)
    return X.T @ X / X.shape[0]


def hessian(X, lam):
    """C + lam I, the (constant) Hessian of L."""
    C = correlation(X)
    return C + lam * np.eye(C.shape[0])


def closed_form(X, y, lam):
    """w* solving (C + lam I) w = (1/n) sum_i y_i x_i, by Cholesky.  [Sec. 3, 'Existing algorithms']

    Unique because L is lam-strongly convex (lam > 0).
    """
    X, y = _f64(X), _f64(y)
    H = hessian(X, lam)
    rhs = X.T @ y / X.shape[0]
    return sla.cho_solve(sla.cho_factor(H, lower=True), rhs)


def closed_forms(X, Y, lams):
    """w*(lam, y) for every lam in lams and every row y of Y, and L(w*): the normal equations of
    closed_form with the correlation matrix and the right-hand sides formed once.  [Sec. 3]

    Returns (W, L) with W of shape (len(lams), len(Y), d) and L of shape (len(lams), len(Y)).
    """
    X, Y = _f64(X), _f64(np.atleast_2d(Y))
    n, d = X.shape
    C = X.T @ X / n
    B = X.T @ Y.T / n                            # d x ny
    yy = np.einsum("ij,ij->i", Y, Y) / n
    W = np.empty((len(lams), Y.shape[0], d))
    L = np.empty((len(lams), Y.shape[0]))
    for j, lam in enumerate(lams):
        Ws = sla.cho_solve(sla.cho_factor(C + lam * np.eye(d), lower=True), B)   # d x ny
        W[j] = Ws.T
        # L(w) = 1/2 w^T (C + lam I) w - w^T X^T y / n + y^T y / (2n), evaluated at w*
        L[j] = 0.5 * np.einsum("ir,ir->r", Ws, (C + lam * np.eye(d)) @ Ws) - np.einsum("ir,ir->r", Ws, B) + 0.5 * yy
    return W, L


def suboptimality(X, lam, w, w_star):
    """L(w) - L(w*) = 1/2 (w - w*)^T (C + lam I) (w - w*), exact for a quadratic."""
    e = _f64(w) - _f64(w_star)
    X = _f64(X)
    Xe = X @ e
    return 0.5 * float(Xe @ Xe) / X.shape[0] + 0.5 * lam * float(e @ e)


def average_condition(H):
    """tr(H) / lambda_min(H) of a symmetric positive definite matrix."""
    ev = np.linalg.eigvalsh(_f64(H))
    return float(ev.sum() / ev[0])


def kappa_hat(X, lam):
    """Average condition number of C + lam I.  [Sec. 1, Eq. (initialCondition)]"""
    ev = np.linalg.eigvalsh(correlation(X))
    return float(np.sum(ev + lam) / (ev[0] + lam))


def kappa_tilde(X, lam, P_mhalf):
    """tr / lambda_min of P^{-1/2}(C + lam I)P^{-1/2}.  [Sec. 5.2, Thm. (condEffect)]"""
    Pm = _f64(P_mhalf)
    return average_condition(Pm @ hessian(X, lam) @ Pm)


def speedup_ratio(eigs, k):
    """sum_i lambda_i / (k lambda_k + sum_{i>k} lambda_i).  [Sec. 2, Eq. (ratioRidge)]

    `eigs` are the eigenvalues of C in descending order; k is 1-based.
    """
    ev = _f64(eigs)
    return float(ev.sum() / (k * ev[k - 1] + ev[k:].sum()))


def predicted_kappa(eigs, lam, k):
    """(k lambda_k + sum_{i>k} lambda_i)/lam + d.  [Sec. 5.3, Eq. (exactCondSketchCond)]"""
    ev = _f64(eigs)
    return float((k * ev[k - 1] + ev[k:].sum()) / lam + ev.size)


def budget_lambdas(eigs, n, k):
    """The regularization at which each method runs in O~(ndk) time (Sec. 2.2): preconditioned SVRG at
    lambda = (k lambda_k + sum_{i>k} lambda_i)/(n k)  [Eq. (decay)], plain SVRG at
    lambda = (sum_i lambda_i)/(n k)  [Eq. (decaySVRG)].

    `eigs` are the eigenvalues of C (any order); k is 1-based. Returns (lambda_precond, lambda_plain).
    """
    ev = np.sort(_f64(eigs))[::-1]
    pre = (k * ev[k - 1] + ev[k:].sum()) / (n * k)
    plain = ev.sum() / (n * k)
    return float(pre), float(plain)


def budget_lambdas_estimated(top, trace, n, k):
    """budget_lambdas with only the k largest eigenvalues known (e.g. sketched ones, descending) and the
    trace of C: the tail sum is trace - sum(top). Equals budget_lambdas when `top` are the exact
    eigenvalues and `trace` the exact trace. Returns (lambda_precond, lambda_plain)."""
    t = np.maximum(_f64(top)[:k], 0.0)
    tail = max(float(trace) - float(t.sum()), 0.0)
    return float((k * t[k - 1] + tail) / (n * k)), float(float(trace) / (n * k))
