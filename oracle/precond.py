"""Preconditioners and the preconditioned n+d components in FP64 (Sec. 5).

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def sketched_preconditioner(U, lam_t, lam):
    """Dense P^{-1/2} = sum_{i<=k} u_i u_i^T / sqrt(lam_i + lam) + (I - sum u_i u_i^T)/sqrt(lam_k + lam).

    [Sec. 5.4, Eq. (condSketch)]; lam_t are the sketched eigenvalue estimates
    (the squared singular values sigma_i^2), in descending order. With k = 0
    (U of width 0) the preconditioner is the identity (plain SVRG).
    """
    U, lam_t = _f64(U), _f64(lam_t)
    d, k = U.shape
    if k == 0:
        return np.eye(d)
    P = np.zeros((d, d))
    proj = np.zeros((d, d))
    for i in range(k):
        uu = np.outer(U[:, i], U[:, i])
        P += uu / np.sqrt(lam_t[i] + lam)
        proj += uu
    P += (np.eye(d) - proj) / np.sqrt(lam_t[k - 1] + lam)
    return P


def exact_preconditioner(C, lam, k):
    """The same formula with the true top-k eigenpairs of C.  [Sec. 5.3]"""
    ev, V = np.linalg.eigh(_f64(C))
    order = np.argsort(ev)[::-1]
    ev, V = ev[order], V[:, order]
    return sketched_preconditioner(V[:, :k], ev[:k], lam), ev, V


class Components:
    """The n+d components of the preconditioned objective.  [Sec. 5.1]

      l_i(w)     = (n+d)/n * 1/2 (w^T xt_i - y_i)^2,   xt_i = P^{-1/2} x_i,  i = 1..n
      l_{n+j}(w) = lam (n+d) * 1/2 (w^T b_j)^2,        b_j  = P^{-1/2} e_j,  j = 1..d

    so that Lt(w) = (1/(n+d)) sum_i l_i(w) = L(P^{-1/2} w). Their smoothness
    constants are beta_i = (n+d)/n ||xt_i||^2 and beta_{n+j} = lam (n+d) ||b_j||^2
    (Alg. 3; the printed ||b_j|| without the square and the missing 1/2 in the
    regularizer component are read as in the Hessian formula of the appendix).
    """

    def __init__(self, X, y, lam, P_mhalf):
        X, y, Pm = _f64(X), _f64(y), _f64(P_mhalf)
        self.n, self.d = X.shape
        self.N = self.n + self.d
        self.lam = float(lam)
        self.y = y
        self.P_mhalf = Pm
        self.Xt = X @ Pm                      # row i is (P^{-1/2} x_i)^T (P symmetric)
        self.B = Pm.copy()                    # row j is b_j^T = (P^{-1/2} e_j)^T

    @classmethod
    def from_rows(cls, Xt, B, y, lam):
        """The same n+d components with their rows given directly: x~_i = row i of Xt (n x d) and
        b_j = row j of B (d x d), e.g. rows already rounded to the precision an implementation stores.
        The components, objective and smoothness are defined from the rows alone.  [Sec. 5.1]"""
        self = cls.__new__(cls)
        self.Xt, self.B = _f64(Xt), _f64(B)
        self.n, self.d = self.Xt.shape
        assert self.B.shape == (self.d, self.d)
        self.N = self.n + self.d
        self.lam = float(lam)
        self.y = _f64(y)
        self.P_mhalf = None
        return self

    def value(self, i, w):
        if i < self.n:
            r = self.Xt[i] @ w - self.y[i]
            return self.N / self.n * 0.5 * r * r
        t = self.B[i - self.n] @ w
        return self.lam * self.N * 0.5 * t * t

    def grad(self, i, w):
        """Gradient of the i-th component at w (0-based i in [0, n+d))."""
        if i < self.n:
            return self.N / self.n * (self.Xt[i] @ w - self.y[i]) * self.Xt[i]
        b = self.B[i - self.n]
        return self.lam * self.N * (b @ w) * b

    def objective(self, w):
        """(1/(n+d)) sum_i l_i(w), the preconditioned objective Lt(w)."""
        w = _f64(w)
        r = self.Xt @ w - self.y
        t = self.B @ w
        total = self.N / self.n * 0.5 * float(r @ r) + self.lam * self.N * 0.5 * float(t @ t)
        return total / self.N

    def full_gradient(self, w):
        """grad F(w) = (1/(n+d)) sum_i grad l_i(w).  [Alg. 1, full gradient at the snapshot]"""
        w = _f64(w)
        g = self.N / self.n * (self.Xt.T @ (self.Xt @ w - self.y))
        g += self.lam * self.N * (self.B.T @ (self.B @ w))
        return g / self.N

    def smoothness(self):
        """beta_i for i = 1..n+d.  [Alg. 3]"""
        bx = self.N / self.n * np.einsum("ij,ij->i", self.Xt, self.Xt)
        bb = self.lam * self.N * np.einsum("ij,ij->i", self.B, self.B)
        return np.concatenate([bx, bb])

    def probabilities(self):
        """q_i = beta_i / sum_j beta_j.  [Alg. 1, sampling step]"""
        beta = self.smoothness()
        return beta / beta.sum()
