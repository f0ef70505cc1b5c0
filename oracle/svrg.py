"""SVRG (Alg. 1) and Sketched Preconditioned SVRG (Alg. 3) in FP64.

Test infrastructure only (see oracle/__init__.py).

Readings of the paper taken here (each is justified where it is used):
  * The variance-reduced direction divides by N q_i (N = n+d components), so
    that it is an unbiased estimate of grad F; with q_i = 1/N it is the usual
    SVRG direction. The printed estimator omits the 1/N.
  * A minibatch of b i.i.d. draws averages b such terms (b = 1 is Alg. 1 as
    printed).
  * The returned weights are w = P^{-1/2} w~ (Sec. 1, Eq. (condRidge)); the
    P^{1/2} printed as Alg. 3's output would not minimize L.
  * The snapshot is the average of the m inner iterates (Alg. 1), or the last
    iterate if average=False.
"""
from __future__ import annotations

import numpy as np

from .precond import Components, sketched_preconditioner
from .sketch import sketch


def _component_grads(comp: Components, idx, w):
    """Rows are grad l_i(w) for i in idx (vectorized form of Components.grad)."""
    idx = np.asarray(idx)
    out = np.empty((idx.size, comp.d))
    data = idx < comp.n
    if data.any():
        rows = comp.Xt[idx[data]]
        r = rows @ w - comp.y[idx[data]]
        out[data] = (comp.N / comp.n) * r[:, None] * rows
    if (~data).any():
        rows = comp.B[idx[~data] - comp.n]
        t = rows @ w
        out[~data] = (comp.lam * comp.N) * t[:, None] * rows
    return out


def beta_hat(comp: Components):
    """Average smoothness (1/N) sum_i beta_i.  [Sec. 4.2, Eq. (conditionSVRG)]"""
    return float(comp.smoothness().mean())


def svrg(comp: Components, w_bar0, m, eta, S, b, epoch_indices, average=True, q=None, trace=None):
    """Alg. 1 on F = (1/N) sum_i l_i, with minibatches of b i.i.d. draws.

    epoch_indices(s) returns the m*b component indices (0-based) used in epoch
    s = 0..S-1, step t using entries [t*b, (t+1)*b). q are the sampling
    probabilities the draws follow: beta_i / sum beta (the default, Alg. 1), or
    e.g. 1/N for the uniform sampling of the original SVRG (Sec. 4.2). Returns
    the final snapshot and the list of snapshots after each epoch. If `trace` is
    a list, every inner iterate w_t is appended to it (a copy), for inspection.
    """
    q = comp.probabilities() if q is None else np.asarray(q, dtype=np.float64)
    N = comp.N
    w_bar = np.asarray(w_bar0, dtype=np.float64).copy()
    snapshots = []
    for s in range(S):
        wb = w_bar
        v_bar = comp.full_gradient(wb)                         # full gradient at the snapshot
        w = wb.copy()
        acc = np.zeros_like(w)
        idx = np.asarray(epoch_indices(s))
        for t in range(m):
            it = idx[t * b:(t + 1) * b]
            diff = _component_grads(comp, it, w) - _component_grads(comp, it, wb)
            v = (diff / (N * q[it])[:, None]).sum(axis=0) / len(it) + v_bar
            w = w - eta * v
            acc += w
            if trace is not None:
                trace.append(w.copy())
        w_bar = acc / m if average else w
        snapshots.append(w_bar.copy())
    return w_bar, snapshots


def preconditioner_from_sketch(X, lam, k, Omega):
    """P^{-1/2} of Eq. (condSketch) from the one-block sketch; identity for k = 0."""
    d = np.asarray(X).shape[1]
    if k == 0:
        return np.eye(d), None, None
    U, lam_t, _ = sketch(X, Omega, k)
    return sketched_preconditioner(U, lam_t, lam), U, lam_t


def scsvrg(X, y, lam, k, Omega, m, S, b, epoch_indices, c=None, eta=None, average=True):
    """Alg. 3: sketch, precondition, SVRG on the n+d components, map back.

    The step is eta = c / beta_hat unless eta is given. Returns
    (w, snapshots_in_w_coordinates, info).
    """
    Pm, U, lam_t = preconditioner_from_sketch(X, lam, k, Omega)
    comp = Components(X, y, lam, Pm)
    bh = beta_hat(comp)
    if eta is None:
        eta = c / bh
    wt, snaps = svrg(comp, np.zeros(comp.d), m, eta, S, b, epoch_indices, average)
    w = Pm @ wt                                                # w = P^{-1/2} w~
    info = dict(P_mhalf=Pm, U=U, lam_t=lam_t, beta_hat=bh, eta=eta, comp=comp)
    return w, [Pm @ s for s in snaps], info
