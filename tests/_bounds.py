"""Per-element rounding-error bounds for comparing the FP32 HIP path with the FP64 oracle.

Each bound follows the FP32 arithmetic of the kernel it covers, with rounding errors modelled as
independent random variables of size <= u = 2^-24 relative to each rounded result (Higham and Mary,
SIAM J. Sci. Comput. 2019). A sum evaluated as short FMA chains of g terms followed by a tree of
lane or row-group reductions rounds every partial sum once; with terms t of mixed signs the
partials of level l are about 2^(l/2) times their terms, so the error has a standard deviation of
about u ||t||_2 sqrt(g + log2(q)) for q terms (the chain adds g roundings of its running sum, each
tree level one). Independent errors add in quadrature; errors that every element shares (a rounded
step size, a rounded input vector) are added as such. The returned arrays are one standard
deviation per element; tests allow a fixed multiple (8) of it and print the largest observed
ratio. A wrong column, a dropped term or a few corrupted elements give errors of the size of the
values themselves, many orders above these scales.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def gradient_scale(X, y, lam, Pm, wt, row_chunks=2048, C=None):
    """Scale of the per-element error of mu = P^{-1/2} [X^T (X w - y)/n + lam w], w = P^{-1/2} wt,
    computed as the full-gradient pass does it:
      * w is formed in FP64 and rounded to FP32 (relative u per element): its effect on g is
        C (w o e), a sum over d columns of independent errors;
      * r_i is an FP32 dot product: each lane accumulates d/64 products with FMA, then 6 levels of
        lane sums, then y_i is subtracted, an error of u ||x_i o w||_2 sqrt(d/64 + 7) + u |r_i|;
        rows round independently, so over the n rows of g_j they add in quadrature;
      * r_i x_ij are accumulated with Kahan compensation and the per-wave partials are rounded to
        FP32 once (u per partial, independent across the row_chunks partials), then summed in FP64;
      * P^{-1/2} is applied in FP64 (errors of g propagate through it in quadrature) and mu is
        rounded to FP32 (u |mu_j|).
    C = X^T X / n may be passed in when the caller already has it.
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Pm = np.asarray(Pm, dtype=np.float64)
    n, d = X.shape
    w = Pm @ np.asarray(wt, dtype=np.float64)
    r = X @ w - y
    e_dot = U32 * np.sqrt(d / 64.0 + 7.0) * np.sqrt((X ** 2) @ (w ** 2)) + U32 * np.abs(r)
    t_dot = np.sqrt((X ** 2).T @ (e_dot ** 2)) / n
    if C is None:
        C = X.T @ X / n
    t_w = U32 * np.sqrt((C ** 2) @ (w ** 2)) + lam * U32 * np.abs(w)
    bounds = np.linspace(0, n, min(row_chunks, n) + 1).astype(int)
    parts = np.stack([r[b0:b1] @ X[b0:b1] for b0, b1 in zip(bounds[:-1], bounds[1:])])
    t_acc = 4.0 * U32 * np.sqrt(np.sum(parts ** 2, axis=0)) / n
    e_g = np.sqrt(t_dot ** 2 + t_w ** 2 + t_acc ** 2)
    mu = Pm @ (X.T @ r / n + lam * w)
    return np.sqrt((Pm ** 2) @ (e_g ** 2)) + U32 * np.abs(mu)


def epoch_scale(rows, scale, idx, trace, wbar, mu, eta, b, gram_rel=0.0):
    """Scale of the per-element error of the averaged step (1/m) sum_t (w_t - wbar) of one inner loop
    run in FP32 on delta = w - wbar (Alg. 1 with minibatches of b), given the oracle's iterates w_t.

    rows(i) returns the rows a_i (FP64 values of what the kernel reads), scale[i] = 1/(n q_i),
    trace[t] = w_{t+1}. Per step, with g = (1/b) sum_j gamma_j a_j, gamma_j = scale_j a_j^T delta:
      * each a_j^T delta is an FP32 dot over d columns: FMA chains of 4 per column thread, sums over
        32 column threads and over the W workgroups' partials (u ||a_j o delta||_2 sqrt(4 + log2 d));
      * gamma_j picks up the FP32 rounding of scale_j, of the product and of the 1/b (3u);
      * the sum over the b rows is FP32: FMA chains of b/16 rows, then 4 butterfly levels
        (u ||gamma o a_k||_2 sqrt(b/16 + 4));
      * delta -= eta (g + mu) rounds eta, the sum and the update (u each).
    The local errors of the m steps propagate through the contracting iteration and add in
    quadrature; the snapshot gradient mu is FP32-rounded (a constant error u |mu| per step).

    gram_rel > 0 models the look-ahead loop, which forms a_j^T delta_t as a_j^T (delta_{t-1} - eta mu)
    - eta sum_i (a_j^T a_i) gamma_i over the previous step's rows a_i, with each product a_j^T a_i carrying
    a relative error of at most gram_rel (times the norms): an extra error of
    eta gram_rel ||a_j|| sum_i |gamma_i| ||a_i|| in the dot, plus an FP32 mat-vec over b terms.
    """
    d = wbar.size
    m = len(trace)
    acc = np.zeros(d)
    sys_mu = np.zeros(d)
    delta = np.zeros(d)
    prev = None
    for t in range(m):
        it = idx[t * b:(t + 1) * b]
        A = rows(it)                                   # b x d
        sc = scale[it]
        gam = sc * (A @ delta) / b
        e_gam = U32 * np.sqrt(4.0 + np.log2(d)) * sc * np.sqrt((A ** 2) @ (delta ** 2)) / b
        e_gam = np.sqrt(e_gam ** 2 + (3.0 * U32 * gam) ** 2)
        if gram_rel > 0.0 and prev is not None:
            A_p, gam_p = prev
            na, na_p = np.linalg.norm(A, axis=1), np.linalg.norm(A_p, axis=1)
            cross = np.abs(gam_p) @ na_p
            e_la = eta * (gram_rel * na * cross + U32 * np.sqrt(b) * np.sqrt((np.abs(A @ A_p.T) ** 2) @ (gam_p ** 2)))
            e_gam = np.sqrt(e_gam ** 2 + (sc * e_la / b) ** 2)
        prev = (A, gam)
        g2 = np.sqrt((gam ** 2) @ (A ** 2))
        e_t = eta * np.sqrt((U32 * np.sqrt(b / 16.0 + 4.0) * g2) ** 2 + (e_gam ** 2) @ (A ** 2)
                            + (2.0 * U32 * (gam @ A + mu)) ** 2)
        delta = trace[t] - wbar
        e_t = e_t + U32 * np.abs(delta)
        acc += e_t ** 2
        sys_mu += eta * U32 * np.abs(mu)
    return np.sqrt(acc) + sys_mu
