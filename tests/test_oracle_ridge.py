"""Pins of the oracle's ridge-regression layer against values fixed by the paper and by mathematics."""
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from oracle import ridge
from paper_1602_02350_amd import inputs


def test_closed_form_hand_example():
    """One-dimensional problem solved in rationals (Eq. (ridge) and its normal equations)."""
    g = read_golden("ridge_scalar.txt")
    x = np.array([float(v) for v in g["x"][0]])[:, None]
    y = np.array([float(v) for v in g["y"][0]])
    lam = float(g["lambda"][0][0])
    w = ridge.closed_form(x, y, lam)
    w_exact = Fraction(int(g["w_star_num"][0][0]), int(g["w_star_den"][0][0]))
    L_exact = Fraction(int(g["L_star_num"][0][0]), int(g["L_star_den"][0][0]))
    assert abs(w[0] - float(w_exact)) < 1e-15
    assert abs(ridge.objective(x, y, lam, w) - float(L_exact)) < 1e-15


def _loop_gradient(X, y, lam, w):
    """grad L written term by term from Eq. (ridge), independent of the matrix form."""
    n, d = X.shape
    g = np.zeros(d)
    for i in range(n):
        r = sum(X[i, j] * w[j] for j in range(d)) - y[i]
        g += r * X[i] / n
    return g + lam * w


def test_closed_form_is_stationary():
    P = inputs.make_ridge(60, 7, 1.0, 1e-2, seed=11, dtype=np.float64)
    w = ridge.closed_form(P.X, P.y, P.lam)
    g = _loop_gradient(P.X, P.y, P.lam, w)
    assert np.linalg.norm(g) < 1e-13
    assert np.allclose(ridge.gradient(P.X, P.y, P.lam, w + 1.0), _loop_gradient(P.X, P.y, P.lam, w + 1.0))


def test_closed_form_matches_augmented_least_squares():
    """Ridge = least squares on [X/sqrt(n); sqrt(lam) I] (LAPACK gelsd, an SVD solver)."""
    P = inputs.make_ridge(300, 20, 2.0, 1e-3, seed=12, dtype=np.float64)
    n, d = P.X.shape
    A = np.vstack([P.X / np.sqrt(n), np.sqrt(P.lam) * np.eye(d)])
    t = np.concatenate([P.y / np.sqrt(n), np.zeros(d)])
    w_ls = np.linalg.lstsq(A, t, rcond=None)[0]
    w = ridge.closed_form(P.X, P.y, P.lam)
    assert np.linalg.norm(w - w_ls) <= 1e-9 * np.linalg.norm(w_ls)


def test_suboptimality_identity():
    """L(w) - L(w*) equals 1/2 (w-w*)^T (C + lam I)(w-w*) for the quadratic L."""
    P = inputs.make_ridge(200, 10, 1.0, 1e-2, seed=13, dtype=np.float64)
    ws = ridge.closed_form(P.X, P.y, P.lam)
    rng = np.random.default_rng(0)
    for scale in [1e-1, 1.0, 10.0]:
        w = ws + scale * rng.standard_normal(10)
        direct = ridge.objective(P.X, P.y, P.lam, w) - ridge.objective(P.X, P.y, P.lam, ws)
        assert abs(direct - ridge.suboptimality(P.X, P.lam, w, ws)) <= 1e-10 * direct
        H = ridge.hessian(P.X, P.lam)
        e = w - ws
        assert abs(0.5 * e @ H @ e - ridge.suboptimality(P.X, P.lam, w, ws)) <= 1e-12 * direct


def test_kappa_hat_on_diagonal_correlation():
    """Eq. (initialCondition) on data with orthogonal columns: C = diag(s^2)."""
    n, s = 8, np.array([2.0, 1.0, 0.5])
    Q = np.linalg.qr(np.random.default_rng(1).standard_normal((n, 3)))[0]
    X = Q * s * np.sqrt(n)                 # X^T X / n = diag(s^2)
    lam = 0.25
    ev = s ** 2
    expect = np.sum(ev + lam) / (ev.min() + lam)
    assert abs(ridge.kappa_hat(X, lam) - expect) < 1e-12 * expect


def test_speedup_ratio_and_bound_on_hand_example():
    g = read_golden("exact_precond_diag.txt")
    ev = np.array([float(v) for v in g["diag"][0]])
    k = int(g["k"][0][0])
    lam = float(g["lambda"][0][0])
    ratio = Fraction(int(g["ratio_num"][0][0]), int(g["ratio_den"][0][0]))
    assert abs(ridge.speedup_ratio(ev, k) - float(ratio)) < 1e-15
    assert abs(ridge.predicted_kappa(ev, lam, k) - float(g["bound"][0][0])) < 1e-12


@pytest.mark.parametrize("lam", [1e-1, 1e-3])
def test_planted_mistake_objective_without_half_is_caught(lam, monkeypatch):
    """A dropped 1/2 in the regularizer moves the minimizer off the normal equations."""
    P = inputs.make_ridge(50, 4, 1.0, lam, seed=14, dtype=np.float64)
    ws = ridge.closed_form(P.X, P.y, P.lam)

    def wrong(X, y, lam_, w):
        r = X @ w - y
        return 0.5 * float(r @ r) / X.shape[0] + lam_ * float(w @ w)

    monkeypatch.setattr(ridge, "objective", wrong)
    # the closed form is no longer the minimizer of the (wrong) objective:
    h = 1e-4
    e0 = np.eye(4)[0]
    fd = (ridge.objective(P.X, P.y, lam, ws + h * e0) - ridge.objective(P.X, P.y, lam, ws - h * e0)) / (2 * h)
    assert abs(fd) > 1e-3 * lam * abs(ws[0])


def test_closed_forms_of_a_path_match_single_closed_forms():
    """Many (lambda, y) normal-equation solves on one X equal the single closed form and objective."""
    from paper_1602_02350_amd import inputs
    P = inputs.make_ridge(300, 12, 1.5, 1e-3, seed=44, dtype=np.float64)
    Y = np.stack([P.y, P.X @ np.arange(12.0) + 0.1, -P.y])
    lams = [1e-4, 1e-2, 3.0]
    W, L = ridge.closed_forms(P.X, Y, lams)
    for j, lam in enumerate(lams):
        for r in range(3):
            ws = ridge.closed_form(P.X, Y[r], lam)
            assert np.allclose(W[j, r], ws, rtol=1e-10, atol=1e-12)
            assert abs(L[j, r] - ridge.objective(P.X, Y[r], lam, ws)) <= 1e-10 * abs(L[j, r])
            # stationarity: the gradient vanishes at the solution
            assert np.linalg.norm(ridge.gradient(P.X, Y[r], lam, W[j, r])) < 1e-9


# ------------------------------------------------------------------ the bias-complexity rule (Sec. 2.2)
def test_budget_lambdas_on_hand_example():
    g = read_golden("budget_lambda_diag.txt")
    ev = np.array([float(v) for v in g["diag"][0]])
    n, k = int(g["n"][0][0]), int(g["k"][0][0])
    pre, plain = ridge.budget_lambdas(ev, n, k)
    assert pre == pytest.approx(float(Fraction(int(g["pre_num"][0][0]), int(g["pre_den"][0][0]))), rel=1e-15)
    assert plain == pytest.approx(float(Fraction(int(g["plain_num"][0][0]), int(g["plain_den"][0][0]))), rel=1e-15)
    # the order in which the eigenvalues are given does not matter
    assert ridge.budget_lambdas(ev[::-1], n, k) == (pre, plain)


@pytest.mark.parametrize("alpha,k", [(1.0, 3), (2.0, 10), (1.5, 1)])
def test_budget_ratio_is_the_speedup_ratio(alpha, k):
    """Sec. 2.2: the ratio of the two regularizations is the speed-up ratio of Eq. (ratioRidge)."""
    ev = np.arange(1, 61, dtype=np.float64) ** -alpha
    pre, plain = ridge.budget_lambdas(ev, 1000, k)
    assert plain / pre == pytest.approx(ridge.speedup_ratio(ev, k), rel=1e-13)
    assert pre <= plain * (1 + 1e-14)  # equal at k = 1


def test_budget_from_top_eigenvalues_and_trace():
    """Knowing only the k largest eigenvalues and tr(C) gives the same values (the tail is the trace minus
    the top sum); sketched (smaller) top values give a larger tail and so a larger lambda_precond."""
    P = inputs.make_ridge(400, 12, 1.5, 1e-3, seed=21, dtype=np.float64)
    C = ridge.correlation(P.X)
    ev = np.sort(np.linalg.eigvalsh(C))[::-1]
    k = 4
    exact = ridge.budget_lambdas(ev, 400, k)
    est = ridge.budget_lambdas_estimated(ev[:k], np.trace(C), 400, k)
    assert est == pytest.approx(exact, rel=1e-12)
    low = ridge.budget_lambdas_estimated(0.9 * ev[:k], np.trace(C), 400, k)
    assert low[0] > exact[0] * (1 + 1e-9) or ev[k - 1] == 0.0
    assert low[1] == pytest.approx(exact[1], rel=1e-14)
