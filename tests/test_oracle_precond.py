"""Pins of the oracle's preconditioner and n+d components (Sec. 5 and the appendix)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import precond, ridge, sketch
from paper_1602_02350_amd import inputs


@pytest.fixture(scope="module")
def problem():
    return inputs.make_ridge(400, 30, 1.5, 1e-3, seed=21, dtype=np.float64)


def _sketched(P, k, seed=3):
    Om = inputs.gaussian((P.X.shape[1], k + 5), seed=seed).astype(np.float64)
    U, lt, _ = sketch.sketch(P.X, Om, k)
    return U, lt, precond.sketched_preconditioner(U, lt, P.lam)


def test_exact_preconditioner_spectrum_hand_example():
    """Lemma (exactCondSketch): spectrum {1}^k and (lam_i+lam)/(lam_k+lam) for i > k."""
    g = read_golden("exact_precond_diag.txt")
    C = np.diag([float(v) for v in g["diag"][0]])
    lam, k = float(g["lambda"][0][0]), int(g["k"][0][0])
    Pm, _, _ = precond.exact_preconditioner(C, lam, k)
    H = Pm @ (C + lam * np.eye(4)) @ Pm
    spec = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert np.allclose(spec, [float(v) for v in g["spectrum"][0]], atol=1e-14)
    assert abs(ridge.average_condition(H) - float(g["kappa_tilde"][0][0])) < 1e-12


def test_exact_preconditioner_spectrum_random(problem):
    C = ridge.correlation(problem.X)
    lam, k = problem.lam, 7
    Pm, ev, _ = precond.exact_preconditioner(C, lam, k)
    H = Pm @ (C + lam * np.eye(C.shape[0])) @ Pm
    expect = np.concatenate([np.ones(k), (ev[k:] + lam) / (ev[k - 1] + lam)])
    assert np.allclose(np.sort(np.linalg.eigvalsh(H)), np.sort(expect), rtol=1e-10, atol=1e-12)
    kt = ridge.kappa_tilde(problem.X, lam, Pm)
    assert kt <= ridge.predicted_kappa(ev, lam, k) * (1 + 1e-12)


def test_whitening_is_optimal(problem):
    """k = d gives P = C + lam I, P^{-1/2}(C+lam I)P^{-1/2} = I and kappa~ = d (Sec. 1, Sec. 5.2)."""
    C = ridge.correlation(problem.X)
    d = C.shape[0]
    Pm, _, _ = precond.exact_preconditioner(C, problem.lam, d)
    H = Pm @ (C + problem.lam * np.eye(d)) @ Pm
    assert np.allclose(H, np.eye(d), atol=1e-10)
    assert abs(ridge.kappa_tilde(problem.X, problem.lam, Pm) - d) < 1e-8 * d


def test_change_of_variables(problem):
    """Lt(w~) = L(P^{-1/2} w~) for the n+d components (Eq. (condRidge), Sec. 5.1)."""
    _, _, Pm = _sketched(problem, 6)
    comp = precond.Components(problem.X, problem.y, problem.lam, Pm)
    rng = np.random.default_rng(5)
    for _ in range(3):
        wt = rng.standard_normal(problem.X.shape[1])
        L = ridge.objective(problem.X, problem.y, problem.lam, Pm @ wt)
        assert abs(comp.objective(wt) - L) <= 1e-12 * L
        # chain rule: grad Lt(w~) = P^{-1/2} grad L(P^{-1/2} w~)
        g = Pm @ ridge.gradient(problem.X, problem.y, problem.lam, Pm @ wt)
        assert np.allclose(comp.full_gradient(wt), g, rtol=1e-10, atol=1e-13)


def test_components_average_to_objective():
    """(1/(n+d)) sum_i l_i(w) = Lt(w), summing the components one by one (Sec. 5.1)."""
    P = inputs.make_ridge(25, 6, 1.0, 1e-2, seed=22, dtype=np.float64)
    _, _, Pm = _sketched(P, 2)
    comp = precond.Components(P.X, P.y, P.lam, Pm)
    w = np.random.default_rng(6).standard_normal(6)
    total = sum(comp.value(i, w) for i in range(comp.N)) / comp.N
    assert abs(total - comp.objective(w)) <= 1e-13 * total
    gsum = sum(comp.grad(i, w) for i in range(comp.N)) / comp.N
    assert np.allclose(gsum, comp.full_gradient(w), rtol=1e-12, atol=1e-14)


def test_trace_identity(problem):
    """(1/(n+d)) sum_i beta_i = tr(P^{-1/2}(C + lam I)P^{-1/2})  (appendix, proof of Thm. (condEffect))."""
    _, _, Pm = _sketched(problem, 8)
    comp = precond.Components(problem.X, problem.y, problem.lam, Pm)
    H = Pm @ ridge.hessian(problem.X, problem.lam) @ Pm
    assert abs(comp.smoothness().mean() - np.trace(H)) <= 1e-12 * np.trace(H)
    # so kappa_hat of Lt (beta_hat / strong convexity) equals kappa~ here (Thm. (condEffect))
    kF = comp.smoothness().mean() / np.linalg.eigvalsh(H)[0]
    assert abs(kF - ridge.kappa_tilde(problem.X, problem.lam, Pm)) <= 1e-9 * kF


def test_hessian_by_finite_differences(problem):
    """grad^2 Lt = P^{-1/2}(C + lam I)P^{-1/2} (appendix): exact differences of the full gradient."""
    _, _, Pm = _sketched(problem, 5)
    comp = precond.Components(problem.X, problem.y, problem.lam, Pm)
    d = problem.X.shape[1]
    H = Pm @ ridge.hessian(problem.X, problem.lam) @ Pm
    w = np.random.default_rng(7).standard_normal(d)
    g0 = comp.full_gradient(w)
    for j in [0, 3, d - 1]:
        col = comp.full_gradient(w + np.eye(d)[j]) - g0      # the gradient is affine: h = 1 is exact
        assert np.allclose(col, H[:, j], rtol=1e-8, atol=1e-10)


def test_preconditioner_properties(problem):
    """Eq. (condSketch): symmetric PD, scales u_i by (lam_i+lam)^{-1/2}, the complement by (lam_k+lam)^{-1/2}."""
    U, lt, Pm = _sketched(problem, 6)
    lam = problem.lam
    assert np.allclose(Pm, Pm.T, atol=1e-15)
    assert np.linalg.eigvalsh(Pm)[0] > 0
    for i in range(6):
        assert np.allclose(Pm @ U[:, i], U[:, i] / np.sqrt(lt[i] + lam), rtol=1e-12, atol=1e-14)
    v = np.random.default_rng(8).standard_normal(U.shape[0])
    v -= U @ (U.T @ v)
    assert np.allclose(Pm @ v, v / np.sqrt(lt[-1] + lam), rtol=1e-12, atol=1e-14)
    # invariant to the signs of the columns of U
    Pm2 = precond.sketched_preconditioner(U * np.array([1, -1, 1, -1, -1, 1]), lt, lam)
    assert np.allclose(Pm, Pm2, atol=1e-14)
    # k = 0 is the identity (plain SVRG)
    assert np.array_equal(precond.sketched_preconditioner(np.zeros((5, 0)), np.zeros(0), lam), np.eye(5))


def test_components_from_rows(problem):
    """Components given by their rows (x~_i, b_j) are the same functions as those formed from X and
    P^{-1/2} (Sec. 5.1); with rows that are no preconditioned pair at all, the full gradient is still
    the brute-force average of the n+d component gradients."""
    _, _, Pm = _sketched(problem, 5)
    ref = precond.Components(problem.X, problem.y, problem.lam, Pm)
    comp = precond.Components.from_rows(problem.X @ Pm, Pm, problem.y, problem.lam)
    w = np.random.default_rng(8).standard_normal(problem.X.shape[1])
    assert np.allclose(comp.full_gradient(w), ref.full_gradient(w), rtol=1e-12, atol=1e-15)
    assert np.allclose(comp.smoothness(), ref.smoothness(), rtol=1e-12)
    assert abs(comp.objective(w) - ref.objective(w)) <= 1e-12 * ref.objective(w)
    rng = np.random.default_rng(9)
    Xt, B, y = rng.standard_normal((7, 3)), rng.standard_normal((3, 3)), rng.standard_normal(7)
    c2 = precond.Components.from_rows(Xt, B, y, 0.3)
    w = rng.standard_normal(3)
    brute = sum(c2.grad(i, w) for i in range(10)) / 10
    assert np.allclose(c2.full_gradient(w), brute, rtol=1e-13, atol=1e-15)
    # component 2 of the data rows and component 1 of the regularizer rows by hand
    assert abs(c2.value(2, w) - 10 / 7 * 0.5 * (Xt[2] @ w - y[2]) ** 2) < 1e-13
    assert abs(c2.value(8, w) - 0.3 * 10 * 0.5 * (B[1] @ w) ** 2) < 1e-13
