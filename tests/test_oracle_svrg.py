"""Pins of the oracle's SVRG (Alg. 1) and the full pipeline (Alg. 3)."""
import numpy as np
import pytest

from oracle import precond, ridge, sampling, svrg
from paper_1602_02350_amd import inputs


def _tiny(seed=41, n=5, d=3, lam=0.3):
    P = inputs.make_ridge(n, d, 1.0, lam, seed=seed, dtype=np.float64)
    Om = inputs.gaussian((d, d), seed=seed).astype(np.float64)
    Pm, _, _ = svrg.preconditioner_from_sketch(P.X, lam, 2, Om)
    return P, precond.Components(P.X, P.y, lam, Pm)


def _estimator_mean(comp, w, wb, scale_by_N=True):
    q = comp.probabilities()
    vbar = comp.full_gradient(wb)
    mean = np.zeros(comp.d)
    for i in range(comp.N):             # enumerate every index with its probability
        v = (comp.grad(i, w) - comp.grad(i, wb)) / ((comp.N if scale_by_N else 1) * q[i]) + vbar
        mean += q[i] * v
    return mean


def test_variance_reduced_direction_is_unbiased():
    """E_q[v_t] = grad F(w_{t-1}) by enumeration over all n+d indices (Alg. 1, with the 1/N reading)."""
    _, comp = _tiny()
    rng = np.random.default_rng(1)
    w, wb = rng.standard_normal(3), rng.standard_normal(3)
    assert np.allclose(_estimator_mean(comp, w, wb), comp.full_gradient(w), rtol=1e-12, atol=1e-14)


def test_planted_mistake_estimator_as_printed_is_biased():
    """Without dividing by N the expectation is off by the factor N: the reading is needed."""
    _, comp = _tiny()
    rng = np.random.default_rng(2)
    w, wb = rng.standard_normal(3), rng.standard_normal(3)
    biased = _estimator_mean(comp, w, wb, scale_by_N=False)
    assert not np.allclose(biased, comp.full_gradient(w), rtol=1e-3)


def _small():
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED)
    X, y = P.X.astype(np.float64), P.y.astype(np.float64)
    Om = inputs.gaussian((cfg["d"], cfg["k"] + 5), seed=inputs.BASE_SEED).astype(np.float64)
    return cfg, X, y, Om


@pytest.mark.slow
def test_scsvrg_reaches_closed_form():
    """Alg. 3 on n=2000, d=100, spectrum j^-2, lam=1e-4, k=10: suboptimality <= 1e-8 (vs Cholesky)."""
    cfg, X, y, Om = _small()
    lam, k, b = cfg["lam"], cfg["k"], cfg["b"]
    ws = ridge.closed_form(X, y, lam)
    m = int(np.ceil(2 * cfg["n"] / b))
    Pm, _, _ = svrg.preconditioner_from_sketch(X, lam, k, Om)
    W = sampling.quantize_weights(precond.Components(X, y, lam, Pm).smoothness())
    w, snaps, info = svrg.scsvrg(X, y, lam, k, Om, m, 12, b,
                                 lambda s: sampling.draw_indices(W, 5, s, m * b), c=8.0)
    so = [ridge.suboptimality(X, lam, s, ws) for s in snaps]
    assert so[-1] <= cfg["eps"]
    assert np.linalg.norm(w - ws) <= 1e-3 * np.linalg.norm(ws)
    # the sketched preconditioner lowers the average condition number (Thm. (sketchCond))
    assert ridge.kappa_tilde(X, lam, info["P_mhalf"]) < ridge.kappa_hat(X, lam) / 4


def test_plain_svrg_reaches_closed_form_on_a_well_conditioned_problem():
    P = inputs.make_ridge(300, 10, 1.0, 1e-2, seed=42, dtype=np.float64)
    ws = ridge.closed_form(P.X, P.y, P.lam)
    comp = precond.Components(P.X, P.y, P.lam, np.eye(10))
    eta = 0.5 / svrg.beta_hat(comp)
    W = sampling.quantize_weights(comp.smoothness())
    m = 2 * 310
    w, _ = svrg.svrg(comp, np.zeros(10), m, eta, 15, 1, lambda s: sampling.draw_indices(W, 1, s, m))
    assert ridge.suboptimality(P.X, P.lam, w, ws) <= 1e-12


def test_k0_pipeline_is_plain_svrg_on_the_same_stream():
    P = inputs.make_ridge(200, 8, 1.0, 1e-2, seed=43, dtype=np.float64)
    idx = inputs.index_stream(208, 3 * 100 * 4, seed=1).reshape(3, -1)
    comp = precond.Components(P.X, P.y, P.lam, np.eye(8))
    eta = 1.0 / svrg.beta_hat(comp)
    w_plain, _ = svrg.svrg(comp, np.zeros(8), 100, eta, 3, 4, lambda s: idx[s])
    w_k0, _, _ = svrg.scsvrg(P.X, P.y, P.lam, 0, None, 100, 3, 4, lambda s: idx[s], eta=eta)
    assert np.array_equal(w_plain, w_k0)


@pytest.mark.slow
def test_planted_mistake_returning_P_half_fails_the_closed_form():
    """Alg. 3 prints w = P^{1/2} w~; the map of Eq. (condRidge) is P^{-1/2} w~. Only the latter is w*."""
    cfg, X, y, Om = _small()
    lam, k, b = cfg["lam"], cfg["k"], cfg["b"]
    ws = ridge.closed_form(X, y, lam)
    m = int(np.ceil(2 * cfg["n"] / b))
    w, _, info = svrg.scsvrg(X, y, lam, k, Om, m, 10, b,
                             lambda s: inputs.index_stream(X.shape[0] + 100, m * b, seed=s), c=4.0)
    Pm = info["P_mhalf"]
    wt = np.linalg.solve(Pm, w)
    w_wrong = np.linalg.inv(Pm) @ wt                          # P^{1/2} w~
    assert ridge.suboptimality(X, lam, w, ws) < 1e-6
    assert ridge.suboptimality(X, lam, w_wrong, ws) > 1e-2


def test_last_iterate_snapshot_option():
    P = inputs.make_ridge(100, 5, 1.0, 1e-1, seed=44, dtype=np.float64)
    comp = precond.Components(P.X, P.y, P.lam, np.eye(5))
    idx = inputs.index_stream(105, 50 * 2, seed=2)
    eta = 0.5 / svrg.beta_hat(comp)
    w_avg, _ = svrg.svrg(comp, np.zeros(5), 50, eta, 1, 2, lambda s: idx, average=True)
    w_last, _ = svrg.svrg(comp, np.zeros(5), 50, eta, 1, 2, lambda s: idx, average=False)
    assert not np.allclose(w_avg, w_last)
    ws = ridge.closed_form(P.X, P.y, P.lam)
    assert ridge.suboptimality(P.X, P.lam, w_last, ws) < ridge.suboptimality(P.X, P.lam, np.zeros(5), ws)


def test_uniform_sampling_is_the_original_svrg_step():
    """With q_i = 1/N the estimator is grad l_i(w) - grad l_i(w~) + grad F(w~), the original SVRG step
    (Sec. 4.2): one epoch of b = 1 steps written out here from the component gradients alone."""
    P, comp = _tiny(seed=43, n=7, d=3, lam=0.2)
    N, m, eta = comp.N, 6, 0.05
    idx = np.array([3, 0, 8, 5, 9, 1])
    w0 = np.array([0.3, -0.2, 0.1])
    w_ref, acc = w0.copy(), np.zeros(3)
    mu = sum(comp.grad(i, w0) for i in range(N)) / N
    for i in idx:
        w_ref = w_ref - eta * (comp.grad(i, w_ref) - comp.grad(i, w0) + mu)
        acc += w_ref
    wb, _ = svrg.svrg(comp, w0, m, eta, 1, 1, lambda s: idx, q=np.full(N, 1.0 / N))
    assert np.allclose(wb, acc / m, rtol=1e-13, atol=1e-15)


def test_uniform_sampling_estimator_is_unbiased():
    P, comp = _tiny(seed=44)
    w, wb = np.array([0.4, -1.0, 0.2]), np.array([-0.3, 0.5, 0.1])
    vbar = comp.full_gradient(wb)
    mean = sum(comp.grad(i, w) - comp.grad(i, wb) + vbar for i in range(comp.N)) / comp.N
    assert np.allclose(mean, comp.full_gradient(w), rtol=1e-12, atol=1e-14)
