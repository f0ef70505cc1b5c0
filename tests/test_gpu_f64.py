"""The FP64 instantiation of the path against the FP64 oracle.

Every quantity is FP64 on both sides, so the two agree to FP64 rounding amplified by the method's
own conditioning: the bounds below are stated per test. FP32 rounding anywhere in the GPU path
(1e-7 relative) would fail them.
"""
import numpy as np
import pytest
import torch

from oracle import precond, ridge, sampling, sketch, svrg
from paper_1602_02350_amd import binding, inputs

pytestmark = pytest.mark.gpu

U64 = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = binding.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def small_problem(seed_offset=0):
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED + seed_offset,
                          dtype=np.float64)
    return cfg, P


def quantized_q(comp):
    """The sampler's distribution: integer weights quantized from beta_i (Alg. 1's q_i = beta_i / sum beta
    on a 2^-B grid), q_i = W_i / T."""
    W = sampling.quantize_weights(comp.smoothness()).astype(np.float64)
    return W / W.sum()


def assert_close_trajectory(w_gpu, w_orc, w_star, tol, what):
    """|(w_gpu - w*) - (w_orc - w*)|_j <= tol (|w_orc - w*|_j + rms(w_orc - w*)), element by element."""
    e_g = np.asarray(w_gpu) - w_star
    e_o = np.asarray(w_orc) - w_star
    bound = tol * (np.abs(e_o) + np.sqrt(np.mean(e_o ** 2)))
    ratio = np.abs(e_g - e_o) / bound
    print(f"\n[{what}] max |dw| / bound = {ratio.max():.3e} at tol {tol:.0e}; "
          f"max |dw| / rms(w_o - w*) = {np.max(np.abs(e_g - e_o)) / np.sqrt(np.mean(e_o ** 2)):.2e}")
    assert np.all(ratio <= 1.0), (int(np.argmax(ratio)), float(ratio.max()))


# ------------------------------------------------------------------ sketch
def test_f64_sketch_matches_the_oracle(ctx):
    """Same Omega: lam~ within 64 n u lam~_1 and each Ritz vector within 64 n u lam~_1 / gap_j (the
    Davis-Kahan scale of a perturbation of B of size n u ||B||), up to sign."""
    cfg, P = small_problem()
    n, d, k = cfg["n"], cfg["d"], cfg["k"]
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED + 1)
    U, lam, rc = ctx.sketch_build_f64(dev(P.X), k, omega=dev(Om, torch.float32))
    assert rc == binding.OK
    Uo, lo, _ = sketch.sketch(P.X, Om.astype(np.float64).T, k)
    Ug, lg = host(U), host(lam)
    scale = 64 * n * U64 * lo[0]
    dl = np.abs(lg - lo)
    print(f"\n[f64 sketch] max |d lam| / lam_1 = {dl.max() / lo[0]:.2e}")
    assert np.all(dl <= scale)
    _, lall, _ = sketch.sketch(P.X, Om.astype(np.float64).T, k + 5)
    gaps = np.minimum(np.abs(lall[:k] - lall[1:k + 1]),
                      np.concatenate([[np.inf], np.abs(lall[1:k] - lall[:k - 1])]))
    for j in range(k):
        s = np.sign(Ug[:, j] @ Uo[:, j])
        err = np.max(np.abs(s * Ug[:, j] - Uo[:, j]))
        assert err <= scale / gaps[j] + 64 * U64, (j, err, scale / gaps[j])


def test_f64_sketch_rejects_what_one_workgroup_cannot_hold(ctx):
    X = dev(np.ones((16, 4097)))
    with pytest.raises(binding.ScsError) as e:
        ctx.sketch_build_f64(X, 2)
    assert e.value.code == binding.EINVAL
    _, P = small_problem()
    with pytest.raises(binding.ScsError) as e:
        ctx.sketch_build_f64(dev(P.X), 10, krylov_blocks=2)
    assert e.value.code == binding.EINVAL


# ------------------------------------------------------------------ epochs on a given stream
@pytest.mark.parametrize("k,uniform", [(10, 0), (0, 0), (10, 1)])
def test_f64_epochs_match_the_oracle_on_an_injected_stream(ctx, k, uniform):
    """Three epochs with the same Omega and index stream: the GPU's iterate follows the oracle's
    (Alg. 3 with Alg. 1, q from the quantized weights, or 1/N) to 1e-11 of its distance to w*
    (measured: about 2e-13)."""
    cfg, P = small_problem()
    n, d, b, lam = cfg["n"], cfg["d"], cfg["b"], cfg["lam"]
    m, S, c = n // b, 3, 4.0
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED + 2)
    idx = inputs.index_stream(n + d, S * m * b, seed=79).reshape(S, -1)
    res = ctx.svrg_solve_f64(dev(P.X), dev(P.y), lam, k, 0.0, omega=dev(Om, torch.float32) if k else None,
                             indices=dev(idx, torch.int32), steps=m, batch=b, max_epochs=S,
                             stop_rule=binding.STOP_EPOCHS, step_scale=c, uniform_sampling=uniform)
    assert res.status == binding.OK and res.report["epochs"] == S
    Pm, _, _ = svrg.preconditioner_from_sketch(P.X, lam, k, Om.astype(np.float64).T)
    comp = precond.Components(P.X, P.y, lam, Pm)
    eta = c / svrg.beta_hat(comp)
    q = np.full(n + d, 1.0 / (n + d)) if uniform else quantized_q(comp)
    wt, _ = svrg.svrg(comp, np.zeros(d), m, eta, S, b, lambda s: idx[s], q=q)
    ws = ridge.closed_form(P.X, P.y, lam)
    assert_close_trajectory(host(res.w), Pm @ wt, ws, 1e-11, f"f64 epochs k={k} uniform={uniform}")
    assert abs(res.report["eta"] - eta) <= 1e-13 * eta


@pytest.mark.parametrize("n,d,k,b", [(1500, 120, 12, 24), (1000, 20, 4, 100), (3000, 300, 20, 64),
                                     (700, 4096, 0, 3)])
def test_f64_epochs_match_the_oracle_at_other_shapes(ctx, n, d, k, b):
    """The inner loop's three forms: rows prefetched a step ahead (b <= 32, d <= 256, b d <= 3072), rows
    staged in LDS (b d <= 3072), rows read twice from memory; d = 4096 is the widest the FP64 path
    takes. Two epochs on an injected stream against the oracle, as above."""
    P = inputs.make_ridge(n, d, 1.5, 1e-3, seed=61 + d, dtype=np.float64)
    lam = P.lam
    m, S, c = max(1, n // (4 * b)), 2, 2.0
    Om = inputs.gaussian((k + 5, d), seed=62 + d)
    idx = inputs.index_stream(n + d, S * m * b, seed=63 + d).reshape(S, -1)
    res = ctx.svrg_solve_f64(dev(P.X), dev(P.y), lam, k, 0.0, omega=dev(Om, torch.float32) if k else None,
                             indices=dev(idx, torch.int32), steps=m, batch=b, max_epochs=S,
                             stop_rule=binding.STOP_EPOCHS, step_scale=c)
    assert res.status == binding.OK and res.report["epochs"] == S
    Pm, _, _ = svrg.preconditioner_from_sketch(P.X, lam, k, Om.astype(np.float64).T)
    comp = precond.Components(P.X, P.y, lam, Pm)
    wt, _ = svrg.svrg(comp, np.zeros(d), m, c / svrg.beta_hat(comp), S, b, lambda s: idx[s], q=quantized_q(comp))
    ws = ridge.closed_form(P.X, P.y, lam)
    assert_close_trajectory(host(res.w), Pm @ wt, ws, 1e-11, f"f64 epochs n={n} d={d} k={k} b={b}")


def test_f64_solve_draws_the_oracles_stream(ctx):
    """No injection: Omega from the counter-based Gaussian and the indices from the integer sampler of
    the seed, which the oracle reproduces (both are exact integer computations up to the FP64 beta_i
    that set the weights), so the two solves run the same trajectory."""
    cfg, P = small_problem(1)
    n, d, b, lam, k = cfg["n"], cfg["d"], cfg["b"], cfg["lam"], cfg["k"]
    m, S, c, seed = n // b, 3, 4.0, 20160211
    res = ctx.svrg_solve_f64(dev(P.X), dev(P.y), lam, k, 0.0, steps=m, batch=b, max_epochs=S,
                             stop_rule=binding.STOP_EPOCHS, step_scale=c, seed=seed)
    assert res.status == binding.OK
    l = k + 5
    Om = sampling.gaussian(seed, l * d).astype(np.float32).astype(np.float64).reshape(l, d)
    Pm, _, _ = svrg.preconditioner_from_sketch(P.X, lam, k, Om.T)
    comp = precond.Components(P.X, P.y, lam, Pm)
    W = sampling.quantize_weights(comp.smoothness())
    draws = [sampling.draw_indices(W, seed=seed, epoch=s, count=m * b) for s in range(S)]
    q = W.astype(np.float64) / W.astype(np.float64).sum()
    wt, _ = svrg.svrg(comp, np.zeros(d), m, c / svrg.beta_hat(comp), S, b, lambda s: draws[s], q=q)
    ws = ridge.closed_form(P.X, P.y, lam)
    assert_close_trajectory(host(res.w), Pm @ wt, ws, 1e-11, "f64 seeded stream")


# ------------------------------------------------------------------ the FP64 workload to its closed form
@pytest.mark.parametrize("k", [10, 0])
def test_f64_solve_reaches_the_closed_form(ctx, k):
    """n = 2000, d = 100, spectrum j^-2, lambda = 1e-4: solved to suboptimality 1e-8 (the gap rule
    against the Cholesky closed form), with the oracle's L(w) - L(w*) confirming it."""
    cfg, P = small_problem()
    lam = cfg["lam"]
    ws = ridge.closed_form(P.X, P.y, lam)
    Ls = ridge.objective(P.X, P.y, lam, ws)
    res = ctx.svrg_solve_f64(dev(P.X), dev(P.y), lam, k, cfg["eps"], batch=cfg["b"], max_epochs=60 if k else 200,
                             stop_rule=binding.STOP_GAP, f_star=Ls, step_scale=8.0 if k else 2.0)
    assert res.status == binding.OK, res.report
    so = ridge.suboptimality(P.X, lam, host(res.w), ws)
    print(f"\n[f64 solve k={k}] epochs {res.report['epochs']}, suboptimality {so:.3e}")
    assert so <= cfg["eps"] * (1 + 1e-6)
    assert abs(res.report["objective"] - ridge.objective(P.X, P.y, lam, host(res.w))) <= 1e-13 * Ls + 1e-16


def test_f64_certificate_bounds_the_true_suboptimality(ctx):
    """The certificate ||mu||^2 (lam_1 + lambda) / (2 lambda) is an upper bound on L(w) - L(w*) (Sec. 4.1,
    H~ >= lambda P^{-1}); in FP64 it can drive the solve to 1e-13."""
    cfg, P = small_problem(2)
    lam = cfg["lam"]
    ws = ridge.closed_form(P.X, P.y, lam)
    res = ctx.svrg_solve_f64(dev(P.X), dev(P.y), lam, cfg["k"], 1e-13, batch=cfg["b"], max_epochs=80,
                             stop_rule=binding.STOP_CERTIFICATE, step_scale=8.0)
    assert res.status == binding.OK, res.report
    so = ridge.suboptimality(P.X, lam, host(res.w), ws)
    print(f"\n[f64 certificate] epochs {res.report['epochs']}, certificate {res.report['certificate']:.3e}, "
          f"suboptimality {so:.3e}")
    assert so <= res.report["certificate"] * (1 + 1e-6) + 1e-18
    assert res.report["certificate"] <= 1e-13


def test_f64_invalid_arguments_are_rejected(ctx):
    _, P = small_problem()
    X, y = dev(P.X), dev(P.y)
    bad = [dict(lam_reg=0.0, k=2), dict(lam_reg=1e-4, k=101), dict(lam_reg=1e-4, k=96),  # k + p > d
           dict(lam_reg=1e-4, k=10, krylov_blocks=2), dict(lam_reg=1e-4, k=10, batch=257),
           dict(lam_reg=1e-4, k=10, w0=torch.zeros(100, device="cuda"))]
    for kw in bad:
        lam, k = kw.pop("lam_reg"), kw.pop("k")
        with pytest.raises(binding.ScsError) as e:
            ctx.svrg_solve_f64(X, y, lam, k, 1e-8, **kw)
        assert e.value.code == binding.EINVAL, kw
    wide = dev(np.zeros((8, 4097)))
    with pytest.raises(binding.ScsError) as e:
        ctx.svrg_solve_f64(wide, dev(np.zeros(8)), 1e-3, 0, 1e-8)
    assert e.value.code == binding.EINVAL


def test_f64_non_finite_input_is_reported(ctx):
    _, P = small_problem()
    y = P.y.copy()
    y[5] = np.nan
    with pytest.raises(binding.ScsError) as e:
        ctx.svrg_solve_f64(dev(P.X), dev(y), 1e-4, 0, 1e-8)
    assert e.value.code == binding.ENONFINITE
