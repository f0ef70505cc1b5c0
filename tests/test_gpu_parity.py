"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, kernel by kernel.

Tolerances follow from the arithmetic: FP32 storage and FP32 accumulation over at most a few
thousand terms give relative errors of a few 1e-6; BF16 operands (8-bit mantissa) give ~1e-2.
"""
import numpy as np
import pytest
import torch

from _bounds import U32, epoch_scale, gradient_scale
from oracle import precond, ridge, sampling, sketch, svrg
from paper_1602_02350_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = binding.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else \
        t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def assert_tracks(w_gpu, w_orc, w_star, tol):
    """Whole solves: the GPU's distance to w* follows the oracle's element by element,
    |(w_gpu - w*) - (w_orc - w*)|_j <= tol (|w_orc - w*|_j + rms(w_orc - w*)). The two sketches differ by
    the GPU's FP32 GEMMs and CholeskyQR2 against the oracle's FP64 Householder QR (a relative change of
    the preconditioner near 1e-6, see the sketch tests), which perturbs every step of the trajectory
    by that relative amount."""
    e_g = np.asarray(w_gpu, dtype=np.float64) - w_star
    e_o = np.asarray(w_orc, dtype=np.float64) - w_star
    bound = tol * (np.abs(e_o) + np.sqrt(np.mean(e_o ** 2)))
    ratio = np.abs(e_g - e_o) / bound
    print(f"\n[solve] max element ratio {ratio.max():.3f} (relative {rel(e_g, e_o):.2e})")
    assert np.all(ratio <= 1.0), (int(np.argmax(ratio)), float(ratio.max()))


# ------------------------------------------------------------------ random numbers
@pytest.mark.parametrize("count", [1, 7, 4096 * 3 + 5])
def test_gaussian_matches_oracle(ctx, count):
    g = host(ctx.gaussian(20160207, count))
    o = sampling.gaussian(20160207, count).astype(np.float32).astype(np.float64)
    assert np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-3)) < 2e-7


@pytest.mark.parametrize("N,count,zeros", [(1, 10, 0.0), (1000, 4097, 0.0), (100003, 65543, 0.1)])
def test_sampler_is_bit_exact(ctx, N, count, zeros):
    rng = np.random.default_rng(N)
    beta = rng.gamma(2.0, 1.0, N).astype(np.float32)
    if zeros:
        beta[rng.random(N) < zeros] = 0.0
        beta[0] = 1.0
    idx = ctx.sample_indices(dev(beta), seed=987654321123, epoch=5, count=count).cpu().numpy()
    W = sampling.quantize_weights(beta.astype(np.float64))
    ref = sampling.draw_indices(W, seed=987654321123, epoch=5, count=count)
    assert np.array_equal(idx, ref)


# ------------------------------------------------------------------ sketch
def _problem(n, d, alpha=1.5, lam=1e-4, seed=1):
    return inputs.make_ridge(n, d, alpha, lam, seed=seed)


# The FP32 Rayleigh-Ritz Gram (X Q)^T (X Q) takes the narrow 64-row-slab kernel for k + p <= 64 and the
# split-K GEMM above: n = 40 is one partial slab, 1500 rows end inside a slab of the last chunk,
# and k + p = 64 and 65 sit on either side of the switch.
@pytest.mark.parametrize("n,d,k,p,mixed", [(700, 40, 6, 5, False), (3000, 130, 20, 5, False),
                                           (3000, 130, 20, 5, True), (517, 61, 9, 4, False),
                                           (40, 30, 6, 5, False), (1500, 100, 59, 5, False),
                                           (1500, 100, 60, 5, False)])
def test_sketch_matches_oracle_with_the_same_omega(ctx, n, d, k, p, mixed):
    P = _problem(n, d, seed=n + d)
    Om = inputs.gaussian((k + p, d), seed=3)                      # Omega^T, (k+p) x d
    U, U64, lam, rc = ctx.sketch_build(dev(P.X), k, oversample=p, omega=dev(Om), sketch_fp32=int(not mixed),
                                       precision=binding.PREC_MIXED if mixed else binding.PREC_FP32)
    assert rc == binding.OK
    Uo, lo, _ = sketch.sketch(P.X.astype(np.float64), Om.T.astype(np.float64), k)
    lam_g = host(lam)
    tol = 3e-2 if mixed else 2e-5
    assert np.all(np.abs(lam_g - lo) <= tol * lo[0])
    Ug = host(U64)
    assert np.allclose(Ug.T @ Ug, np.eye(k), atol=1e-6 if not mixed else 1e-5)
    # compare the preconditioners (invariant to signs and rotations within ties) on probes
    Pg = precond.sketched_preconditioner(Ug, lam_g, P.lam)
    Po = precond.sketched_preconditioner(Uo, lo, P.lam)
    V = np.random.default_rng(0).standard_normal((d, 8))
    assert rel(Pg @ V, Po @ V) < (5e-2 if mixed else 1e-4)


def test_sketch_second_pass_takes_the_cholesky_when_q1_is_not_orthonormal(ctx):
    """Top k + p eigenvalues spanning 1e6: kappa(Y) ~ 3e6 leaves Q1^T Q1 = I + E with (k + p) max|E| ~ 6e-4
    after the first CholeskyQR pass (measured in FP64 on the host), above the 1e-5 up to which the second
    pass uses the series for (I + E)^{-1/2}; the gated Cholesky pass must run, or Q would be built from
    the first pass's inverse and not be orthonormal."""
    rng = np.random.default_rng(11)
    n, d, k, p = 2000, 40, 8, 4
    l = k + p
    Uq, _ = np.linalg.qr(rng.standard_normal((n, d)))
    Vq, _ = np.linalg.qr(rng.standard_normal((d, d)))
    sig = np.concatenate([np.geomspace(1.0, 1e-3, l), 1e-3 * np.geomspace(0.5, 0.1, d - l)]) * np.sqrt(n)
    X = ((Uq * sig) @ Vq.T).astype(np.float32)
    Om = inputs.gaussian((l, d), seed=3)
    U, U64, lam, rc = ctx.sketch_build(dev(X), k, oversample=p, omega=dev(Om), sketch_fp32=1,
                                       precision=binding.PREC_FP32)
    assert rc == binding.OK
    Ug = host(U64)
    assert np.allclose(Ug.T @ Ug, np.eye(k), atol=1e-6)
    _, lo, _ = sketch.sketch(X.astype(np.float64), Om.T.astype(np.float64), k)
    assert np.all(np.abs(host(lam) - lo) <= 2e-5 * lo[0])


def test_full_width_sketch_is_exact_on_gpu(ctx):
    """k + p = d: Rayleigh-Ritz on all of R^d returns the eigenvalues of C."""
    P = _problem(600, 24, alpha=1.0, seed=5)
    U, U64, lam, rc = ctx.sketch_build(dev(P.X), 19, oversample=5, sketch_fp32=1)
    ev = np.sort(np.linalg.eigvalsh(ridge.correlation(P.X.astype(np.float64))))[::-1]
    assert np.allclose(host(lam), ev[:19], rtol=2e-5, atol=1e-6 * ev[0])


def test_rank_deficient_sketch_is_reported(ctx):
    X = torch.zeros(300, 32, device="cuda")
    _, _, _, rc = ctx.sketch_build(X, 4)
    assert rc == binding.SKETCH_RANK_DEFICIENT


@pytest.mark.parametrize("max_epochs", [2, 12])
def test_rank_deficient_solve_falls_back_to_plain(ctx, max_epochs):
    """A zero test matrix Omega makes CholeskyQR break down; the solve learns it only once epochs are
    queued (at its first stop decision, or at the end when there is none), then redoes itself with
    P = I: status SKETCH_RANK_DEFICIENT and the same weights, bit for bit, as a k = 0 solve."""
    P = _problem(700, 40, seed=21)
    X, y = dev(P.X), dev(P.y)
    om = torch.zeros(4 + 5, 40, device="cuda")
    common = dict(batch=8, steps=40, max_epochs=max_epochs, stop_rule=binding.STOP_EPOCHS, seed=5, workgroups=1)
    res = ctx.svrg_solve(X, y, 1e-2, 4, 1e-30, omega=om, **common)
    ref = ctx.svrg_solve(X, y, 1e-2, 0, 1e-30, **common)
    assert res.status == binding.SKETCH_RANK_DEFICIENT
    assert ref.status == binding.OK
    assert res.report["k_used"] == 0 and res.report["epochs"] == ref.report["epochs"] == max_epochs
    assert torch.equal(res.w, ref.w)


# ------------------------------------------------------------------ preconditioning
def _sketch_inputs(d, k, seed):
    U = inputs.random_orthonormal(d, k, seed)
    lt = inputs.decreasing_values(k, seed, lo=1e-3, hi=2.0)
    return U, lt


@pytest.mark.parametrize("n,d,k,bf16", [(1000, 64, 8, False), (777, 101, 13, False), (2048, 256, 50, False),
                                        (1000, 64, 8, True), (300, 40, 0, False)])
def test_apply_matches_oracle(ctx, n, d, k, bf16):
    P = _problem(n, d, seed=7 + d)
    lam_reg = 1e-3
    if k:
        U, lt = _sketch_inputs(d, k, seed=d)
        U32 = U.astype(np.float32)
        Pm = precond.sketched_preconditioner(U32.astype(np.float64), lt, lam_reg)
        Xt, reg, beta = ctx.precondition_apply(dev(P.X), dev(U32), dev(lt, torch.float64), lam_reg, bf16=bf16)
    else:
        Pm = np.eye(d)
        Xt, reg, beta = ctx.precondition_apply(dev(P.X), None, None, lam_reg, bf16=bf16)
    comp = precond.Components(P.X, P.y, lam_reg, Pm)
    Xt_o = comp.Xt
    reg_o = np.sqrt(n * lam_reg) * comp.B
    tol = 1.2e-2 if bf16 else 3e-6
    row_err = np.linalg.norm(host(Xt) - Xt_o, axis=1) / np.linalg.norm(Xt_o, axis=1)
    assert row_err.max() < tol
    assert np.max(np.linalg.norm(host(reg) - reg_o, axis=1) / np.linalg.norm(reg_o, axis=1)) < tol
    beta_o = np.concatenate([np.sum(Xt_o ** 2, 1), np.sum(reg_o ** 2, 1)])
    assert np.max(np.abs(host(beta) - beta_o) / beta_o) < 3 * tol


def test_apply_with_padded_rows(ctx):
    P = _problem(500, 30, seed=9)
    U, lt = _sketch_inputs(30, 4, seed=4)
    Xt, reg, beta = ctx.precondition_apply(dev(P.X), dev(U.astype(np.float32)), dev(lt, torch.float64), 1e-2,
                                           ldt=32)
    Pm = precond.sketched_preconditioner(U.astype(np.float32).astype(np.float64), lt, 1e-2)
    assert rel(host(Xt)[:, :30], P.X.astype(np.float64) @ Pm) < 3e-6


# ------------------------------------------------------------------ full gradient
@pytest.mark.parametrize("n,d,k", [(1000, 64, 8), (4099, 257, 20), (1001, 30, 0), (20000, 1000, 50),
                                   (333, 7, 2), (6000, 2048, 0), (3000, 1100, 120), (1000, 2048, 128),
                                   (1003, 5000, 30), (2000, 2052, 0), (401, 6000, 0)])
def test_full_gradient_matches_oracle(ctx, n, d, k):
    """Where k d >= 20000 (d = 1000 with k = 50, d >= 1100 with k > 0) the P^{-1/2} applies run split
    over many workgroups. For d > 2048 the gradient pass splits each row's columns over the waves of a
    workgroup (2052, 5000 and 6000 columns: 3, 5 and 8 chunks of 256 per wave; n = 1003 leaves a
    workgroup with an odd number of rows)."""
    P = _problem(n, d, seed=11 + d)
    lam_reg = 1e-4
    wt = inputs.random_vector(d, seed=d)
    if k:
        U, lt = _sketch_inputs(d, k, seed=2 * d)
        U32 = U.astype(np.float32)
        Pm = precond.sketched_preconditioner(U32.astype(np.float64), lt, lam_reg)
        g, obj = ctx.full_gradient(dev(P.X), dev(P.y), dev(U32), dev(lt, torch.float64), lam_reg, dev(wt))
    else:
        Pm = np.eye(d)
        g, obj = ctx.full_gradient(dev(P.X), dev(P.y), None, None, lam_reg, dev(wt))
    comp = precond.Components(P.X, P.y, lam_reg, Pm)
    wt32 = wt.astype(np.float32).astype(np.float64)
    go = comp.full_gradient(wt32)
    # element by element, against the FP32 rounding-error scale of the pass (tests/_bounds.py)
    scale = gradient_scale(P.X, P.y, lam_reg, Pm, wt32)
    ratio = np.abs(host(g) - go) / scale
    print(f"\n[gradient n={n} d={d} k={k}] max |g - g_o| / scale = {ratio.max():.3f}; "
          f"scale / |g_o| median {np.median(scale / np.maximum(np.abs(go), 1e-300)):.2e}")
    assert np.all(ratio <= 8.0), (int(np.argmax(ratio)), float(ratio.max()))
    Lo = ridge.objective(P.X, P.y, lam_reg, Pm @ wt32)
    assert abs(obj - Lo) <= 2e-6 * Lo


def test_full_gradient_flags_non_finite_input(ctx):
    P = _problem(200, 16, seed=3)
    X = P.X.copy()
    X[17, 3] = np.nan
    with pytest.raises(binding.ScsError) as e:
        ctx.full_gradient(dev(X), dev(P.y), None, None, 1e-3, dev(np.zeros(16)))
    assert e.value.code == binding.ENONFINITE


# ------------------------------------------------------------------ one SVRG epoch
def _bf16_values(a):
    """Round an FP64 array to BF16 (nearest even) on the host; returns the BF16 tensor and its values."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t, t.float().numpy().astype(np.float64)


def _injected_rows(X, lam_reg, Pm, ldt, bf16):
    """The n + d rows the inner loop reads (x~_i = P^{-1/2} x_i and sqrt(n lam) b_j, Sec. 5.1), formed by
    the oracle in FP64 and stored as FP32 or BF16 with leading dimension ldt. Returns the device rows
    and the FP64 values of what was stored, so both sides run on exactly the same rows."""
    n, d = X.shape
    Xt = np.asarray(X, dtype=np.float64) @ Pm
    R = np.sqrt(n * lam_reg) * Pm
    dev_rows, vals = [], []
    for A in (Xt, R):
        pad = np.zeros((A.shape[0], ldt))
        pad[:, :d] = A
        if bf16:
            t, v = _bf16_values(pad)
            dev_rows.append(t.cuda())
        else:
            t = torch.from_numpy(pad.astype(np.float32))
            v = pad.astype(np.float32).astype(np.float64)
            dev_rows.append(t.cuda())
        vals.append(v[:, :d])
    return dev_rows[0], dev_rows[1], vals[0], vals[1]


def _epoch_parity(ctx, X, y, lam_reg, Pm, b, m, W, bf16, ldt, c, seed, wave_rows=0):
    """One inner loop (Alg. 1) on the GPU and in the oracle from the same rows, snapshot, snapshot
    gradient, step and index stream; the averaged step is compared element by element."""
    n, d = X.shape
    Xt_d, reg_d, Xt64, reg64 = _injected_rows(X, lam_reg, Pm, ldt, bf16)
    comp = precond.Components.from_rows(Xt64, reg64 / np.sqrt(n * lam_reg), y, lam_reg)
    beta64 = np.concatenate([np.sum(Xt64 ** 2, 1), np.sum(reg64 ** 2, 1)])
    beta32 = beta64.astype(np.float32)
    Wq = sampling.quantize_weights(beta32.astype(np.float64)).astype(np.float64)
    q = Wq / Wq.sum()                      # the distribution the integer sampler draws from
    wt0 = inputs.random_vector(d, seed=seed, scale=0.3).astype(np.float32).astype(np.float64)
    mu64 = comp.full_gradient(wt0)
    eta = c / svrg.beta_hat(comp)
    idx = inputs.index_stream(n + d, m * b, seed=seed + 1)
    wt = dev(wt0)
    ctx.svrg_epoch(n, d, Xt_d, reg_d, dev(beta32), dev(mu64), dev(idx, torch.int32), m, b, eta, average=True,
                   workgroups=W, wt=wt, wave_rows=wave_rows)
    trace = []
    wo, _ = svrg.svrg(comp, wt0, m, eta, 1, b, lambda s: idx, average=True, q=q, trace=trace)
    step_o = wo - wt0
    step_g = host(wt) - wt0

    def rows(it):
        it = np.asarray(it)
        return np.where((it < n)[:, None], Xt64[np.minimum(it, n - 1)], reg64[np.maximum(it - n, 0)])

    # the look-ahead loop's Gram block: three BF16 products per FP32 entry (relative error below 2^-16),
    # exact for BF16 rows (FP32 accumulation only)
    gram_rel = 0.0 if wave_rows != binding.LOOKAHEAD else (8 * U32 if bf16 else 2.0 ** -15)
    scale = epoch_scale(rows, 1.0 / (n * q), idx, trace, wt0, mu64, eta, b, gram_rel=gram_rel)
    scale = 8.0 * scale + 2 * U32 * (np.abs(wo) + np.abs(step_o))
    ratio = np.abs(step_g - step_o) / scale
    print(f"\n[epoch n={n} d={d} b={b} m={m} W={W} wave_rows={wave_rows} bf16={bf16}] "
          f"max |step - step_o| / bound = {ratio.max():.3f}; "
          f"relative step error {rel(step_g, step_o):.2e}")
    assert np.all(ratio <= 1.0), (int(np.argmax(ratio)), float(ratio.max()))


@pytest.mark.parametrize("n,d,k,b,W,bf16,ldt,wr", [
    (400, 24, 4, 8, 1, False, 24, 0), (2000, 100, 10, 64, 1, False, 100, 0),
    (2000, 100, 10, 64, 2, False, 128, 0), (1500, 257, 12, 33, 3, False, 260, 0),
    (2000, 100, 10, 64, 1, True, 128, 0), (900, 37, 0, 5, 1, False, 40, 0),
    (400, 24, 4, 8, 16, False, 24, 0), (700, 61, 5, 40, 15, True, 64, 0),
    # minibatches past 64 rows (two and four wave-rows) and every layout on one shape
    (3000, 100, 10, 100, 1, False, 100, 2), (3000, 100, 10, 128, 2, True, 128, 2),
    (4000, 130, 10, 200, 3, False, 132, 4), (4000, 61, 5, 256, 1, False, 64, 4),
    (2000, 100, 10, 37, 2, False, 100, 1), (2000, 100, 10, 37, 2, False, 100, 2),
    (2000, 100, 10, 37, 2, False, 100, 4), (1500, 61, 5, 150, 15, True, 64, 4),
    # the look-ahead loop (b <= 64, at most 64 columns per workgroup)
    (400, 24, 4, 8, 1, False, 24, 8), (2000, 100, 10, 64, 2, False, 100, 8), (2000, 100, 10, 64, 2, True, 128, 8),
    (1500, 257, 12, 33, 5, False, 260, 8), (900, 37, 0, 5, 1, False, 40, 8), (700, 61, 5, 40, 15, True, 64, 8),
    (2000, 100, 10, 17, 2, False, 100, 8)])
def test_epoch_matches_oracle_on_an_injected_stream(ctx, n, d, k, b, W, bf16, ldt, wr):
    """Small and ragged shapes, including more workgroups than column quads (W = 16 at d = 24 and
    W = 15 at d = 61: the last workgroups own no column and only take part in the exchange), minibatches
    up to 256 rows and each split of a workgroup's waves over rows (wr wave-rows; 0 = the default)."""
    P = _problem(n, d, alpha=2.0, seed=13 + d)
    lam_reg = 1e-3
    if k:
        U, lt = _sketch_inputs(d, k, seed=3 * d)
        Pm = precond.sketched_preconditioner(U.astype(np.float32).astype(np.float64), lt, lam_reg)
    else:
        Pm = np.eye(d)
    _epoch_parity(ctx, P.X, P.y, lam_reg, Pm, b, 3 * n // b, W, bf16, ldt, 4.0, seed=n, wave_rows=wr)


@pytest.fixture(scope="module")
def bench_shape_rows():
    """The headline workload's shape: n = 100000, d = 1000, spectrum j^-1.5, lambda = 1e-5, rank-50
    preconditioner."""
    cfg = inputs.WORKLOADS["fp32_n100000_d1000"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED + 60)
    Pm, _, _ = precond.exact_preconditioner(ridge.correlation(P.X), cfg["lam"], cfg["k"])
    return P, Pm, cfg


@pytest.mark.parametrize("W", [16, 8])
@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("b,wr", [(64, 0), (64, 1), (128, 2), (256, 4), (64, binding.LOOKAHEAD),
                                  (32, binding.LOOKAHEAD)])
def test_epoch_at_the_benchmark_launch_shape(ctx, bench_shape_rows, W, bf16, b, wr):
    """The inner loop at the benchmark's shape (n = 100000, d = 1000, rows padded to 1024 columns) with
    16 or 8 cooperating workgroups of 64 or 128 columns, minibatches of 64 to 256 rows and the wave-row
    split each uses; m = 6272 / b steps (98 at b = 64, the benchmark's epoch)."""
    P, Pm, cfg = bench_shape_rows
    if W == 8 and wr in (4, binding.LOOKAHEAD):
        pytest.skip("four wave-rows and the look-ahead loop take slices of at most 64 columns")
    _epoch_parity(ctx, P.X, P.y, cfg["lam"], Pm, b, 6272 // b, W, bf16, 1024, 64.0, seed=101,
                  wave_rows=wr)


# ------------------------------------------------------------------ the paper's synthetic data
@pytest.mark.parametrize("alpha", [1.0, 2.0])
def test_papers_synthetic_data_tracks_the_oracle(ctx, alpha):
    """The experiments' synthetic regression (Sec. 6: singular values 1/q or 1/q^2, unit-norm examples,
    lambda = 1e-8, k = 30) at n = 6000, d = 4200, wider than the 4096 entries the P^{-1/2} apply stages
    in LDS, so it runs the unstaged path. Same Omega and index stream as the oracle: after three epochs
    the GPU's distance to w* matches the oracle's trajectory and its suboptimality."""
    n, d, lam, k, b = 6000, 4200, 1e-8, 30, 64
    X, y, _ = inputs.make_spectral_rows(n, d, alpha, seed=inputs.BASE_SEED + 50)
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED + 51)
    m, S = n // b, 3
    idx = inputs.index_stream(n + d, S * m * b, seed=79).reshape(S, -1)
    res = ctx.svrg_solve(dev(X), dev(y), lam, k, 0.0, omega=dev(Om), indices=dev(idx, torch.int32), steps=m, batch=b,
                         max_epochs=S, stop_rule=binding.STOP_EPOCHS, step_scale=8.0, sketch_fp32=1)
    assert res.status == binding.OK, res.report
    wo, _, info = svrg.scsvrg(X64, y64, lam, k, Om.T.astype(np.float64), m, S, b, lambda s: idx[s], c=8.0)
    ws = ridge.closed_form(X64, y64, lam)
    wg = host(res.w).astype(np.float64)
    assert_tracks(wg, wo, ws, 5e-2)
    so_g, so_o = ridge.suboptimality(X64, lam, wg, ws), ridge.suboptimality(X64, lam, wo, ws)
    assert abs(so_g - so_o) <= 0.1 * so_o, (so_g, so_o)
    assert abs(res.report["eta"] - info["eta"]) <= 1e-4 * info["eta"]


# ------------------------------------------------------------------ whole solve
def test_solve_with_injected_randomness_tracks_the_oracle(ctx):
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED)
    n, d, k, b = cfg["n"], cfg["d"], cfg["k"], cfg["b"]
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED)
    m, S = n // b, 4
    idx = inputs.index_stream(n + d, S * m * b, seed=77).reshape(S, -1)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), cfg["lam"], k, 0.0, omega=dev(Om), indices=dev(idx, torch.int32),
                         steps=m, batch=b, max_epochs=S, stop_rule=binding.STOP_EPOCHS, step_scale=4.0, sketch_fp32=1)
    assert res.status == binding.OK
    wo, _, info = svrg.scsvrg(X64, y64, cfg["lam"], k, Om.T.astype(np.float64), m, S, b, lambda s: idx[s], c=4.0)
    ws = ridge.closed_form(X64, y64, cfg["lam"])
    assert_tracks(host(res.w), wo, ws, 2e-2)      # same trajectory to FP32 accuracy of the sketch
    assert abs(res.report["eta"] - info["eta"]) <= 1e-4 * info["eta"]


@pytest.mark.parametrize("k", [10, 0])
def test_uniform_sampling_tracks_the_oracle(ctx, k):
    """q_i = 1/(n+d) (the original SVRG's sampling, Sec. 4.2) instead of q_i proportional to beta_i: with
    the same Omega and index stream the GPU solve follows the oracle's uniform-sampling trajectory."""
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED + 3)
    n, d, b = cfg["n"], cfg["d"], cfg["b"]
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED + 4)
    m, S, c = n // b, 4, 1.0
    idx = inputs.index_stream(n + d, S * m * b, seed=78).reshape(S, -1)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), cfg["lam"], k, 0.0, omega=dev(Om) if k else None,
                         indices=dev(idx, torch.int32), steps=m, batch=b, max_epochs=S, stop_rule=binding.STOP_EPOCHS,
                         step_scale=c, uniform_sampling=1, sketch_fp32=1)
    assert res.status == binding.OK
    Pm, _, _ = svrg.preconditioner_from_sketch(X64, cfg["lam"], k, Om.T.astype(np.float64))
    comp = precond.Components(X64, y64, cfg["lam"], Pm)
    eta = c / svrg.beta_hat(comp)
    wt, _ = svrg.svrg(comp, np.zeros(d), m, eta, S, b, lambda s: idx[s], q=np.full(n + d, 1.0 / (n + d)))
    wo = Pm @ wt
    ws = ridge.closed_form(X64, y64, cfg["lam"])
    assert_tracks(host(res.w), wo, ws, 2e-2)
    assert abs(res.report["eta"] - eta) <= 1e-4 * eta


@pytest.mark.parametrize("k,mixed", [(10, False), (0, False), (10, True)])
def test_solve_reaches_the_closed_form(ctx, k, mixed):
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, cfg["lam"])
    Ls = ridge.objective(X64, y64, cfg["lam"], ws)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), cfg["lam"], k, 1e-8, batch=cfg["b"], max_epochs=60 if k else 200,
                         stop_rule=binding.STOP_GAP, f_star=Ls, step_scale=8.0 if k else 2.0,
                         precision=binding.PREC_MIXED if mixed else binding.PREC_FP32)
    assert res.status == binding.OK, res.report
    so = ridge.suboptimality(X64, cfg["lam"], host(res.w), ws)
    assert so <= 1.5e-8


def test_solve_fp32_gate_relative_error(ctx):
    """FP32 mode reaches ||w - w*|| <= 1e-5 ||w*|| (the certificate stop rule drives it there)."""
    P = inputs.make_ridge(4000, 120, 1.5, 1e-3, seed=31)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, P.lam)
    # certificate <= 5e-12 bounds ||w - w*||^2 <= 2 * 5e-12 / lambda_min(C + lam I) ~ 6e-9 here
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, 12, 5e-12, batch=32, max_epochs=120,
                         stop_rule=binding.STOP_CERTIFICATE, step_scale=8.0)
    assert res.status == binding.OK, res.report
    assert rel(host(res.w), ws) <= 1e-5


def test_divergence_returns_the_last_good_snapshot(ctx):
    P = inputs.make_ridge(1000, 50, 1.5, 1e-3, seed=32)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, 0, 1e-12, batch=16, max_epochs=10, step_scale=1e4,
                         stop_rule=binding.STOP_EPOCHS)
    assert res.status == binding.DIVERGED
    assert torch.isfinite(res.w).all()


def test_invalid_arguments_are_rejected(ctx):
    P = inputs.make_ridge(100, 10, 1.0, 1e-3, seed=33)
    for lam, k in [(0.0, 2), (-1.0, 2), (1e-3, 11), (1e-3, -1), (1e-3, 8)]:   # k + p > d for k = 8
        with pytest.raises(binding.ScsError) as e:
            ctx.svrg_solve(dev(P.X), dev(P.y), lam, k, 1e-6)
        assert e.value.code == binding.EINVAL


def test_non_finite_input_is_reported(ctx):
    P = inputs.make_ridge(500, 20, 1.0, 1e-3, seed=34)
    y = P.y.copy()
    y[3] = np.inf
    with pytest.raises(binding.ScsError) as e:
        ctx.svrg_solve(dev(P.X), dev(y), P.lam, 0, 1e-6)
    assert e.value.code == binding.ENONFINITE


def test_epoch_cap_reports_not_converged(ctx):
    P = inputs.make_ridge(1000, 50, 2.0, 1e-5, seed=35)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, 0, 1e-30, max_epochs=2)
    assert res.status == binding.NOT_CONVERGED
    assert res.report["epochs"] == 2


# ------------------------------------------------------------------ batched solves
def _uneven_batch(shapes, seed0=40):
    probs = []
    for i, (n, d, alpha, lam, k) in enumerate(shapes):
        P = inputs.make_ridge(n, d, alpha, lam, seed=seed0 + i)
        probs.append((P, k))
    return probs


UNEVEN = [(1500, 100, 2.0, 1e-4, 6), (700, 37, 1.2, 1e-3, 2), (3000, 257, 1.5, 1e-5, 16),
          (400, 64, 2.5, 1e-6, 4), (2200, 130, 1.8, 1e-4, 0), (900, 24, 1.0, 3e-4, 1)]


@pytest.mark.parametrize("mixed", [False, True])
def test_batched_equals_single_solves(ctx, mixed):
    """The batched launches run the same kernels in the same order per problem: bit-identical to
    single solves with one workgroup per inner loop."""
    probs = _uneven_batch(UNEVEN)
    common = dict(batch=16, steps=50, max_epochs=3, stop_rule=binding.STOP_EPOCHS, step_scale=1.0, seed=99,
                  precision=binding.PREC_MIXED if mixed else binding.PREC_FP32, workgroups=1)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    rc, wb, reps = ctx.svrg_solve_batched(Xs, ys, [P.lam for P, _ in probs], [k for _, k in probs], 0.0, **common)
    for i, (P, k) in enumerate(probs):
        r = ctx.svrg_solve(Xs[i], ys[i], P.lam, k, 0.0, **common)
        assert reps[i]["status"] == r.status, (i, reps[i]["status"], r.status)
        assert torch.equal(wb[i], r.w), (i, rel(host(wb[i]), host(r.w)))
        assert reps[i]["epochs"] == r.report["epochs"] and reps[i]["k_used"] == k
    assert rc == binding.OK, [r["status"] for r in reps]


@pytest.mark.parametrize("d,k,W", [(1100, 120, 3), (1000, 50, 2)])
def test_split_apply_is_bit_identical_to_the_one_workgroup_apply(ctx, d, k, W):
    """With k d >= 20000 a single solve spreads the P^{-1/2} applies of the premap and the gradient
    finish over many workgroups (k d = 132000, and 50000 as in the FP32 n = 100000 benchmark); a batch
    of one problem keeps them in one workgroup. Same per-row and per-quad arithmetic: the two solves
    agree bit for bit (with the same W inner-loop workgroups, the fewest that keep d columns within 512
    per workgroup)."""
    probs = _uneven_batch([(3000, d, 1.5, 1e-4, k)], seed0=80)
    assert k * d >= 20000
    common = dict(batch=16, steps=60, max_epochs=3, stop_rule=binding.STOP_EPOCHS, step_scale=2.0, seed=7,
                  workgroups=W)
    (P, k), = probs
    X, y = dev(P.X), dev(P.y)
    rc, wb, reps = ctx.svrg_solve_batched([X], [y], [P.lam], [k], 0.0, **common)
    r = ctx.svrg_solve(X, y, P.lam, k, 0.0, **common)
    assert rc == binding.OK and r.status == binding.OK and reps[0]["workgroups"] == W
    assert torch.equal(wb[0], r.w), rel(host(wb[0]), host(r.w))
    assert reps[0]["objective"] == r.report["objective"]


def test_batched_wide_problem_uses_cooperating_workgroups(ctx):
    probs = _uneven_batch([(2000, 600, 1.5, 1e-4, 8), (800, 90, 2.0, 1e-3, 3), (1200, 513, 1.2, 1e-4, 0)], seed0=60)
    common = dict(batch=32, steps=40, max_epochs=2, stop_rule=binding.STOP_EPOCHS, step_scale=1.0, seed=5)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    # the default is ceil(600 / 256) = 3 cooperating workgroups per problem; 2 (= ceil(600 / 512), the
    # fewest allowed) and 3 must both match single solves with the same count
    for W in (2, 0):
        rc, wb, reps = ctx.svrg_solve_batched(Xs, ys, [P.lam for P, _ in probs], [k for _, k in probs], 0.0,
                                              workgroups=W, **common)
        assert rc == binding.OK
        for i, (P, k) in enumerate(probs):
            assert reps[i]["workgroups"] == (W or 3)
            r = ctx.svrg_solve(Xs[i], ys[i], P.lam, k, 0.0, workgroups=W or 3, **common)
            assert torch.equal(wb[i], r.w), (W, i)


WELL_POSED = [(1500, 100, 2.0, 1e-4, 10), (700, 37, 1.2, 1e-3, 2), (3000, 257, 1.5, 1e-4, 16),
              (400, 64, 2.5, 1e-4, 8), (2200, 130, 1.8, 1e-3, 0), (900, 24, 1.0, 3e-4, 1)]


def test_batched_solves_reach_their_closed_forms(ctx):
    probs = _uneven_batch(WELL_POSED, seed0=70)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    rc, wb, reps = ctx.svrg_solve_batched(Xs, ys, [P.lam for P, _ in probs], [k for _, k in probs], 1e-10,
                                          batch=16, max_epochs=150, stop_rule=binding.STOP_CERTIFICATE,
                                          step_scale=2.0)
    assert rc == binding.OK, [r["status"] for r in reps]
    for i, (P, k) in enumerate(probs):
        X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
        ws = ridge.closed_form(X64, y64, P.lam)
        # the certificate bounds the gap: L(w) - L* <= 1e-10 (plus FP32 evaluation error)
        assert ridge.suboptimality(X64, P.lam, host(wb[i]), ws) <= 2e-10, i
        assert reps[i]["certificate"] <= 1e-10


def test_batched_rejects_what_it_cannot_do(ctx):
    probs = _uneven_batch(UNEVEN[:2])
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    with pytest.raises(binding.ScsError) as e:   # the gap rule needs one optimum per problem
        ctx.svrg_solve_batched(Xs, ys, [1e-3, 1e-3], [2, 2], 1e-6, stop_rule=binding.STOP_GAP)
    assert e.value.code == binding.EINVAL
    with pytest.raises(binding.ScsError) as e:
        ctx.svrg_solve_batched(Xs, ys, [1e-3, 1e-3], [2, 40], 1e-6)   # k + p > d for the second problem
    assert e.value.code == binding.EINVAL


@pytest.mark.parametrize("k", [0, 6])
def test_certificate_bounds_the_gap(ctx, k):
    """Stopping on the certificate guarantees L(w) - L* <= eps, with and without the preconditioner."""
    P = inputs.make_ridge(3000, 80, 1.5, 1e-3, seed=36)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, P.lam)
    eps = 1e-9
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, k, eps, batch=16, max_epochs=200,
                         stop_rule=binding.STOP_CERTIFICATE, step_scale=2.0)
    assert res.status == binding.OK, res.report
    assert res.report["certificate"] <= eps
    assert ridge.suboptimality(X64, P.lam, host(res.w), ws) <= eps * 1.01


# ------------------------------------------------------------------ regularization path (shared sketch)
@pytest.mark.parametrize("implicit", [False, True])
@pytest.mark.parametrize("n,d,k,ny,lams", [(3000, 200, 10, 3, [1e-4, 1e-3, 1e-2]),
                                            (2500, 601, 12, 2, [3e-4, 3e-3])])
def test_path_solves_reach_their_closed_forms(ctx, n, d, k, ny, lams, implicit):
    """Every (lambda, y) solve of a path reaches its own closed form; with implicit_apply the rows
    x~_i are never formed (the inner loop works from x_i and z_i = U~^T x_i)."""
    P = inputs.make_ridge(n, d, 1.5, lams[0], seed=80)
    X64 = P.X.astype(np.float64)
    # right-hand side 0 is the problem's own y; the others come from other planted weights
    extra = [P.X.astype(np.float64) @ inputs.random_vector(d, seed=90 + r) + 0.1 * inputs.random_vector(n, seed=95 + r)
             for r in range(1, ny)]
    Ys = np.stack([P.y.astype(np.float64)] + extra).astype(np.float32)
    eps = 1e-9
    rc, W, reps = ctx.svrg_solve_path(dev(P.X), dev(Ys), lams, k, eps, batch=16, max_epochs=200,
                                      stop_rule=binding.STOP_CERTIFICATE, step_scale=2.0,
                                      implicit_apply=int(implicit))
    assert rc == binding.OK, [r["status"] for r in reps]
    Wh = host(W)
    for j, lam in enumerate(lams):
        for r in range(ny):
            ws = ridge.closed_form(X64, Ys[r].astype(np.float64), lam)
            so = ridge.suboptimality(X64, lam, Wh[j * ny + r], ws)
            assert so <= eps * 1.01, (j, r, so)
            assert reps[j * ny + r]["k_used"] == k


def test_batched_gap_rule_with_per_problem_optima(ctx):
    probs = _uneven_batch(WELL_POSED[:4], seed0=75)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    fs, wss = [], []
    for P, _ in probs:
        X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
        ws = ridge.closed_form(X64, y64, P.lam)
        wss.append(ws)
        fs.append(ridge.objective(X64, y64, P.lam, ws))
    eps = 1e-8
    rc, wb, reps = ctx.svrg_solve_batched(Xs, ys, [P.lam for P, _ in probs], [k for _, k in probs], eps, f_star=fs,
                                          batch=16, max_epochs=150, stop_rule=binding.STOP_GAP, step_scale=2.0)
    assert rc == binding.OK, [r["status"] for r in reps]
    for i, (P, _) in enumerate(probs):
        assert ridge.suboptimality(P.X.astype(np.float64), P.lam, host(wb[i]), wss[i]) <= 1.5 * eps


def test_step_backoff_recovers_from_a_too_large_step(ctx):
    """A snapshot whose objective blows up is rejected, the step halved and the solve goes on."""
    P = inputs.make_ridge(2000, 50, 1.5, 1e-3, seed=37)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, P.lam)
    Ls = ridge.objective(X64, y64, P.lam, ws)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, 0, 1e-9, batch=8, max_epochs=200, step_scale=40.0,
                         stop_rule=binding.STOP_GAP, f_star=Ls)
    assert res.status == binding.OK, res.report
    assert 1 <= res.report["backoffs"] <= 6
    assert ridge.suboptimality(X64, P.lam, host(res.w), ws) <= 1.5e-9


def test_autotuned_workgroups_solve_matches_the_closed_form(ctx):
    P = inputs.make_ridge(3000, 300, 1.5, 1e-4, seed=38)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, P.lam)
    Ls = ridge.objective(X64, y64, P.lam, ws)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), P.lam, 12, 1e-9, batch=32, max_epochs=100, step_scale=4.0,
                         stop_rule=binding.STOP_GAP, f_star=Ls, workgroups=-1)
    assert res.status == binding.OK, res.report
    assert res.report["workgroups"] in (3, 5, 10)   # ceil(300 / 128), ceil(300 / 64), ceil(300 / 32)
    assert ridge.suboptimality(X64, P.lam, host(res.w), ws) <= 1.5e-9


# ------------------------------------------------------------------ the in-library autotuner
def test_autotune_picks_options_that_reach_eps(ctx):
    """scs_autotune scores (b, c, m, launch shape) by wall time to the stop rule; the options it returns must
    themselves solve the problem to eps (gap against the oracle's FP64 optimum) with the caller's seed."""
    P = _problem(6000, 120, alpha=1.5, seed=91)
    lam, k, eps = 1e-4, 8, 1e-7
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    ws = ridge.closed_form(X64, y64, lam)
    Ls = ridge.objective(X64, y64, lam, ws)
    X, y = dev(P.X), dev(P.y)
    with pytest.raises(binding.ScsError):
        ctx.autotune(X, y, lam, k, eps, stop_rule=binding.STOP_EPOCHS)
    tuned, ms = ctx.autotune(X, y, lam, k, eps, stop_rule=binding.STOP_GAP, f_star=Ls, max_epochs=60, seed=7)
    print(f"\n[autotune] {tuned} {ms:.2f} ms")
    assert tuned["batch"] in (32, 64, 128) and tuned["step_scale"] > 0 and tuned["epoch_factor"] > 0
    assert tuned["seed"] == 7
    r = ctx.svrg_solve(X, y, lam, k, eps, **tuned)
    assert r.status == binding.OK, r.report
    assert ridge.objective(X64, y64, lam, host(r.w)) - Ls <= 1.5 * eps


# ------------------------------------------------------------------ warm starts, checkpoints, the lambda rule
def test_resume_from_a_checkpoint_reproduces_the_uninterrupted_solve(ctx):
    """A solve stopped after 3 epochs (its snapshot written to wt_out) and resumed from that snapshot with
    epoch_offset = 3 ends bit for bit where 6 uninterrupted epochs end (same sketch, same index streams)."""
    P = _problem(4000, 150, alpha=1.5, seed=71)
    X, y = dev(P.X), dev(P.y)
    common = dict(batch=32, steps=60, stop_rule=binding.STOP_EPOCHS, step_scale=8.0, seed=11)
    full_wt = torch.empty(150, device="cuda")
    full = ctx.svrg_solve(X, y, 1e-4, 10, 0.0, max_epochs=6, wt_out=full_wt, **common)
    ck = torch.empty(150, device="cuda")
    first = ctx.svrg_solve(X, y, 1e-4, 10, 0.0, max_epochs=3, wt_out=ck, **common)
    assert first.status == binding.OK and first.report["epochs"] == 3
    res_wt = torch.empty(150, device="cuda")
    resumed = ctx.svrg_solve(X, y, 1e-4, 10, 0.0, max_epochs=3, w0=ck, w0_preconditioned=1, epoch_offset=3,
                             wt_out=res_wt, **common)
    assert resumed.status == binding.OK and resumed.report["epochs"] == 3
    assert torch.equal(resumed.w, full.w)
    assert torch.equal(res_wt, full_wt)
    # a wrong offset replays other index streams and ends elsewhere
    other = ctx.svrg_solve(X, y, 1e-4, 10, 0.0, max_epochs=3, w0=ck, w0_preconditioned=1, epoch_offset=0, **common)
    assert not torch.equal(other.w, full.w)


@pytest.mark.parametrize("k", [0, 10])
def test_warm_start_in_the_original_space(ctx, k):
    """w0 given in the original space is mapped by P^{1/2}: started at the optimum the solve stops at its first
    snapshot (no epoch), and started near it needs fewer epochs than from 0."""
    P = _problem(5000, 120, alpha=1.5, seed=72)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    lam, eps = 1e-4, 1e-8
    ws = ridge.closed_form(X64, y64, lam)
    Ls = ridge.objective(X64, y64, lam, ws)
    X, y = dev(P.X), dev(P.y)
    common = dict(batch=32, epoch_factor=0.5, stop_rule=binding.STOP_GAP, f_star=Ls, step_scale=8.0,
                  max_epochs=300, seed=5)
    cold = ctx.svrg_solve(X, y, lam, k, eps, **common)
    at = ctx.svrg_solve(X, y, lam, k, eps, w0=dev(ws), **common)
    near = ctx.svrg_solve(X, y, lam, k, eps, w0=dev(ws + 1e-3 * np.random.default_rng(1).standard_normal(120)),
                          **common)
    print(f"\n[warm start k={k}] epochs cold {cold.report['epochs']}, at w* {at.report['epochs']}, "
          f"near w* {near.report['epochs']}")
    assert cold.status == at.status == near.status == binding.OK
    assert at.report["epochs"] == 0
    assert near.report["epochs"] < cold.report["epochs"]
    assert ridge.objective(X64, y64, lam, host(near.w)) - Ls <= 1.5 * eps


def test_warm_started_path_reaches_every_closed_form_with_fewer_epochs(ctx):
    """Continuation along a regularization path (Sec. 2.2): lambdas from large to small, each lambda's solves
    start from the previous lambda's solutions; every solve reaches its closed form, in fewer epochs in total
    than the same path solved from 0."""
    n, d, k, ny = 4000, 160, 12, 2
    P = _problem(n, d, alpha=1.5, seed=73)
    X64 = P.X.astype(np.float64)
    rng = np.random.default_rng(4)
    Y64 = np.stack([P.y.astype(np.float64), X64 @ rng.standard_normal(d) + 0.1 * rng.standard_normal(n)])
    Y32 = Y64.astype(np.float32)
    lams = list(np.logspace(-2, -5, 7))
    _, Lmat = ridge.closed_forms(X64, Y32.astype(np.float64), lams)
    fs = [float(v) for v in Lmat.reshape(-1)]           # solve j * ny + r
    eps = 1e-8
    common = dict(batch=32, epoch_factor=0.25, stop_rule=binding.STOP_GAP, step_scale=8.0, max_epochs=120, seed=9)
    X, Y = dev(P.X), dev(Y32)
    rc_c, Wc, rep_c = ctx.svrg_solve_path(X, Y, lams, k, eps, f_star=fs, **common)
    rc_w, Ww, rep_w = ctx.svrg_solve_path(X, Y, lams, k, eps, f_star=fs, warm_start=1, **common)
    assert rc_c == binding.OK and rc_w == binding.OK
    ep_c = sum(r["epochs"] for r in rep_c)
    ep_w = sum(r["epochs"] for r in rep_w)
    print(f"\n[path] total epochs cold {ep_c}, warm {ep_w}")
    for p in range(len(lams) * ny):
        j, r = divmod(p, ny)
        gap = ridge.objective(X64, Y32[r].astype(np.float64), lams[j], host(Ww[p])) - fs[p]
        assert gap <= 1.5 * eps, (p, gap)
    assert ep_w < ep_c


@pytest.mark.parametrize("n,d,k", [(3000, 40, 35), (5000, 200, 12)])
def test_budget_regularization_matches_the_oracle(ctx, n, d, k):
    """Sec. 2.2's two regularizations from the GPU sketch (same Omega as the oracle's sketch) and tr(C);
    with k + p = d the sketch is exact and the values are those of the full spectrum."""
    P = _problem(n, d, alpha=1.5, seed=74)
    X64 = P.X.astype(np.float64)
    p = min(5, d - k)
    seed = 123
    Om = sampling.gaussian(seed, (k + p) * d).astype(np.float32).reshape(k + p, d)   # the drawn Omega^T
    pre, plain, rc = ctx.regularization_for_budget(dev(P.X), k, oversample=p, seed=seed, sketch_fp32=1)
    assert rc == binding.OK
    _, lt, _ = sketch.sketch(X64, Om.T.astype(np.float64), k)
    trace = float(np.sum(X64 * X64)) / n
    pre_o, plain_o = ridge.budget_lambdas_estimated(lt, trace, n, k)
    print(f"\n[budget n={n} d={d} k={k}] GPU {pre:.6e} {plain:.6e}  oracle {pre_o:.6e} {plain_o:.6e}")
    assert plain == pytest.approx(plain_o, rel=1e-6)
    assert pre == pytest.approx(pre_o, rel=1e-4)
    if k + p == d:
        ev = np.linalg.eigvalsh(ridge.correlation(X64))
        assert (pre, plain) == pytest.approx(ridge.budget_lambdas(ev, n, k), rel=1e-4)


# ------------------------------------------------------------------ epochs replayed from a captured graph
@pytest.mark.parametrize("mixed", [False, True])
def test_batched_graph_replay_equals_enqueued_epochs(ctx, mixed):
    """The batched solve's epochs replayed from a captured hipGraph (the default; 8 epochs per replay, the
    epoch number read from a device clock) give bit for bit what the host-enqueued epochs give. 21 epochs:
    two replays (with the host waiting on the first while the second runs), then five enqueued epochs and
    the final evaluation; a second graph solve in a row must agree too."""
    probs = _uneven_batch(UNEVEN, seed0=90)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    common = dict(batch=16, steps=30, max_epochs=21, stop_rule=binding.STOP_EPOCHS, step_scale=1.0, seed=3,
                  precision=binding.PREC_MIXED if mixed else binding.PREC_FP32)
    lams, ks = [P.lam for P, _ in probs], [k for _, k in probs]
    rc_e, we, rep_e = ctx.svrg_solve_batched(Xs, ys, lams, ks, 0.0, no_graph=1, **common)
    for rep in range(2):
        rc_g, wg, rep_g = ctx.svrg_solve_batched(Xs, ys, lams, ks, 0.0, **common)
        assert rc_g == rc_e == binding.OK
        for i in range(len(probs)):
            assert torch.equal(wg[i], we[i]), (rep, i)
            assert rep_g[i]["epochs"] == rep_e[i]["epochs"] == 21


def test_batched_graph_replay_stops_with_the_stop_rule(ctx):
    """With the certificate rule every problem stops inside a replay; the graph mode returns the same weights
    and epoch counts as the enqueued mode."""
    probs = _uneven_batch(WELL_POSED, seed0=70)
    Xs = [dev(P.X) for P, _ in probs]
    ys = [dev(P.y) for P, _ in probs]
    common = dict(batch=16, max_epochs=150, stop_rule=binding.STOP_CERTIFICATE, step_scale=2.0)
    lams, ks = [P.lam for P, _ in probs], [k for _, k in probs]
    rc_e, we, rep_e = ctx.svrg_solve_batched(Xs, ys, lams, ks, 1e-10, no_graph=1, **common)
    rc_g, wg, rep_g = ctx.svrg_solve_batched(Xs, ys, lams, ks, 1e-10, **common)
    assert rc_g == rc_e == binding.OK
    for i in range(len(probs)):
        assert torch.equal(wg[i], we[i]), i
        assert rep_g[i]["epochs"] == rep_e[i]["epochs"]


@pytest.mark.parametrize("implicit", [False, True])
def test_path_graph_replay_equals_enqueued_epochs(ctx, implicit):
    n, d, k, ny = 3000, 200, 10, 3
    P = _problem(n, d, alpha=1.5, seed=75)
    rng = np.random.default_rng(5)
    Y = np.stack([P.y] + [(P.X.astype(np.float64) @ rng.standard_normal(d)).astype(np.float32) for _ in range(ny - 1)])
    lams = [1e-2, 1e-3, 1e-4]
    common = dict(batch=32, steps=40, max_epochs=19, stop_rule=binding.STOP_EPOCHS, step_scale=4.0, seed=8,
                  implicit_apply=int(implicit))
    X, Yd = dev(P.X), dev(Y)
    rc_e, We, _ = ctx.svrg_solve_path(X, Yd, lams, k, 0.0, no_graph=1, **common)
    rc_g, Wg, rep_g = ctx.svrg_solve_path(X, Yd, lams, k, 0.0, **common)
    assert rc_e == rc_g == binding.OK
    assert torch.equal(Wg, We)
    assert all(r["epochs"] == 19 for r in rep_g)


# ------------------------------------------------------------------ Block Lanczos (Alg. 2, q blocks)
@pytest.mark.parametrize("n,d,k,p,q", [(3000, 130, 20, 5, 2), (3000, 130, 20, 5, 3), (3000, 130, 20, 5, 4),
                                       (5000, 200, 12, 5, 4), (2000, 61, 9, 4, 3)])
def test_block_lanczos_matches_the_oracle(ctx, n, d, k, p, q):
    """The GPU's q-block sketch against the oracle's Block Lanczos (Alg. 2) started from Pi = X Omega / sqrt(n),
    whose first block is the one-block range C Omega: the Ritz values and P^{-1/2} on probes agree, and the
    Ritz values are at least the one-block sketch's (a larger Krylov space)."""
    P = _problem(n, d, alpha=1.5, seed=n + d + q)
    X64 = P.X.astype(np.float64)
    Om = inputs.gaussian((k + p, d), seed=5)                      # Omega^T
    U, U64, lam, rc = ctx.sketch_build(dev(P.X), k, oversample=p, omega=dev(Om), krylov_blocks=q, sketch_fp32=1)
    assert rc == binding.OK
    Uo, lo, _ = sketch.block_lanczos(X64, X64 @ Om.T.astype(np.float64) / np.sqrt(n), k, q)
    lg = host(lam)
    err = np.max(np.abs(lg - lo)) / lo[0]
    Pg = precond.sketched_preconditioner(host(U64), lg, P.lam)
    Po = precond.sketched_preconditioner(Uo, lo, P.lam)
    V = np.random.default_rng(0).standard_normal((d, 8))
    perr = rel(Pg @ V, Po @ V)
    _, l1, _ = sketch.sketch(X64, Om.T.astype(np.float64), k)
    print(f"\n[block lanczos q={q}] max |d lam~|/lam~_1 = {err:.2e}; P^-1/2 probe rel err = {perr:.2e}; "
          f"lam~_k {lg[-1]:.4e} vs one block {l1[-1]:.4e}")
    assert err <= 2e-5
    assert perr < 1e-4
    assert np.all(lg >= l1 * (1 - 1e-5))
    Ug = host(U64)
    assert np.allclose(Ug.T @ Ug, np.eye(k), atol=1e-6)


def test_block_lanczos_width_is_bounded(ctx):
    P = _problem(2000, 100, seed=3)
    with pytest.raises(binding.ScsError) as e:          # 6 x (20 + 5) = 150 > 136 columns
        ctx.sketch_build(dev(P.X), 20, krylov_blocks=6)
    assert e.value.code == binding.EINVAL


def test_block_lanczos_solve_reaches_the_closed_form(ctx):
    """A whole solve preconditioned from a 3-block sketch stops at the gap against the FP64 optimum."""
    P = _problem(6000, 150, alpha=1.5, seed=77)
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    lam, eps = 1e-5, 1e-8
    ws = ridge.closed_form(X64, y64, lam)
    Ls = ridge.objective(X64, y64, lam, ws)
    r = ctx.svrg_solve(dev(P.X), dev(P.y), lam, 10, eps, krylov_blocks=3, batch=32, epoch_factor=0.25,
                       stop_rule=binding.STOP_GAP, f_star=Ls, step_scale=8.0, max_epochs=100)
    assert r.status == binding.OK, r.report
    assert ridge.objective(X64, y64, lam, host(r.w)) - Ls <= 1.5 * eps



def test_default_bf16_sketch_solve_tracks_the_oracle(ctx):
    """The default FP32 solve runs its sketch GEMMs in BF16 (FP32 accumulation): with the same Omega and index
    stream it follows the oracle's trajectory to the accuracy of a BF16 sketch (P^{-1/2} within about 1e-2),
    and the FP32 accuracy gate still holds (the gradient is exact)."""
    cfg = inputs.WORKLOADS["small_n2000_d100"]
    P = inputs.make_ridge(cfg["n"], cfg["d"], cfg["alpha"], cfg["lam"], seed=inputs.BASE_SEED)
    n, d, k, b = cfg["n"], cfg["d"], cfg["k"], cfg["b"]
    X64, y64 = P.X.astype(np.float64), P.y.astype(np.float64)
    Om = inputs.gaussian((k + 5, d), seed=inputs.BASE_SEED)
    m, S = n // b, 4
    idx = inputs.index_stream(n + d, S * m * b, seed=77).reshape(S, -1)
    res = ctx.svrg_solve(dev(P.X), dev(P.y), cfg["lam"], k, 0.0, omega=dev(Om), indices=dev(idx, torch.int32),
                         steps=m, batch=b, max_epochs=S, stop_rule=binding.STOP_EPOCHS, step_scale=4.0)
    assert res.status == binding.OK
    wo, _, _ = svrg.scsvrg(X64, y64, cfg["lam"], k, Om.T.astype(np.float64), m, S, b, lambda s: idx[s], c=4.0)
    ws = ridge.closed_form(X64, y64, cfg["lam"])
    assert_tracks(host(res.w), wo, ws, 3e-1)
    gate = ctx.svrg_solve(dev(P.X), dev(P.y), cfg["lam"], k, 0.0, batch=b, max_epochs=60,
                          stop_rule=binding.STOP_EPOCHS, step_scale=8.0)
    assert rel(host(gate.w), ws) <= 1e-5
