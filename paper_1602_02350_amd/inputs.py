"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws data. It holds none of the method's arithmetic: no
objective, no sketch, no preconditioner, no sampler. Both the HIP path and the
FP64 oracle consume what it returns, so neither has to import the other.

Recipe (row-major, one instance per row, X is n x d):
  * U  : Haar-random orthogonal d x d matrix (QR of a Gaussian matrix with the
         signs of R's diagonal folded into Q, Mezzadri 2007).
  * X  = G diag(sqrt(spec)) U^T with G ~ N(0,1)^{n x d}, so each row is
         N(0, U diag(spec) U^T).
  * w0 ~ N(0, I_d);  y = X w0 + e with e ~ N(0, noise_var).
  * Omega ~ N(0,1)^{d x l} for the range finder.
Spectra are power laws spec_j = j^{-alpha} (j = 1..d), optionally with a floor.

The synthetic workload of the paper's experiments (Sec. 6) is drawn differently: X has exactly
the singular values q^{-alpha} (q = 1..d) with uniformly random singular vectors (X = V diag(s) U^T,
V an n x d matrix with orthonormal columns from the QR of a Gaussian matrix, U Haar), every example
(row) is then scaled to unit norm, and y = X w* + z with w* ~ N(0, I_d), z ~ N(0, 0.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Base seed of every workload; individual streams are offset from it.
BASE_SEED = 20160207


def power_spectrum(d: int, alpha: float, floor: float = 0.0) -> np.ndarray:
    """Population covariance eigenvalues j^{-alpha} + floor, j = 1..d (descending)."""
    j = np.arange(1, d + 1, dtype=np.float64)
    return j ** (-float(alpha)) + float(floor)


def haar_orthogonal(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed d x d orthogonal matrix."""
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


@dataclass
class RidgeProblem:
    X: np.ndarray        # n x d
    y: np.ndarray        # n
    w0: np.ndarray       # d, the planted weights
    spec: np.ndarray     # d, population covariance eigenvalues
    U: np.ndarray        # d x d, population covariance eigenvectors (columns)
    lam: float           # ridge parameter
    seed: int


def make_ridge(n: int, d: int, alpha: float, lam: float, seed: int,
               noise_var: float = 0.01, floor: float = 0.0,
               dtype=np.float32, block: int = 65536) -> RidgeProblem:
    """Draw one synthetic ridge problem; X and y are rounded to `dtype`."""
    spec = power_spectrum(d, alpha, floor)
    rng_u = np.random.default_rng([seed, 1])
    rng_x = np.random.default_rng([seed, 2])
    rng_w = np.random.default_rng([seed, 3])
    rng_e = np.random.default_rng([seed, 4])
    U = haar_orthogonal(d, rng_u)
    M = (np.sqrt(spec)[:, None] * U.T)          # rows of X are g^T M
    X = np.empty((n, d), dtype=dtype)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        X[r0:r1] = (rng_x.standard_normal((r1 - r0, d)) @ M).astype(dtype)
    w0 = rng_w.standard_normal(d)
    noise = rng_e.standard_normal(n) * np.sqrt(noise_var)
    y = (X.astype(np.float64) @ w0 + noise).astype(dtype)
    return RidgeProblem(X=X, y=y, w0=w0, spec=spec, U=U, lam=float(lam), seed=seed)


def gaussian(shape, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0,1) array (e.g. the range finder's Omega)."""
    return np.random.default_rng([seed, 5]).standard_normal(shape).astype(dtype)


def random_orthonormal(d: int, k: int, seed: int) -> np.ndarray:
    """d x k matrix with orthonormal columns (FP64)."""
    g = np.random.default_rng([seed, 6]).standard_normal((d, k))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def decreasing_values(k: int, seed: int, lo: float = 1e-3, hi: float = 1.0) -> np.ndarray:
    """k positive values sorted descending, log-uniform in [lo, hi]."""
    v = np.exp(np.random.default_rng([seed, 7]).uniform(np.log(lo), np.log(hi), k))
    return np.sort(v)[::-1].copy()


def index_stream(N: int, count: int, seed: int) -> np.ndarray:
    """`count` indices drawn uniformly from [0, N) as int32 (an injected sample stream)."""
    return np.random.default_rng([seed, 8]).integers(0, N, size=count, dtype=np.int64).astype(np.int32)


def integer_weights(N: int, seed: int, max_weight: int = 1 << 20, zero_frac: float = 0.0) -> np.ndarray:
    """N non-negative uint64 sampling weights (some zero if zero_frac > 0, never all)."""
    rng = np.random.default_rng([seed, 9])
    w = rng.integers(1, max_weight, size=N, dtype=np.int64).astype(np.uint64)
    if zero_frac > 0:
        z = rng.random(N) < zero_frac
        z[rng.integers(0, N)] = False
        w[z] = 0
    return w


def make_spectral_rows(n: int, d: int, alpha: float, seed: int, noise_var: float = 0.1,
                       dtype=np.float32, normalize: bool = True):
    """The paper's synthetic regression data (n >= d): singular values q^{-alpha} with uniformly random
    singular vectors, rows scaled to unit norm (skipped with normalize=False), y = X w* + z.
    Returns (X, y, w*); X and y in `dtype`."""
    assert n >= d
    rng_v = np.random.default_rng([seed, 21])
    rng_u = np.random.default_rng([seed, 22])
    rng_w = np.random.default_rng([seed, 23])
    rng_e = np.random.default_rng([seed, 24])
    V, R = np.linalg.qr(rng_v.standard_normal((n, d)))
    V = V * np.sign(np.diag(R))[None, :]
    U = haar_orthogonal(d, rng_u)
    s = np.arange(1, d + 1, dtype=np.float64) ** (-float(alpha))
    X = (V * s[None, :]) @ U.T
    if normalize:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    w = rng_w.standard_normal(d)
    y = X @ w + rng_e.standard_normal(n) * np.sqrt(noise_var)
    return X.astype(dtype), y.astype(dtype), w


def make_spectral_rows_torch(n: int, d: int, alpha: float, seed: int, noise_var: float = 0.1,
                             device: str = "cuda"):
    """make_spectral_rows drawn with torch's generator on a device (a different random stream):
    X (n x d FP32) and y (n FP32) as device tensors."""
    import torch
    assert n >= d
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    V, R = torch.linalg.qr(torch.randn(n, d, generator=g, device=device, dtype=torch.float64))
    V = V * torch.sign(torch.diagonal(R))[None, :]
    del R
    Q, R = torch.linalg.qr(torch.randn(d, d, generator=g, device=device, dtype=torch.float64))
    U = Q * torch.sign(torch.diagonal(R))[None, :]
    s = torch.arange(1, d + 1, device=device, dtype=torch.float64) ** (-float(alpha))
    X = (V * s[None, :]) @ U.T
    del V
    X /= X.norm(dim=1, keepdim=True)
    w = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    y = X @ w + torch.randn(n, generator=g, device=device, dtype=torch.float64) * float(noise_var) ** 0.5
    return X.float().contiguous(), y.float()


def random_vector(d: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng([seed, 10]).standard_normal(d) * scale


# Workload recipes with their sizes. Each returns keyword arguments for make_ridge
# plus the method parameters that go with the workload.
WORKLOADS = {
    # n=2000, d=100, spectrum j^-2, lambda=1e-4, k=10, p=5; solved to 1e-8.
    "small_n2000_d100": dict(n=2000, d=100, alpha=2.0, lam=1e-4, k=10, b=8, eps=1e-8, floor=0.0),
    # the same recipe for the FP64 path (X and y drawn in FP64)
    "fp64_n2000_d100": dict(n=2000, d=100, alpha=2.0, lam=1e-4, k=10, b=8, eps=1e-8, floor=0.0, fp64=True),
    # n=1e5, d=1000, spectrum j^-1.5, lambda=1e-5, k=50, minibatch 64; solved to 1e-6 in FP32.
    "fp32_n100000_d1000": dict(n=100000, d=1000, alpha=1.5, lam=1e-5, k=50, b=64, eps=1e-6, floor=0.0),
    # n=5e5, d=2048, spectrum j^-2 + 1e-6, lambda=1e-6, k=128; BF16 sketch and rows.
    "mixed_n500000_d2048": dict(n=500000, d=2048, alpha=2.0, lam=1e-6, k=128, b=64, eps=1e-6, floor=1e-6),
    # regularization path: one X (n=2e5, d=1024, j^-1.5), 8 right-hand sides, 32 lambda log-spaced
    # from 1e-7 to 1e-2, one shared sketch with k=64: 256 solves.
    "path_n200000_d1024": dict(n=200000, d=1024, alpha=1.5, k=64, b=64, eps=1e-6, floor=0.0, ny=8, nl=32,
                               lam_lo=1e-7, lam_hi=1e-2),
    # 256 independent problems: n ~ U[1000, 50000], d ~ U{64..512}, spectrum j^-a with a ~ U[1, 2.5],
    # lambda ~ logU[1e-6, 1e-3], k = floor(d / 16); BF16 rows in the inner loop.
    "batch256_uneven": dict(nprob=256, n_lo=1000, n_hi=50000, d_lo=64, d_hi=512, a_lo=1.0, a_hi=2.5,
                            lam_lo=1e-6, lam_hi=1e-3, b=64, eps=1e-6, floor=0.0),
    # the paper's synthetic data (Sec. 6): 20000 unit-norm examples in d = 5000 with singular values
    # 1/q (linear decay) and 1/q^2 (quadratic decay), lambda = 1e-8, k = 30
    "synth_linear_n20000_d5000": dict(n=20000, d=5000, alpha=1.0, lam=1e-8, k=30, b=64, eps=1e-6,
                                      spectral_rows=True),
    "synth_quadratic_n20000_d5000": dict(n=20000, d=5000, alpha=2.0, lam=1e-8, k=30, b=64, eps=1e-6,
                                         spectral_rows=True),
}


def uneven_batch_shapes(cfg, seed):
    """Per-problem (n, d, alpha, lambda, k) of an uneven batch, drawn from a seeded generator."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(cfg["nprob"]):
        n = int(rng.integers(cfg["n_lo"], cfg["n_hi"] + 1))
        d = int(rng.integers(cfg["d_lo"], cfg["d_hi"] + 1))
        a = float(rng.uniform(cfg["a_lo"], cfg["a_hi"]))
        lam = float(np.exp(rng.uniform(np.log(cfg["lam_lo"]), np.log(cfg["lam_hi"]))))
        out.append((n, d, a, lam, d // 16))
    return out


def make_ridge_torch(n: int, d: int, alpha: float, seed: int, noise_var: float = 0.01, floor: float = 0.0,
                     device: str = "cuda", block: int = 65536):
    """The same recipe drawn with torch's generator on a device, for the large workloads: returns X
    (n x d FP32) and y (n FP32) as device tensors. (A different random stream from make_ridge.)"""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    G = torch.randn(d, d, generator=g, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(G)
    U = Q * torch.sign(torch.diagonal(R))[None, :]
    j = torch.arange(1, d + 1, device=device, dtype=torch.float64)
    spec = j ** (-float(alpha)) + float(floor)
    M = (spec.sqrt()[:, None] * U.T).float().contiguous()
    X = torch.empty(n, d, device=device, dtype=torch.float32)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        X[r0:r1] = torch.randn(r1 - r0, d, generator=g, device=device) @ M
    w0 = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    noise = torch.randn(n, generator=g, device=device, dtype=torch.float64) * float(noise_var) ** 0.5
    y = (X.double() @ w0 + noise).float()
    return X, y


def make_path_targets_torch(X, y0, ny: int, seed: int, noise_var: float = 0.01):
    """ny right-hand sides for one X (ny x n FP32, device): row 0 is y0, row r >= 1 is X w_r + e_r with
    its own planted w_r ~ N(0, I) and noise e_r ~ N(0, noise_var), from torch's generator."""
    import torch
    n, d = X.shape
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    Y = torch.empty(ny, n, device=X.device, dtype=torch.float32)
    Y[0] = y0
    for r in range(1, ny):
        w0 = torch.randn(d, generator=g, device=X.device, dtype=torch.float64)
        e = torch.randn(n, generator=g, device=X.device, dtype=torch.float64) * float(noise_var) ** 0.5
        Y[r] = (X.double() @ w0 + e).float()
    return Y


def path_lambdas(cfg):
    """The nl values of lambda of a path workload, log-spaced from lam_lo to lam_hi."""
    return np.logspace(np.log10(cfg["lam_lo"]), np.log10(cfg["lam_hi"]), cfg["nl"])
