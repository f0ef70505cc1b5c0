"""Random numbers for the method: Philox4x32-10, an exact weighted sampler, Box-Muller.

Test infrastructure only (see oracle/__init__.py).

SVRG draws component i with probability q_i = beta_i / sum_j beta_j (Alg. 1,
the Xiao-Zhang importance sampling). The sampler below draws from integer
weights W_i (the beta_i quantized to a fixed-point grid) by inverting their
integer CDF, so the distribution it samples is exactly W_i / sum_j W_j and
the draw is an exact integer computation. Uniform bits come from the
counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011).

Stream layout (shared by any implementation that must reproduce these draws):
  * index draw g of epoch s: call c = g // 2 with counter (c mod 2^32, c >> 32, s, 0)
    and key (seed mod 2^32, seed >> 32); even g takes output words (x0, x1),
    odd g takes (x2, x3); r = hi * 2^32 + lo is a uniform 64-bit integer and the
    drawn value is u = floor(r * T / 2^64) for total weight T; the index is the
    first i with cumulative weight > u.
  * Gaussian element e: call c = e // 4 with counter (c mod 2^32, c >> 32, 0, 1);
    words (x0, x1) and (x2, x3) each give two normals by Box-Muller with
    u = (x + 1/2) 2^-32; element e takes normal e mod 4.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57          # Philox4x32 multipliers
W0, W1 = 0x9E3779B9, 0xBB67AE85          # Weyl key increments
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key, rounds=10):
    """Vectorized Philox4x32-R. counter: (..., 4) uint32-valued, key: (2,) -> (..., 4) uint64 words."""
    c = np.asarray(counter, dtype=np.uint64).copy()
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = m0 * c[..., 0]            # < 2^64, exact in uint64
        p1 = m1 * c[..., 2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = np.stack([hi1 ^ c[..., 1] ^ k0, lo1, hi0 ^ c[..., 3] ^ k1, lo0], axis=-1)
    return c


def quantize_weights(beta):
    """Fixed-point sampling weights W_i = max(1, rint(beta_i * 2^B / max beta)) for beta_i > 0, else 0.

    B = 62 - ceil(log2(N)) keeps the total below 2^62. The scale 2^B / max(beta)
    and the product are taken in FP64 (IEEE, round-to-nearest-even).
    """
    beta = np.asarray(beta, dtype=np.float64)
    N = beta.size
    B = 62 - int(np.ceil(np.log2(max(N, 2))))
    bmax = float(beta.max())
    scale = np.float64(2.0 ** B) / np.float64(bmax)
    w = np.rint(beta * scale)
    w = np.where(beta > 0, np.maximum(w, 1.0), 0.0)
    return w.astype(np.uint64)


def _mulhi64(a, b):
    """floor(a * b / 2^64) for uint64 arrays, exactly."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.uint64(b)
    a_lo, a_hi = a & MASK32, a >> np.uint64(32)
    b_lo, b_hi = b & MASK32, b >> np.uint64(32)
    lo_lo = a_lo * b_lo
    hi_lo = a_hi * b_lo
    lo_hi = a_lo * b_hi
    hi_hi = a_hi * b_hi
    cross = (lo_lo >> np.uint64(32)) + (hi_lo & MASK32) + lo_hi
    return hi_hi + (hi_lo >> np.uint64(32)) + (cross >> np.uint64(32))


def uniform64(seed, epoch, start, count):
    """The 64-bit uniforms r_g for draws g = start .. start+count-1 of `epoch`."""
    g = np.arange(start, start + count, dtype=np.uint64)
    c = g >> np.uint64(1)
    ctr = np.stack([c & MASK32, c >> np.uint64(32),
                    np.full_like(c, np.uint64(epoch)), np.zeros_like(c)], axis=-1)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    x = philox4x32(ctr, key)
    odd = (g & np.uint64(1)).astype(bool)
    hi = np.where(odd, x[:, 2], x[:, 0])
    lo = np.where(odd, x[:, 3], x[:, 1])
    return (hi << np.uint64(32)) | lo


def invert_cdf(weights, u):
    """Index i with W_0 + .. + W_{i-1} <= u < W_0 + .. + W_i, for integers 0 <= u < sum W."""
    cum = np.cumsum(np.asarray(weights, dtype=np.uint64), dtype=np.uint64)
    return np.searchsorted(cum, np.asarray(u, dtype=np.uint64), side="right").astype(np.int64)


def draw_indices(weights, seed, epoch, count, start=0):
    """Draw `count` indices i with probability W_i / sum W (exact integer inverse CDF)."""
    total = int(np.sum(np.asarray(weights, dtype=np.uint64), dtype=np.uint64))
    u = _mulhi64(uniform64(seed, epoch, start, count), total)
    return invert_cdf(weights, u)


def gaussian(seed, count):
    """`count` N(0,1) values in FP64 from Philox4x32-10 + Box-Muller (layout in the module docstring)."""
    e = np.arange(count, dtype=np.uint64)
    c = np.unique(e >> np.uint64(2))
    ctr = np.stack([c & MASK32, c >> np.uint64(32), np.zeros_like(c), np.ones_like(c)], axis=-1)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    x = philox4x32(ctr, key).astype(np.float64)
    u = (x + 0.5) * 2.0 ** -32
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    z = np.stack([r01 * np.cos(2 * np.pi * u[:, 1]), r01 * np.sin(2 * np.pi * u[:, 1]),
                  r23 * np.cos(2 * np.pi * u[:, 3]), r23 * np.sin(2 * np.pi * u[:, 3])], axis=-1)
    return z.reshape(-1)[:count]
