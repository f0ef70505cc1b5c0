"""Pins of the oracle's random-number layer: Philox4x32-10 vectors, exact sampler, Box-Muller."""
import os

import numpy as np
import scipy.stats as st

from conftest import GOLDEN
from oracle import sampling
from paper_1602_02350_amd import inputs


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answer_vectors():
    for r in _kat():
        out = sampling.philox4x32(np.array([r[:4]], dtype=np.uint64), r[4:6])[0]
        assert [int(v) for v in out] == r[6:10]


def test_mulhi64_matches_big_integers():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2 ** 63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    for b in [1, 3, 2 ** 40 + 7, 2 ** 62 - 1, 2 ** 64 - 1]:
        got = sampling._mulhi64(a, b)
        assert all(int(g) == (int(x) * b) >> 64 for g, x in zip(got, a))


def test_inverse_cdf_is_exact_on_every_integer():
    """Each index i receives exactly W_i of the integers u in [0, sum W); zero weights none."""
    w = np.array([1, 0, 3, 2, 0, 5], dtype=np.uint64)
    u = np.arange(int(w.sum()), dtype=np.uint64)
    idx = sampling.invert_cdf(w, u)
    assert list(np.bincount(idx, minlength=w.size)) == [1, 0, 3, 2, 0, 5]
    assert list(idx[:4]) == [0, 2, 2, 2]


def test_quantized_weights():
    beta = np.array([1.0, 0.5, 0.0, 1e-30, 0.25])
    w = sampling.quantize_weights(beta)
    B = 62 - 3
    assert list(w) == [2 ** B, 2 ** (B - 1), 0, 1, 2 ** (B - 2)]
    assert int(np.sum(w, dtype=np.uint64)) < 2 ** 62


def test_draws_follow_the_weights():
    w = inputs.integer_weights(40, seed=1, zero_frac=0.2)
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    idx = sampling.draw_indices(w, seed=12345, epoch=3, count=400000)
    assert np.all(p[idx] > 0)
    counts = np.bincount(idx, minlength=40)
    nz = p > 0
    chi = st.chisquare(counts[nz], p[nz] * idx.size)
    assert chi.pvalue > 1e-4


def test_draws_are_a_pure_function_of_the_counter():
    """Counter-based: draws g0..g1 are the same whether generated in one call or from an offset."""
    w = inputs.integer_weights(1000, seed=2)
    a = sampling.draw_indices(w, seed=7, epoch=1, count=100)
    b = sampling.draw_indices(w, seed=7, epoch=1, count=37, start=63)
    assert np.array_equal(a[63:100], b)
    assert not np.array_equal(a, sampling.draw_indices(w, seed=7, epoch=2, count=100))


def test_gaussian_is_standard_normal():
    z = sampling.gaussian(seed=99, count=200000)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert st.kstest(z, "norm").pvalue > 1e-3
    # Box-Muller pairs: the four normals of one call share the radii of (x0,x1) and (x2,x3)
    x = sampling.philox4x32(np.array([[0, 0, 0, 1]], dtype=np.uint64), (99, 0))[0].astype(np.float64)
    u = (x + 0.5) * 2.0 ** -32
    assert np.isclose(z[0] ** 2 + z[1] ** 2, -2 * np.log(u[0]), rtol=1e-12)
    assert np.isclose(z[2] ** 2 + z[3] ** 2, -2 * np.log(u[2]), rtol=1e-12)
