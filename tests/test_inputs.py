"""The paper's synthetic workload generator (Sec. 6): planted singular values, unit-norm examples and
the label model, checked against their definitions."""
import numpy as np

from paper_1602_02350_amd import inputs


def test_spectral_rows_have_the_planted_singular_values():
    for alpha in (1.0, 2.0):
        X, _, _ = inputs.make_spectral_rows(400, 60, alpha, seed=3, dtype=np.float64, normalize=False)
        sv = np.linalg.svd(X, compute_uv=False)
        q = np.arange(1, 61, dtype=np.float64)
        assert np.allclose(sv, q ** -alpha, rtol=1e-10, atol=0.0)


def test_spectral_rows_are_unit_norm_with_planted_labels():
    X, y, w = inputs.make_spectral_rows(3000, 80, 2.0, seed=5, dtype=np.float64)
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, rtol=0, atol=1e-12)
    r = y - X @ w
    assert abs(r.mean()) < 0.03 and abs(r.var() - 0.1) < 0.015   # z ~ N(0, 0.1)
    assert abs(w.var() - 1.0) < 0.4                                # w* ~ N(0, I)


def test_spectral_rows_singular_vectors_are_not_aligned_with_the_axes():
    # uniformly random singular vectors: no coordinate carries the top direction
    X, _, _ = inputs.make_spectral_rows(500, 50, 2.0, seed=7, dtype=np.float64, normalize=False)
    _, _, Vt = np.linalg.svd(X, full_matrices=False)
    assert np.max(np.abs(Vt[0])) < 0.7
