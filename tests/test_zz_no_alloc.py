"""The allocation-free full-gradient entry point against the allocating one, through the C ABI.

Both run the same kernels in the same order, so their outputs must agree bit for bit. Two calls
in a row, the second on a smaller problem, check that the shared scratch array carries nothing
from one call into the next; a problem too large for the array is refused on the host.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1602_02350_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = binding.Context(0)
    yield c
    c.close()


def _problem(n, d, k, seed):
    P = inputs.make_ridge(n, d, 1.5, 1e-5, seed=seed)
    X = torch.from_numpy(P.X).cuda()
    y = torch.from_numpy(P.y).cuda()
    rng = np.random.default_rng(seed)
    if k > 0:
        U = np.linalg.qr(rng.standard_normal((d, k)))[0]
        lam = np.sort(rng.uniform(1e-3, 1.0, k))[::-1].copy()
        Ut = torch.from_numpy(U.astype(np.float32)).cuda()
        lt = torch.from_numpy(lam).cuda()
    else:
        Ut, lt = None, None
    wt = torch.from_numpy(rng.standard_normal(d).astype(np.float32)).cuda()
    return X, y, Ut, lt, wt


@pytest.mark.parametrize("shapes", [((20000, 1000, 50), (3000, 257, 10)), ((4000, 300, 0), (1500, 61, 0))])
def test_noalloc_gradient_equals_the_allocating_entry(ctx, shapes):
    for i, (n, d, k) in enumerate(shapes):
        print(f"[noalloc] call {i}: n={n} d={d} k={k}", flush=True)
        X, y, U, lam, wt = _problem(n, d, k, inputs.BASE_SEED + 50 + i)
        g_ref, obj_ref = ctx.full_gradient(X, y, U, lam, 1e-5, wt)
        g_na, obj_na = ctx.full_gradient_noalloc(X, y, U, lam, 1e-5, wt)
        torch.cuda.synchronize()
        assert torch.equal(g_na, g_ref), float((g_na - g_ref).abs().max())
        assert obj_na == obj_ref
        # the enqueue-only form (no objective, no wait) writes the same gradient
        g2 = torch.full_like(g_ref, float("nan"))
        _, none = ctx.full_gradient_noalloc(X, y, U, lam, 1e-5, wt, g=g2, want_obj=False)
        torch.cuda.synchronize()
        assert none is None
        assert torch.equal(g2, g_ref)


def test_noalloc_refuses_a_problem_larger_than_its_scratch(ctx):
    L = binding.load_library()
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    obj = ctypes.c_double()
    p = ctypes.c_void_p(buf.data_ptr())
    # 512 workgroups x 20000 columns of FP32 partials alone are 41 MB; refused before any launch
    rc = L.scs_full_gradient_noalloc(ctx._h, p, 100000, 20000, 20000, p, None, None, 0, 1e-5, p, p,
                                     ctypes.byref(obj))
    assert rc == binding.EINVAL
    assert b"scratch" in L.scs_last_error()
