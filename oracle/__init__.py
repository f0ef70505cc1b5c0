"""FP64 CPU oracle for Sketched Preconditioned SVRG on ridge regression.

TEST INFRASTRUCTURE ONLY. Nothing in the library path imports, calls, links or
executes anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg do. It is a plain, slow, obviously correct
re-statement of the paper (Gonen, Orabona, Shalev-Shwartz, "Solving Ridge
Regression using Sketched Preconditioned SVRG", arXiv:1602.02350) in NumPy
FP64, sharing no code with the HIP kernels.

Layout: one instance per ROW, X is n x d (the paper stores instances as the
columns of a d x n matrix; every formula here is transposed accordingly).

Modules
  ridge     objective, gradient, closed form, suboptimality, condition numbers
  sketch    randomized range finder + Rayleigh-Ritz (Alg. 2 with one block)
  precond   the sketched / exact preconditioners and the n+d components (Sec. 5)
  sampling  Philox4x32-10, integer-weight inverse-CDF sampler, Box-Muller
  svrg      SVRG (Alg. 1, minibatch form) and the whole pipeline (Alg. 3)

Parity pins: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, identities, brute force or published vectors. The one
function without such a pin is documented as "parity unpinned" in its
docstring (none at present).
"""
from . import ridge, sketch, precond, sampling, svrg  # noqa: F401
