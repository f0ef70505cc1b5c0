"""Sketched Preconditioned SVRG for ridge regression on AMD MI355X (gfx950).

The method (Gonen, Orabona, Shalev-Shwartz, arXiv:1602.02350) runs in libscs.so: HIP
kernels behind the C ABI of include/scs.h. `binding` marshals torch tensors into that
ABI; `inputs` draws seeded synthetic problems; `build` compiles the library.
"""
