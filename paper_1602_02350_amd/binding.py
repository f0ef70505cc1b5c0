"""ctypes binding of libscs (include/scs.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch supplies device memory
(tensors are passed by data_ptr()) and the stream. Importing this module does not load the
library; the first call does, and raises if libscs.so has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscs.so")

OK, EINVAL, ENONFINITE, ENOMEM, EDEVICE = 0, -1, -2, -3, -4
NOT_CONVERGED, DIVERGED, SKETCH_RANK_DEFICIENT = 1, 2, 3
PREC_FP32, PREC_MIXED = 0, 1
LOOKAHEAD = 8   # SCS_LOOKAHEAD: wave_rows value of the look-ahead inner loop
STOP_EPOCHS, STOP_CERTIFICATE, STOP_GAP = 0, 1, 2

EXPORTED = [
    "scs_opts_default", "scs_status_string", "scs_last_error", "scs_create", "scs_destroy",
    "scs_sketch_build", "scs_precondition_apply", "scs_full_gradient", "scs_svrg_epoch",
    "scs_sample_indices", "scs_gaussian", "scs_svrg_solve", "scs_svrg_solve_batched", "scs_svrg_solve_path",
    "scs_full_gradient_noalloc", "scs_autotune", "scs_regularization_for_budget", "scs_sketch_build_f64",
    "scs_svrg_solve_f64",
]


class ScsOpts(ctypes.Structure):
    _fields_ = [
        ("oversample", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("steps", ctypes.c_int64),
        ("step_scale", ctypes.c_double),
        ("max_epochs", ctypes.c_int),
        ("stop_rule", ctypes.c_int),
        ("f_star", ctypes.c_double),
        ("average", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("workgroups", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("omega", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("trace_w", ctypes.c_void_p),
        ("epoch_ms", ctypes.c_void_p),
        ("timing", ctypes.c_int),
        ("epoch_factor", ctypes.c_double),
        ("implicit_apply", ctypes.c_int),
        ("uniform_sampling", ctypes.c_int),
        ("wave_rows", ctypes.c_int),
        ("w0", ctypes.c_void_p),
        ("w0_preconditioned", ctypes.c_int),
        ("epoch_offset", ctypes.c_int),
        ("wt_out", ctypes.c_void_p),
        ("sketch_fp32", ctypes.c_int),
        ("krylov_blocks", ctypes.c_int),
        ("no_graph", ctypes.c_int),
        ("warm_start", ctypes.c_int),
    ]


class ScsReport(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("epochs", ctypes.c_int),
        ("k_used", ctypes.c_int),
        ("steps", ctypes.c_int64),
        ("eta", ctypes.c_double),
        ("beta_hat", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("grad_norm", ctypes.c_double),
        ("certificate", ctypes.c_double),
        ("lam_top", ctypes.c_double),
        ("ms_sketch", ctypes.c_double),
        ("ms_apply", ctypes.c_double),
        ("ms_solve", ctypes.c_double),
        ("ms_grad", ctypes.c_double),
        ("ms_inner", ctypes.c_double),
        ("n_grad", ctypes.c_int),
        ("n_inner", ctypes.c_int),
        ("backoffs", ctypes.c_int),
        ("workgroups", ctypes.c_int),
        ("wave_rows", ctypes.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
# Contexts still open when the interpreter exits are destroyed by an atexit hook, which runs while
# the HIP runtime is still alive; a destructor left to the final garbage collection could instead
# run during the runtime's own teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libscs.so and declare the prototypes (raises FileNotFoundError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with python -m paper_1602_02350_amd.build")
    L = ctypes.CDLL(path)
    vp, i64, i32, dbl, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    P = ctypes.POINTER
    L.scs_opts_default.argtypes = [P(ScsOpts)]
    L.scs_opts_default.restype = None
    L.scs_status_string.argtypes = [i32]
    L.scs_status_string.restype = ctypes.c_char_p
    L.scs_last_error.argtypes = []
    L.scs_last_error.restype = ctypes.c_char_p
    L.scs_create.argtypes = [P(vp), i32, vp]
    L.scs_destroy.argtypes = [vp]
    L.scs_sketch_build.argtypes = [vp, vp, i64, i64, i64, i32, P(ScsOpts), vp, vp, vp]
    L.scs_precondition_apply.argtypes = [vp, vp, i64, i64, i64, vp, vp, i32, dbl, i32, vp, vp, i64, vp]
    L.scs_full_gradient.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp, i32, dbl, vp, vp, P(dbl)]
    L.scs_full_gradient_noalloc.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp, i32, dbl, vp, vp, P(dbl)]
    L.scs_autotune.argtypes = [vp, vp, i64, i64, i64, vp, dbl, i32, dbl, P(ScsOpts), P(ScsOpts), P(dbl)]
    L.scs_regularization_for_budget.argtypes = [vp, vp, i64, i64, i64, i32, P(ScsOpts), P(dbl), P(dbl)]
    L.scs_svrg_epoch.argtypes = [vp, i64, i64, vp, vp, i64, i32, vp, vp, vp, i64, i32, dbl, i32, i32, i32, vp]
    L.scs_sample_indices.argtypes = [vp, vp, i64, u64, i32, i64, vp]
    L.scs_gaussian.argtypes = [vp, u64, i64, vp]
    L.scs_svrg_solve.argtypes = [vp, vp, i64, i64, i64, vp, dbl, i32, dbl, P(ScsOpts), vp, P(ScsReport)]
    L.scs_sketch_build_f64.argtypes = [vp, vp, i64, i64, i64, i32, P(ScsOpts), vp, vp]
    L.scs_svrg_solve_f64.argtypes = [vp, vp, i64, i64, i64, vp, dbl, i32, dbl, P(ScsOpts), vp, P(ScsReport)]
    L.scs_svrg_solve_batched.argtypes = [vp, i32, P(vp), P(i64), P(i64), P(i64), P(vp), P(dbl), P(i32), dbl,
                                         P(dbl), P(ScsOpts), P(vp), P(ScsReport)]
    L.scs_svrg_solve_path.argtypes = [vp, vp, i64, i64, i64, vp, i32, P(dbl), i32, i32, dbl, P(dbl), P(ScsOpts),
                                      vp, P(ScsReport)]
    for name in EXPORTED:
        if name not in ("scs_opts_default", "scs_status_string", "scs_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class ScsError(RuntimeError):
    def __init__(self, code, where):
        L = load_library()
        super().__init__(f"{where}: {L.scs_status_string(code).decode()} ({code}): {L.scs_last_error().decode()}")
        self.code = code


def _check(code, where, allow_positive=True):
    if code < 0 or (code > 0 and not allow_positive):
        raise ScsError(code, where)
    return code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype=None):
    assert t.is_cuda, "expected a device tensor"
    if dtype is not None:
        assert t.dtype == dtype, f"expected {dtype}, got {t.dtype}"
    return t


@dataclass
class SolveResult:
    w: torch.Tensor
    status: int
    report: dict
    epoch_ms: list


class Context:
    """One library context bound to a device and to torch's current stream on that device."""

    def __init__(self, device: int = 0):
        L = load_library()
        self.device = device
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(L.scs_create(ctypes.byref(h), device, ctypes.c_void_p(stream)), "scs_create", False)
        self._h = h
        self._L = L
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._L.scs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- options
    def opts(self, **kw) -> ScsOpts:
        o = ScsOpts()
        self._L.scs_opts_default(ctypes.byref(o))
        for key, v in kw.items():
            if key in ("omega", "indices", "trace_w", "w0", "wt_out"):
                v = None if v is None else v.data_ptr()
            if not hasattr(o, key):
                raise TypeError(f"unknown option {key}")
            setattr(o, key, v)
        return o

    # ---- entry points
    def gaussian(self, seed: int, count: int) -> torch.Tensor:
        out = torch.empty(count, dtype=torch.float32, device=f"cuda:{self.device}")
        _check(self._L.scs_gaussian(self._h, seed, count, _ptr(out)), "scs_gaussian", False)
        return out

    def sample_indices(self, beta: torch.Tensor, seed: int, epoch: int, count: int) -> torch.Tensor:
        _dev(beta, torch.float32)
        out = torch.empty(count, dtype=torch.int32, device=beta.device)
        _check(self._L.scs_sample_indices(self._h, _ptr(beta), beta.numel(), seed, epoch, count, _ptr(out)),
               "scs_sample_indices", False)
        return out

    def sketch_build(self, X: torch.Tensor, k: int, **opts):
        _dev(X, torch.float32)
        n, d = X.shape
        U = torch.empty(d, k, dtype=torch.float32, device=X.device)
        U64 = torch.empty(d, k, dtype=torch.float64, device=X.device)
        lam = torch.empty(k, dtype=torch.float64, device=X.device)
        o = self.opts(**opts)
        rc = _check(self._L.scs_sketch_build(self._h, _ptr(X), n, d, X.stride(0), k, ctypes.byref(o), _ptr(U),
                                             _ptr(U64), _ptr(lam)), "scs_sketch_build")
        return U, U64, lam, rc

    def precondition_apply(self, X: torch.Tensor, U, lam, lam_reg: float, bf16: bool = False, ldt: int = None):
        _dev(X, torch.float32)
        n, d = X.shape
        k = 0 if U is None else U.shape[1]
        ldt = ldt or d
        dt = torch.bfloat16 if bf16 else torch.float32
        Xt = torch.empty(n, ldt, dtype=dt, device=X.device)
        reg = torch.empty(d, ldt, dtype=dt, device=X.device)
        beta = torch.empty(n + d, dtype=torch.float32, device=X.device)
        _check(self._L.scs_precondition_apply(self._h, _ptr(X), n, d, X.stride(0), _ptr(U), _ptr(lam), k,
                                              float(lam_reg), int(bf16), _ptr(Xt), _ptr(reg), ldt, _ptr(beta)),
               "scs_precondition_apply", False)
        return Xt, reg, beta

    def full_gradient(self, X, y, U, lam, lam_reg: float, wt):
        _dev(X, torch.float32)
        n, d = X.shape
        k = 0 if U is None else U.shape[1]
        g = torch.empty(d, dtype=torch.float32, device=X.device)
        obj = ctypes.c_double()
        _check(self._L.scs_full_gradient(self._h, _ptr(X), n, d, X.stride(0), _ptr(y), _ptr(U), _ptr(lam), k,
                                         float(lam_reg), _ptr(wt), _ptr(g), ctypes.byref(obj)),
               "scs_full_gradient", False)
        return g, obj.value

    def full_gradient_noalloc(self, X, y, U, lam, lam_reg: float, wt, g=None, want_obj: bool = True):
        """The allocation-free variant: g (d, FP32) may be passed in; obj is None when want_obj is False."""
        _dev(X, torch.float32)
        n, d = X.shape
        k = 0 if U is None else U.shape[1]
        if g is None:
            g = torch.empty(d, dtype=torch.float32, device=X.device)
        obj = ctypes.c_double()
        _check(self._L.scs_full_gradient_noalloc(self._h, _ptr(X), n, d, X.stride(0), _ptr(y), _ptr(U), _ptr(lam), k,
                                                 float(lam_reg), _ptr(wt), _ptr(g),
                                                 ctypes.byref(obj) if want_obj else None),
               "scs_full_gradient_noalloc", False)
        return g, (obj.value if want_obj else None)

    def svrg_epoch(self, n, d, Xt, reg, beta, mu, idx, m, b, eta, average=True, workgroups=0, wt=None,
                   wave_rows=0):
        bf16 = Xt.dtype == torch.bfloat16
        ldt = Xt.stride(0)
        assert reg.stride(0) == ldt
        _check(self._L.scs_svrg_epoch(self._h, n, d, _ptr(Xt), _ptr(reg), ldt, int(bf16), _ptr(beta), _ptr(mu),
                                      _ptr(idx), m, b, float(eta), int(average), int(workgroups), int(wave_rows),
                                      _ptr(wt)),
               "scs_svrg_epoch", False)
        return wt

    def svrg_solve_batched(self, Xs, ys, lams, ks, eps: float, f_star=None, **opts):
        """Independent problems solved together; returns (status, [w], [report dict])."""
        P = len(Xs)
        assert len(ys) == P and len(lams) == P and len(ks) == P and P > 0
        for X, y in zip(Xs, ys):
            _dev(X, torch.float32)
            _dev(y, torch.float32)
        ws_ = [torch.empty(X.shape[1], dtype=torch.float32, device=X.device) for X in Xs]
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        Xa = (vp * P)(*[X.data_ptr() for X in Xs])
        ya = (vp * P)(*[y.data_ptr() for y in ys])
        wa = (vp * P)(*[w.data_ptr() for w in ws_])
        na = (i64 * P)(*[X.shape[0] for X in Xs])
        da = (i64 * P)(*[X.shape[1] for X in Xs])
        la = (i64 * P)(*[X.stride(0) for X in Xs])
        lama = (ctypes.c_double * P)(*[float(v) for v in lams])
        ka = (ctypes.c_int * P)(*[int(v) for v in ks])
        reps = (ScsReport * P)()
        o = self.opts(**opts)
        fs = None if f_star is None else (ctypes.c_double * P)(*[float(v) for v in f_star])
        rc = _check(self._L.scs_svrg_solve_batched(self._h, P, Xa, na, da, la, ya, lama, ka, float(eps), fs,
                                                   ctypes.byref(o), wa, reps), "scs_svrg_solve_batched")
        return rc, ws_, [r.as_dict() for r in reps]

    def svrg_solve_path(self, X, Y, lams, k: int, eps: float, f_star=None, **opts):
        """All (lambda, y) solves with one shared sketch; returns (status, W (nl*ny x d), [report])."""
        _dev(X, torch.float32)
        _dev(Y, torch.float32)
        n, d = X.shape
        ny = Y.shape[0]
        assert Y.shape[1] == n and Y.is_contiguous()
        nl = len(lams)
        W = torch.empty(nl * ny, d, dtype=torch.float32, device=X.device)
        la = (ctypes.c_double * nl)(*[float(v) for v in lams])
        reps = (ScsReport * (nl * ny))()
        o = self.opts(**opts)
        fs = None if f_star is None else (ctypes.c_double * (nl * ny))(*[float(v) for v in f_star])
        rc = _check(self._L.scs_svrg_solve_path(self._h, _ptr(X), n, d, X.stride(0), _ptr(Y), ny, la, nl, int(k),
                                                float(eps), fs, ctypes.byref(o), _ptr(W), reps),
                    "scs_svrg_solve_path")
        return rc, W, [r.as_dict() for r in reps]

    def regularization_for_budget(self, X, k: int, **opts):
        """(lambda_precond, lambda_plain, status) of the O~(ndk) budget (Sec. 2.2)."""
        _dev(X, torch.float32)
        n, d = X.shape
        o = self.opts(**opts)
        a, b = ctypes.c_double(), ctypes.c_double()
        rc = _check(self._L.scs_regularization_for_budget(self._h, _ptr(X), n, d, X.stride(0), int(k),
                                                          ctypes.byref(o), ctypes.byref(a), ctypes.byref(b)),
                    "scs_regularization_for_budget")
        return a.value, b.value, rc

    def autotune(self, X, y, lam_reg: float, k: int, eps: float, **opts):
        """Tuned options (a dict of the scs_opts fields) and the winner's wall time in milliseconds."""
        _dev(X, torch.float32)
        n, d = X.shape
        o = self.opts(**opts)
        t = ScsOpts()
        ms = ctypes.c_double()
        _check(self._L.scs_autotune(self._h, _ptr(X), n, d, X.stride(0), _ptr(y), float(lam_reg), int(k), float(eps),
                                    ctypes.byref(o), ctypes.byref(t), ctypes.byref(ms)), "scs_autotune", False)
        tuned = {f: getattr(t, f) for f, _ in ScsOpts._fields_
                 if f not in ("omega", "indices", "trace_w", "epoch_ms", "w0", "wt_out")}
        return tuned, ms.value

    def sketch_build_f64(self, X: torch.Tensor, k: int, **opts):
        """FP64 sketch: (U d x k FP64, lam k FP64, status)."""
        _dev(X, torch.float64)
        n, d = X.shape
        U = torch.empty(d, k, dtype=torch.float64, device=X.device)
        lam = torch.empty(k, dtype=torch.float64, device=X.device)
        o = self.opts(**opts)
        rc = _check(self._L.scs_sketch_build_f64(self._h, _ptr(X), n, d, X.stride(0), k, ctypes.byref(o), _ptr(U),
                                                 _ptr(lam)), "scs_sketch_build_f64")
        return U, lam, rc

    def svrg_solve_f64(self, X, y, lam_reg: float, k: int, eps: float, epoch_times: bool = False,
                       **opts) -> SolveResult:
        """FP64 solve (X, y FP64 device tensors); w is FP64. epoch_times as in svrg_solve."""
        _dev(X, torch.float64)
        _dev(y, torch.float64)
        n, d = X.shape
        w = torch.empty(d, dtype=torch.float64, device=X.device)
        o = self.opts(**opts)
        S = o.max_epochs
        ms = (ctypes.c_double * S)() if epoch_times else None
        o.epoch_ms = ctypes.cast(ms, ctypes.c_void_p) if epoch_times else None
        rep = ScsReport()
        rc = _check(self._L.scs_svrg_solve_f64(self._h, _ptr(X), n, d, X.stride(0), _ptr(y), float(lam_reg), int(k),
                                               float(eps), ctypes.byref(o), _ptr(w), ctypes.byref(rep)),
                    "scs_svrg_solve_f64")
        return SolveResult(w=w, status=rc, report=rep.as_dict(), epoch_ms=list(ms) if epoch_times else [])

    def svrg_solve(self, X, y, lam_reg: float, k: int, eps: float, epoch_times: bool = False,
                   **opts) -> SolveResult:
        """FP32 solve; epoch_times asks for the per-epoch times (epoch_ms, which costs an event per epoch)."""
        _dev(X, torch.float32)
        n, d = X.shape
        w = torch.empty(d, dtype=torch.float32, device=X.device)
        o = self.opts(**opts)
        S = o.max_epochs
        ms = (ctypes.c_double * S)() if epoch_times else None
        o.epoch_ms = ctypes.cast(ms, ctypes.c_void_p) if epoch_times else None
        rep = ScsReport()
        rc = _check(self._L.scs_svrg_solve(self._h, _ptr(X), n, d, X.stride(0), _ptr(y), float(lam_reg), int(k),
                                           float(eps), ctypes.byref(o), _ptr(w), ctypes.byref(rep)),
                    "scs_svrg_solve")
        return SolveResult(w=w, status=rc, report=rep.as_dict(), epoch_ms=list(ms) if epoch_times else [])
