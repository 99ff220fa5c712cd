"""Thin ctypes binding of liblsq (include/lsq.h, include/lsq_debug.h).

Argument marshalling only: every step of a solve runs in liblsq's HIP
kernels.  PyTorch provides device memory and the current stream; tensors are
passed by data pointer.  Matrices must be float64 CUDA/HIP tensors in
column-major layout (stride(0) == 1), as produced by `colmajor`.

If liblsq.so has not been built, `load()` raises; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsq.so")
HEADERS = [os.path.join(os.path.dirname(_HERE), "include", h) for h in ("lsq.h", "lsq_debug.h")]

PREC = {"auto": 0, "fp8": 1, "bf16": 2, "fp16": 3, "fp32": 4, "fp64": 5}
PREC_NAME = {v: k for k, v in PREC.items()}
SOLVER = {"auto": 0, "ir": 1, "gmres": 2, "direct": 3}
SOLVER_NAME = {v: k for k, v in SOLVER.items()}
LSE, GLS = 0, 1

c_int, c_double, c_void_p, c_float = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_float


class Opts(ctypes.Structure):
    _fields_ = [("prec", c_int), ("solver", c_int), ("tol", c_double), ("maxit", c_int),
                ("gmres_restart", c_int), ("gmres_tol", c_double), ("gmres_maxit", c_int),
                ("escalate", c_int), ("alpha", c_double), ("beta", c_double), ("nb", c_int),
                ("polish", c_double), ("residual", c_int)]


class Result(ctypes.Structure):
    _fields_ = [("info", c_int), ("prec_used", c_int), ("solver_used", c_int),
                ("attempts", c_int), ("ir_steps", c_int), ("gmres_iters", c_int),
                ("berr", c_double * 3), ("berr_max", c_double), ("ms_convert", c_float),
                ("ms_factor", c_float), ("ms_refine", c_float)]

    def as_dict(self):
        return {"info": self.info, "prec_used": PREC_NAME.get(self.prec_used, self.prec_used),
                "solver_used": SOLVER_NAME.get(self.solver_used, self.solver_used),
                "attempts": self.attempts, "ir_steps": self.ir_steps,
                "gmres_iters": self.gmres_iters, "berr": list(self.berr),
                "berr_max": self.berr_max, "ms_convert": self.ms_convert,
                "ms_factor": self.ms_factor, "ms_refine": self.ms_refine}


class Problem(ctypes.Structure):
    _fields_ = [("type", c_int), ("m", c_int), ("n", c_int), ("p", c_int),
                ("A", c_void_p), ("B", c_void_p), ("b", c_void_p), ("d", c_void_p),
                ("lda", c_int), ("ldb", c_int), ("x", c_void_p), ("y", c_void_p)]


_P = c_void_p
_SIGS = {
    "lsq_create": (c_int, [ctypes.POINTER(c_void_p), c_int]),
    "lsq_destroy": (c_int, [_P]),
    "lsq_set_stream": (c_int, [_P, _P]),
    "lsq_opts_default": (None, [ctypes.POINTER(Opts)]),
    "lse_solve": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P, _P, _P,
                          ctypes.POINTER(Opts), ctypes.POINTER(Result)]),
    "gls_solve": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P, _P,
                          ctypes.POINTER(Opts), ctypes.POINTER(Result)]),
    "zlse_solve": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P, _P, _P,
                           ctypes.POINTER(Opts), ctypes.POINTER(Result)]),
    "zgls_solve": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P, _P,
                           ctypes.POINTER(Opts), ctypes.POINTER(Result)]),
    "lse_factor": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, c_int,
                           ctypes.POINTER(c_void_p)]),
    "gls_factor": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, c_int,
                           ctypes.POINTER(c_void_p)]),
    "lse_solve_factored": (c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Opts),
                                   ctypes.POINTER(Result)]),
    "gls_solve_factored": (c_int, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(Opts),
                                   ctypes.POINTER(Result)]),
    "lse_solve_factored_noalloc": (c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Opts),
                                           ctypes.POINTER(Result)]),
    "lsq_factors_destroy": (c_int, [_P]),
    "lsq_solve_batched": (c_int, [_P, c_int, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                  ctypes.POINTER(Result)]),
    "lsq_batch_plan_create": (c_int, [_P, c_int, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                      ctypes.POINTER(c_void_p)]),
    "lsq_batch_plan_run": (c_int, [_P, ctypes.POINTER(Result)]),
    "lsq_batch_plan_destroy": (c_int, [_P]),
    "lsq_set_batch_workers": (c_int, [_P, c_int]),
    "lsq_set_batch_mode": (c_int, [_P, c_int]),
    "lsq_selector_set": (c_int, [_P, ctypes.POINTER(c_float), c_int]),
    "lsq_selector_features": (c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(c_float),
                                      ctypes.POINTER(c_float), ctypes.POINTER(c_int)]),
    "lse_solve_batched": (c_int, [_P, c_int, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                  ctypes.POINTER(Result)]),
    "gls_solve_batched": (c_int, [_P, c_int, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                  ctypes.POINTER(Result)]),
    "lsq_dbg_qr": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, c_int, _P, _P, _P, _P]),
    "lsq_dbg_trsv": (c_int, [_P, c_int, c_int, c_int, _P, c_int, c_int, _P, _P]),
    "lsq_dbg_lse_residual": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P,
                                     _P, _P, _P, _P, _P, ctypes.POINTER(c_double)]),
    "lsq_dbg_gls_residual": (c_int, [_P, c_int, c_int, c_int, _P, c_int, _P, c_int, _P, _P, _P,
                                     _P, _P, _P, _P, ctypes.POINTER(c_double)]),
    "lsq_dbg_residual_dd": (c_int, [_P, c_int]),
    "lsq_dbg_step_graph": (c_int, [_P, c_int]),
    "lsq_dbg_lse_correction": (c_int, [_P, c_int, c_int, c_int, c_int, _P, c_int, _P, c_int, _P,
                                       _P, _P, _P, _P, _P]),
    "lsq_dbg_gls_correction": (c_int, [_P, c_int, c_int, c_int, c_int, _P, c_int, _P, c_int, _P,
                                       _P, _P, _P, _P, _P]),
    "lsq_dbg_bd_apply": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, _P, c_int, _P, c_int,
                                 c_double, c_double, _P, _P]),
    "lsq_dbg_bd_apply_graph": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, _P, c_int, _P, c_int,
                                       c_double, c_double, _P, _P, c_int, ctypes.POINTER(c_int)]),
    "lsq_dbg_timer_enable": (c_int, [_P, ctypes.c_char_p]),
    "lsq_dbg_timer_read": (c_int, [_P, ctypes.POINTER(c_double), ctypes.POINTER(c_int),
                                   ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "lsq_dbg_copy": (c_int, [_P, _P, _P, ctypes.c_longlong]),
    "lsq_dbg_batch_wait": (c_int, [_P, ctypes.c_double]),
    "lsq_dbg_batch_timeline": (c_int, [_P, c_int, _P]),
    "lsq_dbg_batch_route": (c_int, [_P, ctypes.c_double]),
    "lsq_dbg_batch_split": (c_int, [_P, ctypes.c_double]),
    "lsq_dbg_batch_pre": (c_int, [_P, ctypes.c_double]),
    "lsq_batch_tuning": (c_int, [_P, c_int, _P, _P, _P, _P, _P]),
    "lsq_dbg_batch_regime": (c_int, [_P, ctypes.POINTER(c_double)]),
    "lsq_dbg_history": (c_int, [_P, c_int, _P, _P]),
    "lsq_dbg_deterministic": (c_int, [_P, c_int]),
    "lsq_dbg_lookahead": (c_int, [_P, c_int]),
    "lsq_dbg_factors_bytes": (c_int, [_P, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong)]),
    "lsq_dbg_noalloc_bytes": (c_int, [_P, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong)]),
    "lsq_dbg_noalloc_cap": (c_int, [ctypes.c_longlong]),
    "lsq_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def header_symbols():
    """Function names declared in include/lsq.h and include/lsq_debug.h."""
    names = []
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for mt in re.finditer(r"^(?:[A-Za-z_][\w\s\*]*?)\b([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M):
            name = mt.group(1)
            if name not in names and not name.startswith("LSQ"):
                names.append(name)
    return names


_variants = {}
POISON_LIB_PATH = os.path.join(_HERE, "liblsq_poison.so")


def _bind(path: str) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2406_16499_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblsq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _lib = _bind(path)
    return _lib


def load_variant(path: str) -> ctypes.CDLL:
    """A debug build of the library (e.g. liblsq_poison.so) beside the main
    one, for a Handle(lib=...)."""
    if path not in _variants:
        _variants[path] = _bind(path)
    return _variants[path]


def default_opts(**kw) -> Opts:
    o = Opts()
    load().lsq_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        if k == "solver" and isinstance(v, str):
            v = SOLVER[v]
        setattr(o, k, v)
    return o


# ----------------------------------------------------------- tensors ----

def _torch():
    import torch
    return torch


def colmajor(a, device="cuda"):
    """float64 device tensor with column-major storage (ld = rows) holding `a`."""
    torch = _torch()
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        t = torch.empty(a.shape[0], dtype=torch.float64, device=device)
        t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
        return t
    r, c = a.shape
    t = torch.empty_strided((r, c), (1, max(r, 1)), dtype=torch.float64, device=device)
    t.copy_(torch.from_numpy(np.asfortranarray(a)))
    return t


def colmajor_c(a, device="cuda"):
    """complex128 device tensor with column-major storage holding `a` (the
    interleaved (re, im) layout the complex entry points take)."""
    torch = _torch()
    a = np.asarray(a, dtype=np.complex128)
    if a.ndim == 1:
        t = torch.empty(a.shape[0], dtype=torch.complex128, device=device)
        t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
        return t
    r, c = a.shape
    t = torch.empty_strided((r, c), (1, max(r, 1)), dtype=torch.complex128, device=device)
    t.copy_(torch.from_numpy(np.asfortranarray(a)))
    return t


def empty_c(n, device="cuda"):
    torch = _torch()
    return torch.zeros(max(int(n), 0), dtype=torch.complex128, device=device)


def empty(n, device="cuda"):
    torch = _torch()
    return torch.zeros(max(int(n), 0), dtype=torch.float64, device=device)


def _ptr(t):
    if t is None:
        return None
    torch = _torch()
    assert t.dtype == torch.float64, "liblsq takes float64 tensors"
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(t.data_ptr() or 8)


def _cptr(t):
    if t is None:
        return None
    torch = _torch()
    assert t.dtype == torch.complex128, "the complex entry points take complex128 tensors"
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(t.data_ptr() or 16)


def _ld(t):
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    r, c = t.shape
    if c > 1 and t.stride(0) != 1:
        raise ValueError("matrix must be column-major (stride(0) == 1); use lsq.colmajor")
    return max(int(t.stride(1)) if c > 1 else r, 1)


# Every live handle, factors object and batch plan, closed (factors and plans
# first) by an exit hook that runs before the interpreter tears its modules
# down: a destructor left to the final garbage collection could otherwise
# call into the HIP runtime after a profiler or torch has finalized it.
_LIVE_HANDLES: "weakref.WeakSet" = weakref.WeakSet()
_LIVE_FACTORS: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    for f in list(_LIVE_FACTORS):
        try:
            f.close()
        except Exception:
            pass
    for h in list(_LIVE_HANDLES):
        try:
            h.close()
        except Exception:
            pass


class Factors:
    """Stored factors of one pair (lse_factor / gls_factor); keeps the pair's
    tensors alive, since every solve's FP64 residual reads them."""

    def __init__(self, handle, ptr, kind, shape, keep):
        self.handle, self.f, self.kind, self.shape, self._keep = handle, ptr, kind, shape, keep
        _LIVE_FACTORS.add(self)

    def solve(self, *vecs, opts: Optional[Opts] = None):
        """LSE: solve(b, d, x, r=None, v=None); GLS: solve(d, x, y, z=None)."""
        lib, res = self.handle.lib, Result()
        o = ctypes.byref(opts) if opts is not None else None
        if self.kind == "lse":
            b, d, x, *rest = vecs
            r, v = (rest + [None, None])[:2]
            rc = lib.lse_solve_factored(self.handle.h, self.f, _ptr(b), _ptr(d), _ptr(x), _ptr(r),
                                        _ptr(v), o, ctypes.byref(res))
        else:
            d, x, y, *rest = vecs
            z = (rest + [None])[0]
            rc = lib.gls_solve_factored(self.handle.h, self.f, _ptr(d), _ptr(x), _ptr(y), _ptr(z),
                                        o, ctypes.byref(res))
        return rc, res

    def solve_noalloc(self, b, d, x, r=None, v=None, opts: Optional[Opts] = None):
        """lse_solve_factored_noalloc (LSE factors only)."""
        if self.kind != "lse":
            raise ValueError("the allocation-free solve takes LSE factors")
        lib, res = self.handle.lib, Result()
        o = ctypes.byref(opts) if opts is not None else None
        rc = lib.lse_solve_factored_noalloc(self.handle.h, self.f, _ptr(b), _ptr(d), _ptr(x),
                                            _ptr(r), _ptr(v), o, ctypes.byref(res))
        return rc, res

    def noalloc_bytes(self):
        """(bytes one allocation-free solve needs, bytes it accepts)."""
        need, cap = ctypes.c_longlong(), ctypes.c_longlong()
        rc = self.handle.lib.lsq_dbg_noalloc_bytes(self.f, ctypes.byref(need), ctypes.byref(cap))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_noalloc_bytes = {rc}")
        return need.value, cap.value

    def bytes(self):
        """(bytes in use, bytes held) of the factors' device memory."""
        u, c = ctypes.c_longlong(), ctypes.c_longlong()
        rc = self.handle.lib.lsq_dbg_factors_bytes(self.f, ctypes.byref(u), ctypes.byref(c))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_factors_bytes = {rc}")
        return u.value, c.value

    def close(self):
        if self.f:
            self.handle.lib.lsq_factors_destroy(self.f)
            self.f = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """A captured persistent batch (lsq_batch_plan_create) over a fixed list
    of descriptors; keeps them (and the caller's tensors, via `keep`) alive."""

    def __init__(self, handle, problems, opts: Optional[Opts] = None, keep=None):
        self.handle, self._keep = handle, keep
        self._arr = (Problem * len(problems))(*problems)
        self.count = len(problems)
        ptr = c_void_p()
        rc = handle.lib.lsq_batch_plan_create(handle.h, self.count, self._arr,
                                              ctypes.byref(opts) if opts is not None else None,
                                              ctypes.byref(ptr))
        if rc != 0:
            raise RuntimeError(f"lsq_batch_plan_create = {rc}: {handle.last_error()}")
        self.p = ptr
        _LIVE_FACTORS.add(self)

    def run(self, raw: bool = False):
        """Replay; (rc, [Result] in the order of creation; raw: the ctypes array)."""
        res = (Result * self.count)()
        rc = self.handle.lib.lsq_batch_plan_run(self.p, res)
        return rc, (res if raw else list(res))

    def close(self):
        if self.p:
            self.handle.lib.lsq_batch_plan_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Handle:
    """Owns an lsq_handle bound to the current torch device and stream."""

    def __init__(self, device: Optional[int] = None, load_selector: bool = True, lib=None,
                 load_tuning: bool = True):
        torch = _torch()
        self.lib = lib if lib is not None else load()
        dev = torch.cuda.current_device() if device is None else device
        h = ctypes.c_void_p()
        rc = self.lib.lsq_create(ctypes.byref(h), dev)
        if rc != 0:
            raise RuntimeError(f"lsq_create failed ({rc})")
        self.h = h
        _LIVE_HANDLES.add(self)
        self.sync_stream()
        if load_selector:
            from . import selector
            if os.path.exists(selector.WEIGHTS_PATH):
                self.selector_set(selector.load())
        if load_tuning:
            from . import autotune
            table = autotune.load()
            if table:
                self.batch_tuning(table)

    def selector_set(self, weights):
        """Install selector weights (LSQ_SELECTOR_WEIGHTS floats) or remove them (None)."""
        if weights is None:
            rc = self.lib.lsq_selector_set(self.h, None, 0)
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32)
            rc = self.lib.lsq_selector_set(self.h, w.ctypes.data_as(ctypes.POINTER(c_float)), w.size)
        if rc != 0:
            raise RuntimeError(f"lsq_selector_set = {rc}: {self.last_error()}")

    def selector_features(self, desc, with_logits=False):
        """(features[16], logits[7] or None, classes[2] or None) of one instance descriptor."""
        f = (c_float * 16)()
        lo = (c_float * 7)() if with_logits else None
        cl = (c_int * 2)() if with_logits else None
        rc = self.lib.lsq_selector_features(self.h, ctypes.byref(desc), f, lo, cl)
        if rc != 0:
            raise RuntimeError(f"lsq_selector_features = {rc}: {self.last_error()}")
        return (np.array(f, np.float32), None if lo is None else np.array(lo, np.float32),
                None if cl is None else list(cl))

    def sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream().cuda_stream
        self.lib.lsq_set_stream(self.h, ctypes.c_void_p(s))

    def close(self):
        if self.h:
            self.lib.lsq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return (self.lib.lsq_last_error(self.h) or b"").decode()

    # -------------------------------------------------------- solvers --
    def lse_solve(self, A, B, b, d, x, r=None, v=None, opts: Optional[Opts] = None):
        m, n = A.shape
        p = B.shape[0]
        res = Result()
        rc = self.lib.lse_solve(self.h, m, n, p, _ptr(A), _ld(A), _ptr(B), _ld(B) if p else 1,
                                _ptr(b), _ptr(d), _ptr(x), _ptr(r), _ptr(v),
                                ctypes.byref(opts) if opts is not None else None, ctypes.byref(res))
        return rc, res

    def gls_solve(self, W, V, d, x, y, z=None, opts: Optional[Opts] = None):
        n, m = W.shape
        p = V.shape[1]
        res = Result()
        rc = self.lib.gls_solve(self.h, n, m, p, _ptr(W), _ld(W), _ptr(V), _ld(V), _ptr(d),
                                _ptr(x), _ptr(y), _ptr(z),
                                ctypes.byref(opts) if opts is not None else None, ctypes.byref(res))
        return rc, res

    def zlse_solve(self, A, B, b, d, x, r=None, v=None, opts: Optional[Opts] = None):
        """Complex LSE (complex128 column-major tensors)."""
        m, n = A.shape
        p = B.shape[0]
        res = Result()
        rc = self.lib.zlse_solve(self.h, m, n, p, _cptr(A), _ld(A), _cptr(B), _ld(B) if p else 1,
                                 _cptr(b), _cptr(d), _cptr(x), _cptr(r), _cptr(v),
                                 ctypes.byref(opts) if opts is not None else None, ctypes.byref(res))
        return rc, res

    def zgls_solve(self, W, V, d, x, y, z=None, opts: Optional[Opts] = None):
        """Complex GLS (complex128 column-major tensors)."""
        n, m = W.shape
        p = V.shape[1]
        res = Result()
        rc = self.lib.zgls_solve(self.h, n, m, p, _cptr(W), _ld(W), _cptr(V), _ld(V), _cptr(d),
                                 _cptr(x), _cptr(y), _cptr(z),
                                 ctypes.byref(opts) if opts is not None else None, ctypes.byref(res))
        return rc, res

    def lse_factor(self, A, B, prec: str = "fp32") -> "Factors":
        """Factor (A, B) once at `prec`; A and B must outlive the returned object."""
        m, n = A.shape
        p = B.shape[0]
        f = c_void_p()
        rc = self.lib.lse_factor(self.h, m, n, p, _ptr(A), _ld(A), _ptr(B), _ld(B) if p else 1,
                                 PREC[prec], ctypes.byref(f))
        if rc != 0:
            raise RuntimeError(f"lse_factor = {rc}: {self.last_error()}")
        return Factors(self, f, "lse", (m, n, p), (A, B))

    def gls_factor(self, W, V, prec: str = "fp32") -> "Factors":
        """Factor (W, V) once at `prec`; W and V must outlive the returned object."""
        n, m = W.shape
        p = V.shape[1]
        f = c_void_p()
        rc = self.lib.gls_factor(self.h, n, m, p, _ptr(W), _ld(W), _ptr(V), _ld(V),
                                 PREC[prec], ctypes.byref(f))
        if rc != 0:
            raise RuntimeError(f"gls_factor = {rc}: {self.last_error()}")
        return Factors(self, f, "gls", (n, m, p), (W, V))

    def lsq_solve_batched(self, problems, opts: Optional[Opts] = None, which: str = "lsq", raw: bool = False):
        """(rc, results) of one batched call.  problems: descriptors, or the
        array problem_array() built from them once (no per-call marshalling);
        raw: the results as the ctypes array instead of a list."""
        arr = problems if isinstance(problems, ctypes.Array) else problem_array(problems)
        res = (Result * len(arr))()
        fn = {"lsq": self.lib.lsq_solve_batched, "lse": self.lib.lse_solve_batched,
              "gls": self.lib.gls_solve_batched}[which]
        rc = fn(self.h, len(arr), arr, ctypes.byref(opts) if opts is not None else None, res)
        return rc, (res if raw else list(res))

    def batch_plan(self, problems, opts: Optional[Opts] = None, keep=None) -> "BatchPlan":
        return BatchPlan(self, problems, opts, keep)

    def set_batch_mode(self, mode: str) -> None:
        """"persistent" (default: one work-group per eligible instance, the
        FP64 rung beside the FP32 launch), "sequential" (persistent, the FP64
        rung as a second launch) or "workers" (concurrent per-instance
        solves)."""
        rc = self.lib.lsq_set_batch_mode(self.h, {"persistent": 0, "workers": 1, "sequential": 2}[mode])
        if rc != 0:
            raise RuntimeError(f"lsq_set_batch_mode = {rc}")

    def dbg_batch_timeline(self, count: int) -> np.ndarray:
        """(count, 2, 3) ms: per problem of the last persistent batched call,
        (start, factored, end) of its FP32 and FP64 attempts (NaN: none)."""
        out = np.empty((count, 2, 3), np.float64)
        rc = self.lib.lsq_dbg_batch_timeline(self.h, int(count), out.ctypes.data_as(c_void_p))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_timeline = {rc}: {self.last_error()}")
        return out

    def dbg_history(self, max_steps: int = 256):
        """(berr (k, 3), rung (k, 3): precision, solver, inner iterations) of
        the refinement steps of the last single solve."""
        berr = np.empty((max_steps, 3), np.float64)
        rung = np.empty((max_steps, 3), np.int32)
        n = self.lib.lsq_dbg_history(self.h, int(max_steps), berr.ctypes.data_as(c_void_p),
                                     rung.ctypes.data_as(c_void_p))
        if n < 0:
            raise RuntimeError(f"lsq_dbg_history = {n}: {self.last_error()}")
        k = min(n, max_steps)
        return berr[:k], rung[:k]

    def batch_tuning(self, entries) -> None:
        """Install the persistent batch's launch-shape table: entries of
        (max_dim, route, fp64_share[, pre[, esc_max]]); [] clears it and any
        table resets the handle's escalation regime to 1."""
        n = len(entries)
        md = np.array([e[0] for e in entries], np.int32)
        rt = np.array([e[1] for e in entries], np.float64)
        sh = np.array([e[2] for e in entries], np.float64)
        pr = np.array([e[3] if len(e) > 3 else 0.0 for e in entries], np.float64)
        em = np.array([e[4] if len(e) > 4 else 1.0 for e in entries], np.float64)
        rc = self.lib.lsq_batch_tuning(self.h, n, md.ctypes.data_as(c_void_p), rt.ctypes.data_as(c_void_p),
                                       sh.ctypes.data_as(c_void_p), pr.ctypes.data_as(c_void_p),
                                       em.ctypes.data_as(c_void_p))
        if rc != 0:
            raise RuntimeError(f"lsq_batch_tuning = {rc}: {self.last_error()}")

    def dbg_batch_regime(self) -> float:
        """The escalation fraction of the last FP32-first persistent batch."""
        v = c_double()
        rc = self.lib.lsq_dbg_batch_regime(self.h, ctypes.byref(v))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_regime = {rc}: {self.last_error()}")
        return v.value

    def dbg_batch_pre(self, per_wg: float) -> None:
        rc = self.lib.lsq_dbg_batch_pre(self.h, float(per_wg))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_pre = {rc}: {self.last_error()}")

    def dbg_batch_split(self, fp64_share: float) -> None:
        rc = self.lib.lsq_dbg_batch_split(self.h, float(fp64_share))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_split = {rc}: {self.last_error()}")

    def dbg_batch_route(self, ratio: float) -> None:
        rc = self.lib.lsq_dbg_batch_route(self.h, float(ratio))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_route = {rc}: {self.last_error()}")

    def dbg_batch_wait(self, ms: float) -> None:
        """Bound on an FP64 consumer's wait in the concurrent persistent batch."""
        rc = self.lib.lsq_dbg_batch_wait(self.h, float(ms))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_batch_wait = {rc}: {self.last_error()}")

    # ---------------------------------------------------------- debug --
    def dbg_bd_apply(self, kind, prec, A, B, alpha, beta, u):
        """y = M_l F~ M_r u for LSE (kind "lse": A m x n, B p x n) or GLS (kind
        "gls": A = W n x m, B = V n x p), factors at `prec`."""
        torch = _torch()
        y = torch.zeros_like(u)
        if kind == "lse":
            m, n = A.shape
            p = B.shape[0]
            t = LSE
        else:
            n, m = A.shape
            p = B.shape[1]
            t = GLS
        rc = self.lib.lsq_dbg_bd_apply(self.h, t, PREC[prec], m, n, p, _ptr(A), _ld(A), _ptr(B),
                                       _ld(B), float(alpha), float(beta), _ptr(u), _ptr(y))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_bd_apply = {rc}: {self.last_error()}")
        return y

    def dbg_bd_apply_graph(self, kind, prec, A, B, alpha, beta, U):
        """Y = M_l F~ M_r U column by column through replays of a captured graph;
        returns (Y, graph_used)."""
        torch = _torch()
        N, k = U.shape
        Y = torch.empty_strided((N, k), (1, max(N, 1)), dtype=torch.float64, device=U.device)
        if kind == "lse":
            m, n = A.shape
            p = B.shape[0]
            t = LSE
        else:
            n, m = A.shape
            p = B.shape[1]
            t = GLS
        used = c_int(0)
        rc = self.lib.lsq_dbg_bd_apply_graph(self.h, t, PREC[prec], m, n, p, _ptr(A), _ld(A), _ptr(B),
                                             _ld(B), float(alpha), float(beta), _ptr(U), _ptr(Y), k,
                                             ctypes.byref(used))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_bd_apply_graph = {rc}: {self.last_error()}")
        return Y, bool(used.value)

    def timer_enable(self, kernel: Optional[str]):
        """Time every launch of one kernel kind with HIP events (None disables)."""
        rc = self.lib.lsq_dbg_timer_enable(self.h, (kernel or "").encode())
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_timer_enable({kernel!r}) = {rc}: {self.last_error()}")

    def timer_read(self):
        """(total_ms, launches, flops, bytes) since the last enable / read."""
        ms, n, fl, by = c_double(), c_int(), c_double(), c_double()
        rc = self.lib.lsq_dbg_timer_read(self.h, ctypes.byref(ms), ctypes.byref(n),
                                         ctypes.byref(fl), ctypes.byref(by))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_timer_read = {rc}: {self.last_error()}")
        return ms.value, n.value, fl.value, by.value

    def dbg_copy(self, dst, src, nbytes: int):
        rc = self.lib.lsq_dbg_copy(self.h, _ptr(dst), _ptr(src), int(nbytes))
        if rc != 0:
            raise RuntimeError(f"lsq_dbg_copy = {rc}: {self.last_error()}")

    def dbg_qr(self, prec, M, X=None, want=("R", "Y1", "Y2", "Y3")):
        torch = _torch()
        r, c = M.shape
        k = min(r, c)
        nx = 0 if X is None else X.shape[1]
        R = torch.zeros((k, c), dtype=torch.float64, device=M.device).t().contiguous().t() if "R" in want else None
        outs = {}
        for key in ("Y1", "Y2", "Y3"):
            outs[key] = (torch.empty_strided((r, nx), (1, max(r, 1)), dtype=torch.float64,
                                             device=M.device) if (key in want and nx) else None)
        Rp = None
        if R is not None:
            R = torch.empty_strided((k, c), (1, max(k, 1)), dtype=torch.float64, device=M.device)
            Rp = _ptr(R)
        rc = self.lib.lsq_dbg_qr(self.h, PREC[prec] if isinstance(prec, str) else prec, r, c,
                                 _ptr(M), _ld(M), _ptr(X), _ld(X) if X is not None else max(r, 1), nx,
                                 Rp, _ptr(outs["Y1"]), _ptr(outs["Y2"]), _ptr(outs["Y3"]))
        return rc, R, outs["Y1"], outs["Y2"], outs["Y3"]

    def dbg_trsv(self, prec, U, b, trans=False, tc64=False):
        x = empty(U.shape[0], device=U.device)
        rc = self.lib.lsq_dbg_trsv(self.h, PREC[prec] if isinstance(prec, str) else prec,
                                   1 if tc64 else 0, U.shape[0], _ptr(U), _ld(U),
                                   1 if trans else 0, _ptr(b), _ptr(x))
        return rc, x

    def dbg_lse_residual(self, A, B, b, d, x, r, v):
        m, n = A.shape
        p = B.shape[0]
        f1, f2, f3 = empty(m, A.device), empty(p, A.device), empty(n, A.device)
        out = (c_double * 10)()
        rc = self.lib.lsq_dbg_lse_residual(self.h, m, n, p, _ptr(A), _ld(A), _ptr(B),
                                           _ld(B) if p else 1, _ptr(b), _ptr(d), _ptr(x), _ptr(r),
                                           _ptr(v), _ptr(f1), _ptr(f2), _ptr(f3), out)
        return rc, (f1, f2, f3), list(out)

    def dbg_gls_residual(self, W, V, d, x, y, z):
        n, m = W.shape
        p = V.shape[1]
        f1, f2, f3 = empty(p, W.device), empty(n, W.device), empty(m, W.device)
        out = (c_double * 10)()
        rc = self.lib.lsq_dbg_gls_residual(self.h, n, m, p, _ptr(W), _ld(W), _ptr(V), _ld(V),
                                           _ptr(d), _ptr(x), _ptr(y), _ptr(z), _ptr(f1), _ptr(f2),
                                           _ptr(f3), out)
        return rc, (f1, f2, f3), list(out)

    def dbg_lse_correction(self, prec, A, B, f1, f2, f3):
        m, n = A.shape
        p = B.shape[0]
        dr, dv, dx = empty(m, A.device), empty(p, A.device), empty(n, A.device)
        rc = self.lib.lsq_dbg_lse_correction(self.h, PREC[prec] if isinstance(prec, str) else prec,
                                             m, n, p, _ptr(A), _ld(A), _ptr(B), _ld(B) if p else 1,
                                             _ptr(f1), _ptr(f2), _ptr(f3), _ptr(dr), _ptr(dv),
                                             _ptr(dx))
        return rc, dr, dv, dx

    def dbg_gls_correction(self, prec, W, V, f1, f2, f3):
        n, m = W.shape
        p = V.shape[1]
        dy, dz, dx = empty(p, W.device), empty(n, W.device), empty(m, W.device)
        rc = self.lib.lsq_dbg_gls_correction(self.h, PREC[prec] if isinstance(prec, str) else prec,
                                             n, m, p, _ptr(W), _ld(W), _ptr(V), _ld(V), _ptr(f1),
                                             _ptr(f2), _ptr(f3), _ptr(dy), _ptr(dz), _ptr(dx))
        return rc, dy, dz, dx


def problem_array(problems):
    """The C array of batch descriptors that the batched entry points read."""
    return (Problem * len(problems))(*problems)


def make_problem(kind, tensors, x, y=None) -> Problem:
    """Batch descriptor from device tensors (LSE: A, B, b, d; GLS: W, V, d)."""
    pr = Problem()
    if kind == "lse":
        A, B, b, d = tensors
        pr.type, pr.m, pr.n, pr.p = LSE, A.shape[0], A.shape[1], B.shape[0]
        pr.A, pr.B, pr.b, pr.d = A.data_ptr(), B.data_ptr(), b.data_ptr(), d.data_ptr()
        pr.lda, pr.ldb = _ld(A), (_ld(B) if B.shape[0] else 1)
        pr.x, pr.y = x.data_ptr(), None
    else:
        W, V, d = tensors
        pr.type, pr.n, pr.m, pr.p = GLS, W.shape[0], W.shape[1], V.shape[1]
        pr.A, pr.B, pr.b, pr.d = W.data_ptr(), V.data_ptr(), None, d.data_ptr()
        pr.lda, pr.ldb = _ld(W), _ld(V)
        pr.x, pr.y = x.data_ptr(), y.data_ptr()
    return pr
