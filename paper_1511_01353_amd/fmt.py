"""Thin Python binding of libfmt.so (the C ABI declared in include/fmt.h).

Functions carry the C names and only marshal arguments: device arrays are
torch tensors on the GPU (their data pointers are passed through), host
outputs are numpy arrays, and the stream is torch's current HIP stream unless
one is given.  Every step of fit and evaluation runs in the library's HIP
kernels; if the library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_uint8, c_uint32, c_void_p
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfmt.so")

FMT_OK = 0
FMT_E_INVALID_ARG = 1
FMT_E_DOMAIN = 2
FMT_E_UNDERDETERMINED = 3
FMT_E_OOM = 4
FMT_E_NUMERIC = 5
FMT_E_DEVICE = 6
FMT_E_BUSY = 7
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "DOMAIN", 3: "UNDERDETERMINED", 4: "OOM", 5: "NUMERIC",
                6: "DEVICE", 7: "BUSY"}

FMT_F32 = 0
FMT_F64 = 1
FMT_PATH_FP64 = 0
FMT_PATH_MIXED = 1
FMT_GRAM_MOMENTS = 0
FMT_GRAM_MFMA = 1
FMT_GRAM_MOMENTS_LEVEL = 2
FMT_MAX_P = 14
FMT_MAX_DEPTH = 10
FMT_MAX_LEVELS = FMT_MAX_DEPTH + 1
FMT_REFIT_MAX_FIELDS = 4096

EXPORTED = [
    "fmt_default_opts", "fmt_fit", "fmt_fit_batch", "fmt_eval", "fmt_eval_noalloc", "fmt_tree_wait",
    "fmt_tree_get_info",
    "fmt_tree_export_nodes", "fmt_tree_export_points", "fmt_tree_import", "fmt_refit", "fmt_tree_destroy",
    "fmt_last_error", "fmt_version", "fmt_profile_enable", "fmt_profile_reset", "fmt_profile_read",
    "fmt_rbf_factored",
]


class fmt_fit_opts(ctypes.Structure):
    _fields_ = [("p", c_int), ("tol", c_double), ("max_depth", c_int), ("path", c_int),
                ("refine_steps", c_int), ("box_lo", c_double * 3), ("box_hi", c_double * 3), ("gram", c_int)]


class fmt_tree_info(ctypes.Structure):
    _fields_ = [("nodes", c_int64), ("n_points", c_int64), ("depth", c_int32), ("p", c_int32), ("L", c_int32),
                ("max_depth", c_int32), ("path", c_int32), ("rank_deficient_nodes", c_int32),
                ("per_level", c_int64 * FMT_MAX_LEVELS), ("device_bytes", c_int64)]


class fmt_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int64), ("ms", c_double), ("units", c_double)]


class FmtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfmt.so (once).  Raises if it is not built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfmt.so is not built at {path}; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    T = c_void_p
    lib.fmt_default_opts.argtypes = [POINTER(fmt_fit_opts)]
    lib.fmt_default_opts.restype = None
    lib.fmt_fit.argtypes = [POINTER(fmt_fit_opts), c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p,
                            POINTER(T)]
    lib.fmt_fit.restype = c_int
    lib.fmt_fit_batch.argtypes = [POINTER(fmt_fit_opts), POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                  POINTER(c_void_p), POINTER(c_int64), c_int, c_int, c_void_p, POINTER(T)]
    lib.fmt_fit_batch.restype = c_int
    lib.fmt_eval.argtypes = [T, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p]
    lib.fmt_eval.restype = c_int
    lib.fmt_eval_noalloc.argtypes = [T, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p]
    lib.fmt_eval_noalloc.restype = c_int
    lib.fmt_rbf_factored.argtypes = [c_int, c_double, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                     c_void_p, c_int64, c_int, c_void_p, c_void_p]
    lib.fmt_rbf_factored.restype = c_int
    lib.fmt_tree_wait.argtypes = [T]
    lib.fmt_tree_wait.restype = c_int
    lib.fmt_tree_get_info.argtypes = [T, POINTER(fmt_tree_info)]
    lib.fmt_tree_get_info.restype = c_int
    lib.fmt_tree_export_nodes.argtypes = [T, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.fmt_tree_export_nodes.restype = c_int
    lib.fmt_tree_export_points.argtypes = [T, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.fmt_tree_export_points.restype = c_int
    lib.fmt_tree_import.argtypes = [POINTER(fmt_fit_opts), c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                    POINTER(T)]
    lib.fmt_tree_import.restype = c_int
    lib.fmt_refit.argtypes = [T, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_int, c_void_p,
                              POINTER(c_void_p)]
    lib.fmt_refit.restype = c_int
    lib.fmt_tree_destroy.argtypes = [T]
    lib.fmt_tree_destroy.restype = None
    lib.fmt_last_error.argtypes = []
    lib.fmt_last_error.restype = c_char_p
    lib.fmt_version.argtypes = []
    lib.fmt_version.restype = c_char_p
    lib.fmt_profile_enable.argtypes = [c_int]
    lib.fmt_profile_enable.restype = c_int
    lib.fmt_profile_reset.argtypes = []
    lib.fmt_profile_reset.restype = None
    lib.fmt_profile_read.argtypes = [POINTER(fmt_kernel_stat), c_int]
    lib.fmt_profile_read.restype = c_int
    _lib = lib
    return lib


def _check(st: int):
    if st != FMT_OK:
        raise FmtError(st, load_library().fmt_last_error().decode())


def _dptr(t) -> int:
    """Device pointer of a torch tensor (contiguous, on the GPU)."""
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return FMT_F32
    if t.dtype == torch.float64:
        return FMT_F64
    raise ValueError("coordinates and values must be float32 or float64")


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _hptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(c_void_p)


# ----------------------------------------------------------------------------
# C-named calls
# ----------------------------------------------------------------------------
def fmt_default_opts(**kw) -> fmt_fit_opts:
    o = fmt_fit_opts()
    load_library().fmt_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k in ("box_lo", "box_hi"):
            getattr(o, k)[:] = list(v)
        else:
            setattr(o, k, v)
    return o


def fmt_fit(opts: fmt_fit_opts, x, y, z, f, stream=None) -> "Tree":
    n = x.numel()
    if not (y.numel() == z.numel() == f.numel() == n):
        raise ValueError("x, y, z, f must have the same length")
    dt = _dtype_code(x)
    if not (_dtype_code(y) == _dtype_code(z) == _dtype_code(f) == dt):
        raise ValueError("x, y, z, f must share one dtype")
    h = c_void_p()
    _check(load_library().fmt_fit(ctypes.byref(opts), _dptr(x), _dptr(y), _dptr(z), _dptr(f), n, dt,
                                  _stream(stream), ctypes.byref(h)))
    return Tree(h, opts, n)


def fmt_fit_batch(opts: Sequence[fmt_fit_opts], xs, ys, zs, fs, stream=None) -> list:
    k = len(opts)
    if not (len(xs) == len(ys) == len(zs) == len(fs) == k):
        raise ValueError("one options entry and one array set per problem")
    dt = _dtype_code(xs[0])
    oa = (fmt_fit_opts * k)(*opts)
    P = c_void_p * k
    px = P(*[_dptr(t) for t in xs])
    py = P(*[_dptr(t) for t in ys])
    pz = P(*[_dptr(t) for t in zs])
    pf = P(*[_dptr(t) for t in fs])
    ns = (c_int64 * k)(*[t.numel() for t in xs])
    for group in (xs, ys, zs, fs):
        for t in group:
            if _dtype_code(t) != dt:
                raise ValueError("all arrays of a batch must share one dtype")
    out = (c_void_p * k)()
    _check(load_library().fmt_fit_batch(oa, px, py, pz, pf, ns, k, dt, _stream(stream), out))
    return [Tree(c_void_p(out[i]), opts[i], int(ns[i])) for i in range(k)]


def fmt_eval(tree: "Tree", qx, qy, qz, out, sort_queries: int = -1, stream=None):
    import torch
    nq = qx.numel()
    if not (qy.numel() == qz.numel() == out.numel() == nq):
        raise ValueError("query arrays and output must have the same length")
    if out.dtype != torch.float64:
        raise ValueError("output must be float64")
    dt = _dtype_code(qx)
    _check(load_library().fmt_eval(tree.handle, _dptr(qx), _dptr(qy), _dptr(qz), nq, dt, _dptr(out),
                                   int(sort_queries), _stream(stream)))
    return out


def fmt_eval_noalloc(tree: "Tree", qx, qy, qz, out, sort_queries: int = -1, stream=None):
    """fmt_eval through the entry point that allocates nothing (its sorted mode
    uses the library's fixed per-device scratch array)."""
    import torch
    nq = qx.numel()
    if not (qy.numel() == qz.numel() == out.numel() == nq):
        raise ValueError("query arrays and output must have the same length")
    if out.dtype != torch.float64:
        raise ValueError("output must be float64")
    dt = _dtype_code(qx)
    _check(load_library().fmt_eval_noalloc(tree.handle, _dptr(qx), _dptr(qy), _dptr(qz), nq, dt, _dptr(out),
                                           int(sort_queries), _stream(stream)))
    return out


def fmt_rbf_factored(p: int, eps: float, x, y, z, xq, yq, zq, out=None, stream=None):
    """Truncated Gaussian-RBF factorisation between query points and points:
    an (nq, n) float64 device tensor (out, if given, must be one)."""
    import torch
    n, nq = x.numel(), xq.numel()
    if not (y.numel() == z.numel() == n and yq.numel() == zq.numel() == nq):
        raise ValueError("coordinate arrays must have matching lengths")
    dt = _dtype_code(x)
    if not all(_dtype_code(t) == dt for t in (y, z, xq, yq, zq)):
        raise ValueError("all coordinates must share one dtype")
    if out is None:
        out = torch.empty((nq, n), dtype=torch.float64, device=x.device)
    if out.dtype != torch.float64 or out.numel() != nq * n:
        raise ValueError("out must be a float64 tensor of nq * n entries")
    _check(load_library().fmt_rbf_factored(int(p), float(eps), _dptr(x), _dptr(y), _dptr(z), n, _dptr(xq),
                                           _dptr(yq), _dptr(zq), nq, dt, _dptr(out), _stream(stream)))
    return out


def fmt_tree_wait(tree: "Tree"):
    _check(load_library().fmt_tree_wait(tree.handle))


def fmt_tree_get_info(tree: "Tree") -> fmt_tree_info:
    info = fmt_tree_info()
    _check(load_library().fmt_tree_get_info(tree.handle, ctypes.byref(info)))
    return info


def fmt_tree_export_nodes(tree: "Tree"):
    info = fmt_tree_get_info(tree)
    m = int(info.nodes)
    level = np.zeros(m, np.uint8)
    prefix = np.zeros(m, np.uint32)
    begin = np.zeros(m, np.uint32)
    count = np.zeros(m, np.uint32)
    flags = np.zeros(m, np.uint32)
    coeffs = np.zeros((m, int(info.L)), np.float64)
    _check(load_library().fmt_tree_export_nodes(tree.handle, _hptr(level), _hptr(prefix), _hptr(begin),
                                                _hptr(count), _hptr(flags), _hptr(coeffs)))
    return dict(level=level, prefix=prefix, begin=begin, count=count, flags=flags, coeffs=coeffs)


def fmt_tree_export_points(tree: "Tree"):
    info = fmt_tree_get_info(tree)
    n = int(info.n_points)
    keys = np.zeros(n, np.uint32)
    order = np.zeros(n, np.uint32)
    leaf = np.zeros(n, np.uint32)
    resid = np.zeros(n, np.float64)
    _check(load_library().fmt_tree_export_points(tree.handle, _hptr(keys), _hptr(order), _hptr(leaf),
                                                 _hptr(resid)))
    return dict(keys=keys, order=order, leaf=leaf, residual=resid)


def fmt_tree_import(opts: fmt_fit_opts, level, prefix, coeffs, stream=None) -> "Tree":
    level = np.ascontiguousarray(level, np.uint8)
    prefix = np.ascontiguousarray(prefix, np.uint32)
    coeffs = np.ascontiguousarray(coeffs, np.float64)
    h = c_void_p()
    _check(load_library().fmt_tree_import(ctypes.byref(opts), level.shape[0], _hptr(level), _hptr(prefix),
                                          _hptr(coeffs), _stream(stream), ctypes.byref(h)))
    return Tree(h, opts, 0)


def fmt_refit(tree: "Tree", x, y, z, f, stream=None) -> list:
    """f: (n,) or (m, n) contiguous device tensor of values on the tree's points;
    returns m new trees (the tree's node set, the fields' coefficients)."""
    n = x.numel()
    if not (y.numel() == z.numel() == n):
        raise ValueError("x, y, z must have the same length")
    m = 1 if f.dim() == 1 else f.shape[0]
    if f.numel() != m * n:
        raise ValueError("f must hold m fields of n values")
    dt = _dtype_code(x)
    if not (_dtype_code(y) == _dtype_code(z) == _dtype_code(f) == dt):
        raise ValueError("x, y, z, f must share one dtype")
    out = (c_void_p * max(m, 1))()
    _check(load_library().fmt_refit(tree.handle, _dptr(x), _dptr(y), _dptr(z), _dptr(f), n, m, dt,
                                    _stream(stream), out))
    return [Tree(c_void_p(out[j]), tree.opts, n) for j in range(m)]


def fmt_tree_destroy(tree: "Tree"):
    tree.close()


def fmt_last_error() -> str:
    return load_library().fmt_last_error().decode()


def fmt_version() -> str:
    return load_library().fmt_version().decode()


def fmt_profile_enable(on: bool = True) -> bool:
    return bool(load_library().fmt_profile_enable(1 if on else 0))


def fmt_profile_reset():
    load_library().fmt_profile_reset()


def fmt_profile_read() -> dict:
    """{kernel name: (launches, total ms, total work units)}."""
    lib = load_library()
    n = lib.fmt_profile_read(None, 0)
    rows = (fmt_kernel_stat * n)()
    n = lib.fmt_profile_read(rows, n)
    return {rows[i].name.decode(): (int(rows[i].launches), float(rows[i].ms), float(rows[i].units))
            for i in range(n)}


class Tree:
    """Owner of one fmt_tree handle."""

    def __init__(self, handle: c_void_p, opts: fmt_fit_opts, n: int):
        self.handle = handle
        self.opts = opts
        self.n = n

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().fmt_tree_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> fmt_tree_info:
        return fmt_tree_get_info(self)

    def eval(self, qx, qy, qz, out=None, sort_queries: int = -1, stream=None):
        import torch
        if out is None:
            out = torch.empty(qx.numel(), dtype=torch.float64, device=qx.device)
        return fmt_eval(self, qx, qy, qz, out, sort_queries, stream)

    def export_nodes(self):
        return fmt_tree_export_nodes(self)

    def export_points(self):
        return fmt_tree_export_points(self)
