"""FP64 CPU oracle for the fused BLAS-1/BLAS-2 sequences.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product library. It shares no code
with the GPU path. ``kf_oracle.c`` holds the plain definitions (Table 1 of the
paper, Section 3.3 for the elementary calls); this module only marshals numpy
arrays into it. ``mlp.py`` holds the FP64 reference of the learned cost model.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
OMP_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")
_SRC = os.path.join(_HERE, "kf_oracle.c")
_lib = None
_omp_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def _gcc(out: str, extra) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-fast-math"] + list(extra) + ["-o", tmp, _SRC])
    os.replace(tmp, out)


def build(force: bool = False) -> str:
    """Compile kf_oracle.c with gcc (strict IEEE double, no contraction): the
    one-thread library and the all-core OpenMP build of the same source."""
    for out, extra in ((LIB_PATH, []), (OMP_LIB_PATH, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            _gcc(out, extra)
    return LIB_PATH


def load(path: str):
    """Load a compiled oracle library and declare its signatures."""
    L = ctypes.CDLL(path)
    sig = {
        "kfo_f2d": [_i64, _F, _D],
        "kfo_scal": [_i64, _dbl, _D, _D],
        "kfo_axpy": [_i64, _dbl, _D, _D, _D],
        "kfo_dot": [_i64, _D, _D],
        "kfo_gemv": [_i64, _i64, _dbl, _D, _D, _dbl, _D, _D],
        "kfo_gemtv": [_i64, _i64, _dbl, _D, _D, _dbl, _D, _D],
        "kfo_ger": [_i64, _i64, _dbl, _D, _D, _D, _D],
        "kfo_axpydot": [_i64, _dbl, _F, _F, _F, _D, _D],
        "kfo_waxpby": [_i64, _dbl, _F, _dbl, _F, _D],
        "kfo_bicgk": [_i64, _i64, _i64, _F, _F, _F, _D, _D],
        "kfo_atax": [_i64, _i64, _i64, _F, _F, _D],
        "kfo_gesummv": [_i64, _i64, _i64, _F, _i64, _F, _dbl, _dbl, _F, _D],
        "kfo_gemver": [_i64, _i64, _i64, _F, _F, _F, _F, _F, _dbl, _dbl, _F, _F,
                       _D, _D, _D],
        "kfo_gemv_rows": [_i64, _i64, _i64, _F, _D, _I, _i64, _D],
        "kfo_gemtv_cols": [_i64, _i64, _i64, _F, _D, _I, _i64, _D],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _dbl if name == "kfo_dot" else None
    L.kfo_threads.argtypes = []
    L.kfo_threads.restype = ctypes.c_int
    L.kfo_set_threads.argtypes = [ctypes.c_int]
    L.kfo_set_threads.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def omp_lib():
    """The all-core (OpenMP) build of the same source."""
    global _omp_lib
    if _omp_lib is None:
        if not os.path.exists(OMP_LIB_PATH):
            build()
        _omp_lib = load(OMP_LIB_PATH)
    return _omp_lib


@contextlib.contextmanager
def all_cores(threads: int):
    """Inside the block every oracle function runs on the OpenMP build with
    `threads` threads (bit-identical results: each output entry is still
    summed by one thread in the plain order). Yields the thread count the
    library reports."""
    global _lib
    saved = lib()
    L = omp_lib()
    L.kfo_set_threads(int(threads))
    _lib = L
    try:
        yield L.kfo_threads()
    finally:
        _lib = saved


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_F)


def _d(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _out(n):
    o = np.empty(int(n), dtype=np.float64)
    return o, o.ctypes.data_as(_D)


def _ld(a, cols):
    return a.shape[1] if a.ndim == 2 else cols


# ---- elementary calls on float64 operands -----------------------------------
def scal(alpha, x):
    xk, xp = _d(x)
    y, yp = _out(xk.size)
    lib().kfo_scal(xk.size, alpha, xp, yp)
    return y


def axpy(alpha, x, y):
    xk, xp = _d(x)
    yk, yp = _d(y)
    z, zp = _out(xk.size)
    lib().kfo_axpy(xk.size, alpha, xp, yp, zp)
    return z


def dot(x, y):
    xk, xp = _d(x)
    yk, yp = _d(y)
    return lib().kfo_dot(xk.size, xp, yp)


def gemv(alpha, A, x, beta=0.0, y0=None):
    Ak, Ap = _d(A)
    xk, xp = _d(x)
    y0k, y0p = _d(y0)
    m, n = Ak.shape
    y, yp = _out(m)
    lib().kfo_gemv(m, n, alpha, Ap, xp, beta, y0p, yp)
    return y


def gemtv(alpha, A, x, beta=0.0, y0=None):
    Ak, Ap = _d(A)
    xk, xp = _d(x)
    y0k, y0p = _d(y0)
    m, n = Ak.shape
    y, yp = _out(n)
    lib().kfo_gemtv(m, n, alpha, Ap, xp, beta, y0p, yp)
    return y


def ger(alpha, A, u, v):
    Ak, Ap = _d(A)
    uk, up = _d(u)
    vk, vp = _d(v)
    m, n = Ak.shape
    B = np.empty((m, n), dtype=np.float64)
    lib().kfo_ger(m, n, alpha, Ap, up, vp, B.ctypes.data_as(_D))
    return B


# ---- Table 1 sequences on float32 storage -----------------------------------
def axpydot(alpha, w, v, u):
    wk, wp = _f(w)
    vk, vp = _f(v)
    uk, up = _f(u)
    z, zp = _out(wk.size)
    r = ctypes.c_double()
    lib().kfo_axpydot(wk.size, alpha, wp, vp, up, zp, ctypes.byref(r))
    return z, r.value


def waxpby(alpha, x, beta, y):
    xk, xp = _f(x)
    yk, yp = _f(y)
    w, wp = _out(xk.size)
    lib().kfo_waxpby(xk.size, alpha, xp, beta, yp, wp)
    return w


def bicgk(A, p, r, cols=None):
    Ak, Ap = _f(A)
    m = Ak.shape[0]
    n = int(cols) if cols is not None else Ak.shape[1]
    pk, pp = _f(p)
    rk, rp = _f(r)
    q, qp = _out(m)
    s, sp = _out(n)
    lib().kfo_bicgk(m, n, Ak.shape[1], Ap, pp, rp, qp, sp)
    return q, s


def atax(A, x, cols=None):
    Ak, Ap = _f(A)
    m = Ak.shape[0]
    n = int(cols) if cols is not None else Ak.shape[1]
    xk, xp = _f(x)
    y, yp = _out(n)
    lib().kfo_atax(m, n, Ak.shape[1], Ap, xp, yp)
    return y


def gesummv(alpha, A, beta, B, x, cols=None):
    Ak, Ap = _f(A)
    Bk, Bp = _f(B)
    m = Ak.shape[0]
    n = int(cols) if cols is not None else Ak.shape[1]
    xk, xp = _f(x)
    y, yp = _out(m)
    lib().kfo_gesummv(m, n, Ak.shape[1], Ap, Bk.shape[1], Bp, alpha, beta, xp, yp)
    return y


def gemver(alpha, beta, A, u1, v1, u2, v2, y, z, cols=None, want_b=True):
    Ak, Ap = _f(A)
    m = Ak.shape[0]
    n = int(cols) if cols is not None else Ak.shape[1]
    u1k, u1p = _f(u1)
    v1k, v1p = _f(v1)
    u2k, u2p = _f(u2)
    v2k, v2p = _f(v2)
    yk, yp = _f(y)
    zk, zp = _f(z)
    B = np.empty((m, n), dtype=np.float64) if want_b else None
    Bp = B.ctypes.data_as(_D) if want_b else None
    x, xp = _out(n)
    w, wp = _out(m)
    lib().kfo_gemver(m, n, Ak.shape[1], Ap, u1p, v1p, u2p, v2p, alpha, beta, yp, zp,
                     Bp, xp, wp)
    return B, x, w


def sgemvt(alpha, beta, A, y, z, cols=None):
    """Table 1 SGEMVT: x = beta A^T y + z, then w = alpha A x (A float32 storage)."""
    n = int(cols) if cols is not None else np.asarray(A).shape[1]
    Ad = np.asarray(A)[:, :n].astype(np.float64)
    x = gemtv(beta, Ad, np.asarray(y, dtype=np.float64), 1.0, np.asarray(z, dtype=np.float64))
    w = gemv(alpha, Ad, x)
    return x, w


def vadd(w, y, z):
    """Table 1 VADD: x = w + y + z, as (w + y) + z."""
    f = lambda a: np.asarray(a, dtype=np.float64)
    return axpy(1.0, axpy(1.0, f(w), f(y)), f(z))


def gemv_rows(A, x, idx, cols=None):
    """(A x)[idx] with A float32 storage and x float64."""
    Ak, Ap = _f(A)
    n = int(cols) if cols is not None else Ak.shape[1]
    xk, xp = _d(x)
    ik = np.ascontiguousarray(idx, dtype=np.int64)
    out, op = _out(ik.size)
    lib().kfo_gemv_rows(Ak.shape[0], n, Ak.shape[1], Ap, xp, ik.ctypes.data_as(_I), ik.size, op)
    return out


def gemtv_cols(A, x, idx, cols=None):
    """(A^T x)[idx] with A float32 storage and x float64."""
    Ak, Ap = _f(A)
    n = int(cols) if cols is not None else Ak.shape[1]
    xk, xp = _d(x)
    ik = np.ascontiguousarray(idx, dtype=np.int64)
    out, op = _out(ik.size)
    lib().kfo_gemtv_cols(Ak.shape[0], n, Ak.shape[1], Ap, xp, ik.ctypes.data_as(_I), ik.size, op)
    return out


# ---- selected outputs at full size -------------------------------------------
# The compositions below evaluate the same definitions on a subset of rows or
# on column panels, so that full-size results can be checked without holding
# an n x n double matrix. Every element is computed by the routines above with
# the same arithmetic as the full definition.
def _mat_panel(A, cols):
    """float64 copy of A[:, cols] (A float32 storage)."""
    return np.ascontiguousarray(A[:, cols], dtype=np.float64)


def bicgk_sampled(A, p, r, rows, cols_idx, cols=None):
    n = int(cols) if cols is not None else A.shape[1]
    q = gemv_rows(A, p.astype(np.float64), rows, cols=n)
    s = gemtv_cols(A, r.astype(np.float64), cols_idx, cols=n)
    return q, s


def atax_sampled(A, x, cols_idx, cols=None):
    n = int(cols) if cols is not None else A.shape[1]
    t = gemv_rows(A, x.astype(np.float64), np.arange(A.shape[0]), cols=n)
    return gemtv_cols(A, t, cols_idx, cols=n)


def gesummv_sampled(alpha, A, beta, B, x, rows, cols=None):
    n = int(cols) if cols is not None else A.shape[1]
    xd = x.astype(np.float64)
    Ar = np.ascontiguousarray(A[rows, :n], dtype=np.float64)
    Br = np.ascontiguousarray(B[rows, :n], dtype=np.float64)
    t = gemv(alpha, Ar, xd)
    return gemv(beta, Br, xd, 1.0, t)


def sgemvt_sampled(alpha, beta, A, y, z, rows, cols=None, panel=512):
    """The whole x and w on the given rows (A float32 storage)."""
    n = int(cols) if cols is not None else A.shape[1]
    yd, zd = np.asarray(y, dtype=np.float64), np.asarray(z, dtype=np.float64)
    x = np.empty(n, dtype=np.float64)
    for c0 in range(0, n, panel):
        c = np.arange(c0, min(n, c0 + panel))
        x[c] = gemtv(beta, _mat_panel(A, c), yd, 1.0, zd[c])
    Ar = np.ascontiguousarray(A[rows, :n], dtype=np.float64)
    return x, gemv(alpha, Ar, x)


def gemver_sampled(alpha, beta, A, u1, v1, u2, v2, y, z, rows, cols=None, panel=512, workers=1):
    """B on the given rows, the whole x, and w on the given rows. Column
    panels of x are independent outputs; `workers` threads may take them."""
    n = int(cols) if cols is not None else A.shape[1]
    f = lambda a: np.asarray(a, dtype=np.float64)
    u1d, v1d, u2d, v2d, yd, zd = f(u1), f(v1), f(u2), f(v2), f(y), f(z)
    # x = beta B^T y + z, one column panel of B at a time
    x = np.empty(n, dtype=np.float64)

    def x_panel(c0):
        c = np.arange(c0, min(n, c0 + panel))
        Bp = ger(1.0, ger(1.0, _mat_panel(A, c), u1d, v1d[c]), u2d, v2d[c])
        x[c] = gemtv(beta, Bp, yd, 1.0, zd[c])
    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(x_panel, range(0, n, panel)))
    else:
        for c0 in range(0, n, panel):
            x_panel(c0)
    Ar = np.ascontiguousarray(A[rows, :n], dtype=np.float64)
    Br = ger(1.0, ger(1.0, Ar, u1d[rows], v1d), u2d[rows], v2d)
    w = gemv(alpha, Br, x)
    return Br, x, w
