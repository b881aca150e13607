"""ctypes binding of the C oracle (``dpd_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Inputs are widened to complex128 exactly (complex64 -> complex128 is exact), so
the oracle sees the very values the GPU receives.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def lib_path() -> str:
    return _LIB


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (plain C, no GPU toolchain)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.c_void_p


def _declare(lib):
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_forward.argtypes = [_f64p, ctypes.c_int64, _f64p, _i32p, ctypes.c_int32, _i32p,
                                   ctypes.c_int32, ctypes.c_int32, _f64p, _f64p]
    lib.oracle_forward_at.restype = ctypes.c_int
    lib.oracle_forward_at.argtypes = [_f64p, ctypes.c_int64, _f64p, _i32p, ctypes.c_int32, _i32p,
                                      ctypes.c_int32, ctypes.c_int32, _f64p, _i64p, ctypes.c_int64,
                                      _f64p]
    lib.oracle_backward.restype = ctypes.c_int
    lib.oracle_backward.argtypes = [_f64p, ctypes.c_int64, _f64p, _i32p, ctypes.c_int32, _i32p,
                                    ctypes.c_int32, ctypes.c_int32, _f64p, _f64p, _f64p, _f64p]
    lib.oracle_ls_normal.restype = ctypes.c_int
    lib.oracle_ls_normal.argtypes = [_f64p, ctypes.c_int64, _i32p, ctypes.c_int32, _i32p,
                                     ctypes.c_int32, ctypes.c_int32, _f64p, _f64p, _f64p]
    return lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _orders(o) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(o), dtype=np.int32))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _iptr(a):
    return a.ctypes.data_as(_i32p) if a.size else None


class Oracle:
    """One loaded copy of the C oracle (a path allows loading a variant build)."""

    def __init__(self, path: str | None = None):
        path = path or _LIB
        if path == _LIB and (not os.path.exists(_LIB) or
                             os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        self.lib = _declare(ctypes.CDLL(path))

    def threads(self) -> int:
        return int(self.lib.oracle_threads())

    def set_threads(self, n: int):
        """OpenMP threads of the following calls."""
        self.lib.oracle_set_threads(int(n))

    def forward(self, x, main_orders, conj_orders, L, coeffs, hist=None) -> np.ndarray:
        x = _c128(x)
        co = _c128(coeffs)
        mo, cj = _orders(main_orders), _orders(conj_orders)
        K = (mo.size + cj.size) * L + 1
        if co.size != K:
            raise ValueError("expected %d coefficients, got %d" % (K, co.size))
        h = None if hist is None else _c128(hist)
        if h is not None and h.size != L - 1:
            raise ValueError("history must hold L-1 samples")
        z = np.empty_like(x)
        rc = self.lib.oracle_forward(_ptr(x), x.size, _ptr(h), _iptr(mo), mo.size, _iptr(cj),
                                     cj.size, int(L), _ptr(co), _ptr(z))
        if rc:
            raise ValueError("oracle_forward: invalid arguments")
        return z

    def forward_at(self, x, main_orders, conj_orders, L, coeffs, idx, hist=None) -> np.ndarray:
        x = _c128(x)
        co = _c128(coeffs)
        mo, cj = _orders(main_orders), _orders(conj_orders)
        ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        h = None if hist is None else _c128(hist)
        z = np.empty(ix.size, dtype=np.complex128)
        rc = self.lib.oracle_forward_at(_ptr(x), x.size, _ptr(h), _iptr(mo), mo.size, _iptr(cj),
                                        cj.size, int(L), _ptr(co), ix.ctypes.data_as(_i64p),
                                        ix.size, _ptr(z))
        if rc:
            raise ValueError("oracle_forward_at: invalid arguments")
        return z

    def backward(self, x, main_orders, conj_orders, L, coeffs, G, hist=None, want_dx=True,
                 want_dcoef=True):
        x = _c128(x)
        co = _c128(coeffs)
        g = _c128(G)
        mo, cj = _orders(main_orders), _orders(conj_orders)
        h = None if hist is None else _c128(hist)
        gx = np.empty_like(x) if want_dx else None
        gc = np.empty(co.size, dtype=np.complex128) if want_dcoef else None
        rc = self.lib.oracle_backward(_ptr(x), x.size, _ptr(h), _iptr(mo), mo.size, _iptr(cj),
                                      cj.size, int(L), _ptr(co), _ptr(g), _ptr(gx), _ptr(gc))
        if rc:
            raise ValueError("oracle_backward: invalid arguments")
        return gx, gc

    def ls_normal(self, y, main_orders, conj_orders, L, t):
        y = _c128(y)
        t = _c128(t)
        mo, cj = _orders(main_orders), _orders(conj_orders)
        K = (mo.size + cj.size) * L + 1
        A = np.empty((K, K), dtype=np.complex128)
        b = np.empty(K, dtype=np.complex128)
        rc = self.lib.oracle_ls_normal(_ptr(y), y.size, _iptr(mo), mo.size, _iptr(cj), cj.size,
                                       int(L), _ptr(t), _ptr(A), _ptr(b))
        if rc:
            raise ValueError("oracle_ls_normal: invalid arguments")
        return A, b


_default: Oracle | None = None


def _get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def forward(*a, **k):
    return _get().forward(*a, **k)


def forward_at(*a, **k):
    return _get().forward_at(*a, **k)


def backward(*a, **k):
    return _get().backward(*a, **k)


def ls_normal(*a, **k):
    return _get().ls_normal(*a, **k)


def threads() -> int:
    return _get().threads()
