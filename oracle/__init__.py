"""CPU oracle for the discrete Legendre transform -- TEST INFRASTRUCTURE.

Plain, slow, direct O(N^2) implementations of what the fast GPU path
computes, written from the definitions in Hale & Townsend, "A fast FFT-based
discrete Legendre transform":

  nodes(N)            Legendre nodes theta_k (increasing, x_k = cos theta_k
                      decreasing as in eq. (1)) and Gauss-Legendre weights,
                      Newton's method in theta (Sec. 2.1-2.2).
  dlt(c, theta)       eq. (1)   f = sum_n c_n P_n(cos theta)
                      (dlt/ndct/idlt accept theta_lo: the angle is then the
                      two-double sum theta + theta_lo, honoured by prec="l")
  idlt(f, theta, w)   eq. (2)   c_n = (n+1/2) sum_k w_k f_k P_n(cos theta_k)
  ndct(chat, theta)   eq. (3)   f = sum_n chat_n cos(n theta)
  leg2cheb(c)         Sec. 3    chat = M c (dense, corrected M; see the C
                                header for the reading of the garbled entries)
  leg2cheb_t(y)       Sec. 4    M^T y (dense)
  legendre(N, theta)  P_0..P_{N-1} at cos(theta)

Every function takes prec="d" (FP64, oracle of record) or prec="l"
(x87 long double cross-check).  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may use this package; the product path must
never import it.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        for p in ("d", "l"):
            getattr(lib, f"orc_nodes_{p}").argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _f64p, _f64p]
            getattr(lib, f"orc_dlt_{p}").argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _f64p, _f64p, _f64p]
            getattr(lib, f"orc_ndct_{p}").argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _f64p, _f64p, _f64p]
            getattr(lib, f"orc_idlt_{p}").argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p, _f64p, ctypes.c_int64,
                                                      _i64p, _f64p]
            getattr(lib, f"orc_leg2cheb_{p}").argtypes = [ctypes.c_int64, _f64p, _f64p]
            getattr(lib, f"orc_leg2cheb_t_{p}").argtypes = [ctypes.c_int64, _f64p, _f64p]
            getattr(lib, f"orc_leg2cheb_rows_{p}").argtypes = [ctypes.c_int64, _f64p, ctypes.c_int64, _i64p, _f64p]
            getattr(lib, f"orc_cheb2leg_{p}").argtypes = [ctypes.c_int64, _f64p, _f64p]
            getattr(lib, f"orc_legendre_{p}").argtypes = [ctypes.c_int64, ctypes.c_double, _f64p]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle call failed with status {rc}")


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the number of OpenMP threads the oracle uses."""
    return _load().orc_set_threads(int(n))


def nodes(N, idx=None, prec="d"):
    lib = _load()
    if idx is None:
        cnt, ip = N, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        cnt, ip = len(idx), idx.ctypes.data_as(_i64p)
    th = np.empty(cnt)
    w = np.empty(cnt)
    _check(getattr(lib, f"orc_nodes_{prec}")(N, cnt, ip, th.ctypes.data_as(_f64p), w.ctypes.data_as(_f64p)))
    return th, w


def _lo(theta_lo, n):
    if theta_lo is None:
        return None, None
    a, p = _d(theta_lo)
    if len(a) != n:
        raise ValueError("theta_lo must match theta")
    return a, p


def dlt(c, theta, prec="d", theta_lo=None):
    c, cp = _d(c)
    theta, tp = _d(theta)
    lo, lp = _lo(theta_lo, len(theta))
    f = np.empty(len(theta))
    _check(getattr(_load(), f"orc_dlt_{prec}")(len(c), cp, len(theta), tp, lp, f.ctypes.data_as(_f64p)))
    return f


def ndct(chat, theta, prec="d", theta_lo=None):
    chat, cp = _d(chat)
    theta, tp = _d(theta)
    lo, lp = _lo(theta_lo, len(theta))
    f = np.empty(len(theta))
    _check(getattr(_load(), f"orc_ndct_{prec}")(len(chat), cp, len(theta), tp, lp, f.ctypes.data_as(_f64p)))
    return f


def idlt(f, theta, w, idx=None, prec="d", theta_lo=None):
    f, fp = _d(f)
    theta, tp = _d(theta)
    lo, lp = _lo(theta_lo, len(theta))
    w, wp = _d(w)
    N = len(f)
    if idx is None:
        cnt, ip = N, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        cnt, ip = len(idx), idx.ctypes.data_as(_i64p)
    c = np.empty(cnt)
    _check(getattr(_load(), f"orc_idlt_{prec}")(N, fp, tp, lp, wp, cnt, ip, c.ctypes.data_as(_f64p)))
    return c


def leg2cheb(c, prec="d"):
    c, cp = _d(c)
    out = np.empty(len(c))
    _check(getattr(_load(), f"orc_leg2cheb_{prec}")(len(c), cp, out.ctypes.data_as(_f64p)))
    return out


def leg2cheb_rows(c, idx, prec="d"):
    """(M c)_k for the rows k in idx (Sec. 3, eq. (9)), O(N) per row."""
    c, cp = _d(c)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    _check(getattr(_load(), f"orc_leg2cheb_rows_{prec}")(len(c), cp, len(idx), idx.ctypes.data_as(_i64p),
                                                        out.ctypes.data_as(_f64p)))
    return out


def cheb2leg(chat, prec="d"):
    """Legendre coefficients c = M^{-1} chat (back substitution, Sec. 3)."""
    chat, hp = _d(chat)
    out = np.empty(len(chat))
    _check(getattr(_load(), f"orc_cheb2leg_{prec}")(len(chat), hp, out.ctypes.data_as(_f64p)))
    return out


def leg2cheb_t(y, prec="d"):
    y, yp = _d(y)
    out = np.empty(len(y))
    _check(getattr(_load(), f"orc_leg2cheb_t_{prec}")(len(y), yp, out.ctypes.data_as(_f64p)))
    return out


def legendre(N, theta, prec="d"):
    out = np.empty(N)
    _check(getattr(_load(), f"orc_legendre_{prec}")(N, float(theta), out.ctypes.data_as(_f64p)))
    return out
