"""MI355X (gfx950) fast discrete Legendre transform -- Python binding.

Thin ctypes marshalling over the C ABI in include/dlt.h (libdlt.so, built
in-tree by paper_1505_00354_amd.build).  Every transform runs in the HIP
kernels of that library; this module only passes device pointers, sizes and
the current PyTorch stream.  If the library is missing, every call raises.

Tensors are torch.float64 CUDA (ROCm) tensors, contiguous, with the transform
length N as the last dimension; leading dimensions form the batch.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdlt.so")

DLT_OK = 0
DLT_ERR_INVALID_ARG = -1
DLT_ERR_UNSUPPORTED = -2
DLT_ERR_HIP = -3
DLT_ERR_NOMEM = -4
DLT_ERR_NOT_PREPARED = -5
DLT_MAX_N = 1 << 20
DLT_PREC_FP64 = 0
DLT_PREC_FP32_BULK = 1
DLT_PREC_FP64_RELAXED = 2
PRECISIONS = {"fp64": DLT_PREC_FP64, "fp32bulk": DLT_PREC_FP32_BULK, "fp64relaxed": DLT_PREC_FP64_RELAXED}
DLT_GRID_CHEB1 = 0
DLT_GRID_CHEBSTAR = 1
GRIDS = {"cheb1": DLT_GRID_CHEB1, "chebstar": DLT_GRID_CHEBSTAR}

_lib = None


class DLTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def lib():
    """The loaded libdlt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} not found: build the HIP library first "
                "(python -m paper_1505_00354_amd.build or __graft_entry__.build())"
            )
        L = ctypes.CDLL(LIB_PATH)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        L.leg_nodes_weights.argtypes = [i64, i64, vp, vp, vp, vp]
        L.leg2cheb.argtypes = [i64, i64, vp, vp, vp]
        L.cheb_eval_leggrid.argtypes = [i64, i64, vp, vp, vp]
        L.dlt_forward.argtypes = [i64, i64, vp, vp, vp]
        L.dlt_inverse.argtypes = [i64, i64, vp, vp, vp]
        L.cheb2leg.argtypes = [i64, i64, vp, vp, vp]
        L.cheb_eval_nodes.argtypes = [i64, i64, vp, vp, vp, vp]
        L.cheb_eval_nodes.restype = ctypes.c_int
        for name in ("leg2chebvals", "chebvals2leg"):
            getattr(L, name).argtypes = [i64, i64, vp, vp, vp]
            getattr(L, name).restype = ctypes.c_int
        for name in ("leg2cheb_ex", "cheb_eval_leggrid_ex", "dlt_forward_ex", "dlt_inverse_ex", "cheb2leg_ex"):
            getattr(L, name).argtypes = [i64, i64, vp, vp, ctypes.c_int, vp]
            getattr(L, name).restype = ctypes.c_int
        for name in ("leg2cheb_tol", "cheb_eval_leggrid_tol", "dlt_forward_tol", "dlt_inverse_tol", "cheb2leg_tol"):
            getattr(L, name).argtypes = [i64, i64, vp, vp, ctypes.c_double, vp]
            getattr(L, name).restype = ctypes.c_int
        L.dlt_plan_query_ex.argtypes = [i64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.dlt_plan_query_ex.restype = ctypes.c_int
        L.dlt_plan_query_tol.argtypes = [i64, ctypes.c_double, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.dlt_plan_query_tol.restype = ctypes.c_int
        L.dlt_forward_noalloc.argtypes = [i64, i64, vp, vp, vp]
        L.dlt_forward_noalloc.restype = ctypes.c_int
        L.dlt_batch_ex.argtypes = [i64, vp, vp, vp, vp, vp, ctypes.c_int, vp]
        L.dlt_batch_ex.restype = ctypes.c_int
        L.dlt_batch_grid.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.dlt_batch_grid.restype = ctypes.c_int
        for name in ("cheb_eval_leggrid_grid", "dlt_forward_grid", "dlt_inverse_grid"):
            getattr(L, name).argtypes = [i64, i64, vp, vp, ctypes.c_int, vp]
            getattr(L, name).restype = ctypes.c_int
        L.dlt_status_string.argtypes = [ctypes.c_int]
        L.dlt_status_string.restype = ctypes.c_char_p
        L.dlt_release.argtypes = []
        L.dlt_plan_query.argtypes = [i64, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.dlt_trace_enable.argtypes = [ctypes.c_int]
        L.dlt_trace_collect.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        for name in ("leg_nodes_weights", "leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse", "cheb2leg",
                     "dlt_release", "dlt_plan_query", "dlt_trace_enable", "dlt_trace_collect"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st, what):
    if st != DLT_OK:
        raise DLTError(st, f"{what}: {lib().dlt_status_string(st).decode()} (status {st})")


def _stream(dev=None):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _vec_args(x, out):
    import torch

    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
        raise TypeError("expected a float64 CUDA tensor")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    N = x.shape[-1]
    batch = x.numel() // N if N else 0
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match the input's shape, dtype and device and be contiguous")
    return N, batch, out


def leg_nodes_weights(N, device=None, batch=1, theta=True, w=True, dtheta=True):
    """(theta, w, dtheta) tensors of shape (batch, N) (None where not asked)."""
    import torch

    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    mk = lambda want: torch.empty((batch, N), dtype=torch.float64, device=dev) if want else None
    t, ww, d = mk(theta), mk(w), mk(dtheta)
    ptr = lambda a: ctypes.c_void_p(a.data_ptr()) if a is not None else None
    with torch.cuda.device(dev):
        _check(lib().leg_nodes_weights(N, batch, ptr(t), ptr(ww), ptr(d), _stream(dev)), "leg_nodes_weights")
    return t, ww, d


def _prec(prec):
    if prec not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    return PRECISIONS[prec]


def _unary(name, x, out, prec="fp64", tol=None, grid="cheb1"):
    import torch

    N, batch, out = _vec_args(x, out)
    args = (N, batch, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    if grid not in GRIDS:
        raise ValueError(f"grid must be one of {sorted(GRIDS)}")
    with torch.cuda.device(x.device):
        if grid != "cheb1":
            if prec != "fp64" or tol is not None:
                raise ValueError("the cheb* grid runs in FP64 at the fixed budget (prec 'fp64', no tol)")
            _check(getattr(lib(), name + "_grid")(*args, GRIDS[grid], _stream(x.device)), name + "_grid")
        elif tol is not None:
            if prec != "fp64":
                raise ValueError("a working tolerance runs in FP64 (prec must be 'fp64')")
            _check(getattr(lib(), name + "_tol")(*args, float(tol), _stream(x.device)), name + "_tol")
        elif prec == "fp64":
            _check(getattr(lib(), name)(*args, _stream(x.device)), name)
        else:
            _check(getattr(lib(), name + "_ex")(*args, _prec(prec), _stream(x.device)), name + "_ex")
    return out


def leg2cheb(c, out=None, prec="fp64", tol=None):
    """Chebyshev coefficients of sum_n c_n P_n (chat = M c)."""
    return _unary("leg2cheb", c, out, prec, tol)


def cheb_eval_leggrid(chat, out=None, prec="fp64", tol=None, grid="cheb1"):
    """sum_n chat_n T_n at the N Legendre nodes.  grid: the Taylor expansion
    point, "cheb1" ((k+1/2) pi/N) or "chebstar" ((k+3/4) pi/(N+1/2))."""
    return _unary("cheb_eval_leggrid", chat, out, prec, tol, grid)


def dlt_forward(c, out=None, prec="fp64", tol=None, grid="cheb1"):
    """Discrete Legendre transform f_k = sum_n c_n P_n(x_k).  prec: "fp64",
    "fp32bulk" (FP32 bulk transforms, 5e-6 budget) or "fp64relaxed" (FP64
    with the 5e-6 parameters).  tol: a working tolerance instead (FP64,
    parameters chosen for eps = tol, 5e-14 <= tol <= 0.1; the other entry
    points take it too).  grid: the Taylor expansion point of the evaluation,
    "cheb1" or "chebstar" (FP64, N a power of two)."""
    return _unary("dlt_forward", c, out, prec, tol, grid)


def dlt_forward_noalloc(c, out=None):
    """dlt_forward (FP64) on the library's static scratch: allocates nothing
    (N a power of two <= 65536; the plan of size N must have been built by an
    earlier call of that size)."""
    import torch

    N, batch, out = _vec_args(c, out)
    with torch.cuda.device(c.device):
        _check(lib().dlt_forward_noalloc(N, batch, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         _stream(c.device)), "dlt_forward_noalloc")
    return out


def dlt_inverse(f, out=None, prec="fp64", tol=None, grid="cheb1"):
    """Inverse transform c_n = (n+1/2) sum_k w_k f_k P_n(x_k).  grid: the
    Taylor expansion point of its transposed evaluation, "cheb1" or
    "chebstar" (FP64, N a power of two)."""
    return _unary("dlt_inverse", f, out, prec, tol, grid)


def cheb_eval_nodes(chat, dtheta, out=None):
    """sum_n chat_n cos(n theta_k) at theta_k = (k+1/2) pi/N + dtheta_k
    (|N dtheta_k| <= pi/2); dtheta: float64 CUDA tensor of N offsets."""
    import torch

    N, batch, out = _vec_args(chat, out)
    d = dtheta.contiguous()
    if d.dtype != torch.float64 or d.device != chat.device or d.numel() != N:
        raise ValueError("dtheta must be N float64 values on the device of chat")
    with torch.cuda.device(chat.device):
        _check(lib().cheb_eval_nodes(N, batch, ctypes.c_void_p(chat.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream(chat.device)), "cheb_eval_nodes")
    return out


def leg2chebvals(c, out=None):
    """Values of sum_n c_n P_n at the Chebyshev points cos((j+1/2) pi/N)."""
    return _unary("leg2chebvals", c, out)


def chebvals2leg(v, out=None):
    """Legendre coefficients of the degree < N interpolant of values v at the
    Chebyshev points cos((j+1/2) pi/N)."""
    return _unary("chebvals2leg", v, out)


def cheb2leg(chat, out=None, prec="fp64", tol=None):
    """Legendre coefficients c = M^{-1} chat of a Chebyshev expansion (the
    inverse of leg2cheb)."""
    return _unary("cheb2leg", chat, out, prec, tol)


def dlt_batch(x, sizes, offsets=None, inverse=None, out=None, prec="fp64"):
    """Ragged batch of transforms of uneven sizes in one call (dlt_batch_ex).

    x: 1-D float64 CUDA tensor holding every instance; instance i is
    x[offsets[i] : offsets[i] + sizes[i]] (offsets default to the packed
    layout).  inverse[i] true: IDLT of that instance, else DLT.  Returns (or
    fills) a tensor like x with each instance's result at the same place.
    The first call with a given layout and buffers tunes, captures and
    synchronises; repeated calls replay a cached HIP graph."""
    import numpy as np
    import torch

    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.dim() == 1):
        raise TypeError("expected a 1-D float64 CUDA tensor")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    Ns = np.ascontiguousarray(sizes, dtype=np.int64)
    if offsets is None:
        offs = np.zeros(len(Ns), dtype=np.int64)
        if len(Ns) > 1:
            offs[1:] = np.cumsum(Ns)[:-1]
    else:
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
    if len(offs) != len(Ns):
        raise ValueError("sizes and offsets differ in length")
    if len(Ns) and int((offs + Ns).max()) > x.numel():
        raise ValueError("an instance reaches beyond the input")
    inv = np.zeros(len(Ns), dtype=np.int8) if inverse is None else np.ascontiguousarray(inverse, dtype=np.int8)
    if len(inv) != len(Ns):
        raise ValueError("inverse flags and sizes differ in length")
    if out is None:
        out = torch.zeros_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match the input's shape, dtype and device and be contiguous")
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    with torch.cuda.device(x.device):
        _check(lib().dlt_batch_ex(len(Ns), ptr(Ns), ptr(offs), ptr(inv), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), _prec(prec), _stream(x.device)), "dlt_batch_ex")
    return out


def release():
    _check(lib().dlt_release(), "dlt_release")


PLAN_FIELDS = ("L", "nd", "far_terms", "far_blocks", "far_mmax", "near_items", "near_rows", "N1", "N2",
               "colsA", "rowsB", "tgB", "tnear_wg", "tnear_rg", "near_steps", "boundary_nodes", "ws_bytes",
               "near_work", "tgA", "ws_cap", "chebstar_L")


def plan_info(N, prec="fp64", tol=None):
    """The library's plan parameters for size N (and precision, or working
    tolerance), as a dict."""
    buf = (ctypes.c_int64 * 32)()
    if tol is not None:
        n = lib().dlt_plan_query_tol(N, float(tol), buf, 32)
    else:
        n = lib().dlt_plan_query_ex(N, _prec(prec), buf, 32)
    if n < 0:
        _check(n, "dlt_plan_query")
    return {k: int(buf[i]) for i, k in enumerate(PLAN_FIELDS[:n])}


def batch_grid(N, inverse=False, prec="fp64"):
    """Grid size dlt_batch runs instances of size N on (direction, precision)
    on the current device: the padded power of two or twice it, as timed at
    the first batch holding such instances; 0 before any such batch
    (dlt_batch_grid)."""
    g = ctypes.c_int64(0)
    _check(lib().dlt_batch_grid(int(N), 1 if inverse else 0, _prec(prec), ctypes.byref(g)), "dlt_batch_grid")
    return int(g.value)


def trace_enable(on=True):
    _check(lib().dlt_trace_enable(1 if on else 0), "dlt_trace_enable")


def trace_collect(max_kernels=4096):
    """{kernel name: (total ms, launches)} since the last collect; waits for
    the recorded events."""
    names = ctypes.create_string_buffer(max_kernels * 48)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int64 * max_kernels)()
    n = lib().dlt_trace_collect(max_kernels, names, 48, ms, cnt)
    if n < 0:
        _check(n, "dlt_trace_collect")
    out = {}
    for i in range(n):
        nm = names.raw[i * 48:(i + 1) * 48].split(b"\0", 1)[0].decode()
        out[nm] = (ms[i], int(cnt[i]))
    return out
