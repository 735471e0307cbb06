"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/dlt.h, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dlt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_1505_00354_amd as pk

    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libdlt.so not built")
    return pk.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert set(names) >= {"leg_nodes_weights", "leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse"}
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for st in (0, -1, -2, -3, -4):
        assert L.dlt_status_string(st)
    assert L.dlt_status_string(7) == b"unknown status"


@pytest.mark.parametrize("fn", ["leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse", "cheb2leg",
                                "leg2chebvals", "chebvals2leg"])
def test_rejects_bad_sizes_before_device_work(L, fn):
    f = getattr(L, fn)
    p = ctypes.c_void_p(0x1000)
    q = ctypes.c_void_p(0x100000)
    assert f(0, 1, p, q, None) == -1          # N < 1
    assert f(-5, 1, p, q, None) == -1
    assert f(16, -1, p, q, None) == -1        # batch < 0
    assert f((1 << 20) * 2, 1, p, q, None) == -2   # beyond DLT_MAX_N
    assert f(16, 0, p, q, None) == 0          # empty batch is a no-op
    assert f(16, 1, None, q, None) == -1      # NULL input
    assert f(16, 1, p, None, None) == -1      # NULL output
    # overlapping input/output ranges
    assert f(16, 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000 + 8 * 15), None) == -1


def test_nodes_rejects(L):
    assert L.leg_nodes_weights(0, 1, None, None, None, None) == -1
    assert L.leg_nodes_weights((1 << 20) + 1, 1, None, None, None, None) == -2
    assert L.leg_nodes_weights(16, 1, None, None, None, None) == 0   # nothing requested
    assert L.leg_nodes_weights(24, 1, None, None, None, None) == 0   # any size; nothing requested


@pytest.mark.parametrize("fn", ["leg2cheb_ex", "cheb_eval_leggrid_ex", "dlt_forward_ex", "dlt_inverse_ex", "cheb2leg_ex"])
def test_ex_rejects_bad_precision(L, fn):
    f = getattr(L, fn)
    p, q = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000)
    for prec in (-1, 3, 99):
        assert f(16, 1, p, q, prec, None) == -1
    assert f(0, 1, p, q, 0, None) == -1
    assert f(16, 0, p, q, 1, None) == 0


def test_batch_rejects_bad_descriptors(L):
    import numpy as np

    i64p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    Ns = np.array([16, 100, 7], dtype=np.int64)
    offs = np.array([0, 16, 116], dtype=np.int64)
    inv = np.array([0, 1, 0], dtype=np.int8)
    x, y = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000000)
    f = L.dlt_batch_ex
    assert f(-1, i64p(Ns), i64p(offs), i64p(inv), x, y, 0, None) == -1
    assert f(0, i64p(Ns), i64p(offs), i64p(inv), x, y, 0, None) == 0      # nothing to do
    assert f(3, i64p(Ns), i64p(offs), i64p(inv), x, y, 7, None) == -1     # precision
    assert f(3, None, i64p(offs), i64p(inv), x, y, 0, None) == -1
    assert f(3, i64p(Ns), i64p(offs), i64p(inv), None, y, 0, None) == -1
    bad = Ns.copy(); bad[1] = 0
    assert f(3, i64p(bad), i64p(offs), i64p(inv), x, y, 0, None) == -1   # size 0
    bad[1] = (1 << 20) + 1
    assert f(3, i64p(bad), i64p(offs), i64p(inv), x, y, 0, None) == -2   # too large
    bo = offs.copy(); bo[2] = -4
    assert f(3, i64p(Ns), i64p(bo), i64p(inv), x, y, 0, None) == -1      # negative offset
    bi = inv.copy(); bi[0] = 2
    assert f(3, i64p(Ns), i64p(offs), i64p(bi), x, y, 0, None) == -1     # direction flag
    # output overlapping the input span
    assert f(3, i64p(Ns), i64p(offs), i64p(inv), x, ctypes.c_void_p(0x1000 + 8 * 50), 0, None) == -1
    a = ctypes.c_void_p(0x1000)
    assert L.leg_nodes_weights(16, 1, a, a, None, None) == -1        # overlapping outputs


@pytest.mark.parametrize("fn", ["leg2cheb_tol", "cheb_eval_leggrid_tol", "dlt_forward_tol", "dlt_inverse_tol", "cheb2leg_tol"])
def test_tol_rejects_before_device_work(L, fn):
    f = getattr(L, fn)
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    p, q = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000)
    for eps in (0.0, -1e-6, 1e-15, 4.9e-14, 0.2, float("nan"), float("inf")):
        assert f(16, 1, p, q, eps, None) == -1, eps
    assert f(24, 1, p, q, 1e-6, None) == -2          # power-of-two sizes only
    assert f(0, 1, p, q, 1e-6, None) == -1
    assert f(16, -1, p, q, 1e-6, None) == -1
    assert f(16, 0, p, q, 1e-6, None) == 0           # empty batch is a no-op
    assert f(16, 1, None, q, 1e-6, None) == -1
    assert f(16, 1, p, ctypes.c_void_p(0x1000 + 8), 1e-6, None) == -1   # overlap
    L.dlt_plan_query_tol.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int]
    assert L.dlt_plan_query_tol(16, 1e-20, None, 4) == -1


def test_cheb_eval_nodes_rejects(L):
    f = L.cheb_eval_nodes
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    a, d, o = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    assert f(24, 1, a, d, o, None) == -2                 # power-of-two sizes only
    assert f(0, 1, a, d, o, None) == -1
    assert f(16, 0, a, d, o, None) == 0                  # empty batch
    assert f(16, 1, None, d, o, None) == -1
    assert f(16, 1, a, None, o, None) == -1
    assert f(16, 1, a, d, None, None) == -1
    assert f(16, 1, a, ctypes.c_void_p(0x200000 + 8), o, None) == -1   # offsets overlap the output
    assert f(16, 1, a, d, ctypes.c_void_p(0x1000 + 8), None) == -1     # output overlaps the input
