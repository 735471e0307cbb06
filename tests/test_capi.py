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


@pytest.mark.parametrize("fn", ["leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse"])
def test_rejects_bad_sizes_before_device_work(L, fn):
    f = getattr(L, fn)
    p = ctypes.c_void_p(0x1000)
    q = ctypes.c_void_p(0x100000)
    assert f(0, 1, p, q, None) == -1          # N < 1
    assert f(-5, 1, p, q, None) == -1
    assert f(16, -1, p, q, None) == -1        # batch < 0
    assert f(12, 1, p, q, None) == -2         # not a power of two
    assert f((1 << 20) * 2, 1, p, q, None) == -2   # beyond DLT_MAX_N
    assert f(16, 0, p, q, None) == 0          # empty batch is a no-op
    assert f(16, 1, None, q, None) == -1      # NULL input
    assert f(16, 1, p, None, None) == -1      # NULL output
    # overlapping input/output ranges
    assert f(16, 1, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000 + 8 * 15), None) == -1


def test_nodes_rejects(L):
    assert L.leg_nodes_weights(0, 1, None, None, None, None) == -1
    assert L.leg_nodes_weights(24, 1, None, None, None, None) == -2
    assert L.leg_nodes_weights(16, 1, None, None, None, None) == 0   # nothing requested
    a = ctypes.c_void_p(0x1000)
    assert L.leg_nodes_weights(16, 1, a, a, None, None) == -1        # overlapping outputs
