"""The library's Taylor lengths against Table 1, on the CPU: the library is
linked against the host-only HIP stand-in of tests/lanecheck (plan queries
build the host part of a plan and never run a kernel).

About theta^cheb1 the FP64 plan takes the smallest even L whose factor
0.83845^L/L! (Corollary 2, first bound) is within a tenth of the 5e-14
budget, and about theta^cheb* the smallest L whose factor 1/((6 pi)^L L!)
(second bound) is: both read off the printed table."""
import ctypes
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LC = os.path.join(HERE, "lanecheck")
sys.path.insert(0, LC)
GOLD = os.path.join(HERE, "golden", "table1.txt")

QUERY = r"""
import ctypes, json, sys
sys.path.insert(0, {lc!r})
import build as lbuild
stub = ctypes.CDLL(lbuild.STUB, mode=ctypes.RTLD_GLOBAL)
L = ctypes.CDLL(lbuild.LIB)
L.dlt_plan_query_ex.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
out = {{}}
for N in (16, 1024, 1 << 16, 1 << 20):
    buf = (ctypes.c_int64 * 32)()
    n = L.dlt_plan_query_ex(N, 0, buf, 32)
    out[N] = list(buf[:n])
print(json.dumps(out))
"""


@pytest.fixture(scope="module")
def fields():
    import build as lbuild

    try:
        lbuild.build()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    # a fresh process: the library's HIP references bind to the stand-in
    r = subprocess.run([sys.executable, "-c", QUERY.format(lc=LC)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return {int(k): v for k, v in json.loads(r.stdout.strip().splitlines()[-1]).items()}


def _table():
    rows = []
    with open(GOLD) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                L, a, b = line.split()
                rows.append((int(L), float(a), float(b)))
    return rows


def test_taylor_lengths_from_table1(fields):
    budget = 5e-14 / 10
    cheb1 = next(L for L, a, _ in _table() if a <= budget)
    cheb1 += cheb1 & 1  # the cheb1 terms run in pairs
    star = next(L for L, _, b in _table() if b <= budget)
    assert (cheb1, star) == (16, 8)
    for N, v in fields.items():
        assert len(v) >= 21, N
        assert v[0] == cheb1, (N, v[0])
        assert v[20] == star, (N, v[20])
