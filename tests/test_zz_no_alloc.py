"""dlt_forward_noalloc (the allocation-free form of dlt_forward, for callers
that cannot allocate device memory) against dlt_forward: the same kernels,
so the same bits; two calls in a row, the second with a smaller input (the
static scratch keeps the first call's contents); batches larger than the
scratch holds run in slices; sizes above the limit and sizes whose plan
has not been built are refused."""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def _noalloc(pk, x, y):
    import torch

    N = x.shape[-1]
    batch = x.numel() // N
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return pk.lib().dlt_forward_noalloc(N, batch, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), st)


SCRATCH = 32 << 20  # bytes of the library's static scratch


def _per_slice(pk, N):
    out = (ctypes.c_int64 * 17)()
    assert pk.lib().dlt_plan_query(N, out, 17) >= 17
    shared = 3 * ((8 * N + 255) // 256 * 256)  # theta, w, dtheta
    return (SCRATCH - shared) // out[16] if out[16] else 1 << 62


@pytest.mark.parametrize("cases", [
    [(1 << 16, 2), (1 << 12, 3)],   # 2^16: one instance per slice
    [(4096, 200), (1024, 1)],       # more instances than one slice holds
    [(64, 5), (1, 2)],
])
def test_noalloc_matches_dlt_forward(pk, cases):
    import torch

    for i, (N, batch) in enumerate(cases):
        say("noalloc", N, batch, "call", i)
        c = to_dev(wl.coeffs_algebraic(N, 90 + i, batch=batch))
        ref = to_host(pk.dlt_forward(c))  # also builds the size's plan
        y = torch.full_like(c, float("nan"))
        assert _noalloc(pk, c, y) == 0
        got = to_host(y)
        err = float(np.max(np.abs(got - ref)) / np.max(np.sum(np.abs(to_host(c)), axis=-1)))
        say("  instances per slice", _per_slice(pk, N), "max |diff| / ||c||_1", err)
        if batch <= _per_slice(pk, N):
            # one slice: exactly the launches of dlt_forward
            assert np.array_equal(got, ref)
        else:
            # slices of fewer instances may group the Taylor pairs of the
            # first pass differently (a rounding of the powers), so the
            # forward transform's bar applies
            assert err <= 5e-14


def test_noalloc_refusals(pk):
    import torch

    x = to_dev(np.zeros(1 << 17))
    y = torch.empty_like(x)
    assert _noalloc(pk, x, y) == pk.DLT_ERR_UNSUPPORTED  # above 65536
    x3 = to_dev(np.zeros(3000))
    assert _noalloc(pk, x3, torch.empty_like(x3)) == pk.DLT_ERR_UNSUPPORTED  # not a power of two
    # a size whose plan does not exist yet
    assert pk.lib().dlt_release() == 0
    x2 = to_dev(wl.coeffs_algebraic(2048, 7))
    y2 = torch.empty_like(x2)
    assert _noalloc(pk, x2, y2) == pk.DLT_ERR_NOT_PREPARED
    out = (ctypes.c_int64 * 4)()
    assert pk.lib().dlt_plan_query(2048, out, 4) > 0  # builds it
    assert _noalloc(pk, x2, y2) == 0
    assert np.array_equal(to_host(y2), to_host(pk.dlt_forward(x2)))
