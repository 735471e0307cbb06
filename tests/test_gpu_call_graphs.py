"""Repeated single calls are replayed from a captured HIP graph (the second
call with the same operation, size, batch, precision, buffers and stream
captures it).  Every replay must give the same bits as the direct call on the
same input, also when the input changes in place between replays, with other
direct work and synchronisations in between, and with the trace on (direct
again)."""
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


OPS = ["dlt_forward", "dlt_inverse", "leg2cheb", "cheb_eval_leggrid"]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("N,batch,prec", [(1 << 16, 1, "fp64"), (1 << 13, 3, "fp64"), (1 << 17, 1, "fp32bulk")])
def test_replays_match_direct_calls(pk, op, N, batch, prec):
    import torch

    say("call graph", op, N, batch, prec)
    fn = getattr(pk, op)
    x = to_dev(wl.coeffs_algebraic(N, 21, batch=batch))
    y = torch.empty_like(x)
    other_in = to_dev(wl.values_normal(N, 22, batch=batch))
    other_out = torch.empty_like(other_in)
    ref = to_host(fn(x.clone(), prec=prec))  # direct: fresh buffers
    for rep in range(5):
        # the same buffers every time: direct, captured, then replays
        fn(x, out=y, prec=prec)
        got = to_host(y)
        assert np.array_equal(got, ref), (op, rep)
        # other direct work and host synchronisation between replays
        pk.dlt_inverse(other_in, out=other_out)
        other_out.mul_(0.5)
        torch.cuda.synchronize()
    # new input in place: the replay reads the buffer's current contents
    x2 = wl.values_normal(N, 23, batch=batch)
    x.copy_(to_dev(x2))
    fn(x, out=y, prec=prec)
    got = to_host(y)
    ref2 = to_host(fn(to_dev(x2), prec=prec))
    assert np.array_equal(got, ref2)
    # traced calls run directly and agree too
    pk.trace_enable(True)
    try:
        fn(x, out=y, prec=prec)
        got = to_host(y)
    finally:
        pk.trace_enable(False)
        pk.trace_collect()
    assert np.array_equal(got, ref2)


@pytest.mark.parametrize("op", OPS + ["cheb2leg", "leg2chebvals", "chebvals2leg"])
@pytest.mark.parametrize("Na,Nb", [(1 << 16, 1 << 16), (1 << 16, 1 << 13)])
def test_two_streams_at_once(pk, op, Na, Nb):
    """Calls on two streams (each with its own workspace, side streams and
    graphs) run at the same time, direct, captured and replayed, and give the
    bits of the same calls made alone."""
    import torch

    say("two streams", op, Na, Nb)
    fn = getattr(pk, op)
    xa = to_dev(wl.coeffs_algebraic(Na, 31))
    xb = to_dev(wl.coeffs_algebraic(Nb, 32))
    ref_a = to_host(fn(xa.clone()))
    ref_b = to_host(fn(xb.clone()))
    ya, yb = torch.empty_like(xa), torch.empty_like(xb)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(4):
        ya.fill_(np.nan)
        yb.fill_(np.nan)
        torch.cuda.synchronize()
        for _ in range(2):
            with torch.cuda.stream(s1):
                fn(xa, out=ya)
            with torch.cuda.stream(s2):
                fn(xb, out=yb)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(ya), ref_a), (op, rep, "stream 1")
        assert np.array_equal(to_host(yb), ref_b), (op, rep, "stream 2")


def test_more_distinct_calls_than_kept_graphs(pk):
    """300 distinct repeated calls (one output buffer each), three rounds:
    more than the library keeps graphs for, so graphs are dropped (after the
    device drains) while others are queued; every call still gives the
    bits of the direct call."""
    import torch

    N = 256
    say("many call graphs", N)
    x = to_dev(wl.coeffs_algebraic(N, 41))
    ref = to_host(pk.dlt_forward(x.clone()))
    outs = [torch.empty_like(x) for _ in range(300)]
    for rep in range(3):
        for y in outs:
            y.fill_(np.nan)
        for y in outs:
            pk.dlt_forward(x, out=y)
        torch.cuda.synchronize()
        for i, y in enumerate(outs):
            assert np.array_equal(to_host(y), ref), (rep, i)
