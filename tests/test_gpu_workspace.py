"""The _ws entry points run the transforms on a caller-owned workspace: the
same kernels as on the library's own workspace, so the same bits when the
batch fits; in slices (one instance at a time) when the buffer holds one
instance; nothing written beyond the bytes the caller declared; a buffer
smaller than one instance needs is rejected."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the caller-workspace entry points were withdrawn: the full GPU suite ended in a "
                     "host-side segmentation fault inside the first dlt_forward_ws call of "
                     "test_caller_workspace_slices_and_bounds (it had passed alone); no cause was found"),
]
OPS = ["leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse"]


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def _input(op, N, batch, seed):
    return wl.values_normal(N, seed, batch=batch) if op == "dlt_inverse" else wl.coeffs_algebraic(N, seed, batch=batch)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("N,batch,prec", [(1 << 12, 3, "fp64"), (1 << 16, 2, "fp32bulk"), (1 << 20, 1, "fp64")])
def test_caller_workspace_same_bits(pk, op, N, batch, prec):
    import torch

    say("caller workspace", op, N, batch, prec)
    fn = getattr(pk, op)
    x = to_dev(_input(op, N, batch, 71))
    ref = to_host(fn(x, prec=prec))
    nbytes = pk.workspace_bytes(N, batch, prec)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    for rep in range(3):  # direct, captured, replayed
        y.fill_(np.nan)
        fn(x, out=y, prec=prec, ws=ws)
        assert np.array_equal(to_host(y), ref), rep


@pytest.mark.parametrize("op", OPS)
def test_caller_workspace_slices_and_bounds(pk, op):
    import torch

    N, batch = 1 << 14, 3
    say("caller workspace slices", op, N, batch)
    fn = getattr(pk, op)
    xh = _input(op, N, batch, 72)
    x = to_dev(xh)
    ref = to_host(fn(x))
    one = pk.workspace_bytes(N, 1)
    full = pk.workspace_bytes(N, batch)
    assert full > one
    ws = torch.empty(full, dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    scale = np.sum(np.abs(xh), axis=1, keepdims=True)
    for rep in range(2):  # the whole batch at once (direct, then captured)
        fn(x, out=y, ws=ws)
        assert np.array_equal(to_host(y), ref)
    # the same buffer declared one instance long: slices of one instance, and
    # nothing beyond the declared bytes is touched (the graph of the whole
    # batch must not be replayed)
    ws[one:].fill_(0x5A)
    for rep in range(3):
        y.fill_(np.nan)
        fn(x, out=y, ws=ws[:one])
        got = to_host(y)
        assert np.all(np.abs(got - ref) <= 1e-14 * scale), rep
        assert bool((ws[one:] == 0x5A).all()), rep
    with pytest.raises(pk.DLTError):
        fn(x, out=y, ws=ws[: one - 256])
