"""The exact low block of the Legendre-to-Chebyshev conversion (Sec. 3,
eq. (9): the dense corrected M on columns n < nd) and of its transpose (the
inverse transform, Sec. 4, eq. (10)) for batches of eight or more
instances, where it runs as one contraction on the matrix cores: every
instance against the oracle, at sizes where the block is the whole
conversion (N <= 8192), where it is the low block of a larger one (16384,
2^17) and where it sits inside the sub-plan of a recursion level (2^18); a
batch whose instance count is not a multiple of the 32-instance tile; and
batched against one call per instance (the one-instance kernel), which
agree to the same bar."""
import numpy as np
import pytest

from gpu_util import exact_angles, need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 5e-14


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def _check_rows(pk, orc, N, B, seed):
    c = wl.coeffs_algebraic(N, seed, batch=B)
    chat = to_host(pk.leg2cheb(to_dev(c)))
    nd = pk.plan_info(N)["nd"]
    worst = 0.0
    for b in sorted({0, B // 2, B - 1}):
        if N <= 16384:
            ref = orc.leg2cheb(c[b], prec="l")
            got = chat[b]
        else:
            idx = np.array(sorted(set(int(i) for i in wl.sample_indices(N, 256, 40 + b)) |
                                  {0, 1, 2, nd - 2, nd - 1, nd, nd + 1, N - 1}), dtype=np.int64)
            ref = orc.leg2cheb_rows(c[b], idx, prec="l")
            got = chat[b][idx]
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.sum(np.abs(c[b]))))
    return c, chat, worst


@pytest.mark.parametrize("N,B", [(64, 8), (256, 40), (1024, 33), (8192, 12), (16384, 9), (1 << 17, 8)])
def test_leg2cheb_batched(pk, orc, N, B):
    say("leg2cheb batched", N, B)
    c, chat, err = _check_rows(pk, orc, N, B, 31)
    say("  err", err)
    assert err <= TOL
    # one call per instance takes the one-instance kernel
    single = to_host(pk.leg2cheb(to_dev(c[B - 1])))
    d = float(np.max(np.abs(single - chat[B - 1])) / np.sum(np.abs(c[B - 1])))
    say("  batched vs single", d)
    assert d <= TOL


def test_leg2cheb_batched_subplan(pk, orc):
    # 2^18: the low block is a sub-plan of size 2^15 whose own low block is dense
    N, B = 1 << 18, 8
    say("leg2cheb batched sub-plan", N, B)
    _, _, err = _check_rows(pk, orc, N, B, 32)
    say("  err", err)
    assert err <= TOL


def _idlt_err(c, ref, w, f, idx):
    return float(np.max(np.abs(c - ref) / ((idx + 0.5) * np.sum(w * np.abs(f)))))


@pytest.mark.parametrize("N,B,top", [(1024, 8, 1024), (8192, 10, 8192), (16384, 8, 16384), (1 << 17, 9, 1 << 14)])
def test_inverse_batched(pk, orc, N, B, top):
    say("idlt batched", N, B)
    f = wl.values_normal(N, 33, batch=B)
    c = to_host(pk.dlt_inverse(to_dev(f)))
    _, w, d = (t.cpu().numpy()[0] for t in pk.leg_nodes_weights(N))
    hi, lo = exact_angles(N, d)
    idx = np.arange(top) if top <= 2048 else np.array(
        sorted(set(int(i) for i in wl.sample_indices(top, 200, 34)) | {0, 1, top - 2, top - 1}), dtype=np.int64)
    worst = 0.0
    for b in sorted({0, B - 1}):
        ref = orc.idlt(f[b], hi, w, idx=idx, prec="d", theta_lo=lo)
        worst = max(worst, _idlt_err(c[b][idx], ref, w, f[b], idx))
    say("  err", worst)
    assert worst <= TOL
    single = to_host(pk.dlt_inverse(to_dev(f[B - 1])))
    dd = _idlt_err(single[idx], c[B - 1][idx], w, f[B - 1], idx)
    say("  batched vs single", dd)
    assert dd <= TOL
