"""The Chebyshev evaluation at the Legendre grid (eq. (3)) and the DLT
(eq. (1)) with the Taylor series of Sec. 2.3 taken about the grid
theta^cheb*_k = (k+3/4) pi/(N+1/2) (Sec. 2.2, Lemma 2; Remark 1), against the
oracle at the points the GPU path evaluates at: the full vector up to 16384,
sampled outputs (both ends included) at 2^16 and 2^20; the DLT up to 2^18;
the IDLT (its transposed evaluation about theta^cheb*, eq. (10)) on every
degree up to 2^16 and on sampled degrees up to 2^18 at N = 2^20, and the
round trip; batches, including one that runs in workspace slices; the same
results as about theta^cheb1 to the same bar; the argument checks; the
kernel names in the trace.  Bars: the FP64 targets 5e-14 * ||c||_1 (DLT,
evaluation) and 5e-14 (n+1/2) sum_k w_k |f_k| (IDLT)."""
import ctypes

import numpy as np
import pytest

from gpu_util import dlt_err, exact_angles, need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 5e-14


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def offsets(pk, N):
    return to_host(pk.leg_nodes_weights(N, theta=False, w=False)[2])[0]


def idx_of(N, n, seed):
    if N <= 16384:
        return np.arange(N)
    return np.array(sorted(set(int(i) for i in wl.sample_indices(N, n, seed)) |
                           {0, 1, 2, N // 2 - 1, N // 2, N - 3, N - 2, N - 1}), dtype=np.int64)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64, 256, 1024, 2048, 4096, 16384, 1 << 16, 1 << 20])
def test_chebstar_eval(pk, orc, N):
    say("chebstar ndct", N)
    chat = wl.coeffs_algebraic(N, 4)[0]
    f = to_host(pk.cheb_eval_leggrid(to_dev(chat), grid="chebstar"))
    idx = idx_of(N, 512, 6)
    hi, lo = exact_angles(N, offsets(pk, N), idx)
    ref = orc.ndct(chat, hi, prec="l", theta_lo=lo)
    err = dlt_err(f[idx], ref, chat)
    say("  err", err)
    assert err <= TOL
    # about theta^cheb1: the same values to the same bar
    f1 = to_host(pk.cheb_eval_leggrid(to_dev(chat)))
    d = dlt_err(f, f1, chat)
    say("  vs cheb1", d)
    assert d <= TOL


@pytest.mark.parametrize("N", [1, 16, 1024, 16384, 1 << 18])
def test_chebstar_forward(pk, orc, N):
    say("chebstar dlt", N)
    for fam, c in (("A", wl.coeffs_algebraic(N, 2)[0]), ("B", wl.coeffs_analytic(N, 3)[0])):
        f = to_host(pk.dlt_forward(to_dev(c), grid="chebstar"))
        idx = idx_of(N, 256, 7)
        hi, lo = exact_angles(N, offsets(pk, N), idx)
        ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
        err = dlt_err(f[idx], ref, c)
        say("  family", fam, "err", err)
        assert err <= TOL


def _idlt_err(c, ref, w, f, idx):
    return float(np.max(np.abs(c - ref) / ((idx + 0.5) * np.sum(w * np.abs(f)))))


@pytest.mark.parametrize("N,top", [(1, 1), (2, 2), (16, 16), (1024, 1024), (16384, 16384), (1 << 16, 4096),
                                   (1 << 20, 16384)])
def test_chebstar_inverse(pk, orc, N, top):
    # the inverse transform with its transposed evaluation about theta^cheb*
    # (eq. (10)), against the oracle's IDLT at the GPU's nodes and weights on
    # every degree up to 16384 and on sampled degrees below `top` beyond
    # (the oracle's cost grows with the top degree; the evaluation feeds
    # every degree alike); on every degree against the inverse about
    # theta^cheb1
    say("chebstar idlt", N)
    f = wl.values_normal(N, 33)[0]
    c = to_host(pk.dlt_inverse(to_dev(f), grid="chebstar"))
    _, w, d = (to_host(t)[0] for t in pk.leg_nodes_weights(N))
    hi, lo = exact_angles(N, d)
    if N <= 16384:
        idx = np.arange(top)
    else:
        idx = np.array(sorted(set(int(i) for i in wl.sample_indices(top, 96, 34)) | {0, 1, top - 2, top - 1}),
                       dtype=np.int64)
    ref = orc.idlt(f, hi, w, idx=idx, prec="d", theta_lo=lo)
    err = _idlt_err(c[idx], ref, w, f, idx)
    say("  err", err)
    assert err <= TOL
    c1 = to_host(pk.dlt_inverse(to_dev(f)))
    n = np.arange(N)
    dd = _idlt_err(c, c1, w, f, n)
    say("  vs cheb1, every degree", dd)
    assert dd <= TOL


def test_chebstar_roundtrip(pk):
    # dlt_inverse(dlt_forward(c)) about theta^cheb* returns c (2^16, family A)
    N = 1 << 16
    c = wl.coeffs_algebraic(N, 35)[0]
    f = pk.dlt_forward(to_dev(c), grid="chebstar")
    c2 = to_host(pk.dlt_inverse(f, grid="chebstar"))
    fh = to_host(f)
    w = to_host(pk.leg_nodes_weights(N)[1])[0]
    n = np.arange(N)
    err = float(np.max(np.abs(c2 - c) / ((n + 0.5) * np.sum(w * np.abs(fh)))))
    say("chebstar roundtrip", N, err)
    assert err <= TOL


def test_chebstar_batches(pk, orc):
    # batch 3 at 4096 (full vectors), and 14 instances at 2^20, which the
    # workspace bound splits into slices (the forward's own work plus 8 x 2N
    # complex values per instance): first, middle and last instance sampled
    N, B = 4096, 3
    c = wl.coeffs_algebraic(N, 11, batch=B)
    f = to_host(pk.dlt_forward(to_dev(c), grid="chebstar"))
    hi, lo = exact_angles(N, offsets(pk, N))
    for b in range(B):
        err = dlt_err(f[b], orc.dlt(c[b], hi, prec="l", theta_lo=lo), c[b])
        say("batch", N, b, err)
        assert err <= TOL
    N, B = 1 << 20, 14
    per = 2 * N * 16 * 8 + pk.plan_info(N)["ws_bytes"]
    assert B * per > pk.plan_info(N)["ws_cap"]  # more than one slice
    c = wl.coeffs_algebraic(N, 12, batch=B)
    f = to_host(pk.dlt_forward(to_dev(c), grid="chebstar"))
    idx = idx_of(N, 128, 13)
    hi, lo = exact_angles(N, offsets(pk, N), idx)
    for b in (0, B // 2, B - 1):
        err = dlt_err(f[b][idx], orc.dlt(c[b], hi, prec="l", theta_lo=lo), c[b])
        say("batch", N, b, err)
        assert err <= TOL


def test_chebstar_arguments(pk):
    import torch

    L = pk.lib()
    x = torch.zeros(3000, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    s = pk._stream()
    # not a power of two; unknown grid; overlapping buffers; empty batch
    assert L.cheb_eval_leggrid_grid(3000, 1, vp(x), vp(y), pk.DLT_GRID_CHEBSTAR, s) == pk.DLT_ERR_UNSUPPORTED
    assert L.dlt_forward_grid(3000, 1, vp(x), vp(y), pk.DLT_GRID_CHEBSTAR, s) == pk.DLT_ERR_UNSUPPORTED
    assert L.cheb_eval_leggrid_grid(1024, 1, vp(x), vp(y), 7, s) == pk.DLT_ERR_INVALID_ARG
    assert L.dlt_forward_grid(1024, 1, vp(x), vp(x), pk.DLT_GRID_CHEBSTAR, s) == pk.DLT_ERR_INVALID_ARG
    assert L.dlt_forward_grid(1024, 0, vp(x), vp(y), pk.DLT_GRID_CHEBSTAR, s) == pk.DLT_OK
    assert L.dlt_inverse_grid(3000, 1, vp(x), vp(y), pk.DLT_GRID_CHEBSTAR, s) == pk.DLT_ERR_UNSUPPORTED
    assert L.dlt_inverse_grid(1024, 1, vp(x), vp(y), -1, s) == pk.DLT_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        pk.dlt_forward(x[:1024], grid="chebstar", prec="fp32bulk")
    with pytest.raises(ValueError):
        pk.dlt_forward(x[:1024], grid="cheb2")
    # DLT_GRID_CHEB1 is the plain call, bit for bit
    c = to_dev(wl.coeffs_algebraic(1024, 14)[0])
    a = to_host(pk.dlt_forward(c))
    assert L.dlt_forward_grid(1024, 1, vp(c), vp(y), pk.DLT_GRID_CHEB1, s) == pk.DLT_OK
    assert np.array_equal(to_host(y)[:1024], a)


def test_chebstar_trace(pk):
    N = 1 << 16
    c = to_dev(wl.coeffs_algebraic(N, 15)[0])
    ref = to_host(pk.dlt_forward(c, grid="chebstar"))
    pk.trace_enable(True)
    got = to_host(pk.dlt_forward(c, grid="chebstar"))
    pk.trace_enable(False)
    kern = pk.trace_collect()
    assert np.array_equal(got, ref)
    for k in ("k_star_passA", "k_star_passB", "k_star_passC"):
        assert kern.get(f"{k}/{N}", (0, 0))[1] == 1, sorted(kern)
