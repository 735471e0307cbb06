"""GPU parity of the reduced-precision modes against the CPU oracle.

FP32-bulk (far-field terms and Taylor pairs l >= 2 in FP32, parameters for a
5e-6 budget) and FP64 with the same parameters are checked with the norms of
the FP64 tests -- ||f - f_or||_inf / ||c||_1 (forward, Chebyshev evaluation),
||chat - chat_or||_inf / ||c||_1 (leg2cheb), max_n |c_n - c_or_n| /
((n+1/2) sum_k w_k |f_k|) (inverse, round trip) -- against 5e-6.  The oracle's
extended-precision build evaluated at the GPU's own nodes is the reference."""
import numpy as np
import pytest

from gpu_util import dlt_err, exact_angles, need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 5e-6
MODES = ["fp32bulk", "fp64relaxed"]


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def nodes(pk, N):
    th, w, d = pk.leg_nodes_weights(N)
    return to_host(th)[0], to_host(w)[0], to_host(d)[0]


def idlt_err(c, ref, w, f, idx=None):
    n = np.arange(len(w)) if idx is None else np.asarray(idx)
    scale = (n + 0.5) * np.sum(w * np.abs(f))
    return float(np.max(np.abs(c - ref) / scale))


def test_plan_parameters(pk):
    N = 1 << 20
    p64, p32, prl = pk.plan_info(N), pk.plan_info(N, "fp32bulk"), pk.plan_info(N, "fp64relaxed")
    say("plans", p64, p32, prl)
    assert p64["L"] == 16 and p32["L"] == 10 and prl["L"] == 10
    # each mode picks its own cheapest term count for the 5e-6 budget
    assert p32["far_terms"] < p64["far_terms"] and prl["far_terms"] < p64["far_terms"]
    # FP32 intermediates take less workspace; a batch of 64 at N = 2^20 runs
    # in slices of the per-stream workspace bound
    assert p32["ws_bytes"] < p64["ws_bytes"]
    for p in (p64, p32, prl):
        assert 1 <= p["ws_cap"] // p["ws_bytes"] < 64


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N", [1, 16, 1024, 4096, 16384, 32768])
def test_dlt_forward_full(pk, orc, mode, N):
    say("dlt", mode, N)
    c = wl.coeffs_algebraic(N, 1)[0]
    f = to_host(pk.dlt_forward(to_dev(c), prec=mode))
    _, _, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
    err = dlt_err(f, ref, c)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N", [1 << 16, 1 << 18, 1 << 20])
def test_dlt_forward_sampled(pk, orc, mode, N):
    say("dlt sampled", mode, N)
    for fam, c in (("A", wl.coeffs_algebraic(N, 2)[0]), ("B", wl.coeffs_analytic(N, 3)[0])):
        f = to_host(pk.dlt_forward(to_dev(c), prec=mode))
        _, _, d = nodes(pk, N)
        idx = wl.sample_indices(N, 512, 5)
        hi, lo = exact_angles(N, d, idx)
        ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
        err = dlt_err(f[idx], ref, c)
        say("  family", fam, "err", err)
        assert err <= TOL


@pytest.mark.parametrize("N", [4096, 32768])
def test_leg2cheb(pk, orc, N):
    say("leg2cheb fp32bulk", N)
    c = wl.coeffs_algebraic(N, 2)[0]
    chat = to_host(pk.leg2cheb(to_dev(c), prec="fp32bulk"))
    ref = orc.leg2cheb(c, prec="l")
    err = np.max(np.abs(chat - ref)) / np.sum(np.abs(c))
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [1024, 16384, 1 << 20])
def test_cheb_eval_leggrid(pk, orc, N):
    say("ndct fp32bulk", N)
    chat = wl.coeffs_algebraic(N, 3)[0]
    f = to_host(pk.cheb_eval_leggrid(to_dev(chat), prec="fp32bulk"))
    _, _, d = nodes(pk, N)
    idx = wl.sample_indices(N, min(N, 512), 6)
    hi, lo = exact_angles(N, d, idx)
    ref = orc.ndct(chat, hi, prec="l", theta_lo=lo)
    err = dlt_err(f[idx], ref, chat)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N", [1, 16, 1024, 16384, 1 << 16])
def test_idlt_full(pk, orc, mode, N):
    say("idlt", mode, N)
    f = wl.values_normal(N, 4)[0]
    c = to_host(pk.dlt_inverse(to_dev(f), prec=mode))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    ref = orc.idlt(f, hi, w, prec="l", theta_lo=lo)
    err = idlt_err(c, ref, w, f)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [1 << 18, 1 << 20])
def test_idlt_sampled_low_degrees(pk, orc, N):
    say("idlt sampled fp32bulk", N)
    f = wl.values_normal(N, 4)[0]
    c = to_host(pk.dlt_inverse(to_dev(f), prec="fp32bulk"))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    idx = np.unique(np.concatenate([np.arange(64), wl.sample_indices(4096, 256, 9)]))
    ref = orc.idlt(f, hi, w, idx=idx, prec="l", theta_lo=lo)
    err = idlt_err(c[idx], ref, w, f, idx)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [1024, 1 << 16, 1 << 20])
def test_roundtrip(pk, N):
    say("roundtrip fp32bulk", N)
    for fam, c in (("A", wl.coeffs_algebraic(N, 1)[0]), ("B", wl.coeffs_analytic(N, 3)[0])):
        f = pk.dlt_forward(to_dev(c), prec="fp32bulk")
        c2 = to_host(pk.dlt_inverse(f, prec="fp32bulk"))
        _, w, _ = nodes(pk, N)
        err = idlt_err(c2, c, w, to_host(f))
        say("  family", fam, "err", err)
        assert err <= 2 * TOL


def test_batch_2e20(pk, orc):
    """Four instances of N = 2^20 in one call (the shape of the batched
    mixed-precision workload): each matches its single-instance call bit for
    bit, and 256 sampled outputs of every instance are within the budget."""
    N, B = 1 << 20, 4
    say("batch fp32bulk", N, B)
    c = np.concatenate([wl.coeffs_algebraic(N, 100 + b) for b in range(B)])
    fb = to_host(pk.dlt_forward(to_dev(c), prec="fp32bulk"))
    _, _, d = nodes(pk, N)
    idx = wl.sample_indices(N, 256, 11)
    hi, lo = exact_angles(N, d, idx)
    for b in range(B):
        fs = to_host(pk.dlt_forward(to_dev(c[b]), prec="fp32bulk"))
        assert np.array_equal(fb[b], fs)
        ref = orc.dlt(c[b], hi, prec="l", theta_lo=lo)
        err = dlt_err(fb[b][idx], ref, c[b])
        say("  instance", b, "err", err)
        assert err <= TOL
