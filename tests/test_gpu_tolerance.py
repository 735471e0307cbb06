"""GPU parity of the working-tolerance entry points (*_tol): the same
transforms in FP64 with the Taylor length and the far-field parameters chosen
for a working tolerance eps instead of the fixed budgets (Sec. 3 on working
tolerances; Cor. 1 and Table 1 for the Taylor terms).

Bar: the error norms of the plain entry points with eps in place of 5e-14,
against the extended-precision oracle at the GPU's own nodes: forward DLT,
Chebyshev evaluation and conversion in ||.||_inf / ||c||_1, the IDLT in
max_n |c_n - c_n^or| / ((n+1/2) sum_k w_k |f_k|)."""
import numpy as np
import pytest

from gpu_util import dlt_err, exact_angles, need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS = [1e-12, 1e-9, 1e-6, 1e-3]


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def nodes(pk, N):
    th, w, d = pk.leg_nodes_weights(N)
    return to_host(th)[0], to_host(w)[0], to_host(d)[0]


def test_parameters_follow_the_tolerance(pk):
    # fewer Taylor terms as eps grows (Cor. 1: the smallest L with
    # 0.83845^L / L! <= eps/10); far-field terms trade against near-field rows
    # in the cost model, so only the extremes are compared; at the FP64
    # budget the Taylor length is the plain plan's
    N = 1 << 16
    plans = [pk.plan_info(N, tol=e) for e in (5e-14, 1e-12, 1e-10, 1e-8, 1e-6, 1e-4, 1e-2, 1e-1)]
    say("L", [p["L"] for p in plans], "far terms", [p["far_terms"] for p in plans],
        "near rows", [p["near_rows"] for p in plans])
    assert plans[0]["L"] == pk.plan_info(N)["L"]
    for a, b in zip(plans, plans[1:]):
        assert b["L"] <= a["L"]
    assert plans[-1]["L"] < plans[0]["L"] and plans[-1]["far_terms"] < plans[0]["far_terms"]
    # a tolerance between steps is served by the step below it
    assert pk.plan_info(N, tol=3e-6)["L"] == pk.plan_info(N, tol=2e-6)["L"]


@pytest.mark.parametrize("eps", EPS)
@pytest.mark.parametrize("N", [4096, 1 << 16])
def test_forward_and_evaluation(pk, orc, N, eps):
    say("tol forward", N, eps)
    c = wl.coeffs_algebraic(N, 31)[0]
    f = to_host(pk.dlt_forward(to_dev(c), tol=eps))
    g = to_host(pk.cheb_eval_leggrid(to_dev(c), tol=eps))
    _, _, d = nodes(pk, N)
    idx = None if N <= 4096 else wl.sample_indices(N, 512, 32)
    hi, lo = exact_angles(N, d, idx)
    sel = slice(None) if idx is None else idx
    ef = dlt_err(f[sel], orc.dlt(c, hi, prec="l", theta_lo=lo), c)
    eg = dlt_err(g[sel], orc.ndct(c, hi, prec="l", theta_lo=lo), c)
    say("  dlt err", ef, "ndct err", eg)
    assert ef <= eps and eg <= eps


@pytest.mark.parametrize("eps", EPS)
@pytest.mark.parametrize("N", [4096, 1 << 16])
def test_conversion(pk, orc, N, eps):
    say("tol leg2cheb", N, eps)
    c = wl.coeffs_analytic(N, 33)[0]
    chat = to_host(pk.leg2cheb(to_dev(c), tol=eps))
    idx = np.arange(N) if N <= 4096 else wl.sample_indices(N, 512, 34)
    ref = orc.leg2cheb_rows(c, idx, prec="l")
    err = np.max(np.abs(chat[idx] - ref)) / np.sum(np.abs(c))
    say("  err", err)
    assert err <= eps


@pytest.mark.parametrize("eps", EPS)
def test_inverse(pk, orc, eps):
    N = 4096
    say("tol idlt", N, eps)
    f = wl.values_normal(N, 35)[0]
    c = to_host(pk.dlt_inverse(to_dev(f), tol=eps))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    ref = orc.idlt(f, hi, w, prec="l", theta_lo=lo)
    err = float(np.max(np.abs(c - ref) / ((np.arange(N) + 0.5) * np.sum(w * np.abs(f)))))
    say("  err", err)
    assert err <= eps


@pytest.mark.parametrize("N", [1 << 16, 1 << 20])
def test_roundtrip_and_looser_is_less_accurate(pk, N):
    # IDLT(DLT(c)) = c within the working tolerance, at 2^20 too; a loose
    # tolerance really uses fewer terms (its error is larger than the tight one's)
    c = wl.coeffs_algebraic(N, 36)[0]
    _, w, _ = nodes(pk, N)
    errs = {}
    for eps in (1e-10, 1e-4):
        f = pk.dlt_forward(to_dev(c), tol=eps)
        c2 = to_host(pk.dlt_inverse(f, tol=eps))  # 1-D in, 1-D out
        fh = to_host(f)
        scale = (np.arange(N) + 0.5) * np.sum(w * np.abs(fh))
        errs[eps] = float(np.max(np.abs(c2 - c) / scale))
        say("roundtrip", N, eps, errs[eps])
        assert errs[eps] <= 2 * eps
    assert errs[1e-4] > errs[1e-10]
