"""GPU parity of leg2chebvals / chebvals2leg (Legendre coefficients <->
values at the Chebyshev points x_j = cos((j+1/2) pi/N)) against the oracle.

leg2chebvals: ||v - v_or||_inf / ||c||_1 <= 5e-14, v_or the direct
recurrence sum at the grid angles (extended precision).
chebvals2leg: max_n |c_n - c_n^or| / ((n+1/2) ||chat||_1) <= 2e-13, with
chat the Chebyshev coefficients of the interpolant (scipy's DCT-II of v,
scaled by eps_n / N) and c_or the oracle's back substitution M^{-1} chat.
Round trip at 2^20: the interpolant of the values' errors (<= 5e-14 ||c||_1)
has Legendre coefficients within (n+1/2) 2 Lambda_N times them, Lambda_N <=
1 + (2/pi) ln N the Lebesgue constant of the grid, on top of chebvals2leg's
own 2e-13 (n+1/2) ||chat||_1 with ||chat||_1 <= ||c||_1 (M >= 0, column sums 1)."""
import numpy as np
import pytest

from gpu_util import dlt_err, exact_angles, need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def cheb_coeffs_of_values(v):
    from scipy.fft import dct

    N = len(v)
    y = dct(v, type=2) / 2  # sum_j v_j cos(n (j+1/2) pi/N)
    eps = np.full(N, 2.0)
    eps[0] = 1.0
    return eps / N * y


@pytest.mark.parametrize("N", [1, 2, 16, 1024, 4096, 16384, 1 << 16, 1 << 20])
def test_leg2chebvals(pk, orc, N):
    say("leg2chebvals", N)
    c = wl.coeffs_algebraic(N, 61)[0]
    v = to_host(pk.leg2chebvals(to_dev(c)))
    idx = None if N <= 16384 else wl.sample_indices(N, 512, 62)
    hi, lo = exact_angles(N, np.zeros(N), idx)
    ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
    err = dlt_err(v if idx is None else v[idx], ref, c)
    say("  err", err)
    assert err <= 5e-14


@pytest.mark.parametrize("N", [1, 2, 16, 1024, 4096, 16384, 1 << 16])
def test_chebvals2leg(pk, orc, N):
    say("chebvals2leg", N)
    v = wl.values_normal(N, 63)[0]
    c = to_host(pk.chebvals2leg(to_dev(v)))
    chat = cheb_coeffs_of_values(v)
    ref = orc.cheb2leg(chat, prec="l")
    err = float(np.max(np.abs(c - ref) / ((np.arange(N) + 0.5) * np.sum(np.abs(chat)))))
    say("  err", err)
    assert err <= 2e-13


@pytest.mark.parametrize("N", [1 << 12, 1 << 20])
def test_values_roundtrip(pk, N):
    c = wl.coeffs_algebraic(N, 64)[0]
    back = to_host(pk.chebvals2leg(pk.leg2chebvals(to_dev(c))))
    err = float(np.max(np.abs(back - c) / ((np.arange(N) + 0.5) * np.sum(np.abs(c)))))
    bar = 2e-13 + 2 * (1 + 2 / np.pi * np.log(N)) * 5e-14
    say("values round trip", N, err, "bar", bar)
    assert err <= bar
