"""GPU parity of cheb2leg (Chebyshev to Legendre coefficients, c = M^{-1}
chat, the inverse of leg2cheb, Sec. 3) against the oracle's back
substitution with the upper-triangular M.

Bar: max_n |c_n - c_n^or| / ((n+1/2) ||chat||_1) <= 2e-13: the values at the
Legendre nodes carry at most 5e-14 ||chat||_1 (Chebyshev evaluation) and the
inverse transform adds at most 5e-14 (n+1/2) sum_k w_k |f_k| <=
1e-13 (n+1/2) ||chat||_1 (sum_k w_k = 2, |f_k| <= ||chat||_1)."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, to_host
from paper_1505_00354_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 2e-13


@pytest.fixture(scope="module")
def pk():
    need_gpu()
    import paper_1505_00354_amd as pk

    pk.lib()
    return pk


def err(c, ref, chat):
    n = np.arange(len(c))
    return float(np.max(np.abs(c - ref) / ((n + 0.5) * np.sum(np.abs(chat)))))


@pytest.mark.parametrize("N", [1, 2, 16, 100, 1024, 3000, 4096, 12345, 16384, 1 << 16])
def test_cheb2leg_full(pk, orc, N):
    say("cheb2leg", N)
    for fam, chat in (("A", wl.coeffs_algebraic(N, 41)[0]), ("B", wl.coeffs_analytic(N, 42)[0])):
        c = to_host(pk.cheb2leg(to_dev(chat)))
        e = err(c, orc.cheb2leg(chat, prec="l"), chat)
        say("  family", fam, "err", e)
        assert e <= TOL


def test_cheb2leg_modes(pk, orc):
    N = 4096
    chat = wl.coeffs_algebraic(N, 43)[0]
    ref = orc.cheb2leg(chat, prec="l")
    for prec, tol in (("fp32bulk", 5e-6), ("fp64relaxed", 5e-6)):
        e = err(to_host(pk.cheb2leg(to_dev(chat), prec=prec)), ref, chat)
        say("  mode", prec, e)
        assert e <= 4 * tol
    for eps in (1e-10, 1e-4):
        e = err(to_host(pk.cheb2leg(to_dev(chat), tol=eps)), ref, chat)
        say("  tol", eps, e)
        assert e <= 4 * eps


def test_cheb2leg_2e20_rows(pk, orc):
    # N = 2^20: (M c)_k against chat_k on sampled rows with the exact
    # row-sampled conversion.  |(M dc)_k| <= TOL ||chat||_1 sum_n M_kn (n+1/2)
    # <= TOL ||chat||_1 (2N/pi) (M_kn <= 4/(pi n) for n >= 2k, column sums 1)
    N = 1 << 20
    chat = wl.coeffs_algebraic(N, 44)[0]
    c = to_host(pk.cheb2leg(to_dev(chat)))
    idx = wl.sample_indices(N, 256, 45)
    r = np.max(np.abs(orc.leg2cheb_rows(c, idx, prec="l") - chat[idx])) / np.sum(np.abs(chat))
    bound = TOL * 2 * N / np.pi
    say("cheb2leg 2^20 rows: residual", r, "bound", bound)
    assert r <= bound
