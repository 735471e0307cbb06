"""GPU parity of cheb_eval_nodes: the Taylor NDCT of Sec. 2 at
near-Chebyshev points other than the Legendre nodes (Gauss-Jacobi nodes,
Gauss-Chebyshev nodes of the second kind, random offsets), against the
oracle's direct Chebyshev recurrence at the same angles in extended
precision.  Bar: ||f - f_or||_inf / ||chat||_1 <= 5e-14, for offsets with
|N dtheta| <= pi/2 (the entry point's precondition)."""
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


def offsets(kind, N):
    grid = (np.arange(N) + 0.5) * np.pi / N
    if kind == "cheb2":  # zeros of U_N: theta_k = (k+1) pi/(N+1)
        th = (np.arange(N) + 1) * np.pi / (N + 1)
    elif kind == "jacobi":  # Gauss-Jacobi nodes, alpha = -0.3, beta = 0.4, increasing theta
        from scipy.special import roots_jacobi

        x, _ = roots_jacobi(N, -0.3, 0.4)
        th = np.sort(np.arccos(x))
    else:  # random offsets up to the bound
        th = grid + wl.rng(50).uniform(-1, 1, N) * 0.999 * (np.pi / 2) / N
    d = th - grid
    assert np.max(np.abs(N * d)) <= np.pi / 2
    return d


# Gauss-Jacobi nodes up to 4096 only: scipy's root finder for them is slow
# beyond a few thousand nodes
CASES = [(kind, N) for kind in ("cheb2", "jacobi", "random") for N in (16, 1024, 4096, 1 << 16)
         if not (kind == "jacobi" and N > 4096)]


@pytest.mark.parametrize("kind,N", CASES)
def test_cheb_eval_nodes(pk, orc, kind, N):
    say("nodes eval", kind, N)
    d = offsets(kind, N)
    for fam, chat in (("A", wl.coeffs_algebraic(N, 51)[0]), ("B", wl.coeffs_analytic(N, 52)[0])):
        f = to_host(pk.cheb_eval_nodes(to_dev(chat), to_dev(d)))
        idx = None if N <= 4096 else wl.sample_indices(N, 512, 53)
        hi, lo = exact_angles(N, d, idx)
        ref = orc.ndct(chat, hi, prec="l", theta_lo=lo)
        err = dlt_err(f if idx is None else f[idx], ref, chat)
        say("  family", fam, "err", err)
        assert err <= TOL


def test_cheb_eval_nodes_legendre_matches(pk):
    # at the Legendre offsets it is cheb_eval_leggrid (more Taylor terms, so
    # equal to rounding)
    N = 1 << 14
    chat = to_dev(wl.coeffs_algebraic(N, 54)[0])
    _, _, d = pk.leg_nodes_weights(N)
    a = to_host(pk.cheb_eval_nodes(chat, d[0]))
    b = to_host(pk.cheb_eval_leggrid(chat))
    assert np.max(np.abs(a - b)) / np.sum(np.abs(to_host(chat))) <= 1e-15


def test_cheb_eval_nodes_offsets_beyond_bound(pk, orc):
    # offsets with |N dtheta_k| > pi/2 (outside the precondition the Taylor
    # length is chosen for) give NaN at exactly those outputs; the other
    # outputs keep the bar, and offsets at the bound itself are accepted
    N = 1024
    d = offsets("random", N)
    bad = np.array([0, 5, 300, 511, 512, N - 1])
    d[bad] = np.where(np.arange(bad.size) % 2 == 0, 1, -1) * 0.6 * np.pi / N
    d[7] = 0.5 * np.pi / N  # the bound itself
    chat = wl.coeffs_algebraic(N, 54)[0]
    f = to_host(pk.cheb_eval_nodes(to_dev(chat), to_dev(d)))
    say("beyond bound: NaN at", np.flatnonzero(np.isnan(f)))
    assert np.array_equal(np.flatnonzero(np.isnan(f)), bad)
    good = np.setdiff1d(np.arange(N), bad)
    hi, lo = exact_angles(N, d, good)
    ref = orc.ndct(chat, hi, prec="l", theta_lo=lo)
    err = dlt_err(f[good], ref, chat)
    say("  err at the other points", err)
    assert err <= TOL
