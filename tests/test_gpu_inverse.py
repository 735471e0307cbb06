"""GPU parity of the inverse transform (eq. (2), Sec. 4) against the CPU
oracle, plus the round trip IDLT(DLT(c)) = c and IDLT(1) = e_0.

Error norm (forward-transform analogue for the inverse): for every n,
|c_n - c_n^ref| <= 5e-14 (n + 1/2) sum_k w_k |f_k|; the oracle is evaluated
at the GPU's own nodes (two-double angles) and weights."""
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


def nodes(pk, N):
    th, w, d = pk.leg_nodes_weights(N)
    return to_host(th)[0], to_host(w)[0], to_host(d)[0]


def idlt_err(c, ref, w, f, idx=None):
    n = np.arange(len(w)) if idx is None else np.asarray(idx)
    scale = (n + 0.5) * np.sum(w * np.abs(f))
    return float(np.max(np.abs(c - ref) / scale))


@pytest.mark.parametrize("N", [1, 2, 4, 16, 256, 1024, 4096, 16384, 32768, 1 << 16])
def test_idlt_full(pk, orc, N):
    say("idlt", N)
    f = wl.values_normal(N, 4)[0]
    c = to_host(pk.dlt_inverse(to_dev(f)))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    ref = orc.idlt(f, hi, w, prec="l", theta_lo=lo)
    err = idlt_err(c, ref, w, f)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [1 << 18, 1 << 20])
def test_idlt_sampled_low_degrees(pk, orc, N):
    say("idlt sampled", N)
    f = wl.values_normal(N, 4)[0]
    c = to_host(pk.dlt_inverse(to_dev(f)))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    idx = np.unique(np.concatenate([np.arange(64), wl.sample_indices(4096, 256, 9)]))
    ref = orc.idlt(f, hi, w, idx=idx, prec="l", theta_lo=lo)
    err = idlt_err(c[idx], ref, w, f, idx)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [1, 2, 16, 1024, 4096, 16384, 1 << 16, 1 << 20])
def test_roundtrip(pk, N):
    say("roundtrip", N)
    for fam, c in (("A", wl.coeffs_algebraic(N, 1)[0]), ("B", wl.coeffs_analytic(N, 3)[0])):
        cd = to_dev(c)
        f = pk.dlt_forward(cd)
        c2 = to_host(pk.dlt_inverse(f))
        fh = to_host(f)
        _, w, _ = nodes(pk, N)
        err = idlt_err(c2, c, w, fh)
        say("  family", fam, "err", err)
        assert err <= TOL


@pytest.mark.parametrize("N", [1, 8, 4096, 1 << 16])
def test_idlt_of_constant(pk, N):
    say("idlt const", N)
    c = to_host(pk.dlt_inverse(to_dev(np.ones(N))))
    assert abs(c[0] - 1) <= 1e-14
    n = np.arange(1, N)
    assert np.max(np.abs(c[1:]) / (2 * (n + 0.5)), initial=0) <= TOL
