"""GPU parity for sizes that are not powers of two and for ragged batches
(many transforms of uneven size and direction in one call), against the CPU
oracle evaluated at the GPU's own nodes.  Same norms and FP64 budget as the
power-of-two tests (5e-14); 5e-6 for FP32-bulk."""
import numpy as np
import pytest

from gpu_util import ULP, dlt_err, exact_angles, need_gpu, say, to_dev, to_host
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


@pytest.mark.parametrize("N", [3, 5, 7, 24, 100, 1000, 3000, 6000, 12345, 70000])
def test_nodes_any_size(pk, orc, N):
    say("nodes", N)
    th, w, d = nodes(pk, N)
    idx = wl.sample_indices(N, min(N, 512), 5)
    tho, wo = orc.nodes(N, idx=idx)
    assert np.all(np.abs(th[idx] - tho) <= 4 * ULP * tho), np.max(np.abs(th[idx] - tho) / (ULP * tho))
    assert np.max(np.abs(w[idx] / wo - 1)) <= 1e-14
    assert np.max(np.abs((np.arange(N) + 0.5) * np.pi / N + d - th)) <= 4 * ULP * np.pi


# 2^k - 1 and 2^k - 3: sizes just below the grid size, where the first node
# gaps near the ends are shorter than the grid spacing pi/Ng
@pytest.mark.parametrize("N", [3, 7, 24, 100, 1000, 3000, 6000, 12345, 1021, 1023, 4093, 4095, 16381])
def test_dlt_forward_any_size(pk, orc, N):
    say("dlt", N)
    c = wl.coeffs_algebraic(N, 1)[0]
    f = to_host(pk.dlt_forward(to_dev(c)))
    _, _, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
    err = dlt_err(f, ref, c)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [70000, 300000, 1000000])
def test_dlt_forward_any_size_sampled(pk, orc, N):
    say("dlt sampled", N)
    c = wl.coeffs_algebraic(N, 2)[0]
    f = to_host(pk.dlt_forward(to_dev(c)))
    _, _, d = nodes(pk, N)
    idx = wl.sample_indices(N, 512, 5)
    hi, lo = exact_angles(N, d, idx)
    ref = orc.dlt(c, hi, prec="l", theta_lo=lo)
    err = dlt_err(f[idx], ref, c)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [3, 100, 3000, 12345, 70000])
def test_idlt_any_size(pk, orc, N):
    say("idlt", N)
    f = wl.values_normal(N, 4)[0]
    c = to_host(pk.dlt_inverse(to_dev(f)))
    _, w, d = nodes(pk, N)
    hi, lo = exact_angles(N, d)
    idx = None if N <= 12345 else np.unique(np.concatenate([np.arange(64), wl.sample_indices(N, 256, 9)]))
    ref = orc.idlt(f, hi, w, idx=idx, prec="l", theta_lo=lo)
    err = idlt_err(c if idx is None else c[idx], ref, w, f, idx)
    say("  err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [100, 5000, 40000])
def test_leg2cheb_and_ndct_any_size(pk, orc, N):
    say("leg2cheb/ndct", N)
    c = wl.coeffs_algebraic(N, 2)[0]
    chat = to_host(pk.leg2cheb(to_dev(c)))
    if N <= 16384:
        ref = orc.leg2cheb(c, prec="l")
        assert np.max(np.abs(chat - ref)) / np.sum(np.abs(c)) <= TOL
    f = to_host(pk.cheb_eval_leggrid(to_dev(chat)))
    _, _, d = nodes(pk, N)
    idx = wl.sample_indices(N, min(N, 512), 6)
    hi, lo = exact_angles(N, d, idx)
    ref = orc.ndct(chat, hi, prec="l", theta_lo=lo)
    err = dlt_err(f[idx], ref, chat)
    say("  ndct err", err)
    assert err <= TOL


@pytest.mark.parametrize("N", [100, 5000, 70000])
def test_roundtrip_any_size(pk, N):
    say("roundtrip", N)
    c = wl.coeffs_algebraic(N, 1)[0]
    f = pk.dlt_forward(to_dev(c))
    c2 = to_host(pk.dlt_inverse(f))
    _, w, _ = nodes(pk, N)
    err = idlt_err(c2, c, w, to_host(f))
    say("  err", err)
    assert err <= TOL


def ragged_case(count, lo, hi, seed, mixed=True):
    sizes = wl.log_uniform_sizes(count, lo, hi, seed)
    offs = np.zeros(count, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    inv = (rng.random(count) < 0.5).astype(np.int8) if mixed else np.zeros(count, np.int8)
    x = np.empty(int(sizes.sum()))
    for i, (n, o) in enumerate(zip(sizes, offs)):
        x[o:o + n] = wl.values_normal(int(n), 1000 + i)[0] if inv[i] else wl.coeffs_algebraic(int(n), 1000 + i)[0]
    return sizes, offs, inv, x


@pytest.mark.parametrize("prec,tol", [("fp64", TOL), ("fp32bulk", 5e-6)])
def test_ragged_batch_against_oracle(pk, orc, prec, tol):
    """48 instances, sizes log-uniform in [16, 20000], forward and inverse
    mixed, in one call; every instance against the oracle (full up to 4096,
    sampled above), then the replayed graph on new data."""
    sizes, offs, inv, x = ragged_case(48, 16, 20000, 21)
    say("ragged", prec, int(sizes.min()), int(sizes.max()), int(inv.sum()))
    out = to_host(pk.dlt_batch(to_dev(x), sizes, offs, inv, prec=prec))
    worst = 0.0
    for i, (n, o) in enumerate(zip(sizes, offs)):
        n, o = int(n), int(o)
        xi, yi = x[o:o + n], out[o:o + n]
        _, w, d = nodes(pk, n)
        idx = None if n <= 4096 else wl.sample_indices(n, 256, 30 + i)
        hi, lo = exact_angles(n, d, idx)
        if inv[i]:
            hi_all, lo_all = exact_angles(n, d)
            ref = orc.idlt(xi, hi_all, w, idx=idx, prec="l", theta_lo=lo_all)
            err = idlt_err(yi if idx is None else yi[idx], ref, w, xi, idx)
        else:
            ref = orc.dlt(xi, hi, prec="l", theta_lo=lo)
            err = dlt_err(yi if idx is None else yi[idx], ref, xi)
        worst = max(worst, err)
        assert err <= tol, (i, n, int(inv[i]), err)
    say("  worst err", worst)


def test_ragged_graph_replay_and_single_calls(pk):
    """The second call with the same layout replays the cached graph: with new
    input values it must equal single-instance calls of the same grids."""
    sizes, offs, inv, x = ragged_case(32, 64, 5000, 22)
    xd = to_dev(x)
    out = pk.dlt_batch(xd, sizes, offs, inv)
    first = to_host(out)
    xd.mul_(-0.5)  # new data in the same buffer
    pk.dlt_batch(xd, sizes, offs, inv, out=out)
    second = to_host(out)
    assert np.allclose(second, -0.5 * first, rtol=0, atol=1e-13 * np.max(np.abs(first)))
    pk.dlt_batch(xd, sizes, offs, inv, out=out)
    assert np.array_equal(to_host(out), second)  # replays are deterministic


def test_ragged_graph_cache_bound(pk):
    """70 distinct layouts (the library keeps 64 ragged graphs): each call and
    its replay agree bit for bit, and the earliest layouts, whose graphs were
    dropped, are rebuilt on the same grids with the same bits."""
    import torch

    sizes = np.array([100, 37, 64], dtype=np.int64)
    n = 70
    say("ragged graph cache bound", n)
    xd = to_dev(wl.coeffs_algebraic(int(sizes.sum()) + n, 61)[0])
    base = np.concatenate(([0], np.cumsum(sizes)[:-1]))
    outs = [torch.zeros_like(xd) for _ in range(n)]
    first = []
    for k in range(n):
        pk.dlt_batch(xd, sizes, base + k, out=outs[k])
        first.append(to_host(outs[k]))
        outs[k].zero_()
        pk.dlt_batch(xd, sizes, base + k, out=outs[k])
        assert np.array_equal(to_host(outs[k]), first[k]), k
    for k in range(3):
        outs[k].zero_()
        pk.dlt_batch(xd, sizes, base + k, out=outs[k])
        assert np.array_equal(to_host(outs[k]), first[k]), ("rebuilt", k)


def test_ragged_traced_run_matches_graph(pk):
    """With the kernel trace on, a cached batch runs its kernels directly
    (each traced) instead of its graph: the same bits, and the trace names
    the batched dense block of the classes of eight or more instances."""
    sizes, offs, inv, x = ragged_case(300, 64, 9000, 41, mixed=True)
    say("ragged traced", int(sizes.min()), int(sizes.max()), int(inv.sum()))
    xd = to_dev(x)
    ref = to_host(pk.dlt_batch(xd, sizes, offs, inv))
    ref2 = to_host(pk.dlt_batch(xd, sizes, offs, inv))  # replay
    pk.trace_enable(True)
    got = to_host(pk.dlt_batch(xd, sizes, offs, inv))
    pk.trace_enable(False)
    kern = pk.trace_collect()
    assert np.array_equal(ref, ref2)
    assert np.array_equal(got, ref)
    assert any(k.startswith("k_dense_mm/") for k in kern), sorted(kern)
    assert any(k.startswith("k_dense_mm_t/") for k in kern), sorted(kern)
    # every class ran on the grid dlt_batch_grid reports (its padded size or
    # twice it), and the trace names kernels on those grids only
    grids = set()
    for n, d in zip(sizes.tolist(), inv.tolist()):
        P = 1 << max(0, (int(n) - 1).bit_length())
        G = pk.batch_grid(int(n), bool(d))
        assert G in (P, 2 * P), (n, d, G)
        grids.add(G)
    for k in kern:
        assert int(k.split("/")[1]) in grids, (k, sorted(grids))
