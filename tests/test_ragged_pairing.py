"""The nearest-row pairing of Legendre nodes with a finer Chebyshev grid is
one-to-one (runs without a GPU).

Sizes N that are not powers of two run on the grid theta*_j = (j+1/2) pi/Ng,
Ng = 2^ceil(log2 N), each node theta_k taken to the row
j = rint((2k+1) Ng/(2N) + dtheta_k Ng/pi - 1/2) with dtheta_k its offset from
(k+1/2) pi/N -- the rounding the library's node kernels apply.  Node gaps are
smallest at the ends (about 3.115/(N+1/2) for the first, Sec. 2.2's
asymptotics of the zeros), so only for N close below Ng, and only there, can a
gap fall below the grid spacing pi/Ng.  For every such N up to Ng = 2^12
(all nodes) and a seeded sample of them up to 2^20 (the nodes nearest the
ends), the nodes (oracle, extended precision) must fall on distinct rows,
within pi/2 of them in units of the grid spacing, and with a margin to the
rounding boundary that no rounding difference of the device's offsets could
cross.
"""
import numpy as np
import pytest

from paper_1505_00354_amd import workloads as wl



def rows(N, Ng, th):
    k = np.arange(len(th))
    d = th - (k + 0.5) * np.pi / N
    r = (2.0 * k + 1.0) * Ng / (2.0 * N) + d * Ng / np.pi - 0.5
    return np.rint(r).astype(np.int64), r


def check(orc, N, first):
    Ng = 1 << int(np.ceil(np.log2(N)))
    th, _ = orc.nodes(N, idx=np.arange(min(first, (N + 1) // 2)))
    j, r = rows(N, Ng, th)
    assert np.all(np.diff(j) > 0), (N, j)
    assert np.all(np.abs(Ng * th - (j + 0.5) * np.pi) <= np.pi / 2 + 1e-12)
    # distance of each row coordinate from a rounding boundary (the middle
    # node of an odd N sits at pi/2, halfway between two rows: it is its own
    # mirror image, so either row leaves the pairing one-to-one)
    own = (N % 2 == 1) & (np.arange(len(r)) == (N - 1) // 2)
    assert np.min(np.abs(np.abs(r - np.floor(r)) - 0.5)[~own], initial=1) > 1e-9, N


def sizes_below(Ng):
    return np.arange(int(np.ceil(Ng / 1.0085)) - 2, Ng)


@pytest.mark.slow
def test_pairing_one_to_one_all_sizes_to_2p12(orc):
    # every node of the first half (the second half is its mirror image)
    for e in range(2, 13):
        for N in sizes_below(1 << e):
            if N >= 2:
                check(orc, int(N), N)


@pytest.mark.slow
def test_pairing_one_to_one_sampled_to_2p20(orc):
    # the 64 nodes nearest each end, where the gaps are shortest, for seeded
    # sizes just below every grid size up to 2^20 (always N = Ng - 1, Ng - 3)
    for e in range(13, 21):
        cand = sizes_below(1 << e)
        pick = wl.rng(40 + e).choice(cand, size=min(24, len(cand)), replace=False)
        for N in sorted(set(int(x) for x in pick) | {int(cand[-1]), int(cand[-3])}):
            check(orc, N, 64)
