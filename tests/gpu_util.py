"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np

ULP = np.finfo(np.float64).eps


def need_gpu():
    import pytest
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def dlt_err(f, f_ref, c):
    """max_k |f_k - f_ref_k| / ||c||_1 (the forward-transform norm)."""
    return float(np.max(np.abs(f - f_ref)) / np.sum(np.abs(c)))


PI_L = np.longdouble("3.14159265358979323846264338327950288")


def exact_angles(N, dtheta, idx=None):
    """(hi, lo) two-double angles theta*_k + dtheta_k, theta*_k = (k+1/2) pi/N,
    formed in extended precision: the points the GPU path evaluates at."""
    k = np.arange(N) if idx is None else np.asarray(idx)
    d = np.asarray(dtheta)[k] if len(dtheta) == N else np.asarray(dtheta)
    t = (k.astype(np.longdouble) + np.longdouble(0.5)) * PI_L / np.longdouble(N) + d.astype(np.longdouble)
    hi = t.astype(np.float64)
    lo = (t - hi.astype(np.longdouble)).astype(np.float64)
    return hi, lo
