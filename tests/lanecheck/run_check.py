"""Runs the library's call sequences against the host-only HIP stand-in and
prints the checker's findings as one JSON object (test infrastructure).

Run in a fresh process (tests/test_lanecheck.py does so): the library's
HIP references must bind to the stand-in, not to a HIP runtime that another
module (torch) may already have loaded.

Every entry point is called three times in a row with the same arguments
on each of two caller streams (the null stream and a created one): the
first call runs directly, the second is captured into a graph, the third
replays it.  After every call the checker verifies that the work the call
forked onto other streams is ordered before the caller's stream's end."""
import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build as lbuild  # noqa: E402

PREC = {"fp64": 0, "fp32bulk": 1, "fp64relaxed": 2}


def main(argv):
    quick = "--quick" in argv
    stub = ctypes.CDLL(lbuild.STUB, mode=ctypes.RTLD_GLOBAL)
    L = ctypes.CDLL(lbuild.LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    stub.stub_violation.restype = ctypes.c_char_p
    stub.stub_call_end.argtypes = [vp]
    stub.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
    L.dlt_status_string.restype = ctypes.c_char_p
    s1 = vp()
    assert stub.hipStreamCreateWithFlags(ctypes.byref(s1), 1) == 0
    streams = [vp(0), s1]
    bufs = {}

    def buf(tag, n):
        # host memory stands in for device memory; the stand-in never runs a
        # kernel, so these are only addresses (pages stay untouched)
        key = (tag, n)
        if key not in bufs:
            bufs[key] = np.empty(max(n, 1), dtype=np.float64)
        return vp(bufs[key].ctypes.data)

    calls = []
    errors = []

    def call(name, fn, *args):
        for s in streams:
            for rep in range(3):
                stub.stub_call_begin()
                rc = fn(*args, s)
                stub.stub_call_end(s)
                calls.append(name)
                if rc != 0:
                    errors.append(f"{name} (stream {s.value}, call {rep}): status {rc} "
                                  f"{L.dlt_status_string(rc).decode()}")

    def unary(name, N, batch, prec=None, tol=None):
        x, y = buf("in", N * batch), buf("out", N * batch)
        if tol is not None:
            f = getattr(L, name + "_tol")
            f.argtypes = [i64, i64, vp, vp, ctypes.c_double, vp]
            call(f"{name}_tol N={N} b={batch} eps={tol}", f, N, batch, x, y, tol)
        elif prec is not None:
            f = getattr(L, name + "_ex")
            f.argtypes = [i64, i64, vp, vp, ctypes.c_int, vp]
            call(f"{name}_ex N={N} b={batch} {prec}", f, N, batch, x, y, PREC[prec])
        else:
            f = getattr(L, name)
            f.argtypes = [i64, i64, vp, vp, vp]
            call(f"{name} N={N} b={batch}", f, N, batch, x, y)

    sizes = [1, 16, 1024, 1 << 13, 1 << 14, 1 << 17, 1 << 18, 1 << 20]
    if not quick:
        sizes += [2, 64, 4096, 1 << 16, 1 << 19, 1000, 70000]
    L.leg_nodes_weights.argtypes = [i64, i64, vp, vp, vp, vp]
    for N in sizes:
        call(f"leg_nodes_weights N={N}", L.leg_nodes_weights, N, 2, buf("t", 2 * N), buf("w", 2 * N),
             buf("d", 2 * N))
    ops = ["leg2cheb", "cheb_eval_leggrid", "dlt_forward", "dlt_inverse", "cheb2leg"]
    for name in ops:
        for N in sizes:
            unary(name, N, 1)
            unary(name, N, 3, prec="fp32bulk")
            if N & (N - 1) == 0:
                unary(name, N, 2, tol=1e-9)
        if not quick:
            for N in (1 << 17, 1 << 20):
                unary(name, N, 2, prec="fp64relaxed")
    # a batch that runs in several workspace slices
    for name in ("dlt_forward", "dlt_inverse"):
        unary(name, 1 << 20, 64, prec="fp32bulk")
    # the evaluation about theta^cheb* (every kernel on the caller's stream),
    # and a batch of it in slices
    for name in ("cheb_eval_leggrid_grid", "dlt_forward_grid", "dlt_inverse_grid"):
        f = getattr(L, name)
        f.argtypes = [i64, i64, vp, vp, ctypes.c_int, vp]
        for N, batch in ((1, 2), (1024, 2), (1 << 16, 3), (1 << 20, 2), (1 << 20, 14)):
            call(f"{name} N={N} b={batch}", f, N, batch, buf("in", N * batch), buf("out", N * batch), 1)
    for name in ("leg2chebvals", "chebvals2leg"):
        f = getattr(L, name)
        f.argtypes = [i64, i64, vp, vp, vp]
        for N in (1024, 1 << 18):
            call(f"{name} N={N}", f, N, 2, buf("in", 2 * N), buf("out", 2 * N))
    L.cheb_eval_nodes.argtypes = [i64, i64, vp, vp, vp, vp]
    for N in (1024, 1 << 16):
        call(f"cheb_eval_nodes N={N}", L.cheb_eval_nodes, N, 2, buf("in", 2 * N), buf("d", N), buf("out", 2 * N))
    # ragged batches: mixed sizes and directions, every precision mode
    rng = np.random.default_rng(3)
    Ns = np.round(np.exp(rng.uniform(np.log(64), np.log(1 << 17 if quick else 1 << 18), 200))).astype(np.int64)
    Ns[:4] = [1, 2, 1 << 16, 1 << 18]
    offs = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(np.int64)
    inv = (np.arange(len(Ns)) % 2).astype(np.int8)
    tot = int(Ns.sum())
    L.dlt_batch_ex.argtypes = [i64, vp, vp, vp, vp, vp, ctypes.c_int, vp]
    L.dlt_batch_grid.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(i64)]
    max_n = 1 << 20

    def grids():
        # (status, grid, padded size) of every instance of the batch
        out = []
        for n, d in zip(Ns.tolist(), inv.tolist()):
            g = i64(-7)
            rc = L.dlt_batch_grid(int(n), int(d), PREC["fp64"], ctypes.byref(g))
            out.append((rc, g.value, 1 << max(0, (int(n) - 1).bit_length())))
        return out

    before = grids()
    for prec in ("fp64", "fp32bulk"):
        call(f"dlt_batch_ex count={len(Ns)} {prec}", L.dlt_batch_ex, len(Ns), vp(Ns.ctypes.data),
             vp(offs.ctypes.data), vp(inv.ctypes.data), buf("in", tot), buf("out", tot), PREC[prec])
    after = grids()
    # the grid query: 0 before a batch held the size class (the padded size
    # when there is no larger candidate), the padded size or twice it after;
    # bad arguments refused
    g = i64(0)
    bad = [L.dlt_batch_grid(0, 0, 0, ctypes.byref(g)), L.dlt_batch_grid(5, 2, 0, ctypes.byref(g)),
           L.dlt_batch_grid(5, 0, 9, ctypes.byref(g)), L.dlt_batch_grid(5, 0, 0, None),
           L.dlt_batch_grid(max_n + 1, 0, 0, ctypes.byref(g))]
    batch_grid = {
        "before_ok": all(rc == 0 and gr == (P if 2 * P > max_n else 0) for rc, gr, P in before),
        "after_ok": all(rc == 0 and gr in (P, 2 * P) for rc, gr, P in after),
        "bad_status": bad,
    }
    # more distinct calls than the call-graph cache keeps (its eviction
    # destroys the other graphs), then the first ones again
    N = 1024
    big_in, big_out = np.empty(N * 320), np.empty(N * 320)
    L.dlt_forward.argtypes = [i64, i64, vp, vp, vp]
    for rnd in range(2):
        for i in list(range(300)) + list(range(8)):
            x, y = vp(big_in.ctypes.data + 8 * N * i), vp(big_out.ctypes.data + 8 * N * i)
            for rep in range(2 if rnd == 0 else 3):
                stub.stub_call_begin()
                rc = L.dlt_forward(N, 1, x, y, streams[1])
                stub.stub_call_end(streams[1])
                calls.append("dlt_forward distinct buffers")
                if rc:
                    errors.append(f"dlt_forward distinct buffers {i}: status {rc}")
    # more distinct ragged descriptors than the batch-graph cache keeps
    for i in range(70):
        Ns2 = np.array([100 + i, 300, 1 << 12], dtype=np.int64)
        offs2 = np.array([0, 100 + i, 400 + i], dtype=np.int64)
        inv2 = np.array([0, 1, i % 2], dtype=np.int8)
        for rep in range(2):
            stub.stub_call_begin()
            rc = L.dlt_batch_ex(3, vp(Ns2.ctypes.data), vp(offs2.ctypes.data), vp(inv2.ctypes.data),
                                vp(big_in.ctypes.data), vp(big_out.ctypes.data), 0, streams[rep % 2])
            stub.stub_call_end(streams[rep % 2])
            calls.append("dlt_batch_ex distinct descriptors")
            if rc:
                errors.append(f"dlt_batch_ex distinct descriptor {i}: status {rc}")
    # the allocation-free forward: once its size's plan exists, no allocation,
    # free, stream, event, synchronisation, capture, record or wait at all
    L.dlt_forward_noalloc.argtypes = [i64, i64, vp, vp, vp]
    res0, res1 = (ctypes.c_long * 5)(), (ctypes.c_long * 5)()
    cnt0, cnt1 = (ctypes.c_long * 6)(), (ctypes.c_long * 6)()
    noalloc = {}
    for N, batch in ((1 << 16, 3), (4096, 500), (1024, 2), (1, 4)):
        unary("dlt_forward", N, 1)  # builds the plan
        x, y = buf("in", N * batch), buf("out", N * batch)
        stub.stub_resource_counts(res0)
        stub.stub_counts(cnt0)
        for s in streams:
            for rep in range(2):
                stub.stub_call_begin()
                rc = L.dlt_forward_noalloc(N, batch, x, y, s)
                stub.stub_call_end(s)
                calls.append(f"dlt_forward_noalloc N={N} b={batch}")
                if rc:
                    errors.append(f"dlt_forward_noalloc N={N} b={batch}: status {rc}")
        stub.stub_resource_counts(res1)
        stub.stub_counts(cnt1)
        noalloc[f"{N}x{batch}"] = {
            "resources": [res1[i] - res0[i] for i in range(5)],
            "launches": cnt1[0] - cnt0[0],
            "captures_graphs_records_waits": [cnt1[i] - cnt0[i] for i in (1, 2, 3, 4)],
        }
    # the kernel trace: every kernel on the caller's stream
    L.dlt_trace_enable.argtypes = [ctypes.c_int]
    L.dlt_trace_enable(1)
    unary("dlt_forward", 1 << 18, 1)
    unary("dlt_inverse", 1 << 18, 1)
    # a cached ragged batch runs its kernels directly while traced
    call(f"dlt_batch_ex traced count={len(Ns)}", L.dlt_batch_ex, len(Ns), vp(Ns.ctypes.data),
         vp(offs.ctypes.data), vp(inv.ctypes.data), buf("in", tot), buf("out", tot), PREC["fp64"])
    L.dlt_trace_enable(0)
    L.dlt_release()
    unary("dlt_inverse", 1 << 20, 1)

    counts = (ctypes.c_long * 6)()
    stub.stub_counts(counts)
    viol = [stub.stub_violation(i).decode() for i in range(stub.stub_violation_count())]
    print(json.dumps({
        "calls": len(calls),
        "launches": counts[0], "captures": counts[1], "graph_launches": counts[2],
        "event_records": counts[3], "event_waits": counts[4], "side_to_side_waits": counts[5],
        "errors": errors, "violations": viol[:50], "violation_count": len(viol), "noalloc": noalloc,
        "batch_grid": batch_grid,
    }))


if __name__ == "__main__":
    main(sys.argv[1:])
