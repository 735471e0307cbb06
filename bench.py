#!/usr/bin/env python3
"""Throughput of the fast discrete Legendre transform on one MI355X.

One step = the hot path of the paper's method on one batch of synthetic
input at N = 2^20 (plain FP64): a forward DLT (nodes, Legendre-to-Chebyshev
conversion, Taylor-series Chebyshev evaluation), an inverse DLT (the
transposed pipeline) and a standalone Chebyshev-at-Legendre-grid evaluation.
Inputs are resident in HBM before timing starts.  `value` counts transforms
(3 per instance per step) per second.

Prints one JSON line; diagnostics go to stderr.  Options:
  --gpus N      must be 1 (this build runs on one GPU)
  --steps K     timed steps (default 20)
  --warmup W    untimed steps first (default 3)
  --n N         transform length (default 2^20)
  --batch B     instances per step (default 1)
  --cpu-sample K  output indices the CPU oracle evaluates for cpu_baseline
  --no-cpu      skip the CPU baseline
  --prec P      arithmetic of the headline run: fp64 (default), fp32bulk
                (FP32 bulk transforms, 5e-6 budget) or fp64relaxed (FP64 with
                the 5e-6 parameters)
  --ragged-only run only the ragged-batch workloads (no oracle checks) and
                print their results
  --no-ragged   skip the ragged-batch runs (reported under "ragged": 4096
                FP64 DLTs of sizes log-uniform in [64, 16384] as one cached
                graph launch against one call per transform; 16384 FP32-bulk
                transforms of sizes log-uniform in [256, 2^18], half of them
                inverse, with errors per octave against the oracle)
  --no-modes    skip the short runs of the other modes (reported under
                "modes": step time, speedup at equal stated accuracy,
                FP32-bulk at batch 64, the step at working tolerances
                1e-12 ... 1e-3, errors against the oracle; under
                "sizes" the FP64 step at N = 2^12, 2^14, 2^16, 2^18; and
                under "grids" the evaluation and the DLT with the Taylor
                series about theta^cheb* against theta^cheb1: time per
                call, the theta^cheb* kernels' rooflines, the error)
  --copy-probe BYTES  only run one plain copy kernel (read BYTES, write
                BYTES) and exit: the reference for calibrating the HBM byte
                counters FETCH_SIZE / WRITE_SIZE
"""
import argparse
import faulthandler
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_model(name, N, info, f32=False, bulk=False):
    """Algorithmic work of one launch of `name` at transform size N for one
    instance: ("hbm", bytes) -- inputs read once, outputs and DFT
    intermediates written once -- or ("alu", FP64 flops).  None if the kernel
    has no model.  f32: an FP32 launch of the FP32-bulk mode (complex
    intermediates of 8 bytes; its Taylor launches cover pairs 1..Q-1); bulk:
    an FP64 launch of that mode (its Taylor pass A covers pair 0 only)."""
    T, Q = info["far_terms"], info["L"] // 2
    GA, GB = info["tgA"], info["tgB"]
    hbm = {
        "k_far_passA": 8 * N + 16 * N * T,
        "k_far_passB": 16 * N * T + 8 * N * GB,
        "k_tfar_passA": 8 * N + 16 * N * T,
        "k_tfar_passB": 16 * N * T + 8 * N * GB,
        "k_ndct_passA": 8 * N + 16 * N * Q,
        "k_ndct_passB": 16 * N * Q + 16 * N,
        "k_tndct_passA": 24 * N + 16 * N * Q,
        "k_tndct_passB": 16 * N * Q + 8 * N,
        "k_dct2_passA": 8 * N * GB + 16 * N,
        "k_dct2_passB": 16 * N + 8 * N,
        "k_dct3_passA": 8 * N + 16 * N,
        "k_dct3_passB": 16 * N + 8 * N,
    }
    # evaluation about theta^cheb*: LS slabs of M = 2N complex values
    LS, M = info.get("chebstar_L", 0), 2 * N
    hbm["k_star_passA"] = 8 * N + 16 * M * LS
    hbm["k_star_passB"] = 2 * 16 * M * LS + 16 * M
    hbm["k_star_passC"] = 16 * M * LS + 8 * N + 8 * N
    # near field: per (row, degree >= nd) one recurrence step (3 FMA + 1 add
    # = 7 flops) and one weighted accumulation (FMA, or multiply + add)
    alu = {
        "k_near_sums": 9 * info["near_work"],
        "k_tnear_accum": 9 * info["near_work"],
    }
    if f32:
        hbm = {
            "k_far_passA": 8 * N + 8 * N * T,
            "k_far_passB": 8 * N * T + 8 * N * GB,
            "k_tfar_passA": 8 * N + 8 * N * T,
            "k_tfar_passB": 8 * N * T + 8 * N * GB,
            "k_ndct_passA": 8 * N + 8 * N * (Q - 1),
            "k_ndct_passB": 16 * N + 8 * N * (Q - 1) + 16 * N,
            "k_tndct_passA": 24 * N + 8 * N * (Q - 1),
            "k_tndct_passB": 16 * N + 8 * N * (Q - 1) + 8 * N,
        }
    elif bulk:
        hbm["k_ndct_passA"] = 8 * N + 16 * N
        hbm["k_tndct_passA"] = 24 * N + 16 * N
    if name in hbm:
        return "hbm", hbm[name]
    if name in alu:
        return "alu", alu[name]
    return None


def source_digest():
    """Digest of the kernel sources, to tell whether stored counter data
    still describe the kernels that run."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("dlt_kernels.hip", "dlt_common.hpp", "dlt_plan.cpp", "dlt_plan.hpp"):
        with open(os.path.join(here, "paper_1505_00354_amd", "csrc", f), "rb") as fh:
            data = fh.read()
        if f == "dlt_kernels.hip":  # device code only: the launch code may change freely
            cut = data.find(b"// ================================================================ host ====")
            data = data[:cut] if cut >= 0 else data
        h.update(data)
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` ("name/N") from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when absent or
    taken on other kernel sources."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "hbm_traffic_dlt_step_n1048576.md")
    if not os.path.exists(path):
        return None
    digest, rows = None, {}
    for line in open(path):
        if line.startswith("source digest:"):
            digest = line.split(":", 1)[1].strip().strip("`")
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0].startswith("k_"):
            try:
                rows[cells[0]] = float(cells[4])
            except ValueError:
                pass
    if digest != source_digest() or kernel not in rows:
        return None
    return rows[kernel]


def grid_runs(pk, wl, torch, np, dev, N, reps, checks=None):
    """cheb_eval_leggrid, dlt_forward and dlt_inverse (FP64) with the Taylor
    series about theta^cheb1 and about theta^cheb*, K calls each; the
    theta^cheb* kernels' rooflines from 3 traced evaluations; the
    theta^cheb* forward's error against the oracle (appended to `checks`,
    run in the CPU leg)."""
    c = torch.from_numpy(wl.coeffs_algebraic(N, 2)[0]).to(dev)
    chat = torch.from_numpy(wl.coeffs_algebraic(N, 3)[0]).to(dev)
    f = torch.empty_like(c)

    def timed_fn(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    fin = torch.from_numpy(wl.values_normal(N, 4)[0]).to(dev)
    res = {"N": N}
    for op, x in (("cheb_eval_leggrid", chat), ("dlt_forward", c), ("dlt_inverse", fin)):
        fn = getattr(pk, op)
        t1 = timed_fn(lambda: fn(x, out=f))
        ts = timed_fn(lambda: fn(x, out=f, grid="chebstar"))
        res[op] = {"ms_cheb1": round(t1, 4), "ms_chebstar": round(ts, 4), "chebstar_over_cheb1": round(ts / t1, 3)}
    info = pk.plan_info(N)
    res["taylor_terms"] = {"cheb1": info["L"], "chebstar": info["chebstar_L"]}
    pk.trace_enable(True)
    for _ in range(3):
        pk.cheb_eval_leggrid(chat, out=f, grid="chebstar")
    torch.cuda.synchronize()
    pk.trace_enable(False)
    kern = pk.trace_collect()
    kr = {}
    for key, (ms, cnt) in sorted(kern.items()):
        name, n = key.split("/")
        m = kernel_model(name, int(n), info)
        if m is None or m[0] != "hbm":
            continue
        us = ms / cnt * 1000
        kr[key] = {"avg_launch_us": round(us, 2), "bytes_per_launch": int(m[1]),
                   "achieved": round(m[1] / us / 1e3, 2), "unit": "GB/s",
                   "frac": round(m[1] / us / 1e3 / HBM_PEAK_GBS, 4)}
    res["chebstar_kernels"] = kr
    res["bytes_per_evaluation"] = {
        "cheb1": int(sum(kernel_model(k, N, info)[1] for k in ("k_ndct_passA", "k_ndct_passB"))),
        "chebstar": int(sum(v["bytes_per_launch"] for v in kr.values()))}
    log("grids", res)
    if checks is not None:
        fh = pk.dlt_forward(c, grid="chebstar").cpu().numpy()
        ch = c.cpu().numpy()

        def check(res=res, fh=fh, ch=ch):
            import oracle

            idx = wl.sample_indices(N, 4096, 11)
            th, _ = oracle.nodes(N, idx=idx)
            ref = oracle.dlt(ch, th)
            res["chebstar_forward_error_vs_oracle"] = float(np.max(np.abs(fh[idx] - ref)) / np.sum(np.abs(ch)))
            res["error_check"] = "4096 sampled outputs; the oracle with its own nodes; max |f - f_oracle| / ||c||_1"

        checks.append(check)
    return res


def ragged_runs(pk, wl, torch, np, dev, checks=None):
    """The two ragged-batch workloads; see --no-ragged.  Error checks
    against the oracle are appended to `checks` (run later, in the CPU leg)."""
    res = {}

    def timed_calls(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # batched plain FP64 DLT: 4096 sizes log-uniform in [64, 16384]
    sizes = wl.log_uniform_sizes(4096, 64, 16384, 6)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    x = torch.from_numpy(wl.ragged_inputs(sizes, 6)).to(dev)
    y = torch.zeros_like(x)
    t0 = time.perf_counter()
    pk.dlt_batch(x, sizes, offs, out=y)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ms_graph = timed_calls(lambda: pk.dlt_batch(x, sizes, offs, out=y), 5)
    views = [(x[o:o + n], y[o:o + n]) for n, o in zip(sizes.tolist(), offs.tolist())]

    def one_by_one():
        for xi, yi in views:
            pk.dlt_forward(xi, out=yi)

    ms_single = timed_calls(one_by_one, 1)
    # the same batch with the kernel trace on (the cached batch then runs its
    # kernels directly, each traced): per-kernel times and the roofline of
    # the dominant kernel, the batched dense block on the FP64 matrix cores
    pk.trace_enable(True)
    for _ in range(2):
        pk.dlt_batch(x, sizes, offs, out=y)
    torch.cuda.synchronize()
    pk.trace_enable(False)
    kern = pk.trace_collect()
    tot_ms = sum(v[0] for v in kern.values()) / 2
    ranked = sorted(kern.items(), key=lambda kv: -kv[1][0])
    # instances per grid: each size class (padded power of two P) runs on
    # the grid the batch's first call timed fastest, P or 2P; classes of 8 or
    # more instances take the batched dense block
    classes = {}
    for n in sizes.tolist():
        P = 1 << max(0, (int(n) - 1).bit_length())
        classes[P] = classes.get(P, 0) + 1
    on_grid = {}
    for P, cnt in classes.items():
        if cnt >= 8:
            G = pk.batch_grid(P)
            on_grid[G] = on_grid.get(G, 0) + cnt
    roof3 = None
    mm = {k: v for k, v in kern.items() if k.startswith("k_dense_mm/")}
    if mm and set(int(k.split("/")[1]) for k in mm) == set(on_grid):
        flops = 0.0
        for G, cnt in on_grid.items():
            nd = pk.plan_info(G)["nd"]
            h0, h1 = (nd + 1) // 2, nd // 2
            flops += cnt * (h0 * (h0 + 1) + h1 * (h1 + 1))
        mm_s = sum(v[0] for v in mm.values()) / 2 / 1000.0
        ach = flops / mm_s / 1e12
        roof3 = {"kernel": "k_dense_mm", "bound": "mfma", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
                 "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4), "flops_per_batch": int(flops),
                 "ms_per_batch": round(mm_s * 1000, 3), "share_of_traced_batch": round(mm_s * 1000 / tot_ms, 4),
                 "instances_per_grid": {str(G): c for G, c in sorted(on_grid.items())},
                 "model": "h0 (h0+1) + h1 (h1+1) flops per instance of the dense block (a multiply-add on each of "
                          "the h (h+1)/2 entries of each parity's triangle), h0, h1 = rows of each parity below nd "
                          "of the grid the instance runs on (classes of 8 or more instances)"}
    res["fp64_4096_sizes_64_16384"] = {
        "transforms": 4096, "ms_per_batch_graph": round(ms_graph, 3),
        "transforms_per_s_graph": round(4096 * 1000.0 / ms_graph, 1),
        "ms_per_batch_one_call_each": round(ms_single, 3),
        "speedup_graph_vs_one_call_each": round(ms_single / ms_graph, 2),
        "first_call_s": round(setup_s, 2),
        "traced_ms_per_batch": round(tot_ms, 3),
        "roofline": roof3,
        "top_kernels_ms_per_batch": {k: round(v[0] / 2, 3) for k, v in ranked[:8]},
        "inputs": "c_n = N(0,1)/(n+1), sizes round(exp(U[ln 64, ln 16384])) seed 6, values seed 6"}
    log("ragged fp64 4096:", res["fp64_4096_sizes_64_16384"])
    del x, y, views

    # mixed stream: 16384 sizes in [256, 2^18], half inverse, FP32-bulk
    cnt = 16384
    sizes = wl.log_uniform_sizes(cnt, 256, 1 << 18, 7)
    r = wl.rng(8)
    inv = (np.arange(cnt) % 2 == 1).astype(np.int8)
    analytic = (r.random(cnt) < 0.1) & (inv == 0)
    offs = np.zeros(cnt, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    xh = wl.ragged_inputs(sizes, 9, inverse=inv, analytic=analytic)
    x = torch.from_numpy(xh).to(dev)
    y = torch.zeros_like(x)
    t0 = time.perf_counter()
    pk.dlt_batch(x, sizes, offs, inv, out=y, prec="fp32bulk")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ms = timed_calls(lambda: pk.dlt_batch(x, sizes, offs, inv, out=y, prec="fp32bulk"), 2)
    entry = {"transforms": cnt, "ms_per_batch_graph": round(ms, 2), "transforms_per_s": round(cnt * 1000.0 / ms, 1),
             "gbytes_in_out": round(2 * 8 * int(sizes.sum()) / 1e9, 2), "first_call_s": round(setup_s, 2),
             "inputs": "sizes round(exp(U[ln 256, ln 2^18])) seed 7; odd instances inverse (values N(0,1)); "
                       "10% of forward instances c_n = 0.99^n N(0,1), others N(0,1)/(n+1); values seed 9"}
    if checks is not None:
        yh = y.cpu().numpy()

        def check(entry=entry, yh=yh, xh=xh, sizes=sizes, offs=offs, inv=inv):
            import oracle

            errs = {}
            for octave in range(8, 18):
                lo, hi = 1 << octave, 1 << (octave + 1)
                fwd = [i for i in range(cnt) if lo <= sizes[i] < hi and not inv[i]]
                bwd = [i for i in range(cnt) if lo <= sizes[i] < hi and inv[i]]
                worst = {"forward": 0.0, "inverse": 0.0}
                # two forward instances on 64 sampled outputs; one inverse
                # instance on 64 degrees spread over [0, N), both ends included
                for i in fwd[:2] + bwd[:1]:
                    n, o = int(sizes[i]), int(offs[i])
                    xi, yi = xh[o:o + n], yh[o:o + n]
                    th, w, d = (t.cpu().numpy()[0] for t in pk.leg_nodes_weights(n))
                    if inv[i]:
                        idx = np.unique(np.concatenate([wl.sample_indices(n, 62, 20 + i), [0, n - 1]]))
                        ref = oracle.idlt(xi, th, w, idx=idx)
                        err = np.max(np.abs(yi[idx] - ref) / ((idx + 0.5) * np.sum(w * np.abs(xi))))
                        worst["inverse"] = max(worst["inverse"], float(err))
                    else:
                        idx = wl.sample_indices(n, 64, 10 + i)
                        ref = oracle.dlt(xi, th[idx])
                        err = np.max(np.abs(yi[idx] - ref)) / np.sum(np.abs(xi))
                        worst["forward"] = max(worst["forward"], float(err))
                errs[f"[2^{octave}, 2^{octave + 1})"] = worst
            entry["max_error_vs_oracle_by_octave"] = errs
            entry["error_budget"] = 5e-6
            entry["error_check"] = ("per octave of N: two forward instances on 64 sampled outputs, one inverse "
                                    "instance on 64 degrees spread over [0, N); the oracle at the GPU's nodes")

        checks.append(check)
    res["fp32bulk_16384_sizes_256_262144_mixed"] = entry
    log("ragged fp32bulk 16384:", {k: v for k, v in entry.items() if k != "max_error_vs_oracle_by_octave"})
    del x, y
    return res


def rooflines(pk, kern, N, B, prec):
    """Per-kernel rooflines from a kernel trace ({name: (ms, launches)}) of
    steps at size N, batch B, precision prec: algorithmic bytes (or flops)
    per launch over the average launch time.  A batch whose workspace
    exceeds the library's bound runs in slices, so a launch covers B/slices
    instances on average.  Returns (dominant kernel's roofline, all,
    dominant kernel name); the dominant kernel has the largest share of the
    traced time."""
    infos = {}

    def info(n):
        if n not in infos:
            infos[n] = pk.plan_info(n, prec)
        return infos[n]

    per_inst = max(1, info(N)["ws_bytes"])
    nbmax = max(1, min(B, info(N)["ws_cap"] // per_inst))
    slices = -(-B // nbmax)  # the library splits a batch into equal slices
    inst_per_launch = B / slices
    tot = sum(v[0] for v in kern.values())
    ranked = sorted(kern.items(), key=lambda kv: -kv[1][0])
    per_kernel = {}
    for key, (ms, cnt) in ranked:
        name, n = key.split("/")
        n = int(n)
        m = kernel_model(name.replace("_f32", ""), n, info(n), f32=name.endswith("_f32"), bulk=(prec == "fp32bulk"))
        if m is None:
            continue
        bound, work = m
        avg_s = ms / cnt / 1000.0
        wl = work * inst_per_launch
        if bound == "hbm":
            ach, peak, unit = wl / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = wl / avg_s / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
        per_kernel[key] = {"bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit,
                           "frac": round(ach / peak, 4), "work_per_launch": int(wl),
                           "instances_per_launch": round(inst_per_launch, 3),
                           "avg_launch_us": round(avg_s * 1e6, 2), "share_of_step": round(ms / tot, 4)}
    dominant = ranked[0][0] if ranked else None
    roof = None
    if dominant in per_kernel:
        r = per_kernel[dominant]
        roof = {"kernel": dominant, "bound": r["bound"], "achieved": r["achieved"], "peak": r["peak"],
                "unit": r["unit"], "frac": r["frac"], "traffic": None,
                ("bytes_per_launch" if r["bound"] == "hbm" else "flops_per_launch"): r["work_per_launch"],
                "instances_per_launch": r["instances_per_launch"],
                "avg_launch_us": r["avg_launch_us"], "share_of_step": r["share_of_step"]}
    return roof, per_kernel, dominant


def step_bytes(pk, kern, steps, N, B, prec):
    """Algorithmic HBM bytes of one step from a kernel trace of `steps`
    steps at size N, batch B: each modelled HBM-bound kernel's bytes per
    instance and launch, times the instances a launch covers (B / slices,
    as in rooflines()), times its launches per step.  Kernels without a byte
    model (nodes, dense and near-field blocks, reductions) add nothing."""
    infos = {}

    def info(n):
        if n not in infos:
            infos[n] = pk.plan_info(n, prec)
        return infos[n]

    per_inst = max(1, info(N)["ws_bytes"])
    nbmax = max(1, min(B, info(N)["ws_cap"] // per_inst))
    inst_per_launch = B / -(-B // nbmax)
    tot = 0.0
    for key, (ms, cnt) in kern.items():
        name, n = key.split("/")
        n = int(n)
        m = kernel_model(name.replace("_f32", ""), n, info(n), f32=name.endswith("_f32"), bulk=(prec == "fp32bulk"))
        if m is not None and m[0] == "hbm":
            tot += m[1] * inst_per_launch * cnt / steps
    return tot


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    faulthandler.enable()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32bulk", "fp64relaxed"])
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--ragged-only", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py: this build runs on a single GPU; --gpus must be 1 "
                 "(a batch would shard across GPUs with no exchange, see DESIGN.md)")

    import numpy as np
    import torch

    import paper_1505_00354_amd as pk
    from paper_1505_00354_amd import workloads as wl

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        a = torch.ones(args.copy_probe // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)  # one elementwise kernel: reads and writes BYTES
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} bytes read and written")
        return

    N, B = args.n, args.batch
    pk.lib()
    prec = args.prec
    if args.ragged_only:  # the two ragged-batch workloads alone (for profiling them)
        print(json.dumps({"ragged": ragged_runs(pk, wl, torch, np, dev, checks=None)}), flush=True)
        return
    c = torch.from_numpy(wl.coeffs_algebraic(N, 2, batch=B)).to(dev)
    fin = torch.from_numpy(wl.values_normal(N, 4, batch=B)).to(dev)
    chat = torch.from_numpy(wl.coeffs_algebraic(N, 3, batch=B)).to(dev)
    f = torch.empty_like(c)
    c2 = torch.empty_like(c)
    g = torch.empty_like(c)
    checks = []  # error checks against the oracle, run in the CPU leg

    # first calls of a fresh process: the forward call builds the size's plan
    # (tables formed on the device, synchronous) and the stream's workspace
    first = {}
    torch.cuda.synchronize()
    for name, fn in (("dlt_forward", lambda: pk.dlt_forward(c, out=f, prec=prec)),
                     ("dlt_inverse", lambda: pk.dlt_inverse(fin, out=c2, prec=prec)),
                     ("cheb_eval_leggrid", lambda: pk.cheb_eval_leggrid(chat, out=g, prec=prec))):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        first[name] = round(1000 * (time.perf_counter() - t0), 3)
    log("first calls (ms, host wall clock)", first)
    info = pk.plan_info(N, prec)
    log("plan", prec, info)

    def step(mode=prec, c=c, fin=fin, chat=chat, f=f, c2=c2, g=g):
        pk.dlt_forward(c, out=f, prec=mode)
        pk.dlt_inverse(fin, out=c2, prec=mode)
        pk.cheb_eval_leggrid(chat, out=g, prec=mode)

    def step_tol(eps, c=c, fin=fin, chat=chat, f=f, c2=c2, g=g):
        pk.dlt_forward(c, out=f, tol=eps)
        pk.dlt_inverse(fin, out=c2, tol=eps)
        pk.cheb_eval_leggrid(chat, out=g, tol=eps)

    def timed_tol(eps, steps):
        for _ in range(2):
            step_tol(eps)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            step_tol(eps)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def timed(mode, steps, **kw):
        for _ in range(2):
            step(mode, **kw)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            step(mode, **kw)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps bracketed by synchronisations and events on the
    # current stream (this gives `value`)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = 3 * B * 1000.0 / ms_step
    log(f"ms/step {ms_step:.4f} (wall {1000 * wall / args.steps:.4f})")
    # the same K steps again with the library's kernel trace on: every
    # kernel runs alone on the caller's stream and takes a start and an end
    # event bound to its own dispatch (its duration, as rocprofv3 reports
    # it).  This region runs slower; it gives the per-kernel times only.
    pk.trace_enable(True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    pk.trace_enable(False)
    kern = pk.trace_collect()
    ms_traced = e0.elapsed_time(e1) / args.steps
    log(f"ms/step with the kernel trace {ms_traced:.4f}")
    tot = sum(v[0] for v in kern.values())
    for k, (ms, cnt) in sorted(kern.items(), key=lambda kv: -kv[1][0]):
        log(f"  {k:26s} {ms / cnt * 1000:10.2f} us/launch  x{cnt:4d}  {100 * ms / tot:5.1f}%")

    roof, per_kernel, dominant = rooflines(pk, kern, N, B, prec)
    if roof is not None and B == 1:
        roof["traffic"] = stored_traffic(dominant)
    sb = step_bytes(pk, kern, args.steps, N, B, prec)
    step_hbm = {"algorithmic_bytes_per_step": int(sb), "achieved": round(sb / ms_step / 1e6, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(sb / ms_step / 1e6 / HBM_PEAK_GBS, 4),
                "note": "byte model of the FFT passes only (nodes, dense and near blocks add none), over the "
                        "untraced step time"}
    log("step-level HBM", step_hbm)

    # each transform of the step alone, K calls back to back
    def timed_fn(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    per_transform = {}
    for name, fn in (("dlt_forward", lambda: pk.dlt_forward(c, out=f, prec=prec)),
                     ("dlt_inverse", lambda: pk.dlt_inverse(fin, out=c2, prec=prec)),
                     ("cheb_eval_leggrid", lambda: pk.cheb_eval_leggrid(chat, out=g, prec=prec))):
        ms1 = timed_fn(fn, args.steps)
        per_transform[name] = {"ms": round(ms1, 5), "transforms_per_s": round(B * 1000.0 / ms1, 2),
                               "first_call_ms": first[name]}
    log("per transform", per_transform)

    out = {
        "metric": "DLT transforms/s + HBM GB/s at N=2^16..2^20, plain FP64 vs batched/FP32-bulk",
        "value": round(value, 2),
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "ms_per_step_traced": round(ms_traced, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec != "fp32bulk" else "f32-bulk+f64",
        "data": "synthetic",
        "config": {"workload": f"single {'plain FP64' if prec == 'fp64' else prec} DLT + IDLT + "
                               f"Chebyshev-at-Legendre-grid evaluation, N={N}",
                   "N": N, "batch": B, "prec": prec, "transforms_per_step": 3 * B,
                   "inputs": "c_n=N(0,1)/(n+1) seed 2; IDLT f_k=N(0,1) seed 4; chat_n=N(0,1)/(n+1) seed 3"},
        "dominant_kernel": dominant,
        "roofline": roof,
        "step_hbm": step_hbm,
        "per_transform": per_transform,
        "roofline_by_kernel": per_kernel,
        "kernel_us": {k: round(v[0] / v[1] * 1000, 2) for k, v in kern.items()},
    }

    # the other arithmetic modes, briefly: step time and speedups at equal
    # stated accuracy (FP32-bulk against FP64 with the same 5e-6 budget), and
    # FP32-bulk forward + inverse at batch 64
    modes = {}
    if not args.no_modes:
        for m in ("fp64", "fp32bulk", "fp64relaxed"):
            ms = ms_step if m == prec else timed(m, args.steps)
            pi = pk.plan_info(N, m)
            modes[m] = {"ms_per_step": round(ms, 5), "transforms_per_s": round(3 * B * 1000.0 / ms, 2),
                        "budget": 5e-14 if m == "fp64" else 5e-6, "L": pi["L"], "far_terms": pi["far_terms"],
                        "near_rows": pi["near_rows"]}
            log(f"mode {m}: {ms:.4f} ms/step")
        modes["fp32bulk"]["speedup_vs_fp64"] = round(modes["fp64"]["ms_per_step"] / modes["fp32bulk"]["ms_per_step"], 3)
        modes["fp32bulk"]["speedup_vs_fp64relaxed_equal_accuracy"] = round(
            modes["fp64relaxed"]["ms_per_step"] / modes["fp32bulk"]["ms_per_step"], 3)
        if B == 1:
            BB = 64
            cb = torch.from_numpy(np.concatenate([wl.coeffs_algebraic(N, 100 + i) for i in range(BB)])).to(dev)
            fb, cb2 = torch.empty_like(cb), torch.empty_like(cb)
            for m in ("fp32bulk", "fp64relaxed"):
                def bstep():
                    pk.dlt_forward(cb, out=fb, prec=m)
                    pk.dlt_inverse(fb, out=cb2, prec=m)

                bstep()
                torch.cuda.synchronize()
                a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(3):
                    bstep()
                b2.record()
                torch.cuda.synchronize()
                bms = a.elapsed_time(b2) / 3
                # the same steps with the kernel trace: rooflines of the batched form
                pk.trace_enable(True)
                for _ in range(3):
                    bstep()
                torch.cuda.synchronize()
                pk.trace_enable(False)
                bk = pk.trace_collect()
                broof, bper, _ = rooflines(pk, bk, N, BB, m)
                bsb = step_bytes(pk, bk, 3, N, BB, m)
                top = sorted(bper.items(), key=lambda kv: -kv[1]["share_of_step"])[:8]
                modes[m + "_batch64"] = {"ms_per_step": round(bms, 3), "transforms_per_s": round(2 * BB * 1000.0 / bms, 2),
                                         "step": "forward DLT + inverse DLT of 64 instances (c_n = N(0,1)/(n+1), "
                                                 "seeds 100..163)",
                                         "roofline": broof,
                                         "step_hbm": {"algorithmic_bytes_per_step": int(bsb),
                                                      "achieved": round(bsb / bms / 1e6, 2), "unit": "GB/s",
                                                      "frac": round(bsb / bms / 1e6 / HBM_PEAK_GBS, 4)},
                                         "roofline_by_kernel": {k: {f: v[f] for f in ("frac", "avg_launch_us",
                                                                                      "instances_per_launch")}
                                                                for k, v in top}}
                log(f"{m} batch 64: {bms:.3f} ms per forward+inverse; dominant kernel {broof}")
                # errors: the forward output of four instances on 4096 sampled
                # outputs against the oracle, and the round trip of all 64
                fbh, cbh = fb.cpu().numpy().reshape(BB, N), cb2.cpu().numpy().reshape(BB, N)
                cbin = cb.cpu().numpy().reshape(BB, N)
                entry = modes[m + "_batch64"]
                # round trip in the inverse transform's norm: |c2_n - c_n| /
                # ((n + 1/2) sum_k w_k |f_k|), max over n and the 64 instances
                wN = pk.leg_nodes_weights(N, theta=False, dtheta=False)[1].cpu().numpy()[0]
                scale = (np.arange(N) + 0.5)[None, :] * np.sum(wN[None, :] * np.abs(fbh), axis=1, keepdims=True)
                entry["roundtrip_error"] = float(np.max(np.abs(cbh - cbin) / scale))
                entry["roundtrip_error_relative"] = float(np.max(np.abs(cbh - cbin)) / np.max(np.abs(cbin)))
                if not args.no_cpu:
                    def check(entry=entry, fbh=fbh, cbin=cbin):
                        import oracle

                        idx = wl.sample_indices(N, 4096, 11)
                        th, _ = oracle.nodes(N, idx=idx)
                        worst = 0.0
                        for i in (0, 21, 42, 63):
                            ref = oracle.dlt(cbin[i], th)
                            worst = max(worst, float(np.max(np.abs(fbh[i][idx] - ref)) / np.sum(np.abs(cbin[i]))))
                        entry["forward_error_vs_oracle"] = worst
                        entry["error_budget"] = 5e-6
                        entry["error_check"] = ("instances 0, 21, 42, 63 on 4096 sampled outputs; the oracle with "
                                                "its own nodes; max |f - f_oracle| / ||c||_1")

                    checks.append(check)
            modes["fp32bulk_batch64"]["speedup_vs_fp64relaxed_equal_accuracy"] = round(
                modes["fp64relaxed_batch64"]["ms_per_step"] / modes["fp32bulk_batch64"]["ms_per_step"], 3)
            del cb, fb, cb2
        # working tolerances (the *_tol entry points, FP64): the same step
        # with the parameters chosen for eps
        tols = {}
        for eps in (1e-12, 1e-9, 1e-6, 1e-3):
            ms = timed_tol(eps, args.steps)
            pi = pk.plan_info(N, tol=eps)
            tols[f"{eps:g}"] = {"ms_per_step": round(ms, 5), "transforms_per_s": round(3 * B * 1000.0 / ms, 2),
                                "L": pi["L"], "far_terms": pi["far_terms"], "near_rows": pi["near_rows"],
                                "speedup_vs_fp64": round(ms_step / ms, 3) if prec == "fp64" else None}
            log(f"tolerance {eps:g}: {ms:.4f} ms/step")
        modes["tolerance"] = tols
        out["modes"] = modes

    # the same step at the smaller sizes of the metric's range (FP64, one
    # instance): these are bound by the chain of dependent launches
    if not args.no_modes and B == 1 and prec == "fp64":
        sizes = {}
        for n in (1 << 12, 1 << 14, 1 << 16, 1 << 18):
            cn = torch.from_numpy(wl.coeffs_algebraic(n, 2)).to(dev)
            fn_ = torch.from_numpy(wl.values_normal(n, 4)).to(dev)
            hn = torch.from_numpy(wl.coeffs_algebraic(n, 3)).to(dev)
            a1, a2, a3 = torch.empty_like(cn), torch.empty_like(cn), torch.empty_like(cn)
            ms = timed("fp64", args.steps, c=cn, fin=fn_, chat=hn, f=a1, c2=a2, g=a3)
            pk.trace_enable(True)
            for _ in range(3):
                step("fp64", c=cn, fin=fn_, chat=hn, f=a1, c2=a2, g=a3)
            torch.cuda.synchronize()
            pk.trace_enable(False)
            kn = pk.trace_collect()
            sbn = step_bytes(pk, kn, 3, n, 1, "fp64")
            sizes[str(n)] = {"ms_per_step": round(ms, 5), "transforms_per_s": round(3000.0 / ms, 2),
                             "kernels_per_step": int(round(sum(v[1] for v in kn.values()) / 3)),
                             "step_hbm": {"algorithmic_bytes_per_step": int(sbn),
                                          "achieved": round(sbn / ms / 1e6, 2), "unit": "GB/s",
                                          "frac": round(sbn / ms / 1e6 / HBM_PEAK_GBS, 4)}}
            log(f"N={n}: {ms:.4f} ms/step", sizes[str(n)])
        out["sizes"] = sizes

    # the evaluation about the other grid theta^cheb* against theta^cheb1:
    # time per call, the kernels' rooflines, and the forward error
    if not args.no_modes and B == 1 and prec == "fp64":
        out["grids"] = grid_runs(pk, wl, torch, np, dev, N, args.steps, checks=None if args.no_cpu else checks)

    if not args.no_ragged and B == 1:
        out["ragged"] = ragged_runs(pk, wl, torch, np, dev, checks=None if args.no_cpu else checks)

    if not args.no_cpu:
        import oracle

        cores = oracle.set_threads(0)
        K = min(args.cpu_sample, N)
        idx = wl.sample_indices(N, K, 5)
        cc = wl.coeffs_algebraic(N, 2)[0]
        t0 = time.perf_counter()
        th, _ = oracle.nodes(N, idx=idx)
        fo = oracle.dlt(cc, th)
        dt = time.perf_counter() - t0
        per_transform = dt * N / len(idx)
        out["cpu_baseline"] = {
            "value": round(1.0 / per_transform, 6), "unit": "transforms/s", "cores": cores, "kind": "oracle",
            "sample": f"forward DLT at N={N}: {len(idx)} of {N} outputs (Newton nodes + direct recurrence sum, "
                      f"FP64 build) in {dt:.2f} s, extrapolated x{N / len(idx):.0f} to one transform"}
        # the same oracle on one host core, on a 16x smaller sample
        oracle.set_threads(1)
        idx1 = wl.sample_indices(N, max(8, K // 16), 5)
        t0 = time.perf_counter()
        th1, _ = oracle.nodes(N, idx=idx1)
        oracle.dlt(cc, th1)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        out["cpu_baseline"]["one_core"] = {
            "value": round(len(idx1) / (dt1 * N), 7), "unit": "transforms/s", "cores": 1,
            "sample": f"{len(idx1)} of {N} outputs in {dt1:.2f} s, extrapolated x{N / len(idx1):.0f}"}
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        log("cpu baseline", out["cpu_baseline"])
        for chk in checks:
            chk()
        # end-to-end error of every mode against the FP64 oracle on the same
        # sampled outputs (the oracle with its own nodes), in ||.||_inf/||c||_1
        if modes:
            c1 = torch.from_numpy(cc[None, :]).to(dev)
            for m in ("fp64", "fp32bulk", "fp64relaxed"):
                fg = pk.dlt_forward(c1, prec=m).cpu().numpy()[0]
                modes[m]["forward_error_vs_oracle"] = float(np.max(np.abs(fg[idx] - fo)) / np.sum(np.abs(cc)))
            log("errors", {m: modes[m]["forward_error_vs_oracle"] for m in ("fp64", "fp32bulk", "fp64relaxed")})
            for key in modes.get("tolerance", {}):
                fg = pk.dlt_forward(c1, tol=float(key)).cpu().numpy()[0]
                modes["tolerance"][key]["forward_error_vs_oracle"] = float(
                    np.max(np.abs(fg[idx] - fo)) / np.sum(np.abs(cc)))
            log("tolerance errors", {k: v.get("forward_error_vs_oracle") for k, v in modes.get("tolerance", {}).items()})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
