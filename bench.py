#!/usr/bin/env python3
"""Benchmark: BCSS sttsm  C := [A; X, X, X]  on one MI355X.

Default workload: m=3, n=p=256, bA=bC=16 (816 stored blocks of 16^3), FP32
in/out with FP32 accumulation.  A step is one full sttsm call (padded X
panels, then the three block-contraction levels T^(2), T^(1), C) on inputs
already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|bf16|bf16x3_fp32|bf16x3_bf16]
                    [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3_fp32": 2500.0, "bf16x3_bf16": 2500.0}
PEAK_HBM_GBS = 8000.0
# fp32 FMA on the vector ALUs without packed instructions: 256 CUs x 4 SIMD x
# 16 lanes x 2 flop x 2.4 GHz (packed fp32 would double it; it is disabled).
PEAK_VALU_FP32_TFLOPS = 78.6


def measured_traffic(workload, prec, level):
    """HBM bytes per launch of a level's kernel from the committed rocprofv3
    counter summary, or None when there is none or the level kernels, the
    plan or their shared types have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, prec))
    try:
        d = json.load(open(path))
        if d.get("sources_sha256") != source_digest():
            return None
        e = d["per_level"][str(level)]
        return int(e["fetch_bytes"] + e["write_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def level_bytes(m, n, p, bA, bC, prec, d):
    """Algorithmic HBM bytes of loop level d: its input tensor (A in BCSS, or
    the stored temporary T^(k+1)), the X panel, and its output (T^(k), or C
    in BCSS), each read or written once."""
    from math import comb
    nbar, pbar = -(-n // bA), -(-p // bC)
    k = m - 1 - d
    tbytes = 2 if prec in ("bf16", "bf16x3_bf16") else 4
    in_bytes = 2 if prec == "bf16" else 4

    def temp_elems(kk):   # T^(kk): sorted C-block tuples of length m-kk x sorted prefixes of length kk
        return comb(pbar + m - kk - 1, m - kk) * comb(nbar + kk - 1, kk) * bA ** kk * bC ** (m - kk)
    rd = comb(nbar + m - 1, m) * bA ** m * in_bytes if d == 0 else temp_elems(k + 1) * tbytes
    wr = comb(pbar + m - 1, m) * bC ** m * 4 if k == 0 else temp_elems(k) * tbytes
    return rd + p * n * (2 if prec == "bf16" else 4) + wr


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prec", default="fp32")
    ap.add_argument("--workload", default="m3_n256_b16")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle: no cpu_baseline and no accuracy figures")
    ap.add_argument("--no-bf16", action="store_true", help="FP32 runs: skip the bf16 block on the same workload")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--op", default="sttsm", choices=["sttsm", "all_but_one", "vectors", "rank_update"],
                    help="sttsm, the product in all modes but mode 0, batched vector products, or the "
                         "rank-update form of sttsm")
    ap.add_argument("--rows", default="1,4,16,0",
                    help="--op rank_update: block rows per pass to time (0: all rows in one pass); the first is "
                         "the reported value")
    ap.add_argument("--vectors", type=int, default=64, help="batch size V of --op vectors")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum oracle time for the CPU baseline")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, copy this many MiB device to device once (a plain copy kernel of known "
                         "size, for scaling hardware byte counters)")
    ap.add_argument("--serve", action="store_true", help="run the served mixed-request stream instead")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-window", type=int, default=64, help="outstanding requests in the saturation run")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def serve_bench(args):
    """Served stream: m in {3,4}, n in [32,256], p in [16,n], b = 16 if n >= 128
    else 8, BF16 inputs, FP32 accumulation and output, HBM budget 64 GB.
    (1) saturation: closed loop with a window of outstanding requests gives
    lambda_max; (2) Poisson arrivals at 0.5 and 0.9 lambda_max; (3) the plain
    path, one request at a time on the same arrivals (FIFO), as baseline."""
    import numpy as np
    import torch
    import paper_1301_7744_amd as st
    import synth

    N = args.serve_requests
    shapes = synth.served_stream(N, 11, 1.0)
    flops = np.array([st.sttsm_flops(r["m"], r["n"], r["p"], r["b"], r["b"]) for r in shapes], dtype=np.float64)
    bf = torch.bfloat16

    def inputs(r):
        A = st.bcss_fill_hashed(r["m"], r["n"], r["b"], seed=r["seed_a"], dtype=bf)
        X = torch.from_numpy(synth.change_of_basis(r["p"], r["n"], r["seed_x"])).to(bf).cuda()
        return A, X

    budget = int(args.serve_budget_gb * 2 ** 30)

    # Requests whose C is kept for the accuracy check: small enough for the
    # FP64 oracle chain to take well under a second each.
    sample_ids = [r["id"] for r in shapes if r["n"] ** r["m"] * r["p"] <= 6e8][:12]
    kept = {}

    def run(arrivals, window):
        """Submit in arrival order (open loop: at the arrival times; closed
        loop: keeping `window` outstanding); returns wall time and stats."""
        srv = st.Server(budget, max_inflight=256)
        pending = []
        t0 = time.perf_counter()

        def drain(block):
            """Fetch every finished request (any order); with block, wait
            until at least one has finished."""
            while pending:
                done = []
                for t, rid in pending:
                    st_ = srv.poll(t)
                    if st_ == st.FAILED:
                        raise RuntimeError("served request failed")
                    if st_ == st.DONE:
                        done.append((t, rid))
                for t, rid in done:
                    C = srv.fetch(t)
                    if rid in sample_ids:
                        kept[rid] = C.cpu()
                    pending.remove((t, rid))
                if done or not block:
                    return
                time.sleep(0.00005)

        for i, r in enumerate(shapes):
            if arrivals is not None:
                while time.perf_counter() - t0 < arrivals[i]:
                    drain(False)
                    time.sleep(0.0002)
            else:
                while len(pending) >= window:
                    drain(True)
            A, X = inputs(r)
            pending.append((srv.submit(A, X, r["m"], r["n"], r["p"], r["b"], r["b"], st.PREC_BF16), r["id"]))
            drain(False)
        while pending:
            drain(True)
        wall = time.perf_counter() - t0
        s_ = srv.stats()
        srv.close()
        return wall, s_

    log("serve: warmup")
    keep = shapes
    shapes = keep[:32]
    run(None, 16)
    shapes = keep
    log("serve: saturation, window", args.serve_window)
    wall, sat = run(None, args.serve_window)
    lam = N / wall
    log("serve: lambda_max %.1f req/s, %.1f GFLOP/s" % (lam, flops.sum() / wall / 1e9))
    out = {"saturated": {"req_per_s": round(lam, 2), "gflop_per_s": round(flops.sum() / wall / 1e9, 1),
                         "p50_ms": round(sat["p50_us"] / 1e3, 3), "p99_ms": round(sat["p99_us"] / 1e3, 3),
                         "rounds": sat["rounds"], "launches": sat["launches"]}}
    g = synth.rng(12)
    gaps = g.exponential(1.0, size=N)
    for rho in (0.5, 0.9):
        arr = np.cumsum(gaps) / (rho * lam)
        log("serve: Poisson at %.1f lambda_max" % rho)
        wall, s_ = run(arr, 0)
        out["load_%.1f" % rho] = {"offered_req_per_s": round(rho * lam, 2), "req_per_s": round(N / wall, 2),
                                  "p50_ms": round(s_["p50_us"] / 1e3, 3), "p99_ms": round(s_["p99_us"] / 1e3, 3),
                                  "rounds": s_["rounds"]}
        out["load_%.1f" % rho]["_arrivals"] = arr
    # Plain path: each request alone, timed with events around its kernels
    # only (its plan is built and its C and workspace allocated by a first,
    # untimed call), then a FIFO queue over the same arrivals.
    log("serve: plain path, one request at a time")
    dur = np.zeros(N)
    stream = torch.cuda.current_stream()
    for i, r in enumerate(shapes):
        A, X = inputs(r)
        C, ws = st.sttsm(A, X, r["m"], r["n"], r["p"], r["b"], r["b"], st.PREC_BF16)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.sttsm(A, X, r["m"], r["n"], r["p"], r["b"], r["b"], st.PREC_BF16, C=C, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        dur[i] = e0.elapsed_time(e1) * 1e-3
        del A, X, C, ws
    plain = {"req_per_s_saturated": round(N / dur.sum(), 2), "gflop_per_s": round(flops.sum() / dur.sum() / 1e9, 1)}
    # Accuracy of served results: sampled requests against the FP64 oracle on
    # the same bf16 inputs, and bit for bit against the plain path.
    import oracle
    from oracle import bcss_ref
    errs, same = [], 0
    for rid in sample_ids:
        r = keep[rid]
        m, n, p, b = r["m"], r["n"], r["p"], r["b"]
        A64 = synth.round_to_bf16(synth.hashed_symmetric(m, n, r["seed_a"]).astype(np.float32)).astype(np.float64)
        X64 = synth.round_to_bf16(synth.change_of_basis(p, n, r["seed_x"])).astype(np.float64)
        nb = st.bcss_num_blocks(m, -(-p // b))
        got = kept[rid].double().numpy().reshape(nb, b ** m)
        ref = bcss_ref.pack(oracle.chain(A64, X64), b)
        errs.append((bcss_ref.rel_frobenius_bcss(got, ref, m, p, b), (2 * m) ** 0.5 * 2.0 ** -8))
        A, X = inputs(r)
        Cp, _ = st.sttsm(A, X, m, n, p, b, b, st.PREC_BF16)
        same += int(torch.equal(Cp.cpu(), kept[rid]))
    accuracy = {"sampled_requests": len(sample_ids),
                "max_rel_err_vs_fp64": float("%.3e" % max(e for e, _ in errs)),
                "within_bf16_bound": sum(int(e <= t) for e, t in errs),
                "bitwise_equal_to_plain": same}
    for rho in (0.5, 0.9):
        arr = out["load_%.1f" % rho].pop("_arrivals")
        t_free, lat = 0.0, np.zeros(N)
        for i in range(N):
            start = max(arr[i], t_free)
            t_free = start + dur[i]
            lat[i] = t_free - arr[i]
        plain["load_%.1f" % rho] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                    "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                                    "req_per_s": round(N / t_free, 2)}
    res = {
        "metric": "served sttsm stream: requests/s and p50/p99 latency (continuous batching)",
        "value": out["saturated"]["req_per_s"],
        "unit": "req/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (m in {3,4}, n in [32,256], p in [16,n], hashed symmetric A, X N(0,1)/sqrt(n))",
        "config": {"workload": "served_mixed_stream", "requests": N, "budget_gb": args.serve_budget_gb,
                   "window": args.serve_window, "total_gflop": round(flops.sum() / 1e9, 1)},
        "served": out,
        "plain_one_at_a_time": plain,
        "accuracy": accuracy,
    }
    print(json.dumps(res), flush=True)


def vectors_bench(args):
    """Batched y_v = A x_v^(m-1), s_v = A x_v^m on a named workload's A."""
    import numpy as np
    import torch
    import paper_1301_7744_amd as st
    import synth
    cfg = synth.workload(args.workload)
    m, n, b, V = cfg["m"], cfg["n"], cfg["bA"], args.vectors
    dev = torch.device("cuda:0")
    A_np, _ = synth.make_config_inputs(args.workload)
    X_np = synth.rng((n, V, 97)).standard_normal((V, n)).astype(np.float32) / np.sqrt(n)
    tdt = torch.float32
    if args.prec == "bf16":
        A_np, X_np, tdt = synth.round_to_bf16(A_np), synth.round_to_bf16(X_np), torch.bfloat16
    A = st.bcss_pack(torch.from_numpy(np.ascontiguousarray(A_np.ravel(order="F"))).to(tdt).to(dev), m, n, b)
    X = torch.from_numpy(X_np).to(tdt).to(dev)
    y, s, ws = st.sttsm_vectors(A, X, m, n, b)
    call = lambda: st.sttsm_vectors(A, X, m, n, b, y=y, s=s, ws=ws)
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        call()
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps
    ms = timed(graph.replay)
    ms_eager = timed(call)
    flops = st.sttsm_vectors_flops(m, n, b, V)
    esz = 2 if args.prec == "bf16" else 4
    nbytes = st.bcss_num_elems(m, n, b) * esz + V * n * (esz + 4) + V * 4
    t_alu = flops / (PEAK_VALU_FP32_TFLOPS * 1e12)
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(flops / (ms * 1e-3) / 1e12, 3), "peak": PEAK_VALU_FP32_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = None
    kernels = ("vec_block3_kernel + vec_rows_kernel + vec_dot_kernel" if m == 3 and b in (4, 8, 16)
               else "vec_partial_kernel + vec_reduce_kernel")
    roof["kernel"] = kernels + " (%.3f GFLOP, %.1f MB algorithmic per call)" % (
        flops / 1e9, nbytes / 1e6)
    out = {"metric": "batched vector products A x^(m-1), A x^m GFLOP/s (each stored term once)",
           "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16" if args.prec == "bf16" else "f32", "data": "synthetic",
           "config": {"workload": args.workload + "_V%d" % V, "m": m, "n": n, "b": b, "vectors": V,
                      "launch": "graph replay", "eager_ms_per_step": round(ms_eager, 5)},
           "roofline": roof}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        Y, S = oracle.vectors(A_np.astype(np.float64), X_np.astype(np.float64))
        t_cpu = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(flops / t_cpu / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": "full batch, dense FP64 mode products per vector, %.1f s" % t_cpu}
        out["rel_err_vs_fp64"] = float("%.3e" % (np.linalg.norm(y.double().cpu().numpy() - Y) / np.linalg.norm(Y)))
    print(json.dumps(out), flush=True)


def rank_update_bench(args):
    """The rank-update form (passes of block rows, each a rank update of C)
    against the chain on the same inputs: the chain on the generic kernels
    (the same kernels the form runs on) and on the default kernels, each
    captured in a HIP graph and replayed K times."""
    import numpy as np
    import torch
    import paper_1301_7744_amd as st
    import synth
    cfg = synth.workload(args.workload)
    m, n, p, bA, bC = cfg["m"], cfg["n"], cfg["p"], cfg["bA"], cfg["bC"]
    prec = st.PREC_NAMES[args.prec]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("bench: generating inputs", args.workload)
    A_np, X_np = synth.make_config_inputs(args.workload)
    tdt = torch.float32
    if args.prec == "bf16":
        A_np, X_np, tdt = synth.round_to_bf16(A_np), synth.round_to_bf16(X_np), torch.bfloat16
    A = st.bcss_pack(torch.from_numpy(np.ascontiguousarray(A_np.ravel(order="F"))).to(tdt).to(dev), m, n, bA)
    X = torch.from_numpy(np.ascontiguousarray(X_np)).to(tdt).to(dev)
    nbar = -(-n // bA)
    flops = st.sttsm_flops(m, n, p, bA, bC)
    stream = torch.cuda.current_stream()

    def graph_ms(call):
        for _ in range(max(1, args.warmup)):
            call()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            call()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    rows_list = [int(r) if int(r) > 0 else nbar for r in args.rows.split(",")]
    sweep = {}
    C_main = None
    for rows in rows_list:
        C, ws = st.sttsm_rank_update(A, X, m, n, p, bA, bC, prec, rows)
        ms = graph_ms(lambda: st.sttsm_rank_update(A, X, m, n, p, bA, bC, prec, rows, C=C, ws=ws))
        sweep[str(rows)] = {"ms": round(ms, 5), "passes": -(-nbar // rows), "workspace_mb": round(ws.numel() / 1e6, 2)}
        log("bench: rank update, %d rows per pass: %.4f ms" % (rows, ms))
        if C_main is None:
            C_main = C.clone()
        del C, ws
    os.environ["STTSM_GENERIC_KERNELS"] = "1"
    try:
        Cg, wsg = st.sttsm(A, X, m, n, p, bA, bC, prec)
        ms_gen = graph_ms(lambda: st.sttsm(A, X, m, n, p, bA, bC, prec, C=Cg, ws=wsg))
    finally:
        del os.environ["STTSM_GENERIC_KERNELS"]
    Cd, wsd = st.sttsm(A, X, m, n, p, bA, bC, prec)
    ms_def = graph_ms(lambda: st.sttsm(A, X, m, n, p, bA, bC, prec, C=Cd, ws=wsd))
    log("bench: chain %.4f ms (generic kernels), %.4f ms (default kernels)" % (ms_gen, ms_def))
    ms = sweep[str(rows_list[0])]["ms"]
    peak = PEAK_TFLOPS[args.prec]
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"metric": "sttsm rank-update form GFLOP/s (symmetry-aware count, Table 2 of the paper)",
           "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16" if args.prec == "bf16" else "f32",
           "data": synth.workload_data(args.workload),
           "config": {"workload": args.workload + "_rows%d" % rows_list[0], "m": m, "n": n, "p": p, "bA": bA,
                      "bC": bC, "prec": args.prec, "rows_per_pass": rows_list[0], "launch": "graph replay"},
           "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                        "frac": round(achieved / peak, 4), "traffic": None,
                        "kernel": "whole step (every pass's two generic-kernel launches)"},
           "rows_sweep": sweep,
           "chain": {"generic_kernels_ms": round(ms_gen, 5), "default_kernels_ms": round(ms_def, 5),
                     "workspace_mb": round(wsd.numel() / 1e6, 2),
                     "generic_workspace_mb": round(wsg.numel() / 1e6, 2)}}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import bcss_ref
        t = time.perf_counter()
        Cref = oracle.rank_update(A_np.astype(np.float64), X_np.astype(np.float64), bA, rows_list[0])
        t_cpu = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(flops / t_cpu / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": "full workload, dense FP64 rank-update form, 1 run, %.1f s" % t_cpu}
        nb = st.bcss_num_blocks(m, -(-p // bC))
        got = C_main.double().cpu().numpy().reshape(nb, bC ** m)
        out["rel_err_vs_fp64"] = float("%.3e" % bcss_ref.rel_frobenius_bcss(got, bcss_ref.pack(Cref, bC), m, p, bC))
    print(json.dumps(out), flush=True)


# Relative error per operand of each precision form (the unit of the
# entry-by-entry error scale): bf16 rounding, the two-term bf16 split of an
# fp32 value, FP32 accumulation over Kpad terms (added in accuracy()).
UNIT = {"fp32": 0.0, "bf16": 2.0 ** -9, "bf16x3_fp32": 2.0 ** -17, "bf16x3_bf16": 2.0 ** -9}
DTYPE_NAME = {"fp32": "f32", "bf16": "bf16", "bf16x3_fp32": "bf16x3+f32", "bf16x3_bf16": "bf16x3+bf16"}


def source_digest():
    """sha256 over the sources that decide the level kernels' HBM traffic:
    the kernels, the plan (tiles, task order, tail splits) and their shared
    types."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "stage_bf16.hip", "stage_b64.hip", "plan.cpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1301_7744_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measure(args, prec_name, A_np, X_np, op="sttsm", timing_steps=None):
    """Times one precision form of the operation on the given inputs (K
    graph replays with an event at every step boundary, then K eager steps
    with per-level events) and returns its figures and the result."""
    import numpy as np
    import torch
    import paper_1301_7744_amd as st
    import synth
    cfg = synth.workload(args.workload)
    m, n, p, bA, bC = cfg["m"], cfg["n"], cfg["p"], cfg["bA"], cfg["bC"]
    prec = st.PREC_NAMES[prec_name]
    dev = torch.device("cuda:0")
    steps = timing_steps or args.steps
    if prec_name == "bf16":
        # the bf16 form takes bf16 inputs; the oracle sees the same values
        A_np, X_np = synth.round_to_bf16(A_np), synth.round_to_bf16(X_np)
    tdt = torch.bfloat16 if prec_name == "bf16" else torch.float32
    A_dense = torch.from_numpy(np.ascontiguousarray(A_np.ravel(order="F"))).to(tdt).to(dev)
    X = torch.from_numpy(np.ascontiguousarray(X_np)).to(tdt).to(dev)
    A = st.bcss_pack(A_dense, m, n, bA)
    del A_dense
    if op == "sttsm":
        C, ws = st.sttsm(A, X, m, n, p, bA, bC, prec)
        call = lambda: st.sttsm(A, X, m, n, p, bA, bC, prec, C=C, ws=ws)
        nlev = m
    else:
        C, ws = st.sttsm_all_but_one(A, X, m, n, p, bA, bC, prec)
        call = lambda: st.sttsm_all_but_one(A, X, m, n, p, bA, bC, prec, T=C, ws=ws)
        nlev = m - 1
    torch.cuda.synchronize()
    levels = [st.sttsm_plan_info(m, n, p, bA, bC, prec, d, dtype=st.BF16 if prec_name == "bf16" else st.F32)
              for d in range(nlev)]
    flops = sum(lv["flops"] for lv in levels)
    stream = torch.cuda.current_stream()

    log("bench: %s warmup %d" % (prec_name, args.warmup))
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()

    # Timed region 1 (the reported throughput): K steps, each one replay of
    # a HIP graph holding one whole call (X panels and every level's
    # kernel), synchronised on both sides, with an event at every step
    # boundary (per-step times: median, p10, p90).  The graph removes the
    # host's per-launch cost between the kernels; every replay does all the
    # work.
    graph = None
    if not args.eager:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            call()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            call()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()

    def timed(step):
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t = time.perf_counter()
        ev[0].record(stream)
        for i in range(steps):
            step()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) * 1e3 / steps
        per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
        return ev[0].elapsed_time(ev[steps]) / steps, wall, per

    C_graph = None
    per = None
    if graph is not None:
        ms_step, wall_ms, per = timed(graph.replay)
        C_graph = C.clone()
    # Timed region 2: the same K steps launched eagerly, with HIP events
    # recorded on the launch stream around each level's kernel (per-level
    # kernel times for the roofline).
    st.profile_enable(max(16, steps * m + 8))
    eager_ms, eager_wall, eager_per = timed(call)
    prof = st.profile_read(8)
    st.profile_disable()
    if graph is None:
        ms_step, wall_ms, per = eager_ms, eager_wall, eager_per
    else:
        torch.cuda.synchronize()
        if not torch.equal(C_graph, C):
            raise RuntimeError("graph replay and eager launches gave different C")
    log("bench: %s %.4f ms/step (%s; wall %.4f ms/step), eager %.4f ms/step" %
        (prec_name, ms_step, "graph replay" if graph is not None else "eager", wall_ms, eager_ms))

    # Dominant kernel: the level with the largest flop count (the first on
    # ties); its roofline is MFMA or HBM, whichever bounds it by the model
    # time = max(flops / MFMA peak, algorithmic bytes / HBM peak).
    dom = max(range(nlev), key=lambda d: (levels[d]["flops"], -d))
    dom_ms = prof[dom][0] / prof[dom][1]
    peak = PEAK_TFLOPS[prec_name]
    dom_bytes = level_bytes(m, n, p, bA, bC, prec_name, dom)
    t_mfma = levels[dom]["flops"] / (peak * 1e12)
    t_hbm = dom_bytes / (PEAK_HBM_GBS * 1e9)
    if t_mfma >= t_hbm:
        roof = {"bound": "mfma", "achieved": round(levels[dom]["flops"] / (dom_ms * 1e-3) / 1e12, 3), "peak": peak,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(dom_bytes / (dom_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = measured_traffic(args.workload, prec_name, dom)
    roof["kernel"] = "level %d (%.3f GFLOP, %.1f MB algorithmic per launch)" % (dom, levels[dom]["flops"] / 1e9,
                                                                                 dom_bytes / 1e6)
    roof["kernel_us"] = round(dom_ms * 1e3, 3)
    level_times = {str(d): round(prof[d][0] / prof[d][1] * 1e3, 3) for d in range(nlev) if d in prof}
    res = {"prec": prec_name, "ms_per_step": round(ms_step, 5),
           "step_ms": {"median": round(float(np.median(per)), 5), "p10": round(float(np.percentile(per, 10)), 5),
                       "p90": round(float(np.percentile(per, 90)), 5)},
           "tflops": round(flops / (ms_step * 1e-3) / 1e12, 3),
           "mfma_roofline_frac": round(flops / (ms_step * 1e-3) / 1e12 / peak, 4),
           "launch": "graph replay" if graph is not None else "eager",
           "eager_ms_per_step": round(eager_ms, 5), "level_us": level_times, "roofline": roof,
           "flops_per_step": flops}
    if prec_name.startswith("bf16x3"):
        # the split first level issues three bf16 products per flop of Table 2
        issued = flops + 2 * levels[0]["flops"]
        res["mfma_issued_flops_per_step"] = issued
        res["mfma_issued_tflops"] = round(issued / (ms_step * 1e-3) / 1e12, 3)
        res["mfma_issued_frac"] = round(issued / (ms_step * 1e-3) / 1e12 / peak, 4)
    return res, dict(A=A, X=X, C=C, A_np=A_np, X_np=X_np, m=m, n=n, p=p, bA=bA, bC=bC, tdt=tdt, stream=stream)


def accuracy(res, ctx, prec_name, op="sttsm"):
    """Errors of the result against the FP64 oracle on the same input values:
    relative Frobenius error over the dense tensor, max |error| / max |C|,
    the largest |error_j| / (u S_j) with S_j the oracle's per-entry error
    scale and u the form's relative error per operand, and the largest
    difference between mirrored entries inside blocks with repeated indices
    (computed one by one, §5.4), relative to max |C|."""
    import itertools
    import numpy as np
    import oracle
    import paper_1301_7744_amd as st
    from oracle import bcss_ref
    m, n, p, bA, bC = ctx["m"], ctx["n"], ctx["p"], ctx["bA"], ctx["bC"]
    A64, X64 = ctx["A_np"].astype(np.float64), ctx["X_np"].astype(np.float64)
    if op != "sttsm":
        Tref = oracle.all_but_one(A64, X64)
        nbar, pbar = -(-n // bA), -(-p // bC)
        pad = np.zeros((nbar * bA,) + (pbar * bC,) * (m - 1))
        pad[(slice(0, n),) + tuple(slice(0, p) for _ in range(m - 1))] = Tref
        got = ctx["C"].double().cpu().numpy()
        num = den = 0.0
        for r, J in enumerate(bcss_ref.sorted_block_tuples(m - 1, pbar)):
            for i in range(nbar):
                sl = (slice(i * bA, (i + 1) * bA),) + tuple(slice(j * bC, (j + 1) * bC) for j in J)
                ref = pad[sl].ravel(order="F")
                num += float(np.sum((got[r, i] - ref) ** 2))
                den += float(np.sum(ref ** 2))
        res["rel_err_vs_fp64"] = float("%.3e" % (num / den) ** 0.5)
        return
    Cref, temps = oracle.chain(A64, X64, keep_temps=True)
    S = oracle.error_scale(A64, X64, temps=temps)
    del temps
    nb = st.bcss_num_blocks(m, -(-p // bC))
    got = ctx["C"].double().cpu().numpy().reshape(nb, bC ** m)
    refb, Sb = bcss_ref.pack(Cref, bC), bcss_ref.pack(S, bC)
    res["rel_err_vs_fp64"] = float("%.3e" % bcss_ref.rel_frobenius_bcss(got, refb, m, p, bC))
    cmax = float(np.abs(Cref).max())
    d = np.abs(got - refb)
    res["max_abs_err_over_cmax"] = float("%.3e" % (d.max() / cmax))
    u = UNIT[prec_name] + 2.0 ** -24 * (-(-n // bA) * bA) ** 0.5
    nz = Sb > 0
    res["max_err_over_u_scale"] = round(float((d[nz] / (u * Sb[nz])).max()), 3)
    res["entry_bound"] = "|err_j| <= 16 u S_j, u = %.3g" % u
    D = bcss_ref.unpack(got, m, p, bC)
    asym = 0.0
    for q in itertools.permutations(range(m)):
        asym = max(asym, float(np.abs(D - np.transpose(D, q)).max()))
    res["max_intrablock_asymmetry_over_cmax"] = float("%.3e" % (asym / cmax))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sttsm path here is built and timed on a single MI355X; "
              "multi-GPU sharding is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        return serve_bench(args)
    if args.op == "vectors":
        return vectors_bench(args)
    if args.op == "rank_update":
        return rank_update_bench(args)

    import numpy as np
    import torch
    import paper_1301_7744_amd as st
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy_mb > 0:
        src = torch.ones(args.calibrate_copy_mb * 2 ** 20 // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of %d MiB done" % args.calibrate_copy_mb)
        del src, dst

    log("bench: generating inputs", args.workload)
    A_np, X_np = synth.make_config_inputs(args.workload)
    res, ctx = measure(args, args.prec, A_np, X_np, op=args.op)
    m, n, p, bA, bC = ctx["m"], ctx["n"], ctx["p"], ctx["bA"], ctx["bC"]
    A, C, tdt, stream = ctx["A"], ctx["C"], ctx["tdt"], ctx["stream"]
    ms_step = res["ms_per_step"]
    flops = res["flops_per_step"]
    out = {
        "metric": ("sttsm" if args.op == "sttsm" else "sttsm all-modes-but-one") +
                  " GFLOP/s (symmetry-aware count, Table 2 of the paper)",
        "value": round(flops / (ms_step * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[args.prec],
        "data": synth.workload_data(args.workload),
        "config": {"workload": args.workload, "m": m, "n": n, "p": p, "bA": bA, "bC": bC, "prec": args.prec,
                   "flops_per_step": flops, "mfma_roofline_frac": res["mfma_roofline_frac"],
                   "launch": res["launch"], "eager_ms_per_step": res["eager_ms_per_step"],
                   "level_us": res["level_us"]},
        "step_ms": res["step_ms"],
        "roofline": res["roofline"],
    }
    for k in ("mfma_issued_flops_per_step", "mfma_issued_tflops", "mfma_issued_frac"):
        if k in res:
            out["config"][k] = res[k]

    # Pack and unpack (HBM-bound copies through the block layout), timed
    # apart from the step: K calls each, HIP events around the loop.
    def timed_op(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps
    esz = 2 if args.prec == "bf16" else 4
    dense = torch.empty(n ** m, dtype=tdt, device=dev)
    st.bcss_unpack(A, m, n, bA, out=dense)
    A2 = torch.empty_like(A)
    stored = st.bcss_num_elems(m, n, bA, st.BF16 if args.prec == "bf16" else st.F32)
    ms_pack = timed_op(lambda: st.bcss_pack(dense, m, n, bA, out=A2))
    ms_unpack = timed_op(lambda: st.bcss_unpack(A, m, n, bA, out=dense))
    torch.cuda.synchronize()
    if not torch.equal(A2, A):
        raise RuntimeError("pack(unpack(A)) differs from A")
    # Yardstick: a plain device copy of the same bytes (the BCSS array for
    # pack; the dense tensor, whose bytes dominate, for unpack).
    A3 = torch.empty_like(A)
    dense2 = torch.empty_like(dense)
    ms_copy_pack = timed_op(lambda: A3.copy_(A))
    ms_copy_unpack = timed_op(lambda: dense2.copy_(dense))
    del A3, dense2
    for name, ms, nbytes, ms_copy, copy_bytes in (
            ("pack", ms_pack, 2 * stored * esz, ms_copy_pack, 2 * stored * esz),
            ("unpack", ms_unpack, (n ** m + stored) * esz, ms_copy_unpack, 2 * n ** m * esz)):
        gbs = nbytes / (ms * 1e-3) / 1e9
        copy_gbs = copy_bytes / (ms_copy * 1e-3) / 1e9
        out[name] = {"us": round(ms * 1e3, 2), "algorithmic_mb": round(nbytes / 1e6, 2), "achieved_gbs": round(gbs, 1),
                     "peak_gbs": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4),
                     "plain_copy": {"us": round(ms_copy * 1e3, 2), "mb": round(copy_bytes / 1e6, 2),
                                    "gbs": round(copy_gbs, 1)},
                     "frac_of_plain_copy_gbs": round(gbs / copy_gbs, 4)}
    del dense, A2
    if args.op == "sttsm":
        from math import comb
        C2 = C.clone()
        ms_sym = timed_op(lambda: st.bcss_symmetrize(C2, m, p, bC))
        pbar = -(-p // bC)
        rep_blocks = comb(pbar + m - 1, m) - comb(pbar, m)       # blocks with a repeated index
        nbytes = 2 * rep_blocks * bC ** m * 4
        gbs = nbytes / (ms_sym * 1e-3) / 1e9
        # Yardstick: a plain device copy of the repeated-index blocks' bytes.
        src = torch.empty(rep_blocks * bC ** m, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        ms_copy_sym = timed_op(lambda: dst.copy_(src))
        copy_gbs = nbytes / (ms_copy_sym * 1e-3) / 1e9
        del src, dst
        out["symmetrize"] = {"us": round(ms_sym * 1e3, 2), "algorithmic_mb": round(nbytes / 1e6, 2),
                             "achieved_gbs": round(gbs, 1), "peak_gbs": PEAK_HBM_GBS,
                             "frac": round(gbs / PEAK_HBM_GBS, 4),
                             "plain_copy": {"us": round(ms_copy_sym * 1e3, 2), "mb": round(nbytes / 1e6, 2),
                                            "gbs": round(copy_gbs, 1)},
                             "frac_of_plain_copy_gbs": round(gbs / copy_gbs, 4)}
        del C2

    # The bf16 form on the same workload, reported beside the FP32 line.
    other = None
    if args.op == "sttsm" and args.prec == "fp32" and not args.no_bf16:
        other, octx = measure(args, "bf16", A_np, X_np)

    if not args.no_cpu_baseline:
        import oracle
        log("bench: accuracy against the FP64 oracle")
        accuracy(out, ctx, args.prec, args.op)
        if other is not None:
            accuracy(other, octx, "bf16")
        A64, X64 = A_np.astype(np.float64), X_np.astype(np.float64)
        log("bench: CPU oracle (dense chain, FP64)")
        ref_fn = oracle.chain if args.op == "sttsm" else oracle.all_but_one
        threads = oracle.num_threads()
        runs, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds and runs < 20:
            t = time.perf_counter()
            ref_fn(A64, X64)
            t_cpu += time.perf_counter() - t
            runs += 1
            log("bench: CPU oracle run %d: %.2f s" % (runs, time.perf_counter() - t))
        cpu_gflops = flops / (t_cpu / runs) / 1e9
        # one thread, one run when that is expected to take under a minute
        # (else null); and the literal sum (O1) on the small configuration
        # m3_n16_b4, all threads
        t_one = None
        if t_cpu / runs * threads <= 60.0:
            log("bench: CPU oracle, one thread")
            oracle.set_num_threads(1)
            t = time.perf_counter()
            ref_fn(A64, X64)
            t_one = time.perf_counter() - t
            oracle.set_num_threads(threads)
        A1, X1 = synth.make_config_inputs("m3_n16_b4")
        t = time.perf_counter()
        oracle.direct_sum(A1.astype(np.float64), X1.astype(np.float64))
        t_o1 = time.perf_counter() - t
        dense_flops = 2 * sum(p ** (i + 1) * n ** (m - i) for i in range(m if args.op == "sttsm" else m - 1))
        out["cpu_baseline"] = {
            "value": round(cpu_gflops, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "full workload, dense FP64 mode-product chain (%.1f GFLOP of dense work per run; the "
                      "value divides Table 2's count by its time), %d run(s), %.1f s" % (dense_flops / 1e9, runs,
                                                                                        t_cpu),
            "cpu_model": cpu_model(),
            "one_thread_gflops": round(flops / t_one / 1e9, 3) if t_one else None,
            "one_thread_s": round(t_one, 2) if t_one else None,
            "o1_direct_sum_m3_n16_b4_s": round(t_o1, 4)}
    if other is not None:
        out["bf16"] = other
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
