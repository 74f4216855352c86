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
    counter summary, or None when there is none or the kernel source has
    changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, prec))
    src_name = "stage_bf16.hip" if prec == "bf16" else "kernels.hip"   # the file holding the level kernels
    src = os.path.join(ROOT, "paper_1301_7744_amd", "csrc", src_name)
    try:
        d = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if d.get("source", "kernels.hip") != src_name or d.get("source_sha256", d.get("kernels_hip_sha256")) != cur:
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    # Plain path: each request alone, timed with events, then a FIFO queue
    # over the same arrivals.
    log("serve: plain path, one request at a time")
    dur = np.zeros(N)
    stream = torch.cuda.current_stream()
    for i, r in enumerate(shapes):
        A, X = inputs(r)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        C, ws = st.sttsm(A, X, r["m"], r["n"], r["p"], r["b"], r["b"], st.PREC_BF16)
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
    roof["kernel"] = "vec_partial_kernel + vec_reduce_kernel (%.3f GFLOP, %.1f MB algorithmic per call)" % (
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

    cfg = synth.workload(args.workload)
    m, n, p, bA, bC = cfg["m"], cfg["n"], cfg["p"], cfg["bA"], cfg["bC"]
    prec = st.PREC_NAMES[args.prec]
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
    if args.prec == "bf16":
        # the bf16 form takes bf16 inputs; the oracle sees the same values
        A_np, X_np = synth.round_to_bf16(A_np), synth.round_to_bf16(X_np)
    tdt = torch.bfloat16 if args.prec == "bf16" else torch.float32
    A_dense = torch.from_numpy(np.ascontiguousarray(A_np.ravel(order="F"))).to(tdt).to(dev)
    X = torch.from_numpy(np.ascontiguousarray(X_np)).to(tdt).to(dev)
    A = st.bcss_pack(A_dense, m, n, bA)
    del A_dense
    if args.op == "sttsm":
        C, ws = st.sttsm(A, X, m, n, p, bA, bC, prec)
        call = lambda: st.sttsm(A, X, m, n, p, bA, bC, prec, C=C, ws=ws)
        nlev = m
    else:
        C, ws = st.sttsm_all_but_one(A, X, m, n, p, bA, bC, prec)
        call = lambda: st.sttsm_all_but_one(A, X, m, n, p, bA, bC, prec, T=C, ws=ws)
        nlev = m - 1
    torch.cuda.synchronize()
    levels = [st.sttsm_plan_info(m, n, p, bA, bC, prec, d, dtype=st.BF16 if args.prec == "bf16" else st.F32)
              for d in range(nlev)]
    flops = sum(lv["flops"] for lv in levels)
    stream = torch.cuda.current_stream()

    log("bench: warmup", args.warmup)
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()

    # Timed region 1 (the reported throughput): K steps, each one replay of
    # a HIP graph holding one whole sttsm call (X panels and every level's
    # kernel), synchronised on both sides.  The graph removes the host's
    # per-launch cost between the kernels; every replay does all the work.
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
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, (time.perf_counter() - t) * 1e3 / args.steps

    eager_step = call
    C_graph = None
    if graph is not None:
        ms_step, wall_ms = timed(graph.replay)
        C_graph = C.clone()
    # Timed region 2: the same K steps launched eagerly, with HIP events
    # recorded on the launch stream around each level's kernel (per-level
    # kernel times for the roofline).
    st.profile_enable(max(16, args.steps * m + 8))
    eager_ms, eager_wall = timed(eager_step)
    prof = st.profile_read(8)
    st.profile_disable()
    if graph is None:
        ms_step, wall_ms = eager_ms, eager_wall
    else:
        torch.cuda.synchronize()
        if not torch.equal(C_graph, C):
            raise RuntimeError("graph replay and eager launches gave different C")
    log("bench: %.4f ms/step (%s; wall %.4f ms/step), eager %.4f ms/step" %
        (ms_step, "graph replay" if graph is not None else "eager", wall_ms, eager_ms))
    gflops = flops / (ms_step * 1e-3) / 1e9

    # Dominant kernel: the level with the largest flop count (the first on
    # ties); its roofline is MFMA or HBM, whichever bounds it by the model
    # time = max(flops / MFMA peak, algorithmic bytes / HBM peak).
    dom = max(range(nlev), key=lambda d: (levels[d]["flops"], -d))
    dom_ms = prof[dom][0] / prof[dom][1]
    peak = PEAK_TFLOPS[args.prec]
    dom_bytes = level_bytes(m, n, p, bA, bC, args.prec, dom)
    t_mfma = levels[dom]["flops"] / (peak * 1e12)
    t_hbm = dom_bytes / (PEAK_HBM_GBS * 1e9)
    if t_mfma >= t_hbm:
        roof = {"bound": "mfma", "achieved": round(levels[dom]["flops"] / (dom_ms * 1e-3) / 1e12, 3), "peak": peak,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(dom_bytes / (dom_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = measured_traffic(args.workload, args.prec, dom)
    roof["kernel"] = "level %d (%.3f GFLOP, %.1f MB algorithmic per launch)" % (dom, levels[dom]["flops"] / 1e9,
                                                                                 dom_bytes / 1e6)
    roof["kernel_us"] = round(dom_ms * 1e3, 3)
    level_times = {str(d): round(prof[d][0] / prof[d][1] * 1e3, 3) for d in range(nlev) if d in prof}

    # Accuracy of this run against the FP64 oracle (also the CPU baseline).
    out = {
        "metric": ("sttsm" if args.op == "sttsm" else "sttsm all-modes-but-one") +
                  " GFLOP/s (symmetry-aware count, Table 2 of the paper)",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "bf16x3_fp32": "bf16x3+f32", "bf16x3_bf16": "bf16x3+bf16"}[args.prec],
        "data": synth.workload_data(args.workload),
        "config": {"workload": args.workload, "m": m, "n": n, "p": p, "bA": bA, "bC": bC, "prec": args.prec,
                   "flops_per_step": flops, "mfma_roofline_frac": round(gflops / (peak * 1e3), 4),
                   "launch": "graph replay" if graph is not None else "eager",
                   "eager_ms_per_step": round(eager_ms, 5),
                   "level_us": level_times},
        "roofline": roof,
    }

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
    for name, ms, nbytes in (("pack", ms_pack, 2 * stored * esz), ("unpack", ms_unpack, (n ** m + stored) * esz)):
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"us": round(ms * 1e3, 2), "algorithmic_mb": round(nbytes / 1e6, 2), "achieved_gbs": round(gbs, 1),
                     "peak_gbs": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4)}
    del dense, A2
    if args.op == "sttsm":
        from math import comb
        C2 = C.clone()
        ms_sym = timed_op(lambda: st.bcss_symmetrize(C2, m, p, bC))
        pbar = -(-p // bC)
        rep_blocks = comb(pbar + m - 1, m) - comb(pbar, m)       # blocks with a repeated index
        nbytes = 2 * rep_blocks * bC ** m * 4
        gbs = nbytes / (ms_sym * 1e-3) / 1e9
        out["symmetrize"] = {"us": round(ms_sym * 1e3, 2), "algorithmic_mb": round(nbytes / 1e6, 2),
                             "achieved_gbs": round(gbs, 1), "peak_gbs": PEAK_HBM_GBS,
                             "frac": round(gbs / PEAK_HBM_GBS, 4)}
        del C2

    if not args.no_cpu_baseline:
        import oracle
        from oracle import bcss_ref
        A64, X64 = A_np.astype(np.float64), X_np.astype(np.float64)
        log("bench: CPU oracle (dense chain, FP64)")
        runs, t_cpu = 0, 0.0
        Cref = None
        ref_fn = oracle.chain if args.op == "sttsm" else oracle.all_but_one
        while t_cpu < args.cpu_seconds and runs < 20:
            t = time.perf_counter()
            Cref = ref_fn(A64, X64)
            t_cpu += time.perf_counter() - t
            runs += 1
        cpu_gflops = flops / (t_cpu / runs) / 1e9
        out["cpu_baseline"] = {"value": round(cpu_gflops, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": "full workload, dense FP64 mode-product chain, %d run(s), %.1f s" % (runs, t_cpu)}
        if args.op == "sttsm":
            nb = st.bcss_num_blocks(m, -(-p // bC))
            got = C.double().cpu().numpy().reshape(nb, bC ** m)
            err = bcss_ref.rel_frobenius_bcss(got, bcss_ref.pack(Cref, bC), m, p, bC)
        else:
            # T in its [J][ibar][block] layout against the oracle's dense T
            nbar, pbar = -(-n // bA), -(-p // bC)
            pad = np.zeros((nbar * bA,) + (pbar * bC,) * (m - 1))
            pad[(slice(0, n),) + tuple(slice(0, p) for _ in range(m - 1))] = Cref
            got = C.double().cpu().numpy()
            num = den = 0.0
            for r, J in enumerate(bcss_ref.sorted_block_tuples(m - 1, pbar)):
                for i in range(nbar):
                    sl = (slice(i * bA, (i + 1) * bA),) + tuple(slice(j * bC, (j + 1) * bC) for j in J)
                    ref = pad[sl].ravel(order="F")
                    num += float(np.sum((got[r, i] - ref) ** 2))
                    den += float(np.sum(ref ** 2))
            err = (num / den) ** 0.5
        out["rel_err_vs_fp64"] = float("%.3e" % err)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
