#!/usr/bin/env python3
"""Benchmark of the Bolt hot path on one MI355X.

Workload (single-database scan): N = 1,000,000 database vectors of J = 128
dimensions from the 256-component Gaussian mixture, M = 32 subspaces (16-byte
codes), Q = 1,000 queries, squared-L2 and dot-product tables, top-100.

One step is one pass of the whole hot path over that batch, inputs resident
in HBM: encode all N vectors, build the uint8 tables of the Q queries for both
metrics, scan + top-100 for both metrics.  The reported value is the number
of (query, vector) distances produced per second over the whole step, summed
over both metrics.

Printed: one JSON line (rank 0).  Per-kernel durations come from HIP events
recorded on the launch stream around each call inside the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
VALU_LANE_OPS = 256 * 64 * 2.4e9  # CUs x lanes x clock: 32-bit VALU lane-ops/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--N", type=int, default=1_000_000)
    p.add_argument("--J", type=int, default=128)
    p.add_argument("--M", type=int, default=32)
    p.add_argument("--Q", type=int, default=1000)
    p.add_argument("--k", type=int, default=100)
    p.add_argument("--n-train", type=int, default=100_000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-rows", type=int, default=20_000)
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the scan shards by database rows; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import synth.device as sdev
    import paper_1706_10283_amd.bolt as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, J, M, Q, k = args.N, args.J, args.M, args.Q, args.k
    cfg = 2
    mix_seed = synth.seed_for(cfg, 0)

    # ---------------- inputs (synthetic, generated in HBM) and offline training
    t0 = time.time()
    X = sdev.gmm_rows(mix_seed, synth.seed_for(cfg, 1), 0, N, J)
    Qd = sdev.gmm_rows(mix_seed, synth.seed_for(cfg, 2), 0, Q, J)
    Xtr = sdev.gmm_rows(mix_seed, synth.seed_for(cfg, 3), 0, args.n_train, J).cpu().numpy()
    init = synth.permutation_prefix(synth.seed_for(cfg, 4), args.n_train, 16)
    Qt = Xtr[synth.permutation_prefix(synth.seed_for(cfg, 5), args.n_train, 1000)]
    C, a_l2, off_l2, _ = B.bolt_train_host(Xtr, M, 10, init, Qt, "l2")
    tr_codes = B.bolt_encode(torch.from_numpy(Xtr).to(dev), torch.from_numpy(C).to(dev), M).cpu().numpy()
    a_dot, off_dot, _ = B.bolt_learn_quantizer_host(Qt, tr_codes, C, "dot")
    log("inputs + training: %.1fs" % (time.time() - t0))
    Cd = torch.from_numpy(C).to(dev)
    offd = {"l2": torch.from_numpy(off_l2).to(dev), "dot": torch.from_numpy(off_dot).to(dev)}
    scale = {"l2": a_l2, "dot": a_dot}

    codes = torch.empty((N, M // 2), dtype=torch.uint8, device=dev)
    luts = {m: torch.empty((Q, M, 16), dtype=torch.uint8, device=dev) for m in ("l2", "dot")}
    vals = {m: torch.empty((Q, k), dtype=torch.uint16, device=dev) for m in ("l2", "dot")}
    idx = {m: torch.empty((Q, k), dtype=torch.int32, device=dev) for m in ("l2", "dot")}
    ws = torch.empty(B.bolt_scan_topk_ws_bytes(N, M, Q, k), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    names = ["encode", "luts_l2", "luts_dot", "scan_topk_l2", "scan_topk_dot"]
    ev = {n: [] for n in names}

    def step(record):
        def mark(name, fn):
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                ev[name].append((e0, e1))
            else:
                fn()
        mark("encode", lambda: B.bolt_encode(X, Cd, M, codes=codes))
        for m in ("l2", "dot"):
            mark("luts_" + m, lambda m=m: B.bolt_build_luts(Qd, Cd, M, m, scale[m], offd[m], luts_u8=luts[m]))
        for m in ("l2", "dot"):
            mark("scan_topk_" + m, lambda m=m: B.bolt_scan_topk(codes, luts[m], m, k, vals=vals[m],
                                                                idx=idx[m], ws=ws))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    kern_ms = {n: float(np.mean([a.elapsed_time(b) for a, b in ev[n]])) for n in names}
    dists = 2.0 * Q * N
    value = dists / (ms_per_step * 1e-3) / 1e9

    enc_bytes = 4.0 * N * J + N * M / 2
    scan_lookups = Q * N * M
    scan_ms = 0.5 * (kern_ms["scan_topk_l2"] + kern_ms["scan_topk_dot"])
    result = {
        "metric": "G distances/sec scanned + encode GB/s; p50/p99 latency vs plain per-query scan",
        "value": round(value, 3),
        "unit": "G distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single-database scan: N=%d x J=%d Gaussian-mixture rows, M=%d "
                               "(%d B codes), Q=%d queries, L2 + dot tables, top-%d"
                               % (N, J, M, M // 2, Q, k),
                   "N": N, "J": J, "M": M, "Q": Q, "k": k},
        "encode_GBps": round(4.0 * N * J / (kern_ms["encode"] * 1e-3) / 1e9, 1),
        "kernel_ms": {n: round(v, 4) for n, v in kern_ms.items()},
        "scan_topk_G_distances_per_s": round(Q * N / (scan_ms * 1e-3) / 1e9, 2),
    }
    lookups_per_s = scan_lookups / (scan_ms * 1e-3)
    result["roofline"] = {
        "bound": "alu",
        "kernel": "scan_topk (u8 lookups)",
        "achieved": round(lookups_per_s / 1e12, 3),
        "peak": round(VALU_LANE_OPS / 1e12, 2),
        "unit": "T lookups/s",
        "frac": round(lookups_per_s / VALU_LANE_OPS, 4),
        "traffic": None,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, C, a_l2, off_l2, a_dot, off_dot,
                                              Qd.cpu().numpy(), mix_seed)
    print(json.dumps(result), flush=True)


def cpu_baseline(args, C, a_l2, off_l2, a_dot, off_dot, Qv, mix_seed):
    """The oracle as it stands, one host thread, on a bounded sample of the
    same workload (the first rows of the database, all queries, both metrics)."""
    import oracle
    import synth
    n = args.cpu_sample_rows
    M, k = args.M, args.k
    X = synth.gmm_rows(mix_seed, synth.seed_for(2, 1), 0, n, args.J)
    t0 = time.perf_counter()
    codes = oracle.encode(X, C, M)
    for metric, a, off in (("l2", a_l2, off_l2), ("dot", a_dot, off_dot)):
        _, _, l8 = oracle.luts(Qv, C, M, metric, a, off)
        S = oracle.scan(codes, l8)
        oracle.topk(S, k, metric == "dot")
    dt = time.perf_counter() - t0
    return {"value": round(2.0 * Qv.shape[0] * n / dt / 1e9, 5), "unit": "G distances/s", "cores": 1,
            "kind": "oracle",
            "sample": "first %d of %d rows, all %d queries, L2 + dot, encode + tables + scan + top-%d; "
                      "%.1f s" % (n, args.N, Qv.shape[0], k, dt)}


if __name__ == "__main__":
    main()
