#!/usr/bin/env python3
"""Benchmark of the Bolt hot path on one MI355X.

Headline workload (single-database scan): N = 1,000,000 database vectors of
J = 128 dimensions from the 256-component Gaussian mixture, M = 32 subspaces
(16-byte codes), Q = 1,000 queries, squared-L2 and dot-product tables,
top-100.  One step is one pass of the whole hot path over that batch with
inputs resident in HBM: encode all N vectors, build the uint8 tables of the
Q queries for both metrics, scan + top-100 for both metrics.  `value` is the
number of (query, vector) distances produced per second over the whole step
(both metrics).

Sub-reports on the same line (each its own workload):
  headline extras   the oracle's CPU time on a sample (cpu_baseline), one
           query against the same cache-resident database, Recall@1/10/100
           against exact fp64 search (Sec. 4.5), and the same with the float
           tables (Bolt No Quantize, Sec. 4.2) on 200 of the queries
  msweep   the same step at M = 16 and M = 64 (8 and 32 B codes)
  single_query  one query, top-100, against 2.5e8 rows at M = 16/32/64
           (4/8/16 GB of codes), cache flushed between calls: latency and
           the fraction of the HBM roofline
  amm      approximate matrix product, A 200,000 x 256 N(0,1), M = 32,
           B 256 x K for K in {64, 256, 1024}: throughput and accuracy
           against the exact fp32 product (and the fp32 GEMM's time)
  batched  256 uneven mixture databases (N log-uniform in [1e3, 2e6],
           J in {64,128,256}, M in {16,32,64}, 1..512 queries each, top-100):
           one autotuned persistent launch replayed from a HIP graph vs one
           launch per (database, query), identical results
  serving  8 resident databases of 2.5e8 x 128 at M = 32 (32 GB of codes),
           Poisson requests (90% query batches of 1..64, 10% inserts of
           1e4..1e6 vectors): p50/p99 latency at 0.3/0.6/0.9 of the measured
           saturation rate, against the plain one-query-per-launch FIFO server

Per-kernel durations come from HIP events that the library records on each
kernel's launch stream inside the timed region (bolt_prof_*).  The default
50 warm-up steps let the GPU's clocks settle before the 50 timed steps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz, 64 lanes per CU and clock (32-bit VALU ops)
VALU_LANE_OPS = 256 * 64 * 2.4e9
MFMA_I8_OPS = 5.0e15                 # MI355X dense int8 matrix-core peak (ops/s)
HBM_PEAK_GBPS = 8000.0

# HBM traffic of the dominant kernel, from two rocprofv3 --pmc runs of this
# script's lean headline workload (--profile-kernels headline,single
# --calib-copy: FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
# what the counter reads for a 1 GiB device-to-device copy in the same runs
# (FETCH_SIZE 524309.7 KiB for 1048576 KiB read: factor 2.0; WRITE_SIZE
# 1048576.0 KiB for 1048576 KiB written: factor 1.0).  Valid only for the
# workload and kernel sources they were taken on: the sources are hashed,
# and any change reports traffic as null until measured again.
FETCH_FACTOR = 2.0
WRITE_FACTOR = 1.0
TRAFFIC = {
    "scan_topk_mfma": {
        # Q: queries per launch (both metrics' 1000 each)
        "workload": {"N": 1_000_000, "J": 128, "M": 32, "Q": 2000, "k": 100},
        "fetch_kib": 11912.6,
        "write_kib": 11624.9,
        "sources_sha256": "a11b11cd921198ba83ae22c1efb39d0fab8c7f3b8cc61833923dcfc7216e3494",
    },
}
# the kernel's sources and the build flags (paper_1706_10283_amd/build.py)
TRAFFIC_SOURCES = {
    "scan_topk_mfma": ["fused.hip", "tiles.hpp", "topk_device.hpp", "scan_common.hpp", "../build.py"],
    "scan_topk_grouped": ["fused.hip", "tiles.hpp", "topk_device.hpp", "scan_common.hpp", "../build.py"],
}


def sources_sha256(kernel):
    """Hash of the kernel's code: comments and blank lines stripped, so that
    documentation edits do not invalidate the counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1706_10283_amd", "csrc", f)) as fh:
            text = fh.read()
        if f.endswith(".py"):
            # only the compiler flags of the build script
            text = re.sub(r"#[^\n]*", "", text)
            text = text[text.index("COMMON_FLAGS = "):]
            text = text[:text.index("]", text.index("HIP_FLAGS = ")) + 1]
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()


def traffic_bytes(kernel, workload):
    """Measured HBM bytes per launch, or None if not measured on these sources."""
    t = TRAFFIC.get(kernel)
    if not t or t["fetch_kib"] is None or t["workload"] != workload:
        return None
    if t["sources_sha256"] != sources_sha256(kernel):
        return None
    return 1024.0 * (FETCH_FACTOR * t["fetch_kib"] + WRITE_FACTOR * t["write_kib"])


def scan_roofline(kernel, Q, N, M, ms):
    """Roofline of a many-query scan launch, on the method's own work: one
    table lookup and one add per (query, vector, subspace) (eq. pqDist), 2
    ops each, against the dense int8 matrix-core peak the kernel runs on.
    The one-hot form of the matrix-core kernel spends 16 int8 multiply-adds
    per lookup (dense MFMA), or 8 with the 2:4 structured-sparse MFMA, so it
    can reach at most 1/16 (1/8) of the peak in the method's units; those
    dense-equivalent figures are reported beside it, labelled."""
    lookups = float(Q) * N * M
    t = ms * 1e-3
    ops = 2.0 * lookups
    out = {"bound": "mfma" if kernel.startswith("scan_topk_mfma") else "alu",
           "kernel": kernel,
           "achieved": round(ops / t / 1e12, 3),
           "peak": round(MFMA_I8_OPS / 1e12, 2),
           "unit": "TOP/s",
           "op": "one table lookup + one add per (query, vector, subspace), 2 ops",
           "frac": round(ops / t / MFMA_I8_OPS, 4),
           "lookups_T_per_s": round(lookups / t / 1e12, 3)}
    if kernel.startswith("scan_topk_mfma"):
        slots = matrix_slots_per_lookup(M)
        out["onehot_macs_per_lookup"] = 16
        out["matrix_slots_per_lookup"] = round(slots, 3)
        out["dense_equiv_TOPs"] = round(2.0 * 16 * lookups / t / 1e12, 1)
        out["matrix_ceiling_frac"] = round(slots * ops / t / MFMA_I8_OPS, 4)
        out["note"] = ("the lookups run as a one-hot int8 matrix product (16 multiply-adds per lookup) on the "
                       "4:2-structured sparse instruction, which issues 32 one-hot entries per dense "
                       "multiply-add slot; with the first four subspaces of a pass on the dense instruction, "
                       "a lookup occupies 8 (M + 4) / M dense slots (%.3g at M = %d), so the method's fraction "
                       "of the dense int8 peak is capped at 1/%.3g; matrix_ceiling_frac is the fraction of that "
                       "cap.  The peak is the dense one: the sparse instruction's doubled headline rate is "
                       "never used as the denominator.  LDS/VALU lookup ceilings do not bound a matrix-core "
                       "kernel" % (slots, M, slots))
    else:
        out["note"] = "a lookup-and-add on the vector ALU/LDS; frac against the int8 matrix-core peak"
    return out


def matrix_slots_per_lookup(M):
    """Dense int8 multiply-add slots of the matrix cores one lookup occupies
    in the matrix-core scan: per pass of 32 rows, two dense
    v_mfma_i32_32x32x32_i8 for subspaces 0-3 and M / 4 - 1 sparse
    v_smfmac_i32_32x32x64_i8, each 32 cycles, against M / 2 dense steps of
    16 slots per lookup: 16 (M / 4 + 1) / (M / 2) = 8 (M + 4) / M."""
    return 8.0 * (M + 4) / M


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    # the GPU's clocks settle within a few tens of steps after an idle
    # period: 0.843 ms per step after 3 warm-up steps, 0.815 after 30, 0.811
    # after 100 (the headline, measured)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--N", type=int, default=1_000_000)
    p.add_argument("--J", type=int, default=128)
    p.add_argument("--M", type=int, default=32)
    p.add_argument("--Q", type=int, default=1000)
    p.add_argument("--k", type=int, default=100)
    p.add_argument("--n-train", type=int, default=100_000)
    p.add_argument("--parts", default="headline,msweep,single_query,amm,batched,serving")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-rows", type=int, default=80_000)
    p.add_argument("--batched-dbs", type=int, default=256)
    p.add_argument("--serving-rows", type=int, default=250_000_000)
    p.add_argument("--serving-requests", type=int, default=2000,
                   help="requests per load point of the continuous server")
    p.add_argument("--fifo-requests", type=int, default=300,
                   help="requests per load point of the FIFO baseline (and of the continuous server at FIFO's rates)")
    p.add_argument("--served-check-queries", type=int, default=1000,
                   help="served queries checked against the same queries alone")
    p.add_argument("--calib-copy", action="store_true",
                   help="also run a 1 GiB device-to-device copy (counter calibration for profiles)")
    p.add_argument("--profile-kernels", default="",
                   help="instead of the benchmark, run a lean workload for profiler counters: 'headline' "
                        "(encode, tables, scan + top-k for both metrics, 3 steps) and/or 'single' (one query "
                        "over 2.5e8 rows at M = 16 and 32, 2 calls per metric), comma-separated")
    return p.parse_args()


def event_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


# ------------------------------------------------------------------ headline

def headline(args, torch, B, W, M=None, steps=None, warmup=None, extras=True):
    """One pass of the hot path per step (encode, both tables, scan + top-k for
    both metrics: the two metrics' queries as one two-metric call); with extras, also the oracle's CPU time, the single-query
    latency on the same (cache-resident) database and Recall@R."""
    import synth
    import synth.device as sdev
    dev = "cuda"
    N, J, Q, k = args.N, args.J, args.Q, args.k
    M = M or args.M
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    mix = synth.seed_for(2, 0)
    t0 = time.time()
    X = sdev.gmm_rows(mix, synth.seed_for(2, 1), 0, N, J)
    Qd = sdev.gmm_rows(mix, synth.seed_for(2, 2), 0, Q, J)
    C, quant = W.train(mix, synth.seed_for(2, 3), synth.seed_for(2, 4), synth.seed_for(2, 5), J, M,
                       args.n_train, iters=10)
    log("headline inputs + training: %.1fs" % (time.time() - t0))
    Cd = torch.from_numpy(C).to(dev)
    offd = {m: torch.from_numpy(quant[m][1]).to(dev) for m in quant}
    scale = {m: quant[m][0] for m in quant}
    codes = torch.empty((N, M // 2), dtype=torch.uint8, device=dev)
    # the L2 queries' tables, then the dot queries': 2 Q queries per scan launch
    Q2 = 2 * Q
    luts_all = torch.empty((Q2, M, 16), dtype=torch.uint8, device=dev)
    vals_all = torch.empty((Q2, k), dtype=torch.uint16, device=dev)
    idx_all = torch.empty((Q2, k), dtype=torch.int32, device=dev)
    luts = {"l2": luts_all[:Q], "dot": luts_all[Q:]}
    idx = {"l2": idx_all[:Q], "dot": idx_all[Q:]}
    ws = torch.empty(B.bolt_scan_topk_split_ws_bytes(N, M, Q2, Q, k), dtype=torch.uint8, device=dev)

    def step():
        B.bolt_encode(X, Cd, M, codes=codes)
        for m in ("l2", "dot"):
            B.bolt_build_luts(Qd, Cd, M, m, scale[m], offd[m], luts_u8=luts[m])
        # k smallest sums for the L2 side, k largest for the dot side
        B.bolt_scan_topk_split(codes, luts_all, Q, "l2", "dot", k, vals=vals_all, idx=idx_all, ws=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events only around the scan launches (the dominant
    # kernel; every pair of events costs a few microseconds of stream time)
    B.prof_read(reset=True)
    B.prof_enable(True, only="scan_topk")
    t_start = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    B.prof_enable(False)
    prof_timed = B.prof_read(reset=True)
    # per-kernel breakdown: a few more steps with every launch timed
    for _ in range(min(steps, 5)):
        B.prof_enable(True)
        step()
    torch.cuda.synchronize()
    B.prof_enable(False)
    prof = B.prof_read(reset=True)
    ms_per_step = 1e3 * t_total / steps
    kern = {n: {"launches": c, "avg_ms": round(ms / c, 5)} for n, (c, ms) in prof.items()}
    dists = 2.0 * Q * N
    value = dists / (ms_per_step * 1e-3) / 1e9

    dom = [n for n in ("scan_topk_mfma", "scan_topk_grouped", "scan_topk_few") if n in prof_timed][0]
    dom_ms = prof_timed[dom][1] / prof_timed[dom][0]
    roof = scan_roofline(dom, Q2, N, M, dom_ms)
    enc_ms = prof["encode"][1] / prof["encode"][0]
    traffic = traffic_bytes(dom, {"N": N, "J": J, "M": M, "Q": Q2, "k": k})
    res = {
        "metric": "G distances/sec scanned + encode GB/s; p50/p99 latency vs plain per-query scan",
        "value": round(value, 3),
        "unit": "G distances/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single-database scan: N=%d x J=%d Gaussian-mixture rows, M=%d (%d B "
                               "codes), Q=%d queries, L2 + dot tables, encode + tables + scan + top-%d "
                               "(both metrics' %d queries in one scan call)"
                               % (N, J, M, M // 2, Q, k, Q2),
                   "N": N, "J": J, "M": M, "Q": Q, "k": k},
        "encode_GBps": round(4.0 * N * J / (enc_ms * 1e-3) / 1e9, 1),
        "scan_topk_G_distances_per_s": round(Q2 * N / (dom_ms * 1e-3) / 1e9, 2),
        "kernels": kern,
        "kernels_note": "HIP-event averages from steps timed after the timed region (every launch "
                        "timed); inside it only the scan launches carry events",
        "roofline": dict(roof, **{
            "traffic": None if traffic is None else round(traffic),
            "traffic_unit": "HBM bytes per launch (fetch + write)",
            "algorithmic_bytes": N * M // 2 + Q2 * M * 16,
            "traffic_note": "fetch: the codes once and the query tables once per XCD (eight L2 caches: "
                            "the row blocks, not the query blocks, are spread over them); writes: the "
                            "candidate keys the sampled bound admits (8 bytes each, several times k per query)",
        }),
    }
    if extras:
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(args, C, quant, Qd.cpu().numpy(), mix)
        # one query against the same database (16 MB of codes: cache-resident)
        one = {m: luts[m][:1].contiguous() for m in ("l2", "dot")}
        res["single_query_cache_resident_ms"] = {
            m: round(event_ms(torch, lambda: B.bolt_scan_topk(codes, one[m], m, k), 20), 4)
            for m in ("l2", "dot")}
        res["training"] = training_times(args, torch, B, mix)
        true = exact_nn(torch, X, Qd)
        res["recall"] = {m: recall_at(torch, idx[m], true[m]) for m in ("l2", "dot")}
        res["no_quantize"] = no_quantize(torch, B, codes, Qd, Cd, M, k, idx, true, n_q=200)
    del X, codes, ws
    return res


def training_times(args, torch, B, mix):
    """k-means codebooks for the headline's training set (n_train mixture
    rows, 10 Lloyd iterations): on the GPU (bolt_kmeans) and with the host
    trainer's k-means (threads on the host cores)."""
    import synth
    import synth.device as sdev
    n, J, M = args.n_train, args.J, args.M
    Xtr = sdev.gmm_rows(mix, synth.seed_for(2, 3), 0, n, J)
    init = synth.permutation_prefix(synth.seed_for(2, 4), n, 16)
    B.bolt_kmeans(Xtr, M, 1, init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Cg, _ = B.bolt_kmeans(Xtr, M, 10, init)
    gpu_s = time.perf_counter() - t0
    Xh = Xtr.cpu().numpy()
    Qt = Xh[:64]
    t0 = time.perf_counter()
    Ch, _, _, _ = B.bolt_train_host(Xh, M, 10, init, Qt, "l2")
    host_s = time.perf_counter() - t0
    # the quantiser search (Sec. 3.2: b_m and a from quantiles of the table
    # entries over training pairs, alpha over its grid) for 1000 training
    # queries against the training codes, on the GPU and on the host
    nq = min(1000, n)
    Qtd = Xtr[torch.from_numpy(synth.permutation_prefix(synth.seed_for(2, 5), n, nq)).to(Xtr.device)].contiguous()
    tr_codes = B.bolt_encode(Xtr, Cg, M)
    quant = {}
    for metric in ("l2", "dot"):
        B.bolt_learn_quantizer(Qtd, tr_codes, Cg, metric)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ag, og, ig, _ = B.bolt_learn_quantizer(Qtd, tr_codes, Cg, metric)
        og = og.cpu().numpy()
        qgpu_s = time.perf_counter() - t0
        Qth, codes_h = Qtd.cpu().numpy(), tr_codes.cpu().numpy()
        t0 = time.perf_counter()
        ah, oh, ih = B.bolt_learn_quantizer_host(Qth, codes_h, Cg.cpu().numpy(), metric)
        qhost_s = time.perf_counter() - t0
        quant[metric] = {"gpu_ms": round(qgpu_s * 1e3, 2), "host_ms": round(qhost_s * 1e3, 1),
                         "identical_to_host": bool(np.float32(ag) == np.float32(ah) and np.array_equal(og, oh)
                                                   and int(ig) == int(ih))}
    return {"workload": "k-means, %d x %d mixture rows, M=%d, 10 iterations; quantiser search, %d training "
                        "queries against the training codes" % (n, J, M, nq),
            "kmeans_gpu_ms": round(gpu_s * 1e3, 2),
            "host_trainer_ms": round(host_s * 1e3, 1),
            "host_trainer_note": "k-means plus the quantiser for 64 queries, host threads",
            "identical_codebooks": bool(np.array_equal(Cg.cpu().numpy(), Ch)),
            "quantiser_search": quant}


def exact_nn(torch, X, Qd):
    """Each query's exact nearest neighbour: fp64 squared L2, and the largest
    fp64 dot product (maximum inner product search)."""
    X64 = X.double()
    xx = (X64 * X64).sum(1)
    true = {"l2": [], "dot": []}
    for q0 in range(0, Qd.shape[0], 100):
        dots = Qd[q0:q0 + 100].double() @ X64.t()
        true["dot"].append(dots.argmax(1))
        true["l2"].append((xx[None, :] - 2.0 * dots).argmin(1))
    del X64
    return {m: torch.cat(v).to(torch.int64) for m, v in true.items()}


def recall_at(torch, idx, true):
    """Recall@R (Sec. 4.5): the fraction of queries whose exact nearest
    neighbour is among the first R results."""
    got = idx.to(torch.int64)
    return {"R%d" % R: round((got[:, :R] == true[:, None]).any(1).double().mean().item(), 4)
            for R in (1, 10, 100)}


def no_quantize(torch, B, codes, Qd, Cd, M, k, idx, true, n_q):
    """Bolt No Quantize (Sec. 4.2): the same codes scanned with the float
    tables, on the first n_q queries; Recall@R beside the uint8 tables'
    on the same queries, and the float scan's throughput."""
    N = codes.shape[0]
    Qs = Qd[:n_q].contiguous()
    zeros = torch.zeros(M, dtype=torch.float32, device=Qd.device)
    out = {"queries": n_q, "recall": {}, "recall_uint8_tables": {}}
    for metric in ("l2", "dot"):
        _, lf = B.bolt_build_luts(Qs, Cd, M, metric, 1.0, zeros, want_f32=True)
        S = B.bolt_scan_f32(codes, lf)
        ms = event_ms(torch, lambda: B.bolt_scan_f32(codes, lf, out=S), 3)
        _, i = B.bolt_topk_f32(S, k, largest=metric == "dot")
        out["recall"][metric] = recall_at(torch, i, true[metric][:n_q])
        out["recall_uint8_tables"][metric] = recall_at(torch, idx[metric][:n_q], true[metric][:n_q])
        out["scan_f32_G_distances_per_s"] = round(n_q * N / (ms * 1e-3) / 1e9, 1)
        del S
    return out


def run_msweep(args, torch, B, W):
    """The single-database step at the other code sizes (M = 16 and 64)."""
    out = {}
    for M in (16, 64):
        r = headline(args, torch, B, W, M=M, steps=20, warmup=30, extras=False)
        out["M%d" % M] = {"value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
                          "encode_GBps": r["encode_GBps"],
                          "scan_topk_G_distances_per_s": r["scan_topk_G_distances_per_s"],
                          "kernels": r["kernels"], "roofline_bound": r["roofline"]["bound"],
                          "roofline_frac": r["roofline"]["frac"]}
        log("M=%d: %.1f G distances/s" % (M, r["value"]))
    return out


def run_single_query(args, torch, B, W):
    """One query, top-100, against a 2.5e8-row database (4 / 8 / 16 GB of
    codes at M = 16 / 32 / 64, far beyond the 256 MB last-level cache), with
    a 1 GB write between calls so no call starts with codes in cache.  The
    HBM roofline counts the code bytes once per call."""
    import synth
    import synth.device as sdev
    N, J, k, reps = args.serving_rows, 128, args.k, 10
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    out = {"workload": "N=%.3g x J=%d mixture rows, 1 query, top-%d, cache flushed between calls" % (N, J, k)}
    for M in (16, 32, 64):
        mix = synth.seed_for(5, 0) + 7 * M
        C, quant = W.train(mix, mix + 3, mix + 4, mix + 5, J, M, n_train=20_000, iters=10)
        db = W.build_db(mix, mix + 1, N, J, M, C, quant)
        qv = sdev.gmm_rows(mix, mix + 2, 0, 1, J)
        row = {}
        for metric in ("l2", "dot"):
            luts = db.luts(qv, metric)
            codes = db.codes[:N]
            B.bolt_scan_topk(codes, luts, metric, k)
            # latency with no library events, then the kernel breakdown from
            # as many calls with every launch timed
            ms = []
            for _ in range(reps):
                flush.fill_(1.0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                B.bolt_scan_topk(codes, luts, metric, k)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            B.prof_read(reset=True)
            for _ in range(reps):
                flush.fill_(1.0)
                B.prof_enable(True)
                B.bolt_scan_topk(codes, luts, metric, k)
                B.prof_enable(False)
                torch.cuda.synchronize()
            prof = B.prof_read(reset=True)
            med = float(np.median(ms))
            scan_name = "scan_topk_few" if "scan_topk_few" in prof else "scan_topk_grouped"
            scan_ms = prof[scan_name][1] / prof[scan_name][0]
            nbytes = N * M // 2
            row[metric] = {"ms_per_query": round(med, 4),
                           "G_distances_per_s": round(N / (med * 1e-3) / 1e9, 1),
                           "GBps": round(nbytes / (med * 1e-3) / 1e9, 1),
                           "hbm_frac": round(nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                           "scan_kernel": scan_name,
                           "scan_kernel_ms": round(scan_ms, 4),
                           "scan_kernel_hbm_frac": round(nbytes / (scan_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                           "kernels": {n: round(t / c, 4) for n, (c, t) in prof.items()}}
            log("single query M=%d %s: %.3f ms, %.0f GB/s (kernel %.0f GB/s)"
                % (M, metric, med, nbytes / (med * 1e-3) / 1e9, nbytes / (scan_ms * 1e-3) / 1e9))
            if metric == "l2":
                # the same call with its sampled bound forced to fail: the
                # exact recomputation on the whole GPU, and its result
                v0, i0 = B.bolt_scan_topk(codes, luts, metric, k)
                B.debug_speculation(2)
                try:
                    B.bolt_scan_topk(codes, luts, metric, k)
                    flush.fill_(1.0)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    v1, i1 = B.bolt_scan_topk(codes, luts, metric, k)
                    e1.record()
                    torch.cuda.synchronize()
                finally:
                    B.debug_speculation(-1)
                row[metric]["failed_bound"] = {
                    "ms_per_query": round(e0.elapsed_time(e1), 4),
                    "equals_unforced": bool(torch.equal(v0, v1) and torch.equal(i0, i1))}
                log("single query M=%d, bound forced to fail: %.3f ms" % (M, e0.elapsed_time(e1)))
        out["M%d" % M] = row
        del db, codes
        torch.cuda.empty_cache()
    del flush
    return out


def host_cpu():
    """CPU model and the threads this process may use (the affinity mask,
    capped by OMP_NUM_THREADS where the host sets it)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        n = min(n, int(os.environ["OMP_NUM_THREADS"]))
    return model, max(1, n), os.cpu_count()


def _oracle_step(oracle, X, C, M, quant, Qv, k, threads):
    """The headline step run by the oracle's functions as they stand: encode
    the rows, then per metric tables, scan and top-k.  With threads > 1 the
    rows (encode) and the queries (tables, scan, top-k) are split among host
    threads; each thread calls the unchanged oracle functions on its part
    (ctypes releases the interpreter lock during the C calls)."""
    from concurrent.futures import ThreadPoolExecutor
    out = {}
    if threads <= 1:
        codes = oracle.encode(X, C, M)
        for metric in ("l2", "dot"):
            a, off = quant[metric]
            _, _, l8 = oracle.luts(Qv, C, M, metric, a, off)
            out[metric] = oracle.topk(oracle.scan(codes, l8), k, metric == "dot")
        return codes, out
    threads = min(threads, X.shape[0], Qv.shape[0])
    with ThreadPoolExecutor(threads) as ex:
        rows = np.array_split(np.arange(X.shape[0]), threads)
        codes = np.concatenate(list(ex.map(lambda r: oracle.encode(X[r[0]:r[-1] + 1], C, M), rows)))
        for metric in ("l2", "dot"):
            a, off = quant[metric]

            def part(qs):
                _, _, l8 = oracle.luts(Qv[qs[0]:qs[-1] + 1], C, M, metric, a, off)
                return oracle.topk(oracle.scan(codes, l8), k, metric == "dot")
            parts = list(ex.map(part, np.array_split(np.arange(Qv.shape[0]), threads)))
            out[metric] = (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
    return codes, out


def cpu_baseline(args, C, quant, Qv, mix):
    """The oracle as it stands on the host cores, on a bounded sample of the
    headline workload (the first rows of the database, all queries, both
    metrics, encode + tables + scan + top-k): once on all the threads the
    process may use, once on one thread.  The rate is measured on the sample
    and the whole step's time extrapolated linearly in the rows (the work is
    linear in N, Sec. 3.1)."""
    import oracle
    import synth
    model, threads, ncpu = host_cpu()
    n1 = args.cpu_sample_rows
    nall = min(args.N, n1 * max(1, threads // 2))
    X = synth.gmm_rows(mix, synth.seed_for(2, 1), 0, nall, args.J)
    Qv = np.ascontiguousarray(Qv)
    # all threads: best of 3
    dts = []
    for _ in range(3):
        t0 = time.perf_counter()
        _oracle_step(oracle, X, C, args.M, quant, Qv, args.k, threads)
        dts.append(time.perf_counter() - t0)
    dt_all = min(dts)
    t0 = time.perf_counter()
    _oracle_step(oracle, X[:n1], C, args.M, quant, Qv, args.k, 1)
    dt_one = time.perf_counter() - t0
    rate_all = 2.0 * Qv.shape[0] * nall / dt_all
    rate_one = 2.0 * Qv.shape[0] * n1 / dt_one
    return {"value": round(rate_all / 1e9, 5), "unit": "G distances/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d of %d rows, all %d queries, L2 + dot, encode + tables + scan + top-%d, "
                      "rows encoded and queries split over %d threads, best of 3 runs (%.2f s)"
                      % (nall, args.N, Qv.shape[0], args.k, threads, dt_all),
            "extrapolated": True,
            "full_step_s_extrapolated": round(dt_all * args.N / nall, 2),
            "cpu_model": model, "nproc": ncpu,
            "single_thread": {"value": round(rate_one / 1e9, 5), "unit": "G distances/s", "cores": 1,
                              "sample": "first %d rows, one run (%.1f s)" % (n1, dt_one),
                              "full_step_s_extrapolated": round(dt_one * args.N / n1, 1)},
            "protocol_note": "the paper's best of 5 runs x 10 trials would take hours on the host at "
                             "this size; a bounded sample is timed instead"}


# ------------------------------------------------------------------ approximate matrix product

def run_amm(args, torch, B, W):
    import synth
    dev = "cuda"
    N, J, M = 200_000, 256, 32
    t0 = time.time()
    A = synth.normal(synth.seed_for(3, 1), (N, J))
    Btrain = synth.normal(synth.seed_for(3, 5), (1000, J))
    init = synth.permutation_prefix(synth.seed_for(3, 4), N, 16)
    C, a, offs, _ = B.bolt_train_host(A, M, 10, init, Btrain, "dot")
    log("amm training: %.1fs" % (time.time() - t0))
    Ad = torch.from_numpy(A).to(dev)
    Cd = torch.from_numpy(C).to(dev)
    offd = torch.from_numpy(offs).to(dev)
    bias = float(np.float32(offs.astype(np.float64).sum()))
    scale = float(np.float32(1.0 / a))
    codes = B.bolt_encode(Ad, Cd, M)
    # reconstruction of A (for the per-entry bound) and its row error norms
    cu = torch.stack([codes & 15, codes >> 4], dim=2).reshape(N, M).long()
    xhat = torch.cat([Cd[m][cu[:, m]] for m in range(M)], dim=1)
    err_norm = torch.linalg.norm(Ad - xhat, dim=1)
    out = {"workload": "A %dx%d N(0,1), M=%d, B %dxK N(0,1), dot tables" % (N, J, M, J), "K": {}}
    enc_ms = event_ms(torch, lambda: B.bolt_encode(Ad, Cd, M, codes=codes), 5)
    out["encode_ms"] = round(enc_ms, 4)
    for K in (64, 256, 1024):
        Bm = synth.normal(synth.seed_for(3, 2) + K, (J, K))
        Qv = torch.from_numpy(np.ascontiguousarray(Bm.T)).to(dev)
        luts = B.bolt_build_luts(Qv, Cd, M, "dot", a, offd)
        res = torch.empty((K, N), dtype=torch.float32, device=dev)
        t_luts = event_ms(torch, lambda: B.bolt_build_luts(Qv, Cd, M, "dot", a, offd, luts_u8=luts), 5)
        t_amm = event_ms(torch, lambda: B.bolt_amm(codes, luts, bias, scale, out=res), 5)
        Bd = torch.from_numpy(Bm).to(dev)
        exact = torch.empty((K, N), dtype=torch.float32, device=dev)
        t_gemm = event_ms(torch, lambda: torch.matmul(Bd.t().contiguous(), Ad.t(), out=exact), 5)
        diff = (exact - res).double()
        ex = exact.double()
        r = torch.corrcoef(torch.stack([ex.flatten(), res.double().flatten()]))[0, 1].item()
        rel = (torch.linalg.norm(diff) / torch.linalg.norm(ex)).item()
        bound = torch.linalg.norm(Qv, dim=1)[:, None].double() * err_norm[None].double() + M / a
        within = (diff.abs() <= bound * (1 + 1e-6)).double().mean().item()
        out["K"][str(K)] = {"tables_ms": round(t_luts, 4), "amm_ms": round(t_amm, 4),
                            "fp32_gemm_ms": round(t_gemm, 4),
                            "G_distances_per_s": round(K * N / (t_amm * 1e-3) / 1e9, 2),
                            "pearson_r": round(r, 5), "rel_frobenius_err": round(rel, 5),
                            "frac_within_bound": round(within, 6)}
        log("amm K=%d: %.3f ms, r=%.4f" % (K, t_amm, r))
    return out


# ------------------------------------------------------------------ batched databases

def run_batched(args, torch, B, W):
    from paper_1706_10283_amd import autotune
    t0 = time.time()
    specs = W.batched_specs(args.batched_dbs)
    dbs = W.build_batched(specs, log=log)
    log("batched inputs: %d databases, %.1fs" % (len(dbs), time.time() - t0))
    entries = [{"codes": d["codes"], "luts": d["luts"], "metric": d["metric"], "k": d["k"]} for d in dbs]
    tuner = autotune.BatchTuner(os.path.join(ROOT, "paper_1706_10283_amd", "tuning_cache.json"))
    tuning, trials = tuner.tune(entries, log=log)
    plan = B.BatchPlan(entries, tuning=tuning)
    plan.capture()
    for _ in range(2):
        plan.launch_graph()
    torch.cuda.synchronize()
    B.prof_read(reset=True)
    B.prof_enable(True)
    reps = 5
    t_graph = event_ms(torch, plan.launch_graph, reps)
    B.prof_enable(False)
    torch.cuda.synchronize()
    batched_res = [(v.clone(), i.clone()) for v, i in plan.results()]

    # baseline: one launch (sequence) per (database, query)
    def per_query():
        out = []
        for d in dbs:
            Q = d["luts"].shape[0]
            vs, is_ = [], []
            for q in range(Q):
                v, i = B.bolt_scan_topk(d["codes"], d["luts"][q:q + 1], d["metric"], d["k"])
                vs.append(v)
                is_.append(i)
            out.append((torch.cat(vs), torch.cat(is_)))
        return out
    per_query()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    base = per_query()
    torch.cuda.synchronize()
    t_base = (time.perf_counter() - t1) * 1e3
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(batched_res, base))
    dist = float(sum(s.Q * s.N for s in specs))
    lookups = float(sum(s.Q * s.N * s.M for s in specs))
    info = plan.info()
    plan.close()
    return {"workload": "%d uneven databases, %d queries, %.3g rows, %.3g distances" % (
                len(specs), sum(s.Q for s in specs), sum(s.N for s in specs), dist),
            "tuning": {"rows_per_tile": tuning[0], "few_max_q": tuning[1], "blocks_per_cu": tuning[2]},
            "autotune_trials": trials, "tiles": info["tiles"],
            "graph_ms": round(t_graph, 3), "per_query_launches_ms": round(t_base, 1),
            "speedup": round(t_base / t_graph, 1),
            "G_distances_per_s": round(dist / (t_graph * 1e-3) / 1e9, 1),
            "lookup_TOPs": round(lookups / (t_graph * 1e-3) / 1e12, 3),
            # the method's work (one lookup and one add per query, vector and
            # subspace) against the dense int8 matrix-core peak
            "frac_of_int8_peak": round(2.0 * lookups / (t_graph * 1e-3) / MFMA_I8_OPS, 4),
            # every lookup counted at the dense matrix-core slots it occupies
            # in the one-hot form (most of this workload's lookups run there):
            # the fraction of the matrix cores the lookups keep busy
            "matrix_slot_frac": round(2.0 * sum(s.Q * s.N * s.M * matrix_slots_per_lookup(s.M) for s in specs)
                                      / (t_graph * 1e-3) / MFMA_I8_OPS, 4),
            "identical_to_per_query": bool(same)}


# ------------------------------------------------------------------ serving

def run_serving(args, torch, B, W):
    """Serving (8 resident databases): the continuous-batching server at its
    saturation and at 0.3 / 0.6 / 0.9 of it; the FIFO baseline (one request
    at a time, one launch sequence per query) at its own saturation and at
    0.3 / 0.6 / 0.9 of that, with the continuous server at the same offered
    rates beside it; the peak working memory against the budget and how
    often admission stopped at the budget; and served results checked against
    the same queries run alone at their snapshot."""
    import synth
    import synth.device as sdev
    from paper_1706_10283_amd.serve import GpuExecutor, Server, make_requests, summarize
    n_db, N, J, M, k = 8, args.serving_rows, 128, 32, 100
    t0 = time.time()
    dbs = []
    # capacity: each run starts from the initial rows and appends about 0.1 x
    # requests x 2.15e5 rows over the 8 databases
    headroom = max(4_000_000, int(max(args.serving_requests, args.fifo_requests) * 0.1 * 2.15e5 / n_db * 3))
    for d in range(n_db):
        mix = synth.seed_for(5, 0) + 100 * d
        C, quant = W.train(mix, mix + 3, mix + 4, mix + 5, J, M, n_train=50_000, iters=10)
        dbs.append(W.build_db(mix, mix + 1, N, J, M, C, quant, capacity=N + headroom))
        log("serving database %d/%d built (%.1fs)" % (d + 1, n_db, time.time() - t0))
    torch.cuda.synchronize()
    resident = sum(db.codes.numel() for db in dbs)
    qpool = sdev.gmm_rows(synth.seed_for(5, 0), synth.seed_for(5, 2), 0, 8192, J).cpu().numpy()
    ipool = sdev.gmm_rows(synth.seed_for(5, 0), synth.seed_for(5, 3), 0, 1_000_000, J).cpu().pin_memory()
    budget = 8 << 30   # working memory on top of the resident codes
    ex = GpuExecutor(dbs)

    def serve(mode, rate, n_req, seed, budget=budget):
        reqs = make_requests(n_req, n_db, J, rate, seed, qpool, ipool, k=k)
        srv = Server(ex, dbs, budget, mode=mode)
        wall = srv.run(reqs, realtime=rate > 0)
        torch.cuda.synchronize()
        out = summarize(reqs, wall)
        out["offered_req_per_s"] = round(rate, 2) if rate > 0 else None
        out["peak_in_use_GB"] = round(srv.peak / 1e9, 3)
        out["budget_stalls"] = srv.budget_stalls
        out["group_stalls"] = srv.group_stalls
        log("%s at %s req/s: %s" % (mode, round(rate, 1) if rate else "max", out))
        return reqs, wall, out

    serve("continuous", 0.0, 30, 1)   # warm-up
    reqs, wall, sat_out = serve("continuous", 0.0, args.serving_requests, 2)
    sat = len(reqs) / wall
    out = {"workload": "%d databases x %.3g rows, J=%d, M=%d (%.1f GB codes), budget resident + %d GB"
                       % (n_db, N, J, M, resident / 1e9, budget >> 30),
           "budget_GB": round(budget / 1e9, 3),
           "saturation_req_per_s": round(sat, 2), "continuous": {"saturation": sat_out}, "fifo": {}}
    # the same saturation run under a working-memory budget of 1 GB, below
    # what the batching would use: admission now stops at the budget
    _, _, o = serve("continuous", 0.0, max(args.serving_requests // 4, 100), 2, budget=1 << 30)
    out["continuous"]["saturation_budget_1GB"] = o
    for load in (0.3, 0.6, 0.9):
        reqs, wall, o = serve("continuous", load * sat, args.serving_requests, 10 + int(load * 10))
        out["continuous"]["load_%.1f" % load] = o
        if load == 0.6:
            out["served_equals_alone"] = served_equals_alone(torch, B, dbs, reqs, args.served_check_queries)
    reqs, wall, o = serve("fifo", 0.0, args.fifo_requests, 3)
    fsat = len(reqs) / wall
    out["fifo"]["saturation_req_per_s"] = round(fsat, 2)
    out["fifo"]["saturation"] = o
    out["continuous_at_fifo_rates"] = {}
    for load in (0.3, 0.6, 0.9):
        _, _, o = serve("fifo", load * fsat, args.fifo_requests, 20 + int(load * 10))
        out["fifo"]["load_%.1f" % load] = o
        _, _, o = serve("continuous", load * fsat, args.fifo_requests, 20 + int(load * 10))
        out["continuous_at_fifo_rates"]["load_%.1f_of_fifo" % load] = o
    del dbs, ex
    return out


def served_equals_alone(torch, B, dbs, reqs, n_queries):
    """Served results of the first query requests (at least n_queries
    queries) equal the same requests run alone against their database
    truncated at the request's snapshot; the first 100 of those queries are
    also run one query per call."""
    checked, singles, same = 0, 0, True
    for r in reqs:
        if checked >= n_queries:
            break
        if r.kind != "query" or r.status != "done":
            continue
        db = dbs[r.db]
        qd = torch.from_numpy(np.ascontiguousarray(r.Qv)).to("cuda")
        v, i = B.bolt_scan_topk(db.codes[:r.watermark], db.luts(qd, r.metric), r.metric, r.k)
        same &= bool(np.array_equal(v.cpu().numpy(), r.vals) and np.array_equal(i.cpu().numpy(), r.idx))
        for j in range(r.size):
            if singles >= 100:
                break
            v1, i1 = B.bolt_scan_topk(db.codes[:r.watermark], db.luts(qd[j:j + 1], r.metric), r.metric, r.k)
            same &= bool(np.array_equal(v1.cpu().numpy(), r.vals[j:j + 1]) and
                         np.array_equal(i1.cpu().numpy(), r.idx[j:j + 1]))
            singles += 1
        checked += r.size
    return {"equal": same, "queries_checked": checked, "queries_checked_one_per_call": singles}


def profile_kernels(args, torch, B, W):
    """A lean workload for profiler counter runs (rocprofv3 --pmc serialises
    and instruments every dispatch): the kernels of the headline step and of
    the single-query scan, a few launches each, then a 1 GiB device copy that
    calibrates the memory counters.  Prints the HIP-event averages."""
    import synth
    import synth.device as sdev
    parts = set(args.profile_kernels.split(","))
    out = {}
    if "headline" in parts:
        N, J, M, Q, k = args.N, args.J, args.M, args.Q, args.k
        mix = synth.seed_for(2, 0)
        X = sdev.gmm_rows(mix, synth.seed_for(2, 1), 0, N, J)
        Qd = sdev.gmm_rows(mix, synth.seed_for(2, 2), 0, Q, J)
        C, quant = W.train(mix, synth.seed_for(2, 3), synth.seed_for(2, 4), synth.seed_for(2, 5), J, M,
                           20_000, iters=10)
        Cd = torch.from_numpy(C).to("cuda")
        codes = B.bolt_encode(X, Cd, M)
        luts = torch.cat([_tables(B, torch, Qd, Cd, M, m, quant) for m in ("l2", "dot")])
        torch.cuda.synchronize()
        B.prof_read(reset=True)
        B.prof_enable(True)
        for _ in range(3):
            B.bolt_encode(X, Cd, M, codes=codes)
            for m in ("l2", "dot"):
                _tables(B, torch, Qd, Cd, M, m, quant)
            B.bolt_scan_topk_split(codes, luts, Q, "l2", "dot", k)
        torch.cuda.synchronize()
        B.prof_enable(False)
        out["headline"] = {n: {"launches": c, "avg_ms": round(t / c, 5)}
                           for n, (c, t) in B.prof_read(reset=True).items()}
        log("profile: headline kernels done")
        del X, codes
    if "single" in parts:
        N, J, k = args.serving_rows, 128, args.k
        for M in (16, 32):
            mix = synth.seed_for(5, 0) + 7 * M
            C, quant = W.train(mix, mix + 3, mix + 4, mix + 5, J, M, n_train=20_000, iters=10)
            db = W.build_db(mix, mix + 1, N, J, M, C, quant)
            qv = sdev.gmm_rows(mix, mix + 2, 0, 1, J)
            torch.cuda.synchronize()
            log("profile: single-query database M=%d built" % M)
            B.prof_read(reset=True)
            B.prof_enable(True)
            for metric in ("l2", "dot"):
                luts = db.luts(qv, metric)
                for _ in range(2):
                    B.bolt_scan_topk(db.codes[:N], luts, metric, k)
            torch.cuda.synchronize()
            B.prof_enable(False)
            out["single_M%d" % M] = {n: {"launches": c, "avg_ms": round(t / c, 5)}
                                     for n, (c, t) in B.prof_read(reset=True).items()}
            del db
            torch.cuda.empty_cache()
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"profile_kernels": out}), flush=True)


def _tables(B, torch, Qd, Cd, M, metric, quant):
    a, off = quant[metric]
    return B.bolt_build_luts(Qd, Cd, M, metric, a, torch.from_numpy(off).to("cuda"))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (the scan would shard "
              "by database rows, each GPU keeping its local top-k, merged after one all-gather)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1706_10283_amd.bolt as B
    from paper_1706_10283_amd import workloads as W
    torch.cuda.set_device(0)
    if args.profile_kernels:
        profile_kernels(args, torch, B, W)
        return
    parts = set(args.parts.split(","))
    res = headline(args, torch, B, W)
    log("headline: %.1f G distances/s, %.3f ms/step" % (res["value"], res["ms_per_step"]))
    if args.calib_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    for name, fn in (("msweep", run_msweep), ("single_query", run_single_query), ("amm", run_amm),
                     ("batched", run_batched), ("serving", run_serving)):
        if name in parts:
            t0 = time.time()
            try:
                res[name] = fn(args, torch, B, W)
            except Exception as e:   # a failed sub-report is reported, not fatal to the headline
                res[name] = {"error": repr(e)}
            log("%s done in %.1fs" % (name, time.time() - t0))
            torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
