"""Autotuner for the batched persistent scan (bolt_batch_*).

The tile shape of the persistent launch -- rows per tile, the query count
below which a database takes the pair-table path, and workgroups per CU --
is chosen by timing a few candidates on the actual batch.  The winner is
cached in a JSON file keyed by a coarse signature of the batch (GPU
architecture, mix of M, total queries and total rows in powers of two), so
batches of the same shape reuse it without timing again.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import bolt as B

CANDIDATES = [
    (16384, 2, 3),
    (32768, 2, 3),
    (65536, 2, 2),
    (8192, 2, 3),
    (32768, 4, 3),
]


def signature(entries) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    ms = {}
    q_total = 0
    n_total = 0
    for e in entries:
        M = e["luts"].shape[1]
        ms[M] = ms.get(M, 0) + 1
        q_total += e["luts"].shape[0]
        n_total += e["codes"].shape[0]
    mix = ",".join("M%d:%d" % (m, round(4 * c / max(len(entries), 1))) for m, c in sorted(ms.items()))
    return "%s|%s|Q2^%d|N2^%d" % (arch, mix, int(math.log2(max(q_total, 1))), int(math.log2(max(n_total, 1))))


class BatchTuner:
    def __init__(self, cache_path: str | None = None, candidates=CANDIDATES, reps: int = 3):
        self.cache_path = cache_path
        self.candidates = list(candidates)
        self.reps = reps
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            try:
                with open(cache_path) as f:
                    self.cache = json.load(f)
            except (OSError, ValueError):
                self.cache = {}

    def _time(self, entries, tuning) -> float:
        plan = B.BatchPlan(entries, tuning=tuning)
        try:
            plan.run()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.reps):
                plan.run()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / self.reps
        finally:
            plan.close()

    def tune(self, entries, log=None):
        """(best tuning (rows_per_tile, few_max_q, blocks_per_cu), trials)."""
        key = signature(entries)
        if key in self.cache:
            return tuple(self.cache[key]["tuning"]), []
        trials = []
        for cand in self.candidates:
            ms = self._time(entries, cand)
            trials.append({"tuning": list(cand), "ms": round(ms, 4)})
            if log:
                log("autotune %s: %.3f ms" % (cand, ms))
            torch.cuda.empty_cache()
        best = min(trials, key=lambda t: t["ms"])
        self.cache[key] = {"tuning": best["tuning"], "ms": best["ms"]}
        if self.cache_path:
            try:
                with open(self.cache_path, "w") as f:
                    json.dump(self.cache, f, indent=1, sort_keys=True)
            except OSError:
                pass
        return tuple(best["tuning"]), trials
