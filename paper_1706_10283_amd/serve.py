"""Serving loop for resident encoded databases (continuous batching).

The paper's online phase (Sec. 1.2) receives database vectors to encode and
queries that need their distances to all vectors received so far, with as
little latency as possible.  This server keeps encoded databases resident in
HBM and serves a stream of two request kinds:

* query batches (q queries of J dimensions, one database, one metric, top k):
  tables (bolt_build_luts) then scan + top-k over the rows committed when
  the request is admitted (its snapshot);
* inserts (n fp32 vectors): copied from host memory, encoded (bolt_encode)
  into the database's preallocated rows on their own stream, and made
  visible by advancing the database's committed-row watermark once encoded.

Admission: a request's working memory (query tables, fp32 staging, top-k
outputs, scan workspace) is reserved against an HBM budget; requests wait
in arrival order until their reservation fits, and a request that could
never fit (or an insert beyond the database's capacity) is refused.

Continuous batching: whenever the GPU has free slots, every admitted query
request is grouped by (database, snapshot, k) and each group runs as one
scan per pair of metrics: a metric ranked by the smallest sums (L2) and one
ranked by the largest (dot) share one two-metric call
(bolt_scan_topk_split), so their queries read the codes once; groups go to
several streams, so work admitted while earlier
groups still run overlaps with them on the device, and inserts overlap with
queries.  Results are bit-identical to running each request alone: sums are
exact integers and top-k keys are totally ordered.

The plain baseline (mode "fifo") serves one request at a time in arrival
order and launches one scan per query.

The executor (GPU work) is separate from the scheduler, so the scheduling
logic can be exercised with any executor that implements the same calls.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import bolt as B


def scan_ws_reserve(rows: int, M: int, q: int, k: int) -> int:
    """Fused scan + top-k workspace to reserve for a request of q queries.

    Requests are grouped into one call, so the reservation must cover the
    request's share of any group it can join.  Calls of three or more
    queries run the matrix-core tiles (eight or more at M = 8 or for
    k > 128, where the grouped kernel takes them), whose workspace per query
    is largest at that smallest call and falls slowly after; smaller calls
    run the pair-table kernels, whose workspace per query falls as the call
    grows.  The larger of the request's own workspace and q times the
    per-query workspace of the smallest such call therefore bounds its share
    in every group, up to the alignment padding of the workspace's parts,
    which 64 KiB per request covers.  A two-metric call needs the larger of
    the workspaces of its whole and of either side, and each of those is
    covered by the shares of the requests it holds."""
    qmin = 8 if (M == 8 or k > 128) else 3
    alone = B.bolt_scan_topk_ws_bytes(rows, M, q, k)
    per_min = B.bolt_scan_topk_ws_bytes(rows, M, qmin, k)
    return max(alone, -(-q * per_min // qmin)) + 65536


def metric_calls(reqs):
    """The scan calls of one group: [[(metric, [request indices])], ...],
    each call one metric or two (a smallest-sums metric first, then a
    largest-sums one: one two-metric call); metrics in order of first
    appearance within each direction, leftovers of one direction paired
    among themselves (a two-metric call of one direction is one scan)."""
    parts = {}
    for i, r in enumerate(reqs):
        parts.setdefault(r.metric, []).append(i)
    lo = [(m, ix) for m, ix in parts.items() if not B.metric_largest(m)]
    hi = [(m, ix) for m, ix in parts.items() if B.metric_largest(m)]
    calls = [[a, b] for a, b in zip(lo, hi)]
    n = min(len(lo), len(hi))
    rest = lo[n:] + hi[n:]
    calls += [rest[j:j + 2] for j in range(0, len(rest), 2)]
    return calls


@dataclass
class Request:
    rid: int
    kind: str                     # "query" or "insert"
    db: int
    arrival: float                # seconds after the start of the run
    metric: str = "l2"
    k: int = 100
    Qv: np.ndarray | None = None  # host fp32 [q, J]
    X: np.ndarray | None = None   # host fp32 [n, J] (pinned torch tensor allowed)
    status: str = "pending"       # pending | done | refused | failed
    admitted: float = math.nan
    done: float = math.nan
    watermark: int = -1           # rows visible to a query
    rows: tuple = ()              # rows written by an insert
    vals: np.ndarray | None = None
    idx: np.ndarray | None = None
    error: str = ""
    reserved: int = 0

    @property
    def size(self) -> int:
        if self.kind == "query":
            return self.Qv.shape[0]
        return self.X.shape[0]

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class GpuExecutor:
    """Launches the Bolt kernels for the server on HIP streams."""

    def __init__(self, dbs, n_streams: int = 3, device="cuda"):
        self.dbs = dbs
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.insert_stream = torch.cuda.Stream(device=device)
        self._next = 0

    # -- sizes used for admission
    def query_bytes(self, req: Request, rows: int) -> int:
        """Tables, staging and outputs of the request's queries, plus its share
        of the scan workspace (scan_ws_reserve)."""
        db = self.dbs[req.db]
        q = req.Qv.shape[0]
        ws = scan_ws_reserve(max(rows, 1), db.M, q, req.k)
        return int(q * (db.J * 4 + db.M * 16 + req.k * 6) + ws) + 4096

    def insert_bytes(self, req: Request) -> int:
        return int(req.X.shape[0] * self.dbs[req.db].J * 4) + 4096

    # -- work
    def launch_queries(self, reqs, db_i: int, rows: int, k: int):
        """One group (one database, snapshot and k; any metrics): the queries
        stacked metric by metric, one scan call per pair of metrics."""
        db = self.dbs[db_i]
        s = self.streams[self._next % len(self.streams)]
        self._next += 1
        calls = metric_calls(reqs)
        order = [i for call in calls for _, ix in call for i in ix]
        sizes = [reqs[i].Qv.shape[0] for i in order]
        Q = sum(sizes)
        host_q = torch.empty((Q, db.J), dtype=torch.float32, pin_memory=True)
        o = 0
        for i in order:
            n = reqs[i].Qv.shape[0]
            host_q[o:o + n] = torch.from_numpy(np.ascontiguousarray(reqs[i].Qv, dtype=np.float32))
            o += n
        with torch.cuda.stream(s):
            qd = host_q.to(self.device, non_blocking=True)
            luts = torch.empty((Q, db.M, 16), dtype=torch.uint8, device=self.device)
            vals = torch.empty((Q, k), dtype=torch.uint16, device=self.device)
            idx = torch.empty((Q, k), dtype=torch.int32, device=self.device)
            o = 0
            for call in calls:
                a = o
                for metric, ix in call:
                    n = sum(reqs[i].Qv.shape[0] for i in ix)
                    db.luts(qd[o:o + n], metric, out=luts[o:o + n], stream=s)
                    o += n
                codes = db.codes[:rows]
                if len(call) == 1:
                    B.bolt_scan_topk(codes, luts[a:o], call[0][0], k, vals=vals[a:o], idx=idx[a:o], stream=s)
                else:
                    n_lo = sum(reqs[i].Qv.shape[0] for i in call[0][1])
                    B.bolt_scan_topk_split(codes, luts[a:o], n_lo, call[0][0], call[1][0], k, vals=vals[a:o],
                                           idx=idx[a:o], stream=s)
            hv = torch.empty(vals.shape, dtype=torch.uint16, pin_memory=True)
            hi = torch.empty(idx.shape, dtype=torch.int32, pin_memory=True)
            hv.copy_(vals, non_blocking=True)
            hi.copy_(idx, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"event": ev, "keep": (host_q, qd, luts, vals, idx), "hv": hv, "hi": hi, "sizes": sizes,
                "order": order}

    def launch_insert(self, req: Request, row0: int):
        db = self.dbs[req.db]
        s = self.insert_stream
        X = req.X if isinstance(req.X, torch.Tensor) else torch.from_numpy(req.X)
        n = X.shape[0]
        with torch.cuda.stream(s):
            xd = X.to(self.device, non_blocking=True)
            B.bolt_encode(xd, db.centroids, db.M, codes=db.codes[row0:row0 + n], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"event": ev, "keep": (X, xd)}

    def ready(self, handle) -> bool:
        return handle["event"].query()

    def query_results(self, handle):
        """Per request of the group, in the order launch_queries was given them."""
        hv, hi = handle["hv"].numpy(), handle["hi"].numpy()
        out, o = [None] * len(handle["order"]), 0
        for i, q in zip(handle["order"], handle["sizes"]):
            out[i] = (hv[o:o + q].copy(), hi[o:o + q].copy())
            o += q
        return out

    def plain_query(self, req: Request, rows: int):
        """Baseline: one launch sequence per query, waited for."""
        db = self.dbs[req.db]
        vals, idx = [], []
        for j in range(req.Qv.shape[0]):
            qd = torch.from_numpy(np.ascontiguousarray(req.Qv[j:j + 1], dtype=np.float32)).to(self.device)
            luts = db.luts(qd, req.metric)
            v, i = B.bolt_scan_topk(db.codes[:rows], luts, req.metric, req.k)
            vals.append(v)
            idx.append(i)
        v = torch.cat(vals).cpu().numpy()
        i = torch.cat(idx).cpu().numpy()
        return v, i

    def plain_insert(self, req: Request, row0: int):
        h = self.launch_insert(req, row0)
        h["event"].synchronize()


class Server:
    """Continuous-batching server (mode "continuous") or the plain FIFO
    baseline (mode "fifo") over resident databases."""

    def __init__(self, executor, dbs, budget_bytes: int, mode: str = "continuous", max_groups: int = 6,
                 clock=time.perf_counter):
        self.ex = executor
        self.dbs = dbs
        self.budget = int(budget_bytes)
        self.mode = mode
        self.max_groups = max_groups
        self.clock = clock
        self.in_use = 0
        self.peak = 0
        self.budget_stalls = 0   # admission rounds stopped by a request that did not fit the budget
        self.group_stalls = 0    # admission rounds stopped by the limit on query groups in flight
        self.committed = [db.n_rows for db in dbs]   # visible rows per database
        self.reserved = [db.n_rows for db in dbs]    # rows handed out to inserts

    # ---------------------------------------------------------------- helpers
    def _footprint(self, r: Request) -> int:
        if r.kind == "query":
            return self.ex.query_bytes(r, self.committed[r.db])
        return self.ex.insert_bytes(r)

    def _refuse_reason(self, r: Request):
        if r.kind == "insert" and self.reserved[r.db] + r.size > self.dbs[r.db].capacity:
            return "insert exceeds the database's capacity"
        if self._footprint(r) > self.budget:
            return "request larger than the whole HBM budget"
        return None

    def _insert_failed(self, r: Request, insert_queue):
        """An insert whose encode failed after it was enqueued.  Its rows hold
        no valid codes, so the watermark must never cover them.  If no later
        insert has reserved rows, the range is handed back; otherwise the
        failed entry stays at its place in the commit queue and holds the
        watermark below it (later inserts of that database stay invisible,
        which keeps every query's snapshot valid)."""
        q = insert_queue.get(r.db, deque())
        if r.rows and self.reserved[r.db] == r.rows[1] and q and q[-1] is r:
            q.pop()
            self.reserved[r.db] = r.rows[0]
            r.rows = ()

    # ---------------------------------------------------------------- run
    def run(self, requests, realtime: bool = True):
        """Serve `requests` (sorted by arrival).  With realtime, arrivals are
        honoured against the wall clock; otherwise all have arrived at t=0.
        Returns the wall time of the run."""
        if self.mode == "fifo":
            return self._run_fifo(requests, realtime)
        return self._run_continuous(requests, realtime)

    def _run_fifo(self, requests, realtime):
        t0 = self.clock()
        for r in requests:
            if realtime:
                while self.clock() - t0 < r.arrival:
                    pass
            why = self._refuse_reason(r)
            if why:
                r.status, r.error, r.done = "refused", why, self.clock() - t0
                continue
            r.admitted = self.clock() - t0
            try:
                if r.kind == "query":
                    r.watermark = self.committed[r.db]
                    r.vals, r.idx = self.ex.plain_query(r, r.watermark)
                else:
                    row0 = self.reserved[r.db]
                    self.reserved[r.db] += r.size
                    r.rows = (row0, row0 + r.size)
                    self.ex.plain_insert(r, row0)
                    self.committed[r.db] = self.reserved[r.db]
                r.status = "done"
            except Exception as e:   # a failed request does not stop the server
                r.status, r.error = "failed", str(e)
                if r.kind == "insert" and r.rows:
                    # its rows were never encoded: hand them back (one request
                    # at a time, so the range is the newest one)
                    self.reserved[r.db] = r.rows[0]
                    r.rows = ()
            r.done = self.clock() - t0
        return self.clock() - t0

    def _run_continuous(self, requests, realtime):
        t0 = self.clock()
        pending = deque(requests)
        waiting = deque()
        inflight = []          # (kind, handle, [requests], footprint)
        insert_queue = {}      # db -> deque of in-flight inserts in order
        while pending or waiting or inflight:
            now = self.clock() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # completions
            still = []
            for item in inflight:
                kind, handle, reqs, fp = item
                try:
                    if not self.ex.ready(handle):
                        still.append(item)
                        continue
                    err = None
                except Exception as e:      # the device reported the work as failed
                    err = str(e)
                t_done = self.clock() - t0
                if err is not None:
                    for r in reqs:
                        r.status, r.error, r.done = "failed", err, t_done
                    if kind == "insert":
                        self._insert_failed(reqs[0], insert_queue)
                elif kind == "query":
                    try:
                        for r, (v, i) in zip(reqs, self.ex.query_results(handle)):
                            r.vals, r.idx, r.status, r.done = v, i, "done", t_done
                    except Exception as e:
                        for r in reqs:
                            r.status, r.error, r.done = "failed", str(e), t_done
                else:
                    r = reqs[0]
                    q = insert_queue[r.db]
                    r.status, r.done = "done", t_done
                    # commit in order: the watermark covers every finished prefix
                    while q and q[0].status == "done":
                        self.committed[r.db] = q.popleft().rows[1]
                self.in_use -= fp
            inflight = still
            # admission (arrival order; stops at the first request that does not fit)
            groups = {}
            n_groups = sum(1 for it in inflight if it[0] == "query")
            while waiting:
                r = waiting[0]
                why = self._refuse_reason(r)
                if why:
                    waiting.popleft()
                    r.status, r.error, r.done = "refused", why, self.clock() - t0
                    continue
                fp = self._footprint(r)
                if self.in_use + fp > self.budget:
                    self.budget_stalls += 1
                    break
                if r.kind == "query":
                    key = (r.db, self.committed[r.db], r.k)
                    if key not in groups and n_groups + len(groups) >= self.max_groups:
                        self.group_stalls += 1
                        break
                    waiting.popleft()
                    r.admitted, r.watermark, r.reserved = self.clock() - t0, self.committed[r.db], fp
                    groups.setdefault(key, []).append(r)
                    self.in_use += fp
                else:
                    waiting.popleft()
                    r.admitted, r.reserved = self.clock() - t0, fp
                    row0 = self.reserved[r.db]
                    self.reserved[r.db] += r.size
                    r.rows = (row0, row0 + r.size)
                    self.in_use += fp
                    try:
                        h = self.ex.launch_insert(r, row0)
                    except Exception as e:
                        r.status, r.error, r.done = "failed", str(e), self.clock() - t0
                        self.in_use -= fp
                        # nothing was enqueued and no later insert has reserved
                        # rows yet: hand the range back
                        self.reserved[r.db] = row0
                        r.rows = ()
                        continue
                    insert_queue.setdefault(r.db, deque()).append(r)
                    inflight.append(("insert", h, [r], fp))
                self.peak = max(self.peak, self.in_use)
            for (db_i, rows, k), reqs in groups.items():
                fp = sum(r.reserved for r in reqs)
                try:
                    h = self.ex.launch_queries(reqs, db_i, rows, k)
                except Exception as e:
                    for r in reqs:
                        r.status, r.error, r.done = "failed", str(e), self.clock() - t0
                    self.in_use -= fp
                    continue
                inflight.append(("query", h, reqs, fp))
            if not groups and inflight:
                time.sleep(0)   # yield; completions are polled on the next turn
        return self.clock() - t0


# -------------------------------------------------------------------- workload and report

def make_requests(n_req: int, n_db: int, J: int, rate: float, seed: int, query_pool, insert_pool,
                  frac_insert: float = 0.1, batch_lo: int = 1, batch_hi: int = 64,
                  ins_lo: float = 1e4, ins_hi: float = 1e6, k: int = 100):
    """Poisson arrivals at `rate` requests/s (rate 0: all at t = 0).  Query
    batches of U[batch_lo, batch_hi] queries on a uniform database, L2 or dot
    with equal odds; inserts of round(exp(U[ln ins_lo, ln ins_hi])) vectors.
    query_pool: host fp32 [P, J] rows to draw queries from; insert_pool: host
    fp32 (pinned) [R, J] rows whose prefix is each insert's payload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for i in range(n_req):
        if rate > 0:
            t += rng.exponential(1.0 / rate)
        db = int(rng.integers(0, n_db))
        if rng.random() < frac_insert:
            n = int(round(math.exp(rng.uniform(math.log(ins_lo), math.log(ins_hi)))))
            n = min(n, insert_pool.shape[0])
            reqs.append(Request(i, "insert", db, t, X=insert_pool[:n], k=k))
        else:
            q = int(rng.integers(batch_lo, batch_hi, endpoint=True))
            off = int(rng.integers(0, query_pool.shape[0] - q + 1))
            metric = "l2" if rng.random() < 0.5 else "dot"
            reqs.append(Request(i, "query", db, t, metric=metric, k=k, Qv=query_pool[off:off + q]))
    return reqs


def summarize(reqs, wall: float):
    def pct(xs, p):
        return float(np.percentile(xs, p)) * 1e3 if len(xs) else math.nan
    q = [r.latency for r in reqs if r.kind == "query" and r.status == "done"]
    ins = [r.latency for r in reqs if r.kind == "insert" and r.status == "done"]
    wait = [r.admitted - r.arrival for r in reqs if r.status == "done"]
    dist = sum(r.size * r.watermark for r in reqs if r.kind == "query" and r.status == "done")
    return {"requests": len(reqs), "done": sum(r.status == "done" for r in reqs),
            "refused": sum(r.status == "refused" for r in reqs),
            "failed": sum(r.status == "failed" for r in reqs),
            "refused_reasons": sorted({r.error for r in reqs if r.status == "refused"}),
            "wall_s": round(wall, 4),
            "query_p50_ms": round(pct(q, 50), 3), "query_p99_ms": round(pct(q, 99), 3),
            "insert_p50_ms": round(pct(ins, 50), 3), "insert_p99_ms": round(pct(ins, 99), 3),
            "admission_wait_p50_ms": round(pct(wait, 50), 3), "admission_wait_p99_ms": round(pct(wait, 99), 3),
            "G_distances_per_s": round(dist / wall / 1e9, 3) if wall > 0 else math.nan}
