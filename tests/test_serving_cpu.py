"""The serving scheduler on the CPU, with a fake executor whose "kernels" are
oracle calls: admission by budget, refusal, failure isolation, grouping,
snapshot visibility of inserts, and mix-equals-alone results."""
import numpy as np
import pytest

import oracle
import synth
from paper_1706_10283_amd.serve import Request, Server, summarize


class FakeDB:
    def __init__(self, seed, N, cap, J=16, M=8):
        self.J, self.M, self.n_rows = J, M, N
        X = synth.normal(seed, (N, J))
        init = synth.permutation_prefix(seed + 1, N, 16)
        C, a, offs, _ = oracle.train(X, M, 3, init, X[:200], "l2")
        self.C, self.a, self.offs = C, a, offs
        self.codes = np.zeros((cap, M // 2), np.uint8)
        self.codes[:N] = oracle.encode(X, C, M)

    @property
    def capacity(self):
        return self.codes.shape[0]


class FakeExecutor:
    """Runs the work at launch time; a handle becomes ready after `delay` polls."""

    def __init__(self, dbs, delay=2, fail_on=(), fail_ready_on=()):
        self.dbs, self.delay, self.fail_on = dbs, delay, set(fail_on)
        self.fail_ready_on = set(fail_ready_on)   # launches whose completion reports a device error
        self.launches = []

    def query_bytes(self, r, rows):
        return 100 * r.Qv.shape[0]

    def insert_bytes(self, r):
        return 10 * r.X.shape[0]

    def _alone(self, db, Qv, metric, k, rows):
        _, _, l8 = oracle.luts(Qv, db.C, db.M, metric, db.a, db.offs)
        return oracle.topk(oracle.scan(db.codes[:rows], l8), k, metric == "dot")

    def launch_queries(self, reqs, db_i, rows, k):
        self.launches.append(("query", db_i, len(reqs)))
        if len(self.launches) in self.fail_on:
            raise RuntimeError("injected failure")
        db = self.dbs[db_i]
        out = [self._alone(db, r.Qv, r.metric, k, rows) for r in reqs]
        v, i = np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out])
        sizes = [r.Qv.shape[0] for r in reqs]
        return {"left": self.delay, "v": v, "i": i, "sizes": sizes}

    def launch_insert(self, r, row0):
        self.launches.append(("insert", r.db, 1))
        if len(self.launches) in self.fail_on:
            raise RuntimeError("injected insert failure")
        db = self.dbs[r.db]
        if len(self.launches) in self.fail_ready_on:
            # the encode "fails on the device": its rows keep stale contents
            db.codes[row0:row0 + r.X.shape[0]] = 0xEE
            return {"left": self.delay, "fail": True}
        db.codes[row0:row0 + r.X.shape[0]] = oracle.encode(r.X, db.C, db.M)
        return {"left": self.delay}

    def ready(self, h):
        h["left"] -= 1
        if h["left"] < 0 and h.get("fail"):
            raise RuntimeError("injected device error")
        return h["left"] < 0

    def query_results(self, h):
        out, o = [], 0
        for q in h["sizes"]:
            out.append((h["v"][o:o + q], h["i"][o:o + q]))
            o += q
        return out

    def plain_query(self, r, rows):
        return self._alone(self.dbs[r.db], r.Qv, r.metric, r.k, rows)

    def plain_insert(self, r, row0):
        self.launch_insert(r, row0)


def _requests(dbs, n=40, seed=3):
    rng = np.random.default_rng(seed)
    pool = synth.normal(seed + 100, (500, dbs[0].J))
    reqs = []
    for i in range(n):
        d = int(rng.integers(0, len(dbs)))
        if i % 7 == 3:
            m = int(rng.integers(5, 60))
            reqs.append(Request(i, "insert", d, 0.0, X=synth.normal(seed + i, (m, dbs[0].J))))
        else:
            q = int(rng.integers(1, 6))
            off = int(rng.integers(0, 400))
            metric = "l2" if i % 3 else "dot"
            reqs.append(Request(i, "query", d, 0.0, metric=metric, k=7, Qv=pool[off:off + q]))
    return reqs


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_mix_equals_alone_and_snapshots(mode):
    dbs = [FakeDB(10, 300, 2000), FakeDB(20, 500, 2000)]
    ex = FakeExecutor(dbs)
    reqs = _requests(dbs)
    srv = Server(ex, dbs, budget_bytes=10 ** 9, mode=mode)
    srv.run(reqs, realtime=False)
    assert all(r.status == "done" for r in reqs)
    for r in reqs:
        if r.kind == "query":
            v, i = ex._alone(dbs[r.db], r.Qv, r.metric, r.k, r.watermark)
            assert np.array_equal(v, r.vals) and np.array_equal(i, r.idx)
            assert dbs[r.db].n_rows <= r.watermark <= srv.committed[r.db]
        else:
            a, b = r.rows
            assert np.array_equal(dbs[r.db].codes[a:b], oracle.encode(r.X, dbs[r.db].C, dbs[r.db].M))
    # inserts are appended in admission order and all committed at the end
    for d in range(len(dbs)):
        assert srv.committed[d] == srv.reserved[d]
    if mode == "continuous":
        # requests that arrive together are served in shared launches
        assert sum(1 for l in ex.launches if l[0] == "query") < sum(r.kind == "query" for r in reqs)
    s = summarize(reqs, 1.0)
    assert s["done"] == len(reqs) and s["refused"] == 0


def test_budget_admission_and_refusal():
    dbs = [FakeDB(30, 200, 260)]
    ex = FakeExecutor(dbs, delay=5)
    pool = synth.normal(31, (50, 16))
    reqs = [Request(0, "query", 0, 0.0, k=5, Qv=pool[:3]),          # 300 bytes: fits
            Request(1, "query", 0, 0.0, k=5, Qv=pool[:4]),          # 400: waits for 0
            Request(2, "query", 0, 0.0, k=5, Qv=pool[:9]),          # 900 > budget: refused
            Request(3, "insert", 0, 0.0, X=synth.normal(32, (100, 16)))]   # beyond capacity: refused
    srv = Server(ex, dbs, budget_bytes=500)
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["done", "done", "refused", "refused"]
    assert srv.peak <= 500
    assert reqs[1].admitted >= reqs[0].done   # it had to wait for the first to release memory
    assert "budget" in reqs[2].error and "capacity" in reqs[3].error


def test_failure_is_isolated():
    dbs = [FakeDB(40, 200, 1000)]
    ex = FakeExecutor(dbs, fail_on={2})
    pool = synth.normal(41, (50, 16))
    # separate arrival times keep the launches apart
    reqs = [Request(i, "query", 0, 0.0, k=5, Qv=pool[i:i + 2]) for i in range(4)]
    srv = Server(ex, dbs, budget_bytes=250, max_groups=1)
    srv.run(reqs, realtime=False)
    st = [r.status for r in reqs]
    assert st.count("failed") == 1 and st.count("done") == 3
    assert "injected" in [r for r in reqs if r.status == "failed"][0].error


def _insert_then_query(dbs, seed):
    pool = synth.normal(seed, (40, 16))
    return [Request(0, "insert", 0, 0.0, X=synth.normal(seed + 1, (30, 16))),   # fails
            Request(1, "insert", 0, 0.0, X=synth.normal(seed + 2, (20, 16))),   # succeeds
            Request(2, "query", 0, 0.0, k=5, Qv=pool[:3])]


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_failed_insert_rows_never_become_visible(mode):
    """An insert that fails at launch hands its rows back: the next insert
    takes them, and no query's snapshot ever covers unencoded rows."""
    N = 200
    dbs = [FakeDB(50, N, 1000)]
    ex = FakeExecutor(dbs, fail_on={1})
    reqs = _insert_then_query(dbs, 51)
    srv = Server(ex, dbs, budget_bytes=10 ** 9, mode=mode, max_groups=1)
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["failed", "done", "done"]
    assert reqs[0].rows == ()
    assert reqs[1].rows == (N, N + 20)
    assert srv.committed[0] == srv.reserved[0] == N + 20
    q = reqs[2]
    assert q.watermark in (N, N + 20)
    db = dbs[0]
    assert np.array_equal(db.codes[N:N + 20], oracle.encode(reqs[1].X, db.C, db.M))
    v, i = ex._alone(db, q.Qv, q.metric, q.k, q.watermark)
    assert np.array_equal(v, q.vals) and np.array_equal(i, q.idx)


def test_insert_failing_on_the_device_blocks_the_watermark():
    """An insert reported failed at completion while a later insert holds the
    rows after it: the failed rows stay below no watermark, so neither they
    nor the later rows become visible; a failed newest insert is handed back."""
    N = 200
    dbs = [FakeDB(60, N, 1000)]
    pool = synth.normal(61, (40, 16))
    ex = FakeExecutor(dbs, delay=3, fail_ready_on={1})
    reqs = [Request(0, "insert", 0, 0.0, X=synth.normal(62, (30, 16))),     # fails on the device
            Request(1, "insert", 0, 0.0, X=synth.normal(63, (20, 16))),     # encoded after it
            Request(2, "query", 0, 0.0, k=5, Qv=pool[:3])]
    srv = Server(ex, dbs, budget_bytes=10 ** 9, max_groups=1)
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["failed", "done", "done"]
    assert srv.committed[0] == N                       # blocked below the failed rows
    assert reqs[2].watermark == N
    # the newest range failing is handed back instead
    dbs = [FakeDB(64, N, 1000)]
    ex = FakeExecutor(dbs, delay=3, fail_ready_on={2})
    reqs = [Request(0, "insert", 0, 0.0, X=synth.normal(65, (30, 16))),
            Request(1, "insert", 0, 0.0, X=synth.normal(66, (20, 16)))]   # fails, newest
    srv = Server(ex, dbs, budget_bytes=10 ** 9, max_groups=1)
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["done", "failed"]
    assert srv.committed[0] == srv.reserved[0] == N + 30


def test_metric_calls_pairs_directions():
    """A group's scan calls: a smallest-sums metric and a largest-sums one
    share a call (smallest first); the rest pair up within their direction;
    every request lands in exactly one call."""
    from paper_1706_10283_amd.serve import metric_calls

    def reqs(metrics):
        return [Request(i, "query", 0, 0.0, metric=m, k=5, Qv=np.zeros((1, 4))) for i, m in enumerate(metrics)]

    def names(calls):
        return [[m for m, _ in c] for c in calls]

    assert names(metric_calls(reqs(["l2"]))) == [["l2"]]
    assert names(metric_calls(reqs(["dot", "l2", "dot", "l2"]))) == [["l2", "dot"]]
    assert metric_calls(reqs(["dot", "l2", "dot", "l2"])) == [[("l2", [1, 3]), ("dot", [0, 2])]]
    assert names(metric_calls(reqs(["l2", "l1", "dot"]))) == [["l2", "dot"], ["l1"]]
    assert names(metric_calls(reqs(["l2", "l1", "lp3", "cosine"]))) == [["l2", "cosine"], ["l1", "lp3"]]
    assert names(metric_calls(reqs(["dot", "cosine", "dot"]))) == [["dot", "cosine"]]
    for ms in (["l2", "dot", "l1", "cosine", "lp4", "dot"], ["dot"] * 3 + ["l2"]):
        calls = metric_calls(reqs(ms))
        got = sorted(i for c in calls for _, ix in c for i in ix)
        assert got == list(range(len(ms)))
        for c in calls:
            assert 1 <= len(c) <= 2

