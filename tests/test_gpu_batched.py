"""Batched persistent scan + top-k over many uneven databases: bit-identical to
the oracle and to bolt_scan_topk on each database alone, under every tuning,
and when replayed from a HIP graph with new query tables."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available()
    return b


# (M, N, Q, k, metric, table kind)
DBS = [
    (32, 70000, 40, 100, "l2", "rand"), (16, 5000, 3, 10, "dot", "rand"), (64, 140000, 17, 256, "l2", "coarse"),
    (8, 100, 5, 100, "dot", "rand"), (32, 1, 8, 1, "l2", "rand"), (64, 33000, 1, 50, "dot", "const"),
    (16, 70000, 9, 100, "l2", "coarse"), (32, 0, 4, 10, "l2", "rand"), (8, 20000, 2, 7, "l2", "rand"),
    (32, 16385, 33, 100, "dot", "rand"), (64, 9000, 6, 100, "l2", "rand"), (16, 123457, 7, 256, "dot", "rand"),
    # matrix-core tiles at M = 64 (their own launch): ragged rows and query block, ties
    (64, 50001, 45, 100, "dot", "rand"), (64, 20000, 32, 64, "l2", "coarse"),
]


def _make(seed, M, N, Q, kind):
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 32).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 9)
    return codes, luts


def _build(bolt, seed0=500):
    host, dev = [], []
    for i, (M, N, Q, k, metric, kind) in enumerate(DBS):
        codes, luts = _make(seed0 + 7 * i, M, N, Q, kind)
        host.append((codes, luts, k, metric))
        dev.append({"codes": torch.from_numpy(codes).to(DEV), "luts": torch.from_numpy(luts).to(DEV),
                    "k": k, "metric": metric})
    return host, dev


@pytest.mark.parametrize("tuning", [None, (4096, 0, 1), (65536, 7, 8), (1024, 2, 3)])
def test_batched_matches_oracle_and_single(bolt, tuning):
    print("[case] batched tuning", tuning, flush=True)
    host, dev = _build(bolt)
    plan = bolt.BatchPlan(dev, tuning=tuning)
    print("[case] plan", plan.info(), flush=True)
    plan.run()
    torch.cuda.synchronize()
    for (codes, luts, k, metric), d, (v, i) in zip(host, dev, plan.results()):
        vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
        assert np.array_equal(v.cpu().numpy(), vr)
        assert np.array_equal(i.cpu().numpy(), ir)
        if codes.shape[0] > 0:
            vs, is_ = bolt.bolt_scan_topk(d["codes"], d["luts"], metric, k)
            assert np.array_equal(vs.cpu().numpy(), vr) and np.array_equal(is_.cpu().numpy(), ir)
    plan.close()


def test_batched_graph_replays_with_new_tables(bolt):
    """Capture once, replay three times with the query tables rewritten in
    place between replays (eager work and synchronisation in between); every
    replay equals the eager single-database result."""
    host, dev = _build(bolt, seed0=900)
    plan = bolt.BatchPlan(dev, tuning=(16384, 4, 3))
    plan.capture()
    for rep in range(3):
        print("[case] graph replay", rep, flush=True)
        for j, d in enumerate(dev):
            M = d["luts"].shape[1]
            new = synth.random_luts(3000 + 31 * rep + j, d["luts"].shape[0], M)
            d["luts"].copy_(torch.from_numpy(new).to(DEV))
        torch.cuda.synchronize()
        plan.launch_graph()
        torch.cuda.synchronize()
        for d, (v, i) in zip(dev, plan.results()):
            if d["codes"].shape[0] == 0:
                assert (i.cpu().numpy() == -1).all()
                continue
            vs, is_ = bolt.bolt_scan_topk(d["codes"], d["luts"], d["metric"], d["k"])
            torch.cuda.synchronize()
            assert np.array_equal(v.cpu().numpy(), vs.cpu().numpy())
            assert np.array_equal(i.cpu().numpy(), is_.cpu().numpy())
    plan.close()


def test_batched_rejects_bad_input(bolt):
    codes = torch.zeros((10, 5), dtype=torch.uint8, device=DEV)
    luts = torch.zeros((2, 10, 16), dtype=torch.uint8, device=DEV)
    with pytest.raises(bolt.BoltError):
        bolt.BatchPlan([{"codes": codes, "luts": luts, "k": 5}])
    codes = torch.zeros((10, 16), dtype=torch.uint8, device=DEV)
    luts = torch.zeros((2, 32, 16), dtype=torch.uint8, device=DEV)
    with pytest.raises(bolt.BoltError):
        bolt.BatchPlan([{"codes": codes, "luts": luts, "k": 300}])


# databases large enough for speculative bounds (2^16 rows),
# with matrix-core tiles (M = 16, 32 or 64, 8 or more queries), beside others
SPEC_DBS = [
    (32, 140000, 40, 100, "l2", "rand"), (16, 150000, 70, 64, "dot", "coarse"), (32, 131072, 33, 1, "dot", "const"),
    (64, 140000, 40, 100, "l2", "rand"), (16, 20000, 50, 10, "l2", "rand"), (32, 160000, 5, 100, "dot", "rand"),
    # 8 to 31 queries: one part-filled 32-query matrix-core tile per database
    (32, 140000, 8, 100, "l2", "rand"), (16, 150000, 9, 64, "dot", "coarse"), (64, 131100, 17, 100, "dot", "rand"),
    (32, 135000, 31, 128, "l2", "coarse"),
]


@pytest.mark.parametrize("mode", [1, 2])
def test_batched_speculation(bolt, mode):
    """Sampled starting bounds (mode 1), and all of them failing (mode 2: every
    speculative query recomputed exactly): results equal the oracle's."""
    print("[case] batched speculation mode", mode, flush=True)
    host, dev = [], []
    for i, (M, N, Q, k, metric, kind) in enumerate(SPEC_DBS):
        codes, luts = _make(700 + 11 * i, M, N, Q, kind)
        host.append((codes, luts, k, metric))
        dev.append({"codes": torch.from_numpy(codes).to(DEV), "luts": torch.from_numpy(luts).to(DEV),
                    "k": k, "metric": metric})
    bolt.debug_speculation(mode)
    try:
        plan = bolt.BatchPlan(dev, tuning=(16384, 4, 2))
        plan.run()
        torch.cuda.synchronize()
        res = [(v.cpu().numpy(), i.cpu().numpy()) for v, i in plan.results()]
        plan.close()
    finally:
        bolt.debug_speculation(-1)
    for (codes, luts, k, metric), (v, i) in zip(host, res):
        vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
        assert np.array_equal(v, vr)
        assert np.array_equal(i, ir)
