"""Scan + top-k over row ranges (bolt_scan_topk_ranges) against the oracle on
the same rows, through the C ABI: bit-exact values and global row indices,
ties by index across ranges."""
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return b


def _say(*a):
    print("[case]", *a, flush=True)


def _expected(codes, luts, ranges, k, largest):
    rows = np.concatenate([np.arange(a, b) for a, b in ranges] + [np.zeros(0, np.int64)]).astype(np.int64)
    S = oracle.scan(codes[rows], luts)
    vr, ir = oracle.topk(S, k, largest)
    gi = np.where(ir >= 0, rows[np.maximum(ir, 0)] if len(rows) else -1, -1).astype(np.int32)
    return vr, gi


CASES = [
    # (M, Q, N, k, ranges, lut kind)
    (32, 1, 50_000, 100, [(0, 50_000)], "rand"),
    (32, 1, 300_000, 100, [(100, 70_000), (150_000, 150_000), (200_001, 290_000)], "rand"),
    (16, 3, 120_000, 50, [(5, 10), (20, 70_000), (80_000, 120_000)], "coarse"),
    (32, 20, 100_000, 100, [(1000, 17_000), (40_000, 99_999)], "rand"),
    (64, 9, 90_000, 64, [(0, 1), (3, 5), (10, 90_000)], "rand"),
    (8, 40, 70_000, 10, [(0, 35_000), (35_000, 70_000)], "const"),
    (32, 2, 10_000, 100, [(100, 150)], "rand"),
    (32, 5, 10_000, 10, [], "rand"),
    (32, 12, 10_000, 10, [(7, 7), (9, 9)], "rand"),
]


@pytest.mark.parametrize("metric", ["l2", "dot", "l1"])
@pytest.mark.parametrize("M,Q,N,k,ranges,kind", CASES)
def test_scan_topk_ranges_parity(bolt, metric, M, Q, N, k, ranges, kind):
    seed = M + 3 * Q + N + k + len(ranges)
    _say("ranges", metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k, "ranges", ranges)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 2)
    vr, ir = _expected(codes, luts, ranges, k, metric == "dot")
    v, i = bolt.bolt_scan_topk_ranges(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV), metric,
                                      k, np.array(ranges, dtype=np.int64).reshape(-1, 2))
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


def test_whole_range_equals_scan_topk(bolt):
    N, M, Q, k = 200_000, 32, 10, 100
    codes = torch.from_numpy(synth.random_codes(5, N, M)).to(DEV)
    luts = torch.from_numpy(synth.random_luts(6, Q, M)).to(DEV)
    v, i = bolt.bolt_scan_topk(codes, luts, "l2", k)
    vr, ir = bolt.bolt_scan_topk_ranges(codes, luts, "l2", k, [[0, N]])
    assert torch.equal(v, vr) and torch.equal(i, ir)


def test_ranges_errors(bolt):
    codes = torch.zeros((1000, 16), dtype=torch.uint8, device=DEV)
    luts = torch.zeros((2, 32, 16), dtype=torch.uint8, device=DEV)
    for bad in ([[10, 5]], [[0, 10], [5, 20]], [[0, 1001]], [[-1, 3]]):
        with pytest.raises(bolt.BoltError):
            bolt.bolt_scan_topk_ranges(codes, luts, "l2", 10, bad)
