"""GPU parity of the two-metric scan + top-k (bolt_scan_topk_split) against
the oracle, through the C ABI.

Queries [0, q_split) rank under one metric and [q_split, Q) under another;
each side must equal the oracle's top-k of its own tables and direction, bit
for bit.  The cases cover one set of launches for both directions (the
matrix-core tiles, with sampled bounds holding, all failing or off, the split
inside a query tile and on its edge), the two sides run one after the other
(few-query, grouped and unfused shapes), metrics of one direction, the empty
sides q_split = 0 and Q, padding (N < k, N = 0) and total ties.  Each case
prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
LARGEST = {"l2": False, "l1": False, "lp3": False, "dot": True, "cosine": True}


@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return b


def _say(*a):
    print("[case]", *a, flush=True)


def _luts(seed, Q, M, kind):
    luts = synth.random_luts(seed, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    return luts


def _expected(codes, luts, q_split, lo, hi, k):
    """The oracle's top-k of each side under its own direction, stacked."""
    vs, ix = [], []
    for a, b, metric in ((0, q_split, lo), (q_split, luts.shape[0], hi)):
        if b > a:
            v, i = oracle.topk(oracle.scan(codes, luts[a:b]), k, LARGEST[metric])
            vs.append(v)
            ix.append(i)
    return np.concatenate(vs), np.concatenate(ix)


SPLIT_CASES = [
    # (M, Q, q_split, N, k, lut kind, metric_lo, metric_hi, speculation mode)
    # both directions in one set of launches (matrix-core tiles)
    (32, 70, 31, 200_000, 100, "rand", "l2", "dot", 1),
    (32, 70, 31, 200_000, 100, "rand", "dot", "l2", 2),
    (32, 70, 64, 180_000, 64, "coarse", "l2", "cosine", 1),
    (16, 40, 17, 150_000, 64, "coarse", "l2", "dot", 0),
    (64, 33, 32, 140_000, 128, "rand", "cosine", "l1", 1),
    (64, 33, 1, 140_000, 128, "rand", "dot", "l2", 2),
    (8, 40, 20, 160_000, 50, "rand", "l2", "dot", -1),
    (32, 5, 2, 300_001, 100, "coarse", "l2", "dot", 1),
    (16, 6, 5, 170_000, 1, "rand", "dot", "l2", 2),
    (32, 40, 13, 150_000, 256, "const", "l2", "dot", 1),
    (32, 40, 13, 150_000, 100, "const", "dot", "l2", 2),
    (32, 20, 7, 5, 100, "rand", "l2", "dot", -1),
    (32, 64, 32, 16_384 * 2 + 77, 100, "rand", "dot", "l2", 0),
    # the two sides one after the other: few-query, grouped (k above the
    # matrix-core cap), M = 6 (unfused) and an empty database
    (32, 2, 1, 200_000, 100, "rand", "l2", "dot", -1),
    (16, 50, 25, 70_000, 200, "rand", "l2", "dot", -1),
    (6, 9, 4, 1000, 7, "rand", "dot", "l2", -1),
    (32, 30, 10, 0, 10, "rand", "l2", "dot", -1),
    # one direction on both sides, and empty sides
    (32, 40, 11, 150_000, 100, "rand", "l2", "l1", -1),
    (32, 40, 40, 150_000, 100, "rand", "l2", "dot", -1),
    (32, 40, 0, 150_000, 100, "rand", "l2", "dot", -1),
]


@pytest.mark.parametrize("M,Q,q_split,N,k,kind,lo,hi,mode", SPLIT_CASES)
def test_scan_topk_split_parity(bolt, M, Q, q_split, N, k, kind, lo, hi, mode):
    seed = 19 * M + 3 * Q + 7 * q_split + N + k
    _say("split scan_topk", lo, hi, kind, "mode", mode, "seed", seed, "M", M, "Q", Q, "q_split", q_split, "N", N,
         "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = _luts(seed + 1, Q, M, kind)
    vr, ir = _expected(codes, luts, q_split, lo, hi, k)
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_speculation(mode)
    try:
        v, i = bolt.bolt_scan_topk_split(cd, ld, q_split, lo, hi, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_speculation(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


@pytest.mark.parametrize("force", ["unfused", "grouped"])
def test_scan_topk_split_forced_paths(bolt, force):
    """With the unfused path or the grouped kernel forced, the call runs the
    two sides one after the other and still equals the oracle."""
    M, Q, q_split, N, k = 32, 45, 20, 90_000, 100
    seed = 1234 + len(force)
    _say("split scan_topk forced", force, "seed", seed, "M", M, "Q", Q, "q_split", q_split, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = _luts(seed + 1, Q, M, "rand")
    vr, ir = _expected(codes, luts, q_split, "l2", "dot", k)
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    if force == "unfused":
        bolt.debug_force_unfused_topk(True)
    else:
        bolt.debug_force_fused_kind(2)
    try:
        v, i = bolt.bolt_scan_topk_split(cd, ld, q_split, "l2", "dot", k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_force_unfused_topk(False)
        bolt.debug_force_fused_kind(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


def test_scan_topk_split_errors(bolt):
    codes = torch.zeros((100, 16), dtype=torch.uint8, device=DEV)
    luts = torch.zeros((4, 32, 16), dtype=torch.uint8, device=DEV)
    for q_split in (-1, 5):
        _say("split scan_topk error", "q_split", q_split)
        with pytest.raises(bolt.BoltError) as e:
            bolt.bolt_scan_topk_split(codes, luts, q_split, "l2", "dot", 10)
        assert e.value.status == bolt.BOLT_ERR_INVALID
        assert "q_split" in bolt.last_error()
    assert bolt.bolt_scan_topk_split_ws_bytes(100, 32, 4, 5, 10) == 0
    need = bolt.bolt_scan_topk_split_ws_bytes(100, 32, 4, 2, 10)
    assert need > 0
    ws = torch.empty(need - 1, dtype=torch.uint8, device=DEV)
    with pytest.raises(bolt.BoltError) as e:
        bolt.bolt_scan_topk_split(codes, luts, 2, "l2", "dot", 10, ws=ws)
    assert e.value.status == bolt.BOLT_ERR_NOMEM
