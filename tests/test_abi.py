"""The C-ABI library loads on the host and exports every symbol include/bolt.h
declares; argument validation runs on the host without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bolt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1706_10283_amd.bolt as b
    return b


def test_exports_every_declared_symbol(lib):
    names = _declared("bolt.h")
    assert "bolt_encode" in names and "bolt_scan_topk" in names
    for n in names:
        assert hasattr(lib.lib(), n), n


def test_validation_without_gpu(lib):
    L = lib.lib()
    # J % M != 0, odd M, M > 256: shape errors before any device work
    assert L.bolt_encode(None, 10, 30, 30, None, 4, None, None) == lib.BOLT_ERR_SHAPE
    assert L.bolt_encode(None, 10, 30, 30, None, 3, None, None) == lib.BOLT_ERR_SHAPE
    assert L.bolt_scan_l2(None, 10, 258, None, 1, None, 10, None) == lib.BOLT_ERR_SHAPE
    # empty work is a no-op
    assert L.bolt_encode(None, 0, 32, 32, None, 8, None, None) == lib.BOLT_OK
    assert L.bolt_scan_l2(None, 0, 8, None, 5, None, 0, None) == lib.BOLT_OK
    # null pointers with work, bad k, bad ld
    assert L.bolt_encode(None, 10, 32, 32, None, 8, None, None) == lib.BOLT_ERR_INVALID
    assert L.bolt_topk(None, 1, 10, 10, 0, 0, None, None, None, 0, None) == lib.BOLT_ERR_INVALID
    assert L.bolt_topk(None, 1, 10, 10, 4096, 0, None, None, None, 0, None) == lib.BOLT_ERR_UNSUPPORTED
    assert L.bolt_scan_l2(None, 10, 8, None, 1, None, 5, None) == lib.BOLT_ERR_INVALID
    assert "ldo" in lib.last_error()
    # metric codes: L_p for 1 <= p <= 16 (3 + 256 p), cosine 4; others rejected
    for bad in (3, 5, 3 + 256 * 17, -1, 3 + 128):
        assert L.bolt_build_luts(None, 0, 32, 32, None, 8, bad, 1.0, None, None, None, None) \
            == lib.BOLT_ERR_INVALID
    for good in (0, 1, 2, 4, lib.metric_lp(1), lib.metric_lp(16)):
        assert L.bolt_build_luts(None, 0, 32, 32, None, 8, good, 1.0, None, None, None, None) == lib.BOLT_OK
    assert lib.metric_id("lp3") == 3 + 256 * 3 and lib.metric_largest("cosine") and not lib.metric_largest("lp2")
    # two-metric scan + top-k: split index, metrics and shape checked first
    split = lambda N, M, Q, q_split, lo, hi, k: L.bolt_scan_topk_split(
        None, N, M, None, Q, q_split, lo, hi, k, None, None, None, 0, None)
    assert split(10, 32, 4, 5, 0, 1, 3) == lib.BOLT_ERR_INVALID
    assert "q_split" in lib.last_error()
    assert split(10, 32, 4, -1, 0, 1, 3) == lib.BOLT_ERR_INVALID
    assert split(10, 32, 4, 2, 0, 5, 3) == lib.BOLT_ERR_INVALID
    assert split(10, 31, 4, 2, 0, 1, 3) == lib.BOLT_ERR_SHAPE
    assert split(10, 32, 0, 0, 0, 1, 3) == lib.BOLT_OK
    assert split(10, 32, 4, 2, 0, 1, 3) == lib.BOLT_ERR_INVALID   # null pointers with work
    # misaligned codes or tables are rejected before anything is enqueued (the
    # pointers are never dereferenced on the host)
    P = ctypes.c_void_p
    for c, t in ((0x10001, 0x20000), (0x10000, 0x20008)):
        assert L.bolt_scan_topk(P(c), 1000, 32, P(t), 4, 0, 10, P(0x30000), P(0x40000), P(0x50000),
                                1 << 30, None) == lib.BOLT_ERR_INVALID
        assert "aligned" in lib.last_error()
    # M = 12 has no fused kernel: room for the [Q][N] sums
    assert lib.bolt_scan_topk_ws_bytes(1000, 12, 10, 100) >= 1000 * 10 * 2
    # M = 32 takes the fused path: candidate buffers only, far below the sums
    assert 0 < lib.bolt_scan_topk_ws_bytes(10**8, 32, 64, 100) < 10**8 * 64 * 2 // 20


def test_train_host_matches_oracle_definition(lib):
    """Host trainer of the library vs the oracle's (same definition, written
    independently; the oracle's k-means is pinned to scikit-learn's Lloyd
    iterations in test_oracle_pins.py)."""
    J, M = 32, 8
    X = synth.normal(201, (3000, J))
    init = synth.permutation_prefix(202, 3000, 16)
    Qt = X[synth.permutation_prefix(203, 3000, 300)]
    for metric in ("l2", "dot", "lp3", "cosine"):
        C, a, offs, ai = lib.bolt_train_host(X, M, 6, init, Qt, metric)
        Co, ao, offso, aio = oracle.train(X, M, 6, init, Qt, metric)
        np.testing.assert_allclose(C, Co, rtol=1e-5, atol=1e-6)
        assert ai == aio
        assert a == pytest.approx(ao, rel=1e-5)
        np.testing.assert_allclose(offs, offso, rtol=1e-4, atol=1e-3)


def test_serving_workspace_reservation_covers_any_group(lib):
    """The serving admission reserves scan_ws_reserve(q) per request of q
    queries; admitted requests of one database run as one call, so the call's
    workspace must not exceed the sum of its members' reservations, also when
    the group's requests form the two sides of a two-metric call.  Checked
    over the serving shapes (one to 64 queries per request: the few-query,
    part-filled matrix-core and many-query paths, with and without sampled
    bounds)."""
    from paper_1706_10283_amd.serve import scan_ws_reserve
    rng = np.random.default_rng(7)
    for N in (60_000, 1_000_000, 250_000_000):
        for M in (8, 16, 32, 64):
            for _ in range(60):
                sizes = rng.integers(1, 65, size=int(rng.integers(1, 7)))
                if rng.random() < 0.3:
                    sizes = rng.integers(1, 8, size=int(rng.integers(2, 7)))
                k = int(rng.choice([10, 100, 128, 256]))
                group = lib.bolt_scan_topk_ws_bytes(N, M, int(sizes.sum()), k)
                reserved = sum(scan_ws_reserve(N, M, int(q), k) for q in sizes)
                assert group <= reserved, (N, M, sizes.tolist(), k, group, reserved)
                # the same requests as the two sides of one two-metric call
                cut = int(rng.integers(0, len(sizes) + 1))
                q_lo, Q = int(sizes[:cut].sum()), int(sizes.sum())
                split = lib.bolt_scan_topk_split_ws_bytes(N, M, Q, q_lo, k)
                assert split >= group
                assert split <= reserved, (N, M, sizes.tolist(), cut, k, split, reserved)
