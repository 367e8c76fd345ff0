"""bolt_scan_topk_noalloc through the C ABI: the same result as
bolt_scan_topk (which takes a caller workspace), on two calls in a row, the
second with a smaller input, so that the shared static scratch is reused
with the first call's contents still in it; an oversized request is
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"

# (M, Q, N, k, metric): matrix-core tiles with sampled bounds, then the
# few-query kernel on a smaller database, then a shape without a fused
# kernel (M = 12: scan into the scratch, then select)
CASES = [(32, 40, 600_000, 100, "l2"), (16, 5, 20_000, 10, "dot"), (12, 3, 5_000, 7, "l2")]


@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fn = b.lib().bolt_scan_topk_noalloc
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    fn.argtypes = [P, I64, I32, P, I64, I32, I32, P, P, P]
    fn.restype = ctypes.c_int
    return b


def _noalloc(b, codes, luts, metric, k):
    Q, M = luts.shape[0], luts.shape[1]
    vals = torch.empty((Q, k), dtype=torch.uint16, device=DEV)
    idx = torch.empty((Q, k), dtype=torch.int32, device=DEV)
    st = b.lib().bolt_scan_topk_noalloc(codes.data_ptr(), codes.shape[0], M, luts.data_ptr(), Q,
                                        b.metric_id(metric), k, vals.data_ptr(), idx.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)
    assert st == 0, b.last_error()
    return vals, idx


def test_noalloc_equals_workspace_entry_point(bolt):
    for M, Q, N, k, metric in CASES:
        print("[case] noalloc M", M, "Q", Q, "N", N, "k", k, metric, flush=True)
        codes = synth.random_codes(7 * M + N, N, M)
        luts = synth.random_luts(7 * M + N + 1, Q, M)
        cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
        v, i = _noalloc(bolt, cd, ld, metric, k)
        vr, ir = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), vr.cpu().numpy())
        assert np.array_equal(i.cpu().numpy(), ir.cpu().numpy())
        if N <= 20_000:
            vo, io = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
            assert np.array_equal(v.cpu().numpy(), vo) and np.array_equal(i.cpu().numpy(), io)


def test_noalloc_refuses_beyond_its_scratch(bolt):
    """A request whose workspace exceeds the scratch is refused on the host
    (the pointers are never used)."""
    N, M, Q, k = 1_000_000, 32, 4000, 100
    assert bolt.bolt_scan_topk_ws_bytes(N, M, Q, k) > 64 << 20
    P = ctypes.c_void_p
    st = bolt.lib().bolt_scan_topk_noalloc(P(0x1000), N, M, P(0x2000), Q, 0, k, P(0x3000), P(0x4000), None)
    assert st == bolt.BOLT_ERR_UNSUPPORTED
    assert "scratch" in bolt.last_error()
