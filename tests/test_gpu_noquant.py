"""Bolt No Quantize (float-table scan and float top-k) on the GPU against the
oracle, through the C ABI.  The float sums are defined in one order
(ascending m, fp32 adds), so they must match bit for bit; top-k must match
exactly, ties by index."""
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


def _float_luts(seed, Q, J, M, metric):
    Qv = synth.normal(seed, (Q, J)) * 2
    C = synth.normal(seed + 1, (M, 16, J // M)) * 2
    _, l32, _ = oracle.luts(Qv, C, M, metric)
    return l32


SCAN_CASES = [(8, 1, 1000), (32, 13, 5000), (16, 8, 70_000), (64, 3, 1234), (256, 2, 300), (2, 9, 777),
              (130, 4, 513), (32, 20, 1), (32, 5, 0)]


@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N", SCAN_CASES)
def test_scan_f32_parity(bolt, metric, M, Q, N):
    seed = 3 * M + 7 * Q + N
    _say("scan_f32", metric, "seed", seed, "M", M, "Q", Q, "N", N)
    J = M * (2 if M <= 64 else 1)
    lut = _float_luts(seed, Q, J, M, metric)
    codes = synth.random_codes(seed + 5, N, M)
    ref = oracle.scan_f32(codes, lut)
    got = bolt.bolt_scan_f32(torch.from_numpy(codes).to(DEV), torch.from_numpy(lut).to(DEV)).cpu().numpy()
    assert got.shape == ref.shape
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


TOPK_CASES = [(1, 1000, 1, "rand"), (6, 70_000, 100, "rand"), (3, 5000, 2048, "rand"), (4, 3000, 100, "ties"),
              (2, 37, 100, "rand"), (5, 100_000, 10, "coarse")]


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("Q,N,k,kind", TOPK_CASES)
def test_topk_f32_parity(bolt, largest, Q, N, k, kind):
    seed = Q + N + k
    _say("topk_f32", kind, "largest", largest, "seed", seed, "Q", Q, "N", N, "k", k)
    d = synth.normal(seed, (Q, N)).astype(np.float32)
    if kind == "ties":
        d[:] = np.float32(2.5)
    elif kind == "coarse":
        d = (np.round(d * 2) / 2).astype(np.float32)
    vr, ir = oracle.topk_f32(d, k, largest)
    v, i = bolt.bolt_topk_f32(torch.from_numpy(d).to(DEV), k, largest)
    assert np.array_equal(i.cpu().numpy(), ir)
    assert np.array_equal(v.cpu().numpy().view(np.uint32), vr.view(np.uint32))


@pytest.mark.parametrize("metric", ["l2", "dot"])
def test_no_quantize_end_to_end(bolt, metric):
    """GPU float tables -> GPU float scan -> GPU float top-k equals the oracle."""
    N, J, M, Q, k = 20_000, 64, 16, 7, 25
    _say("no quantize end to end", metric, "N", N, "M", M, "Q", Q)
    X = synth.normal(81, (N, J))
    Qv = synth.normal(82, (Q, J))
    C = synth.normal(83, (M, 16, J // M))
    codes = oracle.encode(X, C, M)
    _, l32, _ = oracle.luts(Qv, C, M, metric)
    S = oracle.scan_f32(codes, l32)
    vr, ir = oracle.topk_f32(S, k, metric == "dot")
    Cd = torch.from_numpy(C).to(DEV)
    _, lf = bolt.bolt_build_luts(torch.from_numpy(Qv).to(DEV), Cd, M, metric, 1.0,
                                 torch.zeros(M, device=DEV), want_f32=True)
    Sg = bolt.bolt_scan_f32(torch.from_numpy(codes).to(DEV), lf)
    v, i = bolt.bolt_topk_f32(Sg, k, metric == "dot")
    assert np.array_equal(Sg.cpu().numpy().view(np.uint32), S.view(np.uint32))
    assert np.array_equal(i.cpu().numpy(), ir)


def test_no_quantize_errors(bolt):
    codes = torch.zeros((10, 4), dtype=torch.uint8, device=DEV)
    lut = torch.zeros((2, 7, 16), dtype=torch.float32, device=DEV)
    with pytest.raises(bolt.BoltError):
        bolt.bolt_scan_f32(codes, lut)          # odd M
    with pytest.raises(bolt.BoltError):
        bolt.bolt_topk_f32(torch.zeros((2, 5), device=DEV), 0)
