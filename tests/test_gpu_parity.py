"""GPU parity of every hot-path step against the CPU oracle, through the C ABI.

Integer results (codes, uint8 tables, sums, top-k) must be bit-exact; fp32
tables match the exact fp64 tables to 1e-5 relative (L2) or 1e-5 of
sum_j |q_j c_j| (dot) and equal the oracle's canonical fp32 order bit for bit.
Each case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return b


DEV = "cuda"


def _say(*a):
    print("[case]", *a, flush=True)


def _unpack(codes, M):
    out = np.empty((codes.shape[0], M), dtype=np.int64)
    out[:, 0::2] = codes & 15
    out[:, 1::2] = codes >> 4
    return out


def _train(X, M, seed, metric="l2", n_q=200):
    init = synth.permutation_prefix(seed + 4, X.shape[0], 16)
    Qt = X[synth.permutation_prefix(seed + 5, X.shape[0], n_q)]
    C, a, offs, _ = oracle.train(X, M, 4, init, Qt, metric)
    return C, a, offs


# ------------------------------------------------------------------ encode

ENCODE_CASES = [
    # (N, J, M): subspace widths 1, 2, 4, 8, 16, 32 (tuned) and 3, 64 (generic)
    (0, 32, 8), (1, 32, 8), (63, 32, 8), (64, 32, 8), (65, 32, 8), (1000, 32, 8),
    (777, 16, 16), (517, 32, 16), (300, 128, 32), (129, 128, 16), (200, 256, 16),
    (257, 64, 2), (100, 24, 8), (50, 128, 2), (70, 6, 2), (333, 256, 256), (130, 130, 130),
]


@pytest.mark.parametrize("N,J,M", ENCODE_CASES)
def test_encode_parity(bolt, N, J, M):
    seed = 7 * N + J + M
    _say("encode", "seed", seed, "N", N, "J", J, "M", M)
    X = synth.normal(seed, (N, J)) * 3
    C = synth.normal(seed + 1, (M, 16, J // M)) * 3
    ref = oracle.encode(X, C, M)
    got = bolt.bolt_encode(torch.from_numpy(X).to(DEV), torch.from_numpy(C).to(DEV), M)
    torch.cuda.synchronize()
    assert got.shape == ref.shape
    assert np.array_equal(got.cpu().numpy(), ref)


def test_encode_mixture_full_tile_and_strided(bolt):
    """Mixture data (integer-valued, many exact ties between centroids made
    from data rows), a strided X and an unaligned output pointer."""
    N, J, M = 5000, 128, 32
    _say("encode mixture strided", "N", N, "J", J, "M", M)
    X = synth.gmm_rows(21, 22, 0, N, J)
    init = synth.permutation_prefix(23, N, 16)
    C, _ = oracle.kmeans(X, M, 3, init)
    ref = oracle.encode(X, C, M)
    Xp = np.zeros((N, J + 12), np.float32)
    Xp[:, :J] = X
    Xd = torch.from_numpy(Xp).to(DEV)[:, :J]
    buf = torch.zeros(N * M // 2 + 1, dtype=torch.uint8, device=DEV)
    out = buf[1:].view(N, M // 2)
    bolt.bolt_encode(Xd, torch.from_numpy(C).to(DEV), M, codes=out)
    got = bolt.bolt_encode(torch.from_numpy(X).to(DEV), torch.from_numpy(C).to(DEV), M)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(got.cpu().numpy(), ref)


def test_encode_gap_report(bolt):
    """Any code that differs from the fp64 argmin is a near tie (gap <= 1e-6)."""
    N, J, M = 4000, 64, 16
    X = synth.normal(31, (N, J))
    C = synth.normal(32, (M, 16, J // M))
    got = bolt.bolt_encode(torch.from_numpy(X).to(DEV), torch.from_numpy(C).to(DEV), M).cpu().numpy()
    d64 = oracle.subspace_dists_f64(X, C, M)
    gu = _unpack(got, M)
    best = d64.argmin(-1)
    n, m = np.nonzero(gu != best)
    gap = (d64[n, m, gu[n, m]] - d64[n, m, best[n, m]]) / np.maximum(d64[n, m, best[n, m]], 1e-38)
    print("fp64 near-tie exceptions: %d of %d" % (len(n), N * M))
    assert (gap <= 1e-6).all()


# ------------------------------------------------------------------ tables

@pytest.mark.parametrize("metric", ["l2", "dot", "l1", "lp1", "lp2", "lp3", "lp5", "cosine"])
@pytest.mark.parametrize("Q,J,M", [(1, 32, 8), (17, 128, 32), (100, 64, 16), (5, 256, 16),
                                   (9, 6, 2), (3, 256, 256)])
def test_luts_parity(bolt, metric, Q, J, M):
    seed = Q + J + M
    _say("luts", metric, "seed", seed, "Q", Q, "J", J, "M", M)
    Qv = synth.normal(seed, (Q, J)) * 2
    C = synth.normal(seed + 1, (M, 16, J // M)) * 2
    a = np.float32(4.3)
    offs = synth.uniform(seed + 2, (M,), -20.0, 20.0)
    l64, l32, l8 = oracle.luts(Qv, C, M, metric, float(a), offs)
    u8, f32 = bolt.bolt_build_luts(torch.from_numpy(Qv).to(DEV), torch.from_numpy(C).to(DEV), M,
                                   metric, float(a), torch.from_numpy(offs).to(DEV), want_f32=True)
    torch.cuda.synchronize()
    f32 = f32.cpu().numpy()
    assert np.array_equal(u8.cpu().numpy(), l8)
    assert np.array_equal(f32.view(np.uint32), l32.view(np.uint32))
    if metric not in ("dot", "cosine"):
        assert (np.abs(f32 - l64) <= 1e-5 * l64 + 1e-30).all()
    else:
        sub = J // M
        Qs = Qv.astype(np.float64)
        if metric == "cosine":
            Qs = Qs / np.linalg.norm(Qs, axis=1, keepdims=True)
        scale = (np.abs(Qs.reshape(Q, M, 1, sub)) * np.abs(C[None])).sum(-1)
        assert (np.abs(f32 - l64) <= 1e-5 * scale).all()


@pytest.mark.parametrize("N,J", [(0, 8), (1, 32), (300, 128), (1000, 7), (257, 256)])
def test_normalize_rows_parity(bolt, N, J):
    """Unit rows (cosine similarity) bit for bit against the oracle, a zero
    row included; strided input, separate and in-place output."""
    _say("normalize rows", "N", N, "J", J)
    X = synth.normal(N + J, (N, J)) * 7
    if N > 3:
        X[3] = 0.0
    ref = oracle.normalize_rows(X)
    Xp = torch.zeros((N, J + 5), dtype=torch.float32, device=DEV)
    Xp[:, :J] = torch.from_numpy(X).to(DEV)
    got = bolt.bolt_normalize_rows(Xp[:, :J])
    inplace = torch.from_numpy(X).to(DEV)
    bolt.bolt_normalize_rows(inplace, out=inplace)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(inplace.cpu().numpy().view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------------------ scan

SCAN_M = [2, 4, 6, 8, 16, 32, 64, 128, 256]


@pytest.mark.parametrize("kind", [-1, 0, 1, 2, 3])
@pytest.mark.parametrize("M", SCAN_M)
@pytest.mark.parametrize("Q", [1, 3, 7, 8, 9, 33, 70])
def test_scan_parity(bolt, kind, M, Q):
    tuned = M in (8, 16, 32, 64, 128, 256)
    if kind == 2 and not tuned:
        pytest.skip("the grouped kernel takes power-of-two M in 8..256")
    if kind == 3 and M not in (8, 16, 32, 64):
        pytest.skip("the matrix-core kernel takes M in {8, 16, 32, 64}")
    if kind == 1 and M not in (8, 16, 32, 64):
        pytest.skip("the few-query kernel takes M in {8, 16, 32, 64}")
    if kind == 1 and Q >= 8:
        pytest.skip("few-query kernel takes Q < 8")
    N = 3000 + 37
    seed = 1000 * M + Q
    _say("scan kind", kind, "seed", seed, "N", N, "M", M, "Q", Q)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    ref = oracle.scan(codes, luts)
    bolt.debug_force_scan_kernel(kind)
    try:
        got = bolt.bolt_scan_l2(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV))
        got2 = bolt.bolt_scan_dot(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV))
        torch.cuda.synchronize()
    finally:
        bolt.debug_force_scan_kernel(-1)
    assert np.array_equal(got.cpu().numpy(), ref)
    assert np.array_equal(got2.cpu().numpy(), ref)


def test_scan_extremes_and_edges(bolt):
    """All-255 tables at M = 256 reach the largest sum 65280; N = 0, 1; ldo > N."""
    M, N, Q = 256, 1001, 9
    codes = synth.random_codes(5, N, M)
    luts = np.full((Q, M, 16), 255, np.uint8)
    got = bolt.bolt_scan_l2(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV))
    assert (got.cpu().numpy() == 65280).all()
    for n in (0, 1):
        c = synth.random_codes(6, n, 32)
        lt = synth.random_luts(7, 10, 32)
        got = bolt.bolt_scan_l2(torch.from_numpy(c).to(DEV), torch.from_numpy(lt).to(DEV))
        assert np.array_equal(got.cpu().numpy(), oracle.scan(c, lt))
    c = synth.random_codes(8, 500, 16)
    lt = synth.random_luts(9, 12, 16)
    big = torch.full((12, 640), 7, dtype=torch.uint16, device=DEV)
    bolt.bolt_scan_l2(torch.from_numpy(c).to(DEV), torch.from_numpy(lt).to(DEV), out=big[:, :500])
    b = big.cpu().numpy()
    assert np.array_equal(b[:, :500], oracle.scan(c, lt))
    assert (b[:, 500:] == 7).all()


# ------------------------------------------------------------------ top-k

@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("N,k,hi", [(0, 5, 10), (1, 1, 10), (5, 10, 3), (100, 7, 1000),
                                    (10000, 100, 65535), (10000, 100, 20), (4097, 2048, 500),
                                    (3000, 2048, 65535), (50000, 1, 3)])
def test_topk_parity(bolt, largest, N, k, hi):
    Q = 6
    seed = N + k + hi
    _say("topk", "seed", seed, "N", N, "k", k, "largest", largest)
    d = synth.integers(seed, 0, hi, (Q, N)).astype(np.uint16)
    vr, ir = oracle.topk(d, k, largest)
    vals, idx = bolt.bolt_topk(torch.from_numpy(d).to(DEV), k, largest)
    torch.cuda.synchronize()
    assert np.array_equal(vals.cpu().numpy(), vr)
    assert np.array_equal(idx.cpu().numpy(), ir)


def test_topk_constant_rows_and_stride(bolt):
    d = np.full((3, 999), 1234, np.uint16)
    vals, idx = bolt.bolt_topk(torch.from_numpy(d).to(DEV), 50, False)
    assert idx.cpu().numpy().tolist() == [list(range(50))] * 3
    big = torch.from_numpy(synth.integers(3, 0, 9, (4, 1000)).astype(np.uint16)).to(DEV)
    sub = big[:, 1:998]
    vr, ir = oracle.topk(sub.cpu().numpy(), 33, True)
    v, i = bolt.bolt_topk(sub, 33, True)
    assert np.array_equal(v.cpu().numpy(), vr) and np.array_equal(i.cpu().numpy(), ir)


@pytest.mark.parametrize("metric", ["l2", "dot", "lp4", "cosine"])
@pytest.mark.parametrize("M,Q,k", [(8, 16, 10), (32, 1, 100), (32, 40, 100), (64, 9, 33), (6, 5, 7)])
def test_scan_topk_parity(bolt, metric, M, Q, k):
    N = 20011
    seed = M * Q + k
    _say("scan_topk", metric, "seed", seed, "N", N, "M", M, "Q", Q, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = (synth.random_luts(seed + 1, Q, M) // 16).astype(np.uint8)   # many ties
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric in ("dot", "cosine"))
    v, i = bolt.bolt_scan_topk(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV),
                               metric, k)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


# ------------------------------------------------------------------ approximate matrix product

@pytest.mark.parametrize("kernel", [-1, 2, 3])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("K", [1, 5, 64, 97])
def test_amm_parity(bolt, kernel, transpose, K):
    N, M = 2345, 32
    if kernel >= 2 and K < 8:
        pytest.skip("the grouped and matrix-core kernels are for 8 or more queries")
    _say("amm", "N", N, "M", M, "K", K, "transpose", transpose, "kernel", kernel)
    codes = synth.random_codes(K, N, M)
    luts = synth.random_luts(K + 1, K, M)
    bias, scale = np.float32(-311.25), np.float32(1.0 / 3.3)
    S = oracle.scan(codes, luts)
    ref = oracle.rescale_f32(S, float(bias), float(scale))
    bolt.debug_force_scan_kernel(kernel)
    try:
        got = bolt.bolt_amm(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV), float(bias),
                            float(scale), transpose=transpose).cpu().numpy()
    finally:
        bolt.debug_force_scan_kernel(-1)
    if transpose:
        got = got.T
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------------------ end to end

@pytest.mark.parametrize("metric", ["l2", "dot", "l1", "lp3", "cosine"])
def test_end_to_end_tiny_workload(bolt, metric):
    """The tiny workload: 10k x 32 N(0,1), M = 8, 16 queries, top-10, every
    intermediate equal to the oracle.  Cosine encodes unit rows (normalised
    on the GPU and compared with the oracle's) with codebooks learned on
    them."""
    cfg = synth.configs.TINY
    X = synth.normal(synth.seed_for(1, 1), (cfg.N, cfg.J))
    Xd = torch.from_numpy(X).to(DEV)
    if metric == "cosine":
        X = oracle.normalize_rows(X)
        Xd = bolt.bolt_normalize_rows(Xd)
        assert np.array_equal(Xd.cpu().numpy().view(np.uint32), X.view(np.uint32))
    Qv = synth.normal(synth.seed_for(1, 2), (cfg.Q, cfg.J))
    init = synth.permutation_prefix(synth.seed_for(1, 4), cfg.N, 16)
    Qt = X[synth.permutation_prefix(synth.seed_for(1, 5), cfg.N, 1000)]
    C, a, offs, _ = oracle.train(X, cfg.M, cfg.kmeans_iters, init, Qt, metric)
    codes_ref = oracle.encode(X, C, cfg.M)
    _, _, l8 = oracle.luts(Qv, C, cfg.M, metric, a, offs)
    S_ref = oracle.scan(codes_ref, l8)
    vr, ir = oracle.topk(S_ref, cfg.k, metric in ("dot", "cosine"))
    Cd = torch.from_numpy(C).to(DEV)
    codes = bolt.bolt_encode(Xd, Cd, cfg.M)
    luts = bolt.bolt_build_luts(torch.from_numpy(Qv).to(DEV), Cd, cfg.M, metric, a,
                                torch.from_numpy(offs).to(DEV))
    v, i = bolt.bolt_scan_topk(codes, luts, metric, cfg.k)
    torch.cuda.synchronize()
    assert np.array_equal(codes.cpu().numpy(), codes_ref)
    assert np.array_equal(luts.cpu().numpy(), l8)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


def test_device_generator_matches_host(bolt):
    import synth.device as sd
    got = sd.gmm_rows(2000, 2001, 123456, 300, 128).cpu().numpy()
    ref = synth.gmm_rows(2000, 2001, 123456, 300, 128)
    assert np.array_equal(got, ref)


def test_errors_are_reported(bolt):
    """Shape errors come back as status codes through the C ABI, nothing is launched."""
    import ctypes
    X = torch.zeros((10, 30), device=DEV)
    C = torch.zeros(16 * 30, device=DEV)
    codes = torch.zeros(10 * 2, dtype=torch.uint8, device=DEV)
    st = bolt.lib().bolt_encode(ctypes.c_void_p(X.data_ptr()), 10, 30, 30, ctypes.c_void_p(C.data_ptr()),
                                4, ctypes.c_void_p(codes.data_ptr()), None)
    assert st == bolt.BOLT_ERR_SHAPE
    assert "multiple of M" in bolt.last_error()
    d = torch.zeros((2, 10), dtype=torch.uint16, device=DEV)
    with pytest.raises(bolt.BoltError) as e:
        bolt.bolt_topk(d, 4096)
    assert e.value.status == bolt.BOLT_ERR_UNSUPPORTED


# ------------------------------------------------------------------ fused scan + top-k

FUSED_CASES = [
    # (M, Q, N, k, lut kind)
    (32, 1, 1, 1, "rand"), (32, 1, 300, 100, "rand"), (32, 3, 16384, 100, "rand"),
    (32, 7, 16385, 100, "coarse"), (16, 5, 70000, 256, "rand"), (8, 2, 40000, 10, "coarse"),
    (64, 4, 50001, 100, "rand"), (32, 1, 70000, 100, "const"), (32, 8, 33000, 100, "rand"),
    (32, 17, 50000, 100, "coarse"), (32, 40, 20000, 10, "rand"), (16, 16, 70000, 256, "rand"),
    (8, 33, 17000, 64, "coarse"), (64, 9, 40000, 100, "rand"), (64, 12, 30000, 100, "const"),
    (32, 64, 16384 * 3 + 5, 100, "rand"), (32, 20, 5, 100, "rand"), (16, 100, 4000, 1, "coarse"),
    (16, 24, 140_000, 100, "const"), (8, 8, 65_537, 100, "rand"), (32, 15, 131_073, 200, "coarse"),
    # many candidate lists per query: two-level merge (few-query and grouped kernels)
    (32, 2, 2_000_000, 100, "rand"), (16, 9, 1_200_000, 256, "coarse"), (64, 7, 300_000, 50, "rand"),
]


@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", FUSED_CASES)
def test_scan_topk_fused_parity(bolt, metric, M, Q, N, k, kind):
    """The fused path (scan + in-LDS candidate selection + merge) gives exactly
    the oracle's top-k, including heavy and total ties (coarse / constant
    tables) and ragged row blocks."""
    seed = 17 * M + 31 * Q + N + k
    _say("fused scan_topk", metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
    bolt.debug_force_unfused_topk(True)
    try:
        vu, iu = bolt.bolt_scan_topk(cd, ld, metric, k)
    finally:
        bolt.debug_force_unfused_topk(False)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)
    assert np.array_equal(vu.cpu().numpy(), vr)
    assert np.array_equal(iu.cpu().numpy(), ir)


# many queries: the grouped LDS-table kernel and the int8 matrix-core kernel
# (kind 3 falls back to the grouped kernel for k > 128)
MANY_CASES = [
    # (M, Q, N, k, lut kind)
    (32, 64, 16384 * 2 + 77, 100, "rand"), (32, 100, 50_000, 128, "coarse"), (16, 65, 33_000, 100, "rand"),
    (8, 40, 20_000, 10, "const"), (64, 33, 40_001, 100, "rand"), (64, 96, 16_384, 1, "coarse"),
    (32, 200, 5, 100, "rand"), (32, 37, 1, 7, "rand"), (16, 128, 70_000, 129, "rand"),
    (8, 300, 9_000, 64, "coarse"), (32, 36, 700_000, 128, "rand"), (64, 32, 129, 100, "const"),
]


@pytest.mark.parametrize("kernel", [2, 3])
@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", MANY_CASES)
def test_scan_topk_many_queries_parity(bolt, kernel, metric, M, Q, N, k, kind):
    """Both many-query kernels give exactly the oracle's top-k: ragged query
    blocks and passes, N < k, ties (coarse / constant tables), two-level merge."""
    seed = 13 * M + 7 * Q + N + k
    _say("many-query scan_topk kernel", kernel, metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_force_fused_kind(kernel)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_force_fused_kind(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


# three to seven queries take the matrix-core tiles by default (one
# part-filled 32-query tile); with sampled bounds (mode 1), all of them
# failing (mode 2) and without them (mode 0)
FEW_MFMA_CASES = [
    # (M, Q, N, k, lut kind)
    (16, 3, 200_000, 100, "rand"), (32, 5, 300_001, 64, "coarse"), (64, 7, 150_000, 128, "rand"),
    (32, 4, 131_072, 1, "const"), (16, 6, 170_000, 100, "coarse"), (32, 7, 16_385, 100, "rand"),
]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", FEW_MFMA_CASES)
def test_scan_topk_three_to_seven_queries_parity(bolt, mode, metric, M, Q, N, k, kind):
    """The default path for three to seven queries (matrix-core tiles) equals
    the oracle, whether the sampled bounds hold, all fail or are off."""
    seed = 17 * M + 3 * Q + N + k
    _say("three to seven queries mode", mode, metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_speculation(mode)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_speculation(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


# speculative starting bounds from a row sample (mode 1), and the same with
# every bound failing so that each query takes the exact recomputation (mode 2)
SPEC_CASES = [
    # (M, Q, N, k, lut kind)
    (32, 64, 200_000, 100, "rand"), (16, 40, 150_000, 10, "coarse"), (64, 33, 140_000, 128, "rand"),
    (8, 100, 131_072, 1, "const"), (32, 48, 300_001, 256, "rand"), (32, 70, 180_000, 64, "coarse"),
    # 8 to 31 queries: one part-filled 32-query matrix-core tile is the only query block
    (32, 8, 140_000, 100, "rand"), (16, 9, 150_000, 64, "coarse"), (64, 17, 131_100, 100, "rand"),
    (8, 31, 160_000, 128, "coarse"),
    # every d tied: a recomputed query's exact bound admits all of every
    # tile's kept keys, more than the merge buffer holds at once
    (32, 40, 140_000, 256, "const"),
]


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("kernel", [2, 3])
@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", SPEC_CASES)
def test_scan_topk_speculation_parity(bolt, mode, kernel, metric, M, Q, N, k, kind):
    """Sampled starting bounds select candidates only: the result equals the
    oracle's whether the bounds hold or all fail (exact recomputation)."""
    seed = 11 * M + 5 * Q + N + k
    _say("speculation mode", mode, "kernel", kernel, metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_force_fused_kind(kernel)
    bolt.debug_speculation(mode)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_speculation(-1)
        bolt.debug_force_fused_kind(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


TIE_CASES = [
    # (M, Q, N, k, lut kind): one merge level with more than 1024 candidate keys
    # at or below the boundary bin, most of them tied at the k-th sum
    (8, 40, 200_000, 100, "coarse"), (16, 33, 150_000, 100, "const"), (8, 64, 300_001, 256, "coarse"),
    (32, 40, 250_000, 128, "const"),
]


@pytest.mark.parametrize("kernel", [2, 3])
@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", TIE_CASES)
def test_scan_topk_crowded_ties_parity(bolt, kernel, metric, M, Q, N, k, kind):
    """Thousands of keys tied at the k-th sum: the merge bounds the ties by row
    before it selects; ties still resolve by the lowest row."""
    seed = 17 * M + 3 * Q + N + k
    _say("crowded ties kernel", kernel, metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    else:
        luts = np.full_like(luts, 5)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_force_fused_kind(kernel)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_force_fused_kind(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


SPEC_FEW_CASES = [
    # (M, Q, N, k, lut kind): the one- and few-query kernels from sampled bounds
    (32, 1, 200_000, 100, "rand"), (16, 1, 131_072, 1, "const"), (64, 3, 150_001, 256, "rand"),
    (8, 7, 140_000, 10, "coarse"), (32, 2, 300_000, 64, "coarse"),
    (16, 1, 300_000, 256, "const"),   # every d tied (as in SPEC_CASES)
]


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", SPEC_FEW_CASES)
def test_scan_topk_speculation_few_parity(bolt, mode, metric, M, Q, N, k, kind):
    """Sampled starting bounds with one to seven queries: the result equals
    the oracle's whether the bounds hold or all fail."""
    seed = 13 * M + 7 * Q + N + k
    _say("speculation few mode", mode, metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    elif kind == "const":
        luts = np.full_like(luts, 3)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_speculation(mode)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_speculation(-1)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


@pytest.mark.parametrize("metric", ["l2", "dot"])
@pytest.mark.parametrize("M,Q,N,k,kind", [(32, 12, 600_000, 100, "rand"), (16, 31, 524_288, 128, "coarse"),
                                          (64, 8, 530_000, 100, "rand")])
def test_scan_topk_default_large_part_filled_tile(bolt, metric, M, Q, N, k, kind):
    """The automatic path at 5e5 rows or more with 8 to 31 queries: sampled
    bounds and one part-filled 32-query matrix-core tile (what groups of a
    served workload mostly take); equal to the oracle."""
    seed = 19 * M + 3 * Q + N + k
    _say("default large part-filled tile", metric, kind, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    v, i = bolt.bolt_scan_topk(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV), metric, k)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


def test_scan_topk_fused_repeatable(bolt):
    """Cross-workgroup bounds depend on timing; the answer must not."""
    M, Q, N, k = 32, 24, 200_000, 100
    codes = synth.random_codes(77, N, M)
    luts = (synth.random_luts(78, Q, M) // 8).astype(np.uint8)
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    outs = [bolt.bolt_scan_topk(cd, ld, "l2", k) for _ in range(5)]
    torch.cuda.synchronize()
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, False)
    for v, i in outs:
        assert np.array_equal(v.cpu().numpy(), vr) and np.array_equal(i.cpu().numpy(), ir)


# the matrix-core tiles with the dense instruction (the sparse one is the
# default and runs in every case above): same results, same oracle
DENSE_CASES = [
    # (M, Q, N, k, metric, lut kind, speculation mode)
    (32, 70, 100_003, 100, "l2", "rand", 0), (16, 40, 70_000, 64, "dot", "coarse", 0),
    (64, 33, 50_001, 128, "l2", "rand", 0), (8, 64, 40_000, 10, "dot", "rand", 0),
    (32, 48, 140_000, 100, "dot", "rand", 1), (16, 9, 150_000, 100, "l2", "coarse", 2),
    (64, 40, 131_100, 64, "dot", "rand", 1), (8, 31, 160_000, 128, "l2", "coarse", 2),
]


@pytest.mark.parametrize("M,Q,N,k,metric,kind,mode", DENSE_CASES)
def test_scan_topk_dense_mfma_parity(bolt, M, Q, N, k, metric, kind, mode):
    seed = 29 * M + 3 * Q + N + k
    _say("dense matrix-core", metric, kind, "mode", mode, "seed", seed, "M", M, "Q", Q, "N", N, "k", k)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    if kind == "coarse":
        luts = (luts // 64).astype(np.uint8)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    cd, ld = torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV)
    bolt.debug_sparse_mfma(False)
    bolt.debug_force_fused_kind(3)
    bolt.debug_speculation(mode)
    try:
        v, i = bolt.bolt_scan_topk(cd, ld, metric, k)
        torch.cuda.synchronize()
    finally:
        bolt.debug_speculation(-1)
        bolt.debug_force_fused_kind(-1)
        bolt.debug_sparse_mfma(True)
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)
