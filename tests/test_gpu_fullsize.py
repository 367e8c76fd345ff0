"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times, through the C ABI.

* Single database: N = 1e6 mixture vectors of J = 128, M in {16, 32, 64},
  Q = 1000 queries, L2 and dot, top-100.  Every code and every uint8 table
  entry is compared with the oracle; the scan + top-k of all 1000 queries
  runs as one call and a seeded sample of queries is compared with the
  oracle's full scan and top-k over all N rows; both metrics' queries then
  run as one two-metric call, as the benchmark step runs them.
* Matrix product: A 200000 x 256, M = 32, K = 1024 dot tables; the full
  [K][N] fp32 output is computed and a sample of its rows is compared with
  the oracle bit for bit.
* Single-query and small-batch scans over a 2.5e8-row database (the
  serving size, 4-16 GB of codes): every row holds one constant code byte
  except a seeded set of planted rows, so the exact top-k is that of a small
  problem the oracle solves (the planted rows plus the lowest-index
  constant rows, which win all ties at the constant sum).

Inputs come from the seeded generators (the mixture rows from the device
generator, which equals the host definition bit for bit) and from the
oracle (codebooks, quantiser, reference codes and tables).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import synth.device as sdev

pytestmark = pytest.mark.gpu

DEV = "cuda"
N1, J1, Q1, K1 = 1_000_000, 128, 1000, 100


@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return b


def _say(*a):
    print("[case]", *a, flush=True)


def _unpack(codes, M):
    out = np.empty((codes.shape[0], M), dtype=np.int64)
    out[:, 0::2] = codes & 15
    out[:, 1::2] = codes >> 4
    return out


@pytest.fixture(scope="module")
def mixture():
    mix = synth.seed_for(2, 0)
    X = sdev.gmm_rows(mix, synth.seed_for(2, 1), 0, N1, J1, device=DEV)
    Qd = sdev.gmm_rows(mix, synth.seed_for(2, 2), 0, Q1, J1, device=DEV)
    Xtrain = synth.gmm_rows(mix, synth.seed_for(2, 3), 0, 20_000, J1)
    Qtrain = synth.gmm_rows(mix, synth.seed_for(2, 5), 0, 500, J1)
    torch.cuda.synchronize()
    return X, X.cpu().numpy(), Qd, Qd.cpu().numpy(), Xtrain, Qtrain


@pytest.mark.parametrize("M", [16, 32, 64])
def test_single_database_full_size(bolt, mixture, M):
    X, Xh, Qd, Qh, Xtrain, Qtrain = mixture
    _say("single database", "N", N1, "J", J1, "M", M, "Q", Q1, "k", K1)
    C, _ = oracle.kmeans(Xtrain, M, 10, synth.permutation_prefix(synth.seed_for(2, 4), Xtrain.shape[0], 16))
    Cd = torch.from_numpy(C).to(DEV)

    # a1: every code of the million rows, bit-exact against the oracle's fp32
    # decision (the same operations in the same order)
    ref_codes = oracle.encode(Xh, C, M)
    got_codes = bolt.bolt_encode(X, Cd, M).cpu().numpy()
    bad = np.nonzero((got_codes != ref_codes).any(axis=1))[0]
    print("rows with a code differing from the oracle: %d of %d" % (len(bad), N1))
    assert len(bad) == 0
    # separately, the fp64 argmin: the fp32 decision may differ from it only on
    # near ties (relative gap <= 1e-6), which are counted and reported
    n_near = 0
    for lo in range(0, N1, 100_000):
        d64 = oracle.subspace_dists_f64(Xh[lo:lo + 100_000], C, M)
        gu = _unpack(got_codes[lo:lo + 100_000], M)
        best = d64.argmin(-1)
        r, m = np.nonzero(gu != best)
        if len(r):
            b = d64[r, m, best[r, m]]
            gap = (d64[r, m, gu[r, m]] - b) / np.maximum(b, np.finfo(np.float32).tiny)
            assert (gap <= 1e-6).all()
            n_near += len(r)
    print("codes differing from the fp64 argmin (near ties, gap <= 1e-6): %d of %d" % (n_near, N1 * M))

    codes_d = torch.from_numpy(ref_codes).to(DEV)
    sample = synth.permutation_prefix(synth.seed_for(2, 6) + M, Q1, 12)
    tables, results = [], []
    for metric in ("l2", "dot"):
        a, offs, _, _ = oracle.learn_quantizer(Qtrain, oracle.encode(Xtrain, C, M), C, metric)
        # a2: all 1000 queries' tables
        _, l32, l8 = oracle.luts(Qh, C, M, metric, a, offs)
        u8, f32 = bolt.bolt_build_luts(Qd, Cd, M, metric, a, torch.from_numpy(offs).to(DEV), want_f32=True)
        assert np.array_equal(u8.cpu().numpy(), l8)
        assert np.array_equal(f32.cpu().numpy().view(np.uint32), l32.view(np.uint32))
        # a3 + a4: one call for all queries, sampled queries against the oracle
        v, i = bolt.bolt_scan_topk(codes_d, torch.from_numpy(l8).to(DEV), metric, K1)
        v, i = v.cpu().numpy(), i.cpu().numpy()
        S = oracle.scan(ref_codes, l8[sample])
        vr, ir = oracle.topk(S, K1, metric == "dot")
        assert np.array_equal(v[sample], vr)
        assert np.array_equal(i[sample], ir)
        tables.append(l8)
        results.append((v, i, vr, ir))
    # both metrics' 2000 queries as one two-metric call: each side equals its
    # one-metric call over all queries, and the sampled queries the oracle
    v2, i2 = bolt.bolt_scan_topk_split(codes_d, torch.from_numpy(np.concatenate(tables)).to(DEV), Q1, "l2", "dot",
                                       K1)
    v2, i2 = v2.cpu().numpy(), i2.cpu().numpy()
    for side, (v, i, vr, ir) in enumerate(results):
        vs, is_ = v2[side * Q1:(side + 1) * Q1], i2[side * Q1:(side + 1) * Q1]
        assert np.array_equal(vs, v) and np.array_equal(is_, i)
        assert np.array_equal(vs[sample], vr) and np.array_equal(is_[sample], ir)


def test_matrix_product_full_size(bolt):
    N, J, M, K = 200_000, 256, 32, 1024
    _say("matrix product", "N", N, "J", J, "M", M, "K", K)
    A = synth.normal(synth.seed_for(3, 1), (N, J))
    Bt = synth.normal(synth.seed_for(3, 5), (500, J))
    C, _ = oracle.kmeans(A[:20_000], M, 10, synth.permutation_prefix(synth.seed_for(3, 4), 20_000, 16))
    a, offs, _, _ = oracle.learn_quantizer(Bt, oracle.encode(A[:20_000], C, M), C, "dot")
    codes = oracle.encode(A, C, M)
    Bm = synth.normal(synth.seed_for(3, 2) + K, (J, K))
    Qv = np.ascontiguousarray(Bm.T)
    _, _, l8 = oracle.luts(Qv, C, M, "dot", a, offs)
    bias = float(np.float32(offs.astype(np.float64).sum()))
    scale = float(np.float32(1.0 / a))
    codes_d, l8_d = torch.from_numpy(codes).to(DEV), torch.from_numpy(l8).to(DEV)
    sample = synth.permutation_prefix(synth.seed_for(3, 6), K, 16)
    ref = oracle.rescale_f32(oracle.scan(codes, l8[sample]), bias, scale)
    for transpose in (False, True):
        out = bolt.bolt_amm(codes_d, l8_d, bias, scale, transpose=transpose).cpu().numpy()
        got = out.T[sample] if transpose else out[sample]
        assert np.array_equal(np.ascontiguousarray(got).view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("M", [16, 32, 64])
@pytest.mark.parametrize("Q", [1, 7, 64])
def test_large_database_planted(bolt, M, Q):
    N, k, n_plant = 250_000_000, 100, 150
    seed = 5000 + 10 * M + Q
    _say("planted rows", "N", N, "M", M, "Q", Q, "k", k, "seed", seed)
    bg = np.uint8(0x5A)                       # codes 10 (even subspaces) and 5 (odd)
    rows = np.sort(synth.permutation_prefix(seed, N, n_plant)).astype(np.int64)
    planted = synth.random_codes(seed + 1, n_plant, M)
    luts = synth.random_luts(seed + 2, Q, M)
    codes_d = torch.full((N, M // 2), int(bg), dtype=torch.uint8, device=DEV)
    codes_d[torch.from_numpy(rows).to(DEV)] = torch.from_numpy(planted).to(DEV)
    # the reduced problem: planted rows and the first k + n_plant rows overall
    head = np.arange(k + n_plant, dtype=np.int64)
    sub_rows = np.union1d(rows, head)
    sub_codes = np.full((len(sub_rows), M // 2), bg, dtype=np.uint8)
    pos = np.searchsorted(sub_rows, rows)
    sub_codes[pos] = planted
    S = oracle.scan(sub_codes, luts)
    luts_d = torch.from_numpy(luts).to(DEV)
    for metric in ("l2", "dot"):
        vr, ir = oracle.topk(S, k, metric == "dot")
        ir = sub_rows[ir]
        v, i = bolt.bolt_scan_topk(codes_d, luts_d, metric, k)
        assert np.array_equal(v.cpu().numpy(), vr)
        assert np.array_equal(i.cpu().numpy(), ir)
    del codes_d
    torch.cuda.empty_cache()
