"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: numpy brute force,
closed forms, textbook special cases, library routines (np.quantile,
np.lexsort, np.searchsorted) and hand-derived values under tests/golden/.
Each is chosen so that a plausible mistake in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong nibble order or tie rule)
fails at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unpack(codes, M):
    """Nibble unpacking written independently: byte t = sub 2t (low) | sub 2t+1 (high)."""
    lo = codes & 0x0F
    hi = codes >> 4
    out = np.empty((codes.shape[0], M), dtype=np.int64)
    out[:, 0::2] = lo
    out[:, 1::2] = hi
    return out


def _brute_codes_f64(X, C, M):
    sub = X.shape[1] // M
    Xs = X.astype(np.float64).reshape(X.shape[0], M, 1, sub)
    d = ((Xs - C.astype(np.float64)[None]) ** 2).sum(-1)      # [N, M, 16]
    return np.argmin(d, axis=-1), d


def _reconstruct(codes_unpacked, C):
    M = C.shape[0]
    return np.concatenate([C[m][codes_unpacked[:, m]] for m in range(M)], axis=1).astype(np.float64)


def _round_f32(x):
    """Round a rational to the nearest fp32, ties to even (IEEE 754 default
    rounding), written from the definition: scale so that one unit in the last
    place is 1, round the integer part, scale back.  Subnormals keep the
    quantum 2^-149."""
    x = Fraction(x)
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    e = max(e, -126)
    q = 23 - e
    scaled = x * Fraction(2) ** q
    m = scaled.numerator // scaled.denominator
    rem = scaled - m
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and m % 2 == 1):
        m += 1
    return np.float32(sign * m * 2.0 ** (-q))


def _fr(v):
    return Fraction(float(v))


def _canonical_f32_entry(qv, c, metric):
    """One fp32 table entry by exact rational arithmetic, one correct rounding
    per step in the canonical order: acc = 0, then for j ascending
    L2: t = round(q_j - c_j), acc = round(t * t + acc) (one fused rounding);
    dot: acc = round(q_j * c_j + acc)."""
    acc = np.float32(0.0)
    for j in range(len(qv)):
        if metric == "l2":
            t = _round_f32(_fr(qv[j]) - _fr(c[j]))
            acc = _round_f32(_fr(t) * _fr(t) + _fr(acc))
        else:
            acc = _round_f32(_fr(qv[j]) * _fr(c[j]) + _fr(acc))
    return acc


# ---------------------------------------------------------------- golden

def test_golden_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    M, J = g["M"], g["J"]
    C = np.zeros((2, 16, 2), dtype=np.float32)
    C[0, :, 0] = np.arange(16)
    C[1, :, 1] = 2 * np.arange(16)
    x = np.array([g["x"]], dtype=np.float32)
    q = np.array([g["q"]], dtype=np.float32)
    codes = oracle.encode(x, C, M)
    assert codes[0, 0] == g["codes_byte"]
    _, _, l8 = oracle.luts(q, C, M, "l2", 1.0, np.zeros(M, np.float32))
    assert l8[0].tolist() == g["lut_l2"]
    _, _, d8 = oracle.luts(q, C, M, "dot", 1.0, np.zeros(M, np.float32))
    assert d8[0].tolist() == g["lut_dot"]
    assert int(oracle.scan(codes, l8)[0, 0]) == g["sum_l2"]
    assert int(oracle.scan(codes, d8)[0, 0]) == g["sum_dot"]


def test_golden_paper_numbers():
    """Byte accounting of the codes against the compression ratios and encode
    rate the paper states (Sec. 4.3, Sec. 4.6)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    for case in g["compression"]["cases"]:
        M = 2 * case["code_bytes"]              # 4-bit codes: M subspaces -> M/2 bytes
        J = case["J"]
        Jp = -(-J // M) * M                     # the paper's MNIST row keeps J = 784
        X = np.zeros((1, Jp), dtype=np.float32)
        C = np.zeros((M, 16, Jp // M), dtype=np.float32)
        codes = oracle.encode(X, C, M)
        ratio = (4 * J) / codes.shape[1]
        assert ratio == case["ratio"], case
    e = g["encode_rate"]
    rate = e["vectors_per_s"] * e["J"] * 4
    assert abs(rate - e["bytes_per_s_approx"]) / e["bytes_per_s_approx"] < 0.03
    assert abs(1e6 / e["vectors_per_s"] - e["sift1m_s"]) < 1e-12
    assert abs(1e9 / e["vectors_per_s"] - e["sift1b_s"]) < 1e-9
    assert g["codebook_size"]["pq_K"] // g["codebook_size"]["K"] == 16
    assert 2 ** g["codebook_size"]["bits"] == g["codebook_size"]["K"]
    assert list(oracle.ALPHAS) == g["alpha_grid"]["values"]


# ---------------------------------------------------------------- encode

@pytest.mark.parametrize("J,M", [(32, 8), (16, 16), (64, 8), (24, 2), (128, 32)])
def test_encode_matches_exhaustive_argmin(J, M):
    X = synth.normal(11 + J + M, (300, J))
    C = synth.normal(12 + J + M, (M, 16, J // M))
    codes, d32 = oracle.encode(X, C, M, want_dists=True)
    ref, d64 = _brute_codes_f64(X, C, M)
    got = _unpack(codes, M)
    mism = got != ref
    # fp32 and fp64 decisions may only differ on near-ties
    if mism.any():
        n, m = np.nonzero(mism)
        gap = (d64[n, m, got[n, m]] - d64[n, m, ref[n, m]]) / np.maximum(d64[n, m, ref[n, m]], 1e-38)
        assert (gap <= 1e-6).all()
    assert mism.mean() < 1e-3
    # the fp32 distances agree with the exact ones to fp32 accuracy
    np.testing.assert_allclose(d32, d64, rtol=1e-5, atol=1e-6)


def test_encode_exact_centroid_and_ties():
    M, J = 4, 8
    C = synth.normal(21, (M, 16, 2)).astype(np.float32)
    # subvector equal to a centroid -> that centroid's index
    rng = np.random.default_rng(0)
    pick = rng.integers(0, 16, size=(50, M))
    X = np.concatenate([C[m][pick[:, m]] for m in range(M)], axis=1)
    assert (_unpack(oracle.encode(X, C, M), M) == pick).all()
    # duplicate centroids: the lower index wins
    C2 = C.copy()
    C2[:, 9] = C2[:, 4]
    X2 = np.concatenate([C2[m][np.full(50, 9)] for m in range(M)], axis=1)
    assert (_unpack(oracle.encode(X2, C2, M), M) == 4).all()


def test_encode_scalar_quantizer_special_case():
    """J/M = 1: each subspace is a 16-level scalar quantiser; the nearest level
    is found by binary search over the midpoints of the sorted levels."""
    M = 8
    levels = np.sort(synth.normal(31, (M, 16)), axis=1)
    C = levels[:, :, None].astype(np.float32)
    X = synth.normal(32, (500, M))
    got = _unpack(oracle.encode(X, C, M), M)
    for m in range(M):
        mids = (levels[m, 1:].astype(np.float64) + levels[m, :-1]) / 2
        ref = np.searchsorted(mids, X[:, m].astype(np.float64), side="left")
        near = np.abs(X[:, m][:, None] - mids[None]).min(1) < 1e-6
        assert (got[~near, m] == ref[~near]).all()


def test_encode_m1_is_vector_quantisation():
    """M = 1 (oracle-only): plain k-means vector quantisation, Sec. 3.1."""
    C = synth.normal(41, (1, 16, 6))
    X = synth.normal(42, (200, 6))
    # M=1 is odd; pad a second empty-weight subspace by duplicating the space
    X2 = np.concatenate([X, X], axis=1)
    C2 = np.concatenate([C, C], axis=0)
    got = _unpack(oracle.encode(X2, C2, 2), 2)
    ref = np.argmin(((X[:, None, :].astype(np.float64) - C[0][None]) ** 2).sum(-1), axis=1)
    assert (got[:, 0] == ref).mean() > 0.999
    assert (got[:, 0] == got[:, 1]).all()


def test_round_f32_helper_matches_ieee():
    """The rational rounding helper used by the pins below agrees with the
    hardware's round-to-nearest-even conversion from fp64 (numpy), including
    exact halfway cases and subnormals."""
    rng = np.random.default_rng(5)
    vals = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-40, 38, 2000))
    one = 1.0
    vals += [one + 2.0 ** -24, one + 3 * 2.0 ** -24, -(one + 2.0 ** -24), 2.0 ** -149, 3 * 2.0 ** -150,
             2.0 ** -150, 1e-45, 0.0, 16777217.0, 16777219.0]
    for v in vals:
        assert _round_f32(Fraction(v)).view(np.uint32) == np.float32(v).view(np.uint32), v
    # a fused step differs from two roundings: (1 + 2^-12)^2 - 1 - 2^-11 = 2^-24 exactly
    t = np.float32(1 + 2.0 ** -12)
    fused = _round_f32(_fr(t) * _fr(t) + _fr(np.float32(-(1 + 2.0 ** -11))))
    assert fused == np.float32(2.0 ** -24)
    assert np.float32(t * t) + np.float32(-(1 + 2.0 ** -11)) == np.float32(0.0)


def test_encode_fp32_decision_exact():
    """The encoding decision is taken on fp32 distances in the canonical order
    (t = x_j - c_j rounded, acc = fma(t, t, acc), j ascending), ties to the
    lowest index: each distance equals the exact-rational emulation of those
    roundings bit for bit, and each code is the first index of their minimum.
    Inputs include exact ties (duplicated centroids) and a subvector equal to a
    centroid."""
    N, J, M = 24, 12, 4
    sub = J // M
    X = synth.normal(181, (N, J)) * 3
    C = synth.normal(182, (M, 16, sub)) * 3
    C[:, 11] = C[:, 6]                                  # exact tie: index 6 must win
    X[0, :sub] = C[0, 6]
    codes, d32 = oracle.encode(X, C, M, want_dists=True)
    got = _unpack(codes, M)
    for n in range(N):
        for m in range(M):
            ref = np.array([_canonical_f32_entry(X[n, m * sub:(m + 1) * sub], C[m, i], "l2")
                            for i in range(16)], dtype=np.float32)
            assert np.array_equal(d32[n, m].view(np.uint32), ref.view(np.uint32)), (n, m)
            assert got[n, m] == int(np.argmin(ref)), (n, m)
    assert got[0, 0] == 6


def test_subspace_dists_f64_pins():
    """The fp64 subspace distances (the checker of near-tie encodings):
    on integer-valued inputs every step is exact in fp64, so they equal the
    int64 brute force exactly; on continuous inputs they are within
    sub * 2^-52 relative of the exact rational sum; a subvector equal to a
    centroid has distance 0 there.  A dropped or transposed index, a wrong
    subspace offset or a missing square fails one of these."""
    N, J, M = 50, 24, 6
    sub = J // M
    Xi = synth.integers(191, -60, 60, (N, J))
    Ci = synth.integers(192, -60, 60, (M, 16, sub))
    got = oracle.subspace_dists_f64(Xi.astype(np.float32), Ci.astype(np.float32), M)
    diff = Xi.astype(np.int64).reshape(N, M, 1, sub) - Ci.astype(np.int64)[None]
    assert np.array_equal(got, (diff * diff).sum(-1).astype(np.float64))
    X = synth.normal(193, (8, J))
    C = synth.normal(194, (M, 16, sub))
    X[3, 2 * sub:3 * sub] = C[2, 9]
    got = oracle.subspace_dists_f64(X, C, M)
    assert got[3, 2, 9] == 0.0
    for n in range(8):
        for m in range(M):
            for i in range(16):
                exact = sum((_fr(X[n, m * sub + j]) - _fr(C[m, i, j])) ** 2 for j in range(sub))
                assert abs(Fraction(float(got[n, m, i])) - exact) <= exact * Fraction(sub, 2 ** 52)


# ---------------------------------------------------------------- LUTs

@pytest.mark.parametrize("J,M", [(32, 8), (64, 16), (128, 32), (16, 2)])
def test_lut_closed_form_reconstruction(J, M):
    """Sum of the fp64 table entries selected by h(x) equals the distance to the
    reconstruction x_hat (Sec. 3.1 sum of table entries; Sec. 3.3 Definition)."""
    X = synth.normal(51 + J, (64, J))
    Qv = synth.normal(52 + J, (8, J))
    C = synth.normal(53 + J, (M, 16, J // M))
    codes = oracle.encode(X, C, M)
    cu = _unpack(codes, M)
    xh = _reconstruct(cu, C)
    l64, _, _ = oracle.luts(Qv, C, M, "l2")
    d64, _, _ = oracle.luts(Qv, C, M, "dot")
    q64 = Qv.astype(np.float64)
    for q in range(len(Qv)):
        s_l2 = l64[q][np.arange(M)[None, :], cu].sum(1)
        s_dot = d64[q][np.arange(M)[None, :], cu].sum(1)
        ref_l2 = ((q64[q][None] - xh) ** 2).sum(1)
        ref_dot = xh @ q64[q]
        np.testing.assert_allclose(s_l2, ref_l2, rtol=1e-12)
        np.testing.assert_allclose(s_dot, ref_dot, rtol=1e-12, atol=1e-12 * np.abs(xh).sum())


def test_lut_l2_dot_identity_and_fp32():
    J, M = 64, 16
    Qv = synth.normal(61, (10, J))
    C = synth.normal(62, (M, 16, J // M))
    l64, l32, _ = oracle.luts(Qv, C, M, "l2")
    d64, d32, _ = oracle.luts(Qv, C, M, "dot")
    sub = J // M
    qn = (Qv.astype(np.float64).reshape(10, M, sub) ** 2).sum(-1)          # ||q^(m)||^2
    cn = (C.astype(np.float64) ** 2).sum(-1)                                # ||c_i^(m)||^2
    np.testing.assert_allclose(l64, qn[:, :, None] - 2 * d64 + cn[None], rtol=1e-12, atol=1e-12)
    # the fp32 canonical tables match the exact ones to 1e-5 relative
    assert (np.abs(l32 - l64) <= 1e-5 * l64 + 1e-30).all()
    scale = (np.abs(Qv.astype(np.float64).reshape(10, M, 1, sub)) * np.abs(C[None])).sum(-1)
    assert (np.abs(d32 - d64) <= 1e-5 * scale).all()


@pytest.mark.parametrize("metric", ["l2", "dot"])
def test_lut_fp32_canonical_order_exact(metric):
    """The fp32 tables equal, bit for bit, the exact-rational emulation of the
    canonical order (acc = 0; j ascending; one rounding for the difference and
    one per fused multiply-add), the order the GPU tables must reproduce.  A
    different summation order, separately rounded products or fp64
    accumulation each change some entries of this input."""
    J, M, Q = 24, 4, 3
    sub = J // M
    Qv = synth.normal(201, (Q, J)) * 7
    C = synth.normal(202, (M, 16, sub)) * 7
    _, l32, _ = oracle.luts(Qv, C, M, metric)
    for q in range(Q):
        for m in range(M):
            for i in range(16):
                ref = _canonical_f32_entry(Qv[q, m * sub:(m + 1) * sub], C[m, i], metric)
                assert l32[q, m, i].view(np.uint32) == ref.view(np.uint32), (q, m, i)


def test_lut_u8_formula_exact():
    """beta = clamp(floor(fma(a, y, -b')), 0, 255) (Sec. 3.2), checked with exact
    rational arithmetic and round-to-nearest-even to fp32."""
    J, M = 32, 8
    Qv = synth.normal(71, (6, J))
    C = synth.normal(72, (M, 16, J // M))
    offs = synth.uniform(73, (M,), -3.0, 40.0)
    a = np.float32(5.37)
    _, l32, l8 = oracle.luts(Qv, C, M, "l2", float(a), offs)
    for e in np.ndindex(l32.shape):
        exact = Fraction(float(a)) * Fraction(float(l32[e])) - Fraction(float(offs[e[1]]))
        r = np.float32(float(exact))            # float(Fraction) rounds to nearest double
        # float(Fraction) -> double -> fp32 can double-round; re-round exactly when close
        lo = np.nextafter(r, np.float32(-np.inf))
        hi = np.nextafter(r, np.float32(np.inf))
        cands = [lo, r, hi]
        r = min(cands, key=lambda c: (abs(Fraction(float(c)) - exact),
                                       int(np.float32(c).view(np.uint32)) & 1))
        ref = min(max(int(np.floor(r)), 0), 255)
        assert int(l8[e]) == ref, (e, float(l32[e]))


def test_lut_u8_monotone_clamp_and_lemma1():
    """Monotone, clamped, and inside the learned range the reconstruction error
    satisfies 0 <= y - y_hat < 1/a (Sec. 3.3 Lemma 1, with the step 1/a)."""
    J, M = 32, 8
    Qv = synth.normal(81, (40, J))
    C = synth.normal(82, (M, 16, J // M))
    a = np.float32(3.0)
    b = np.linspace(0.5, 4.0, M).astype(np.float64)
    offs = (a * b).astype(np.float32)
    _, l32, l8 = oracle.luts(Qv, C, M, "l2", float(a), offs)
    for m in range(M):
        y = l32[:, m, :].ravel().astype(np.float64)
        beta = l8[:, m, :].ravel().astype(np.float64)
        order = np.argsort(y, kind="stable")
        assert (np.diff(beta[order]) >= 0).all()
        lo = offs[m] / a
        hi = lo + 255.0 / a
        yh = (beta + offs[m]) / a
        inside = (y >= lo) & (y < hi)
        err = y - yh
        slack = 1e-5 * np.maximum(np.abs(y), 1)
        assert (err[inside] >= -slack[inside]).all()
        assert (err[inside] < 1.0 / a + slack[inside]).all()
        assert (beta[y < lo - 1e-6] == 0).all()
        assert (beta[y >= hi + 1e-3] == 255).all()


# ---------------------------------------------------------------- scan

@pytest.mark.parametrize("M", [2, 8, 16, 32, 64, 256])
def test_scan_brute_force(M):
    codes = synth.random_codes(91 + M, 257, M)
    lut = synth.random_luts(92 + M, 5, M)
    S = oracle.scan(codes, lut)
    cu = _unpack(codes, M)
    ref = lut[:, np.arange(M)[None, :], cu].astype(np.int64).sum(-1)   # [Q, N]
    assert (S.astype(np.int64) == ref).all()
    assert ref.max() < 65536


def test_scan_identity_constant_onehot_permutation():
    M, N = 16, 300
    codes = synth.random_codes(101, N, M)
    cu = _unpack(codes, M)
    # identity table on one subspace extracts that subspace's code
    for m in (0, 1, 7, 14, 15):
        lut = np.zeros((1, M, 16), np.uint8)
        lut[0, m] = np.arange(16)
        assert (oracle.scan(codes, lut)[0] == cu[:, m]).all()
    # constant 255 tables -> 255*M everywhere
    lut = np.full((1, M, 16), 255, np.uint8)
    assert (oracle.scan(codes, lut)[0] == 255 * M).all()
    # one-hot on code value v -> number of subspaces whose code is v
    for v in (0, 5, 15):
        lut = np.zeros((1, M, 16), np.uint8)
        lut[0, :, v] = 1
        assert (oracle.scan(codes, lut)[0] == (cu == v).sum(1)).all()
    # permuting rows permutes outputs
    lut = synth.random_luts(102, 3, M)
    perm = np.random.default_rng(1).permutation(N)
    assert (oracle.scan(codes[perm], lut) == oracle.scan(codes, lut)[:, perm]).all()
    # pairs agree with the full scan
    qs = np.array([0, 2, 1, 2]); ns = np.array([5, 0, 299, 17])
    assert (oracle.scan_pairs(codes, lut, qs, ns) == oracle.scan(codes, lut)[qs, ns]).all()


# ---------------------------------------------------------------- top-k

@pytest.mark.parametrize("largest", [False, True])
def test_topk_lexsort(largest):
    d = synth.integers(111, 0, 40, (7, 500)).astype(np.uint16)   # many ties
    k = 25
    vals, idx = oracle.topk(d, k, largest)
    for q in range(7):
        key = (-d[q].astype(np.int64)) if largest else d[q].astype(np.int64)
        order = np.lexsort((np.arange(500), key))[:k]
        assert (idx[q] == order).all()
        assert (vals[q] == d[q][order]).all()


def test_topk_pad_and_constant():
    d = np.full((2, 5), 77, np.uint16)
    vals, idx = oracle.topk(d, 8, False)
    assert idx[0].tolist() == [0, 1, 2, 3, 4, -1, -1, -1]
    assert vals[0].tolist() == [77] * 5 + [65535] * 3
    vals, idx = oracle.topk(d, 8, True)
    assert vals[1].tolist() == [77] * 5 + [0] * 3


# ---------------------------------------------------------------- rescale and AMM bound

def test_rescale_f32_matches_numpy_single():
    S = synth.integers(121, 0, 65535, (1000,)).astype(np.uint16)
    bias, scale = np.float32(-123.456), np.float32(1 / 7.77)
    got = oracle.rescale_f32(S, float(bias), float(scale))
    ref = (S.astype(np.float32) + bias) * scale
    assert (got.view(np.uint32) == ref.view(np.uint32)).all()


def test_amm_error_bound_lemma3_plus_lemma1():
    """|q.x - S_hat| <= ||q|| ||x - x_hat|| + M/a when no entry is clipped
    (Sec. 3.3 Lemma 3 for the codebook error plus Lemma 1, step 1/a, per table)."""
    J, M = 64, 16
    X = synth.normal(131, (400, J))
    Qv = synth.normal(132, (12, J))
    init = synth.permutation_prefix(133, 400, 16)
    C, _ = oracle.kmeans(X, M, 5, init)
    codes = oracle.encode(X, C, M)
    cu = _unpack(codes, M)
    xh = _reconstruct(cu, C)
    d64, d32, _ = oracle.luts(Qv, C, M, "dot")
    b = d64.min(axis=(0, 2))                                  # per-table minimum: no clipping at 0
    a = np.float32(250.0 / (d64.max(axis=(0, 2)) - b).max())  # no clipping at 255
    offs = (a * b).astype(np.float32)
    _, _, l8 = oracle.luts(Qv, C, M, "dot", float(a), offs)
    S = oracle.scan(codes, l8)
    Sh = oracle.rescale_f64(S, float(a), offs)
    exact = Qv.astype(np.float64) @ X.astype(np.float64).T
    bound = (np.linalg.norm(Qv.astype(np.float64), axis=1)[:, None] *
             np.linalg.norm(X.astype(np.float64) - xh, axis=1)[None] + M / float(a) * 1.0001)
    assert (np.abs(exact - Sh) <= bound).all()
    # Lemma 4 (triangle inequality) for the L2 side
    for q in range(len(Qv)):
        lhs = np.abs(np.linalg.norm(Qv[q] - X, axis=1) - np.linalg.norm(Qv[q] - xh, axis=1))
        assert (lhs <= np.linalg.norm(X - xh, axis=1) + 1e-9).all()


# ---------------------------------------------------------------- training (no trained values in the paper: an
# independent Lloyd implementation, invariants and numpy quantiles)

def test_kmeans_invariants():
    J, M = 32, 8
    X = synth.normal(141, (3000, J))
    init = synth.permutation_prefix(142, 3000, 16)
    C, obj = oracle.kmeans(X, M, 8, init)
    assert (np.diff(obj) <= 1e-9 * obj[0]).all()               # Lloyd never increases the objective
    # well-separated clusters, one initial row in each: the centroids become
    # the cluster means
    centers = np.array([[0, 0], [10, 0], [0, 10], [10, 10]] * 4, dtype=np.float32) \
        + np.repeat(np.arange(4), 4)[:, None] * 40
    pts = np.repeat(centers, 30, axis=0) + synth.normal(143, (16 * 30, 2)) * 0.1
    init2 = np.arange(0, 16 * 30, 30)
    C2, _ = oracle.kmeans(np.concatenate([pts, pts], 1), 2, 3, init2)
    np.testing.assert_allclose(np.sort(C2[0, :, 0]), np.sort(centers[:, 0]), atol=0.1)


def test_kmeans_matches_scikit_learn_lloyd():
    """Per subspace, the oracle's k-means equals scikit-learn's Lloyd
    iterations from the same initial rows (an independent implementation of
    the same algorithm, in fp64): centroids within the fp32 rounding the
    oracle applies to every mean, and the objective of the final
    assignment.  Continuous data, no cluster empties on the way."""
    cluster = pytest.importorskip("sklearn.cluster")
    J, M, n, iters = 32, 8, 3000, 6
    X = synth.normal(171, (n, J))
    init = synth.permutation_prefix(172, n, 16)
    C, obj = oracle.kmeans(X, M, iters, init)
    sub = J // M
    total = 0.0
    for m in range(M):
        Xm = X[:, m * sub:(m + 1) * sub].astype(np.float64)
        km = cluster.KMeans(n_clusters=16, init=Xm[init], n_init=1, max_iter=iters, tol=0.0,
                            algorithm="lloyd").fit(Xm)
        np.testing.assert_allclose(C[m], km.cluster_centers_, rtol=1e-5, atol=1e-6)
        total += km.inertia_
    assert obj[iters] == pytest.approx(total, rel=1e-6)


def test_quantizer_learning_matches_expanded_quantiles():
    """The weighted quantiles equal np.quantile (linear, type 7) of the expanded
    sample of y = D_m[h(x)_m](q) over all (query, vector) pairs, and the chosen
    alpha is the grid argmin of the loss (Sec. 3.2)."""
    J, M = 16, 4
    X = synth.normal(151, (60, J))
    init = synth.permutation_prefix(152, 60, 16)
    C, _ = oracle.kmeans(X, M, 3, init)
    codes = oracle.encode(X, C, M)
    Qt = synth.normal(153, (7, J))
    a, offs, best, losses = oracle.learn_quantizer(Qt, codes, C, "l2")
    assert best == int(np.argmin(losses))
    alpha = oracle.ALPHAS[best]
    l64, _, _ = oracle.luts(Qt, C, M, "l2")
    cu = _unpack(codes, M)
    Y = np.stack([l64[:, m, :][:, cu[:, m]].ravel() for m in range(M)])    # [M, nq*n]
    b = np.quantile(Y, alpha, axis=1)
    pool = (Y - b[:, None]).ravel()
    top = np.quantile(pool, 1 - alpha)
    a_ref = np.float32(255.0 / top)
    assert a == pytest.approx(float(a_ref), rel=1e-6)
    np.testing.assert_allclose(offs, (np.float64(a_ref) * b).astype(np.float32), rtol=1e-5, atol=1e-4)
    # loss of the chosen alpha recomputed from the expanded sample
    beta = np.clip(np.floor(np.float64(a) * Y - offs[:, None].astype(np.float64)), 0, 255)
    yh = (beta + offs[:, None]) / np.float64(a)
    assert losses[best] == pytest.approx(((yh - Y) ** 2).mean(), rel=1e-9)


# ------------------------------------------------------------------ Bolt No Quantize (Sec. 4.2)

def test_scan_f32_integer_tables_equal_integer_scan():
    """Integer-valued float tables: every partial sum is an exact fp32 integer,
    so the float scan must equal the (pinned) integer scan exactly."""
    N, M, Q = 3000, 32, 5
    codes = synth.random_codes(71, N, M)
    lut8 = synth.random_luts(72, Q, M)
    got = oracle.scan_f32(codes, lut8.astype(np.float32))
    assert np.array_equal(got, oracle.scan(codes, lut8).astype(np.float32))


@pytest.mark.parametrize("metric", ["l2", "dot"])
def test_scan_f32_reconstruction_closed_form(metric):
    """Float tables over h(x): the sum is the squared distance to (or the dot
    product with) the reconstruction x_hat, up to fp32 rounding of the M
    table entries and M adds (Sec. 3.1; Sec. 3.3 Definition)."""
    J, M = 64, 16
    X = synth.normal(73, (200, J))
    Qv = synth.normal(74, (6, J))
    C = synth.normal(75, (M, 16, J // M))
    codes = oracle.encode(X, C, M)
    xh = _reconstruct(_unpack(codes, M), C)
    _, l32, _ = oracle.luts(Qv, C, M, metric)
    got = oracle.scan_f32(codes, l32).astype(np.float64)
    q64 = Qv.astype(np.float64)
    if metric == "l2":
        ref = ((q64[:, None, :] - xh[None]) ** 2).sum(-1)
        np.testing.assert_allclose(got, ref, rtol=4 * M * 2.0 ** -24)
    else:
        ref = q64 @ xh.T
        scale = np.abs(q64)[:, None, :] * np.abs(xh)[None]
        assert (np.abs(got - ref) <= 4 * M * 2.0 ** -24 * scale.sum(-1)).all()


def test_scan_f32_adds_in_ascending_m_order():
    """The sum is left to right in ascending m with fp32 rounding after each
    add: for entries 1, 1e8, -1e8 that gives (1 + 1e8) - 1e8 = 0 in fp32,
    where the exact sum (or fp64, or another order) gives 1."""
    M = 4
    lut = np.zeros((1, M, 16), dtype=np.float32)
    lut[0, 0, 0], lut[0, 1, 0], lut[0, 2, 0], lut[0, 3, 0] = 1.0, 1e8, -1e8, 0.0
    codes = np.zeros((1, M // 2), dtype=np.uint8)
    assert oracle.scan_f32(codes, lut)[0, 0] == np.float32(0.0)
    lut[0, 0, 0], lut[0, 1, 0], lut[0, 2, 0] = 1e8, -1e8, 1.0
    assert oracle.scan_f32(codes, lut)[0, 0] == np.float32(1.0)


@pytest.mark.parametrize("largest", [False, True])
def test_topk_f32_lexsort(largest):
    """Float top-k against numpy.lexsort on (value, index), with forced ties."""
    d = (np.round(synth.normal(76, (7, 900)) * 4) / 4).astype(np.float32)
    k = 50
    vals, idx = oracle.topk_f32(d, k, largest)
    for q in range(d.shape[0]):
        keys = -d[q].astype(np.float64) if largest else d[q].astype(np.float64)
        order = np.lexsort((np.arange(d.shape[1]), keys))[:k]
        assert np.array_equal(idx[q], order)
        assert np.array_equal(vals[q], d[q][order])
    v, i = oracle.topk_f32(d[:, :3], 5, largest)
    assert (i[:, 3:] == -1).all()
    assert (v[:, 3:] == (-np.inf if largest else np.inf)).all()


def test_lut_l1_closed_form_and_fp32():
    """L1 tables (the L_p distance with p = 1, eq. distFuncForm): the fp64
    entries selected by h(x) sum to ||q - x_hat||_1, and the fp32 entries are
    the ascending-j fp32 sum of |q_j - c_j|."""
    J, M = 64, 16
    X = synth.normal(91, (64, J))
    Qv = synth.normal(92, (8, J))
    C = synth.normal(93, (M, 16, J // M))
    codes = oracle.encode(X, C, M)
    cu = _unpack(codes, M)
    xh = _reconstruct(cu, C)
    l64, l32, _ = oracle.luts(Qv, C, M, "l1")
    for q in range(len(Qv)):
        s = l64[q][np.arange(M)[None, :], cu].sum(1)
        np.testing.assert_allclose(s, np.abs(Qv[q].astype(np.float64)[None] - xh).sum(1), rtol=1e-12)
    sub = J // M
    ref = np.zeros((8, M, 16), dtype=np.float32)
    for j in range(sub):
        ref = ref + np.abs(Qv.reshape(8, M, 1, sub)[..., j] - C[None, :, :, j]).astype(np.float32)
    assert np.array_equal(l32.view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------------------ L_p and cosine tables (eq. distFuncForm)

def test_lut_lp_reduces_to_l1_and_l2_and_closed_form():
    """L_p tables (|q - c|^p per dimension): p = 1 and p = 2 are the L1 and
    squared-L2 tables bit for bit (fp32) and equal in fp64; for p = 3 and 4
    the fp64 entries selected by h(x) sum to ||q - x_hat||_p^p."""
    J, M = 32, 8
    X = synth.normal(211, (60, J))
    Qv = synth.normal(212, (6, J)) * 2
    C = synth.normal(213, (M, 16, J // M))
    for p, base in ((1, "l1"), (2, "l2")):
        a64, a32, _ = oracle.luts(Qv, C, M, "lp%d" % p)
        b64, b32, _ = oracle.luts(Qv, C, M, base)
        assert np.array_equal(a32.view(np.uint32), b32.view(np.uint32))
        np.testing.assert_allclose(a64, b64, rtol=1e-13)
    cu = _unpack(oracle.encode(X, C, M), M)
    xh = _reconstruct(cu, C)
    for p in (3, 4):
        l64, l32, _ = oracle.luts(Qv, C, M, "lp%d" % p)
        for q in range(len(Qv)):
            s = l64[q][np.arange(M)[None, :], cu].sum(1)
            ref = (np.abs(Qv[q].astype(np.float64)[None] - xh) ** p).sum(1)
            np.testing.assert_allclose(s, ref, rtol=1e-12)
        assert (np.abs(l32 - l64) <= 1e-5 * l64 + 1e-30).all()


def test_lut_lp3_fp32_order_exact():
    """The canonical fp32 order of the L_p entries at p = 3, by exact rational
    arithmetic: t = |round(q - c)|, w = round(t * t), acc = round(w * t + acc)
    (one fused rounding), j ascending."""
    J, M, Q = 16, 4, 2
    sub = J // M
    Qv = synth.normal(221, (Q, J)) * 3
    C = synth.normal(222, (M, 16, sub)) * 3
    _, l32, _ = oracle.luts(Qv, C, M, "lp3")
    for q in range(Q):
        for m in range(M):
            for i in range(16):
                acc = np.float32(0.0)
                for j in range(sub):
                    t = abs(_round_f32(_fr(Qv[q, m * sub + j]) - _fr(C[m, i, j])))
                    w = _round_f32(_fr(t) * _fr(t))
                    acc = _round_f32(_fr(w) * _fr(t) + _fr(acc))
                assert l32[q, m, i].view(np.uint32) == acc.view(np.uint32), (q, m, i)


def test_normalize_rows_pins():
    """Unit rows: the fused sum of squares emulated exactly, then numpy's IEEE
    fp32 square root and division (correctly rounded, like the oracle's);
    the result has unit norm to fp32 accuracy and the direction of x; a zero
    row stays zero."""
    X = synth.normal(231, (20, 12)) * 5
    X[7] = 0.0
    Y = oracle.normalize_rows(X)
    for r in range(X.shape[0]):
        s = np.float32(0.0)
        for j in range(X.shape[1]):
            s = _round_f32(_fr(X[r, j]) * _fr(X[r, j]) + _fr(s))
        n = np.sqrt(np.float32(s))
        ref = (X[r] / n).astype(np.float32) if n > 0 else np.zeros(X.shape[1], np.float32)
        assert np.array_equal(Y[r].view(np.uint32), ref.view(np.uint32)), r
    norms = np.linalg.norm(Y.astype(np.float64), axis=1)
    assert abs(norms[7]) == 0.0
    np.testing.assert_allclose(np.delete(norms, 7), 1.0, atol=4e-7)
    cosang = (Y.astype(np.float64) * X).sum(1) / np.maximum(np.linalg.norm(X.astype(np.float64), axis=1), 1e-30)
    np.testing.assert_allclose(np.delete(cosang, 7), 1.0, atol=1e-6)


def test_lut_cosine_is_dot_of_the_unit_query():
    """Cosine tables are the dot tables of the unit query (bit for bit in
    fp32), and over h(x) of unit database rows the fp64 entries sum to
    q . x_hat / |q|, the cosine of q with the reconstruction times |x_hat|."""
    J, M = 32, 8
    Qv = synth.normal(241, (7, J)) * 4
    X = oracle.normalize_rows(synth.normal(242, (80, J)))
    init = synth.permutation_prefix(243, 80, 16)
    C, _ = oracle.kmeans(X, M, 3, init)
    c64, c32, _ = oracle.luts(Qv, C, M, "cosine")
    _, d32, _ = oracle.luts(oracle.normalize_rows(Qv), C, M, "dot")
    assert np.array_equal(c32.view(np.uint32), d32.view(np.uint32))
    cu = _unpack(oracle.encode(X, C, M), M)
    xh = _reconstruct(cu, C)
    q64 = Qv.astype(np.float64)
    for q in range(len(Qv)):
        s = c64[q][np.arange(M)[None, :], cu].sum(1)
        ref = xh @ q64[q] / np.linalg.norm(q64[q])
        np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-12)
        cos = ref / np.linalg.norm(xh, axis=1)
        assert (np.abs(cos) <= 1 + 1e-12).all()
