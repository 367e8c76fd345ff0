"""The seeded input generators follow their stated definition."""
import numpy as np

import synth

MASK = (1 << 64) - 1


def _sm64(x):
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def _ref_value(mix, draw, r, j, J, C=256):
    """Pure-Python-int evaluation of the mixture generator's definition."""
    base = lambda seed, s: _sm64((seed * 16 + s) & MASK)
    comp = ((_sm64((base(draw, 1) + r) & MASK) >> 32) * C) >> 32
    mean = (_sm64((base(mix, 2) + comp * J + j) & MASK) >> 40) * 100
    S = 0
    for k in range(3):
        h = _sm64((base(draw, 3) + 3 * (r * J + j) + k) & MASK)
        for t in range(4):
            S += (h >> (16 * t)) & 0xFFFF
    v = mean + 10 * (S - 393210) * 256
    q, rem = divmod(v, 1 << 24)
    if rem > (1 << 23) or (rem == (1 << 23) and q % 2 == 1):
        q += 1
    return float(min(max(q, 0), 255))


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 seeded with 0 (state advanced by the golden gamma)
    got = [int(v) for v in synth.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))]
    assert got[0] == _sm64(0)
    assert got[0] == 0xE220A8397B1DCDAF
    assert got[1] == 0x6E789E6AA1B965F4


def test_gmm_matches_definition():
    J = 16
    rows = synth.gmm_rows(7, 8, 1000, 20, J)
    for r in range(20):
        for j in range(J):
            assert rows[r, j] == _ref_value(7, 8, 1000 + r, j, J)


def test_gmm_chunks_are_consistent_and_shaped():
    J = 128
    full = synth.gmm_rows(2000, 2001, 0, 3000, J)
    part = synth.gmm_rows(2000, 2001, 1000, 500, J)
    assert (full[1000:1500] == part).all()
    assert full.min() >= 0 and full.max() <= 255
    assert (full == np.round(full)).all()
    means = synth.gmm_means(2000, J)
    assert 0 <= means.min() and means.max() < 100
    # per-row residual from the nearest component mean has std close to 10
    d = ((full[:, None, :].astype(np.float64) - means[None]) ** 2).sum(-1)
    res = full - means[np.argmin(d, 1)]
    inner = (means[np.argmin(d, 1)] > 35) & (means[np.argmin(d, 1)] < 65)
    assert abs(res[inner].std() - 10.0) < 0.5


def test_normal_and_permutation_seeded():
    a = synth.normal(5, (100, 3))
    b = synth.normal(5, (100, 3))
    assert (a == b).all() and a.dtype == np.float32
    p = synth.permutation_prefix(9, 50, 16)
    assert len(set(p.tolist())) == 16 and p.max() < 50
