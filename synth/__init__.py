"""Seeded synthetic inputs for the Bolt hot path.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It holds random draws only, none of the method's arithmetic
(no distances, no codes, no lookup tables, no quantisation).

Two kinds of inputs are produced:

* i.i.d. N(0, 1) fp32 matrices, drawn with numpy's PCG64 generator.  These
  stand in for the "random data" the paper times on (Sec. 4, timing
  protocol) and for the approximate matrix product workload (Sec. 4.4).

* A 256-component Gaussian mixture shaped like the descriptor datasets the
  paper evaluates on (Sec. 4.1): component means uniform in [0, 100] per
  dimension, per-dimension noise of standard deviation 10, values rounded to
  integers and clipped to [0, 255].  This generator is counter based and
  written in exact integer arithmetic, so that any row can be regenerated on
  the host, bit for bit, from (mixture seed, draw seed, row index) after the
  GPU generated the same rows at full scale (``synth/gmm.hip`` implements the
  identical definition).  The Gaussian noise is the classical Irwin-Hall
  approximation: the sum of twelve uniform variates minus six, which has mean
  0 and variance 1.  The uniform variates are 16-bit fields of SplitMix64
  outputs (Steele, Lea & Flood, OOPSLA 2014).

Definition of the mixture generator (all arithmetic modulo 2**64 unless
stated otherwise):

    splitmix64(x):  z = x + 0x9E3779B97F4A7C15
                    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
                    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
                    return z ^ (z >> 31)
    base(seed, s) = splitmix64(seed * 16 + s)          s = 1 comp, 2 mean, 3 noise
    comp(r)       = (splitmix64(base(draw, 1) + r) >> 32) * C >> 32     (C components)
    mean(c, j)    = (splitmix64(base(mix, 2) + c*J + j) >> 40) * 100   [units of 2^-24]
    S(r, j)       = sum over k < 3, t < 4 of 16-bit field t of
                    splitmix64(base(draw, 3) + 3*(r*J + j) + k)
    v(r, j)       = mean(comp(r), j) + 10 * (S - 393210) * 256          [units of 2^-24]
    x(r, j)       = clip(round_half_even(v / 2^24), 0, 255)              (as fp32)

``S - 393210`` equals 2^16 times (sum of the twelve variates, each taken at the
centre of its 16-bit bin, minus 6).
"""
from __future__ import annotations

import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_COMP = 1
STREAM_MEAN = 2
STREAM_NOISE = 3
N_COMPONENTS = 256


def splitmix64(x):
    """SplitMix64 output function of state ``x`` (uint64 array, wraps mod 2^64)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_base(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * np.uint64(16) + np.uint64(stream)
    return splitmix64(np.array([s], dtype=np.uint64))[0]


def gmm_rows(mix_seed: int, draw_seed: int, row0: int, nrows: int, J: int,
             n_comp: int = N_COMPONENTS) -> np.ndarray:
    """Rows ``row0 .. row0+nrows-1`` of the mixture sample, fp32 [nrows, J]."""
    if nrows <= 0:
        return np.zeros((0, J), dtype=np.float32)
    rows = np.arange(row0, row0 + nrows, dtype=np.uint64)
    b_comp = stream_base(draw_seed, STREAM_COMP)
    b_mean = stream_base(mix_seed, STREAM_MEAN)
    b_noise = stream_base(draw_seed, STREAM_NOISE)
    with np.errstate(over="ignore"):
        h = splitmix64(b_comp + rows)
        comp = ((h >> np.uint64(32)) * np.uint64(n_comp)) >> np.uint64(32)
        jj = np.arange(J, dtype=np.uint64)
        mean_idx = comp[:, None] * np.uint64(J) + jj[None, :]
        mean = (splitmix64(b_mean + mean_idx) >> np.uint64(40)).astype(np.int64) * 100
        elem = rows[:, None] * np.uint64(J) + jj[None, :]
        S = np.zeros((nrows, J), dtype=np.int64)
        for k in range(3):
            hk = splitmix64(b_noise + elem * np.uint64(3) + np.uint64(k))
            for t in range(4):
                S += ((hk >> np.uint64(16 * t)) & np.uint64(0xFFFF)).astype(np.int64)
    v = mean + 10 * (S - 393210) * 256
    q = v >> 24                       # floor division by 2^24
    rem = v - (q << 24)
    half = 1 << 23
    q = q + (rem > half) + ((rem == half) & ((q & 1) == 1))
    return np.clip(q, 0, 255).astype(np.float32)


def gmm_means(mix_seed: int, J: int, n_comp: int = N_COMPONENTS) -> np.ndarray:
    """Component means of the mixture (float64 [n_comp, J]), for reporting."""
    b_mean = stream_base(mix_seed, STREAM_MEAN)
    idx = np.arange(n_comp * J, dtype=np.uint64)
    with np.errstate(over="ignore"):
        m = (splitmix64(b_mean + idx) >> np.uint64(40)).astype(np.float64) * 100.0
    return (m / float(1 << 24)).reshape(n_comp, J)


def normal(seed: int, shape) -> np.ndarray:
    """i.i.d. N(0,1) fp32 draws from numpy's PCG64 generator."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=shape, dtype=np.float32)


def uniform(seed: int, shape, lo=0.0, hi=1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def permutation_prefix(seed: int, n: int, k: int) -> np.ndarray:
    """First ``k`` entries of a seeded permutation of ``range(n)`` (int64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.permutation(n)[: min(k, n)].astype(np.int64)


def integers(seed: int, lo: int, hi: int, size) -> np.ndarray:
    """Seeded integers in [lo, hi] inclusive."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi, size=size, endpoint=True)


def random_codes(seed: int, N: int, M: int) -> np.ndarray:
    """Uniform random packed 4-bit codes, uint8 [N, M/2] (any byte is valid)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 256, size=(N, M // 2), dtype=np.uint8)


def random_luts(seed: int, Q: int, M: int) -> np.ndarray:
    """Uniform random uint8 lookup tables [Q, M, 16]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 256, size=(Q, M, 16), dtype=np.uint8)


def seed_for(config: int, purpose: int) -> int:
    """Seed layout: 1000*config + purpose.

    purpose: 0 mixture parameters, 1 database, 2 queries, 3 training set,
    4 k-means initial rows, 5 quantiser-training queries, 6 schedule/arrivals.
    """
    return 1000 * config + purpose


from . import configs  # noqa: E402  (re-export of the workload presets)
