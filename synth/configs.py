"""Workload presets: sizes and seeds of the five synthetic workloads.

Each preset describes shapes only; the data itself comes from the
generators in ``synth``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

LUT_ALPHAS = (0.0, 0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1)


@dataclass(frozen=True)
class Tiny:
    """N(0,1) data, 10k x 32, M=8, 16 queries, squared L2, top-10."""
    config: int = 1
    N: int = 10_000
    J: int = 32
    M: int = 8
    Q: int = 16
    k: int = 10
    kmeans_iters: int = 10
    metric: str = "l2"


@dataclass(frozen=True)
class SingleDB:
    """Mixture data, 1e6 x 128, M in {16,32,64}, 1000 queries, L2 and dot, top-100."""
    config: int = 2
    N: int = 1_000_000
    J: int = 128
    Ms: Tuple[int, ...] = (16, 32, 64)
    Q: int = 1000
    k: int = 100
    n_train: int = 100_000
    n_lut_train: int = 1000
    kmeans_iters: int = 10


@dataclass(frozen=True)
class AMM:
    """A: 2e5 x 256 N(0,1) encoded with M=32; B: 256 x K N(0,1), K in {64,256,1024}."""
    config: int = 3
    N: int = 200_000
    J: int = 256
    M: int = 32
    Ks: Tuple[int, ...] = (64, 256, 1024)
    n_lut_train: int = 1000
    kmeans_iters: int = 10


@dataclass(frozen=True)
class Batched:
    """256 mixture databases, N log-uniform in [1e3, 2e6], J in {64,128,256}, M in {16,32,64}."""
    config: int = 4
    n_db: int = 256
    N_lo: float = 1e3
    N_hi: float = 2e6
    Js: Tuple[int, ...] = (64, 128, 256)
    Ms: Tuple[int, ...] = (16, 32, 64)
    Q_lo: int = 1
    Q_hi: int = 512
    k: int = 100
    n_train: int = 20_000
    kmeans_iters: int = 10


@dataclass(frozen=True)
class Serving:
    """8 resident mixture databases of 2.5e8 x 128 at M=32 (32 GB of codes)."""
    config: int = 5
    n_db: int = 8
    N_per_db: int = 250_000_000
    J: int = 128
    M: int = 32
    batch_lo: int = 1
    batch_hi: int = 64
    k: int = 100
    insert_lo: float = 1e4
    insert_hi: float = 1e6
    insert_frac: float = 0.1
    n_train: int = 100_000
    kmeans_iters: int = 10


TINY = Tiny()
SINGLE_DB = SingleDB()
AMM_CFG = AMM()
BATCHED = Batched()
SERVING = Serving()
