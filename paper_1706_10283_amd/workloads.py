"""Encoded databases built from the seeded synthetic inputs, at any scale.

The offline phase (Sec. 1.2) runs on the host with bolt_train_host: k-means
codebooks on a training sample, then the quantiser of each metric from
training queries taken from the training set (Sec. 4.1).  The database rows
are generated on the GPU chunk by chunk and encoded straight into HBM with
bolt_encode, so the fp32 data never has to exist in full.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import synth
import synth.device as sdev

from . import bolt as B


@dataclass
class EncodedDB:
    codes: torch.Tensor                 # uint8 [capacity, M/2]; rows [0, n_rows) valid
    n_rows: int
    J: int
    M: int
    centroids: torch.Tensor             # fp32 [M, 16, J/M] on the device
    centroids_host: np.ndarray
    scale: dict = field(default_factory=dict)     # metric -> a
    offsets: dict = field(default_factory=dict)   # metric -> fp32 [M] device tensor
    offsets_host: dict = field(default_factory=dict)
    mix_seed: int = 0
    draw_seed: int = 0

    @property
    def capacity(self) -> int:
        return self.codes.shape[0]

    def luts(self, Qv: torch.Tensor, metric: str, out=None, stream=None):
        return B.bolt_build_luts(Qv, self.centroids, self.M, metric, self.scale[metric],
                                 self.offsets[metric], luts_u8=out, stream=stream)


def train(mix_seed: int, train_seed: int, init_seed: int, lut_seed: int, J: int, M: int,
          n_train: int, iters: int = 10, n_lut_train: int = 1000, device="cuda"):
    """Training on a GPU-generated mixture sample: k-means on the GPU, the
    quantisers on the host.  Returns (centroids, {metric: (a, offsets)})."""
    Xtr = sdev.gmm_rows(mix_seed, train_seed, 0, n_train, J, device=device)
    init = synth.permutation_prefix(init_seed, n_train, 16)
    Qt = Xtr[torch.from_numpy(synth.permutation_prefix(lut_seed, n_train, n_lut_train)).to(device)].cpu().numpy()
    # codebooks on the GPU (bit-identical to the host k-means on this
    # integer-valued data), quantisers on the host
    Cd, _ = B.bolt_kmeans(Xtr, M, iters, init)
    C = Cd.cpu().numpy()
    tr_codes = B.bolt_encode(Xtr, Cd, M).cpu().numpy()
    a_l2, off_l2, _ = B.bolt_learn_quantizer_host(Qt, tr_codes, C, "l2")
    a_dot, off_dot, _ = B.bolt_learn_quantizer_host(Qt, tr_codes, C, "dot")
    return C, {"l2": (a_l2, off_l2), "dot": (a_dot, off_dot)}


def build_db(mix_seed: int, draw_seed: int, N: int, J: int, M: int, C: np.ndarray, quant: dict,
             capacity: int | None = None, chunk_rows: int = 8_000_000, device="cuda") -> EncodedDB:
    """Generate N mixture rows on the GPU in chunks and encode them into HBM."""
    capacity = max(capacity or N, N, 1)
    codes = torch.empty((capacity, M // 2), dtype=torch.uint8, device=device)
    Cd = torch.from_numpy(C).to(device)
    buf = torch.empty((min(chunk_rows, max(N, 1)), J), dtype=torch.float32, device=device)
    for r0 in range(0, N, chunk_rows):
        n = min(chunk_rows, N - r0)
        X = sdev.gmm_rows(mix_seed, draw_seed, r0, n, J, out=buf[:n])
        B.bolt_encode(X, Cd, M, codes=codes[r0:r0 + n])
    db = EncodedDB(codes=codes, n_rows=N, J=J, M=M, centroids=Cd, centroids_host=C,
                   mix_seed=mix_seed, draw_seed=draw_seed)
    for metric, (a, off) in quant.items():
        db.scale[metric] = float(a)
        db.offsets[metric] = torch.from_numpy(np.ascontiguousarray(off, dtype=np.float32)).to(device)
        db.offsets_host[metric] = np.ascontiguousarray(off, dtype=np.float32)
    del buf
    return db


# ------------------------------------------------------------------ the batched workload

@dataclass
class BatchedSpec:
    N: int
    J: int
    M: int
    Q: int
    metric: str
    seed: int


def batched_specs(n_db: int = 256, seed: int = 4006, N_lo: float = 1e3, N_hi: float = 2e6,
                  Js=(64, 128, 256), Ms=(16, 32, 64), Q_lo: int = 1, Q_hi: int = 512):
    """Uneven databases: N log-uniform in [N_lo, N_hi], J and M uniform over
    their sets, Q uniform in [Q_lo, Q_hi], metric L2 or dot with equal odds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n_db):
        N = int(round(math.exp(rng.uniform(math.log(N_lo), math.log(N_hi)))))
        J = int(rng.choice(Js))
        M = int(rng.choice(Ms))
        Q = int(rng.integers(Q_lo, Q_hi, endpoint=True))
        metric = "l2" if rng.random() < 0.5 else "dot"
        specs.append(BatchedSpec(N, J, M, Q, metric, 100_000 + 10 * i))
    return specs


def build_batched(specs, n_train: int = 20_000, iters: int = 10, k: int = 100, device="cuda", log=None):
    """Encode every database of the batched workload and the tables of its queries."""
    dbs = []
    t0 = time.time()
    for i, s in enumerate(specs):
        C, quant = train(s.seed, s.seed + 3, s.seed + 4, s.seed + 5, s.J, s.M, n_train, iters,
                         n_lut_train=min(1000, n_train), device=device)
        db = build_db(s.seed, s.seed + 1, s.N, s.J, s.M, C, quant, device=device)
        Qv = sdev.gmm_rows(s.seed, s.seed + 2, 0, s.Q, s.J, device=device)
        luts = db.luts(Qv, s.metric)
        dbs.append({"db": db, "codes": db.codes[:s.N], "luts": luts, "Qv": Qv, "metric": s.metric,
                    "k": k, "spec": s})
        if log and (i + 1) % 32 == 0:
            log("built %d/%d databases (%.1fs)" % (i + 1, len(specs), time.time() - t0))
    return dbs
