"""CPU oracle for the Bolt hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

The arithmetic lives in ``bolt_oracle.c`` (plain scalar C, see its header
for the definitions and the paper passages they follow); this module only
compiles it with gcc and marshals numpy arrays.

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):
  encode              pinned: the fp32 decision (canonical order, ties to the
                      lowest index) against an exact-rational emulation of
                      each rounding, and against the fp64 argmin (near ties
                      only)
  subspace_dists_f64  pinned: integer-valued inputs against int64 brute force
                      (exact), continuous inputs against exact rationals
  luts                pinned: fp64 closed forms; the canonical fp32 order bit
                      for bit against an exact-rational emulation; uint8 by
                      the formula in exact arithmetic; L_p against L1/L2 at
                      p = 1, 2, the L_p closed form and an exact-rational
                      emulation at p = 3; cosine against dot tables of the
                      unit query and the closed form q.x_hat / |q|
  normalize_rows      pinned: numpy's IEEE fp32 sqrt and division after the
                      exact-rational fused sum of squares; unit norm
  scan, scan_pairs, topk, scan_f32, topk_f32,
  rescale_f64, rescale_f32                      pinned
  kmeans                                        pinned to scikit-learn's Lloyd
                                                iterations from the same initial
                                                rows (the paper prints no trained
                                                values)
  learn_quantizer                               pinned to numpy quantiles of the
                                                expanded sample and the argmin of
                                                the recomputed grid losses
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bolt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ALPHAS = np.array([0.0, 0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1], dtype=np.float64)
METRICS = {"l2": 0, "dot": 1, "l1": 2, "cosine": 4}


def _metric(metric):
    """(code, p) of a metric name: "l2", "dot", "l1", "cosine" or "lp<p>"
    (the L_p distance to the p, integer p >= 1)."""
    if metric in METRICS:
        return METRICS[metric], 0
    if metric.startswith("lp") and metric[2:].isdigit() and int(metric[2:]) >= 1:
        return 3, int(metric[2:])
    raise ValueError("unknown metric %r" % (metric,))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


I64 = ctypes.c_int64
I32 = ctypes.c_int32


def encode(X, C, M, want_dists=False):
    """Codes uint8 [N, M/2] (and fp32 distances [N, M, 16] if asked)."""
    X = _f32(X)
    C = _f32(C)
    N, J = X.shape
    codes = np.zeros((N, M // 2), dtype=np.uint8)
    d = np.zeros((N, M, 16), dtype=np.float32) if want_dists else None
    _load().orc_encode(_p(X), I64(N), I32(J), I64(J), _p(C), I32(M), _p(codes), _p(d))
    return (codes, d) if want_dists else codes


def subspace_dists_f64(X, C, M):
    X = _f32(X)
    C = _f32(C)
    N, J = X.shape
    out = np.zeros((N, M, 16), dtype=np.float64)
    _load().orc_subspace_dists_f64(_p(X), I64(N), I32(J), I64(J), _p(C), I32(M), _p(out))
    return out


def luts(Qv, C, M, metric="l2", a=1.0, offsets=None):
    """(lut64 fp64, lut32 fp32, lut8 uint8), each [Q, M, 16]."""
    Qv = _f32(Qv)
    C = _f32(C)
    Q, J = Qv.shape
    if offsets is None:
        offsets = np.zeros(M, dtype=np.float32)
    offsets = _f32(offsets)
    l64 = np.zeros((Q, M, 16), dtype=np.float64)
    l32 = np.zeros((Q, M, 16), dtype=np.float32)
    l8 = np.zeros((Q, M, 16), dtype=np.uint8)
    code, p = _metric(metric)
    _load().orc_luts(_p(Qv), I64(Q), I32(J), I64(J), _p(C), I32(M), I32(code), I32(p),
                     ctypes.c_float(a), _p(offsets), _p(l64), _p(l32), _p(l8))
    return l64, l32, l8


def normalize_rows(X):
    """Unit-norm rows fp32 [N, J] (cosine similarity); zero rows stay zero."""
    X = _f32(X)
    N, J = X.shape
    Y = np.zeros((N, J), dtype=np.float32)
    _load().orc_normalize_rows(_p(X), I64(N), I32(J), I64(J), _p(Y), I64(J))
    return Y


def scan(codes, lut8):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lut8 = np.ascontiguousarray(lut8, dtype=np.uint8)
    N = codes.shape[0]
    Q, M, _ = lut8.shape
    out = np.zeros((Q, N), dtype=np.uint16)
    _load().orc_scan(_p(codes), I64(N), I32(M), _p(lut8), I64(Q), _p(out))
    return out


def scan_pairs(codes, lut8, qs, ns):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lut8 = np.ascontiguousarray(lut8, dtype=np.uint8)
    qs = np.ascontiguousarray(qs, dtype=np.int64)
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    M = lut8.shape[1]
    out = np.zeros(len(qs), dtype=np.uint32)
    _load().orc_scan_pairs(_p(codes), I32(M), _p(lut8), _p(qs), _p(ns), I64(len(qs)), _p(out))
    return out


def topk(d, k, largest=False):
    d = np.ascontiguousarray(d, dtype=np.uint16)
    Q, N = d.shape
    vals = np.zeros((Q, k), dtype=np.uint16)
    idx = np.zeros((Q, k), dtype=np.int32)
    _load().orc_topk(_p(d), I64(Q), I64(N), I64(N), I32(k), I32(1 if largest else 0),
                     _p(vals), _p(idx))
    return vals, idx


def scan_f32(codes, lutf):
    """Bolt No Quantize: fp32 sums [Q, N] of float tables [Q, M, 16], ascending m."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lutf = _f32(lutf)
    N = codes.shape[0]
    Q, M, _ = lutf.shape
    out = np.zeros((Q, N), dtype=np.float32)
    _load().orc_scan_f32(_p(codes), I64(N), I32(M), _p(lutf), I64(Q), _p(out))
    return out


def topk_f32(d, k, largest=False):
    """(vals fp32 [Q, k], idx int32 [Q, k]): k smallest (largest) values, ties by index."""
    d = _f32(d)
    Q, N = d.shape
    vals = np.zeros((Q, k), dtype=np.float32)
    idx = np.zeros((Q, k), dtype=np.int32)
    _load().orc_topk_f32(_p(d), I64(Q), I64(N), I64(N), I32(k), I32(1 if largest else 0),
                         _p(vals), _p(idx))
    return vals, idx


def rescale_f64(S, a, offsets):
    S = np.ascontiguousarray(S, dtype=np.uint16)
    offsets = _f32(offsets)
    out = np.zeros(S.shape, dtype=np.float64)
    _load().orc_rescale_f64(_p(S), I64(S.size), ctypes.c_float(a), _p(offsets),
                            I32(len(offsets)), _p(out))
    return out


def rescale_f32(S, bias, scale):
    S = np.ascontiguousarray(S, dtype=np.uint16)
    out = np.zeros(S.shape, dtype=np.float32)
    _load().orc_rescale_f32(_p(S), I64(S.size), ctypes.c_float(bias), ctypes.c_float(scale),
                            _p(out))
    return out


def kmeans(X, M, iters, init_rows):
    """Centroids fp32 [M, 16, J/M] and the objective before each update [iters+1]."""
    X = _f32(X)
    n, J = X.shape
    init_rows = np.ascontiguousarray(init_rows, dtype=np.int64)
    assert len(init_rows) == 16
    C = np.zeros((M, 16, J // M), dtype=np.float32)
    obj = np.zeros(iters + 1, dtype=np.float64)
    _load().orc_kmeans(_p(X), I64(n), I32(J), I64(J), I32(M), I32(iters), _p(init_rows),
                       _p(C), _p(obj))
    return C, obj


def learn_quantizer(Qt, codes, C, metric="l2", alphas=ALPHAS):
    """(a, offsets[M], chosen alpha index, losses[len(alphas)])."""
    Qt = _f32(Qt)
    C = _f32(C)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    alphas = np.ascontiguousarray(alphas, dtype=np.float64)
    nq, J = Qt.shape
    M = C.shape[0]
    a = np.zeros(1, dtype=np.float32)
    offs = np.zeros(M, dtype=np.float32)
    losses = np.zeros(len(alphas), dtype=np.float64)
    lib = _load()
    lib.orc_learn_quantizer.restype = ctypes.c_int
    code, p = _metric(metric)
    best = lib.orc_learn_quantizer(_p(Qt), I64(nq), I32(J), I64(J), _p(codes), I64(codes.shape[0]),
                                   _p(C), I32(M), I32(code), I32(p), _p(alphas),
                                   I32(len(alphas)), _p(a), _p(offs), _p(losses))
    return float(a[0]), offs, int(best), losses


def train(Xtrain, M, iters, init_rows, Qtrain, metric="l2"):
    """Full offline phase: codebooks, then the quantiser for ``metric``.

    Returns (centroids, a, offsets, alpha_index)."""
    C, _ = kmeans(Xtrain, M, iters, init_rows)
    codes = encode(Xtrain, C, M)
    a, offs, best, _ = learn_quantizer(Qtrain, codes, C, metric)
    return C, a, offs, best
