"""Python binding of libbolt.so: the same entry points as include/bolt.h.

Only argument marshalling happens here (torch tensors -> device pointers,
the current HIP stream); every step of the hot path runs in the HIP
kernels.  The library must be built (``python -m paper_1706_10283_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbolt.so")

BOLT_OK = 0
BOLT_ERR_INVALID = -1
BOLT_ERR_SHAPE = -2
BOLT_ERR_UNSUPPORTED = -3
BOLT_ERR_DEVICE = -4
BOLT_ERR_NOMEM = -5
METRIC_L2 = 0
METRIC_DOT = 1
METRIC_L1 = 2
METRIC_COSINE = 4
TOPK_MAX_K = 2048
ALPHAS = (0.0, 0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1)

_STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "SHAPE", -3: "UNSUPPORTED", -4: "DEVICE", -5: "NOMEM"}


class BoltError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("bolt status %d (%s): %s" % (status, _STATUS_NAMES.get(status, "?"), message))
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError("libbolt.so is not built: run `python -m paper_1706_10283_amd.build` "
                      "(the HIP library is required; there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F32 = ctypes.c_float
_SZ = ctypes.c_size_t

_SIGS = {
    "bolt_last_error": ([], ctypes.c_char_p),
    "bolt_version": ([], ctypes.c_char_p),
    "bolt_encode": ([_P, _I64, _I32, _I64, _P, _I32, _P, _P], ctypes.c_int),
    "bolt_normalize_rows": ([_P, _I64, _I32, _I64, _P, _I64, _P], ctypes.c_int),
    "bolt_build_luts": ([_P, _I64, _I32, _I64, _P, _I32, _I32, _F32, _P, _P, _P, _P], ctypes.c_int),
    "bolt_scan_l2": ([_P, _I64, _I32, _P, _I64, _P, _I64, _P], ctypes.c_int),
    "bolt_scan_dot": ([_P, _I64, _I32, _P, _I64, _P, _I64, _P], ctypes.c_int),
    "bolt_topk_ws_bytes": ([_I64, _I64, _I32], _SZ),
    "bolt_topk": ([_P, _I64, _I64, _I64, _I32, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "bolt_scan_topk_ws_bytes": ([_I64, _I32, _I64, _I32], _SZ),
    "bolt_scan_topk": ([_P, _I64, _I32, _P, _I64, _I32, _I32, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "bolt_amm": ([_P, _I64, _I32, _P, _I64, _F32, _F32, _P, _I64, _I32, _P], ctypes.c_int),
    "bolt_scan_f32": ([_P, _I64, _I32, _P, _I64, _P, _I64, _P], ctypes.c_int),
    "bolt_scan_topk_split_ws_bytes": ([_I64, _I32, _I64, _I64, _I32], _SZ),
    "bolt_scan_topk_split": ([_P, _I64, _I32, _P, _I64, _I64, _I32, _I32, _I32, _P, _P, _P, _SZ, _P],
                             ctypes.c_int),
    "bolt_scan_topk_ranges_ws_bytes": ([_P, _I32, _I32, _I64, _I32], _SZ),
    "bolt_scan_topk_ranges": ([_P, _I64, _I32, _P, _I64, _I32, _I32, _P, _I32, _P, _P, _P, _SZ, _P],
                              ctypes.c_int),
    "bolt_kmeans_ws_bytes": ([_I32, _I32, _I32], _SZ),
    "bolt_kmeans": ([_P, _I64, _I32, _I64, _I32, _I32, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "bolt_topk_f32": ([_P, _I64, _I64, _I64, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "bolt_train_host": ([_P, _I64, _I32, _I64, _I32, _I32, _P, _P, _I64, _I64, _I32, _P, _I32,
                         _P, _P, _P, _P], ctypes.c_int),
    "bolt_learn_quantizer_host": ([_P, _I64, _I32, _I64, _P, _I64, _P, _I32, _I32, _P, _I32,
                                   _P, _P, _P], ctypes.c_int),
    "bolt_learn_quantizer_ws_bytes": ([_I64, _I32, _I32], _SZ),
    "bolt_learn_quantizer": ([_P, _I64, _I32, _I64, _P, _I64, _P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P,
                              _SZ, _P], ctypes.c_int),
    "bolt_debug_force_scan_kernel": ([_I32], ctypes.c_int),
    "bolt_debug_force_unfused_topk": ([_I32], ctypes.c_int),
    "bolt_debug_force_fused_kind": ([_I32], ctypes.c_int),
    "bolt_debug_speculation": ([_I32], ctypes.c_int),
    "bolt_debug_sparse_mfma": ([_I32], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def lib():
    return _lib


def last_error() -> str:
    return _lib.bolt_last_error().decode()


def version() -> str:
    return _lib.bolt_version().decode()


def _check(status):
    if status != BOLT_OK:
        raise BoltError(status, last_error())


def _stream(stream):
    if stream is None:
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    return t


def _ptr(t):
    return _P(t.data_ptr()) if t is not None else _P(0)


def _rows(t, name):
    """(rows, cols, row stride) of a 2-D tensor with unit column stride."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.numel() == 0:
        return t.shape[0], t.shape[1], t.shape[1]
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("%s must have contiguous rows" % name)
    return t.shape[0], t.shape[1], max(t.stride(0), t.shape[1])


def metric_id(metric):
    """The library's metric code of a name ("l2", "dot", "l1", "cosine" or
    "lp<p>", the L_p distance to the p) or of a code."""
    if isinstance(metric, (int, np.integer)):
        return int(metric)
    names = {"l2": METRIC_L2, "dot": METRIC_DOT, "l1": METRIC_L1, "cosine": METRIC_COSINE}
    if metric in names:
        return names[metric]
    if metric.startswith("lp") and metric[2:].isdigit():
        return metric_lp(int(metric[2:]))
    raise ValueError("unknown metric %r" % (metric,))


def metric_lp(p):
    """Metric code of the L_p distance to the p (bolt.h BOLT_METRIC_LP)."""
    return 3 + 256 * int(p)


def metric_largest(metric):
    """True for the similarities (dot, cosine), whose top-k takes the largest sums."""
    return metric_id(metric) in (METRIC_DOT, METRIC_COSINE)


# ------------------------------------------------------------------ hot path

def bolt_encode(X, centroids, M, codes=None, stream=None):
    """codes uint8 [N, M/2] of fp32 rows X [N, J] (nearest centroid per subspace)."""
    _dev(X, torch.float32, "X")
    _dev(centroids, torch.float32, "centroids")
    N, J, ldx = _rows(X, "X")
    if not centroids.is_contiguous() or centroids.numel() != 16 * J:
        raise ValueError("centroids must be contiguous [M, 16, J/M]")
    if codes is None:
        codes = torch.empty((N, M // 2), dtype=torch.uint8, device=X.device)
    _dev(codes, torch.uint8, "codes")
    _check(_lib.bolt_encode(_ptr(X), N, J, ldx, _ptr(centroids), M, _ptr(codes), _stream(stream)))
    return codes


def bolt_normalize_rows(X, out=None, stream=None):
    """Unit rows fp32 [N, J] of X [N, J] (cosine similarity); zero rows stay
    zero.  out may be X itself (in place)."""
    _dev(X, torch.float32, "X")
    N, J, ldx = _rows(X, "X")
    if out is None:
        out = torch.empty((N, J), dtype=torch.float32, device=X.device)
    _dev(out, torch.float32, "out")
    M_, J_, ldy = _rows(out, "out")
    if (M_, J_) != (N, J):
        raise ValueError("out must be [N, J]")
    _check(_lib.bolt_normalize_rows(_ptr(X), N, J, ldx, _ptr(out), ldy, _stream(stream)))
    return out


def bolt_build_luts(Qv, centroids, M, metric, a, offsets, luts_u8=None, luts_f32=None,
                    want_f32=False, want_u8=True, stream=None):
    """uint8 tables [Q, M, 16] (and fp32 tables if asked) of the queries Qv [Q, J]."""
    _dev(Qv, torch.float32, "Qv")
    _dev(centroids, torch.float32, "centroids")
    Q, J, ldq = _rows(Qv, "Qv")
    if offsets is not None:
        _dev(offsets, torch.float32, "offsets")
    if want_u8 and luts_u8 is None:
        luts_u8 = torch.empty((Q, M, 16), dtype=torch.uint8, device=Qv.device)
    if want_f32 and luts_f32 is None:
        luts_f32 = torch.empty((Q, M, 16), dtype=torch.float32, device=Qv.device)
    _check(_lib.bolt_build_luts(_ptr(Qv), Q, J, ldq, _ptr(centroids), M, metric_id(metric),
                                float(a), _ptr(offsets), _ptr(luts_f32), _ptr(luts_u8),
                                _stream(stream)))
    if want_f32 and want_u8:
        return luts_u8, luts_f32
    return luts_u8 if want_u8 else luts_f32


def _scan(fn, codes, luts_u8, out, stream):
    _dev(codes, torch.uint8, "codes")
    _dev(luts_u8, torch.uint8, "luts_u8")
    N = codes.shape[0]
    Q, M = luts_u8.shape[0], luts_u8.shape[1]
    if codes.dim() != 2 or codes.shape[1] != M // 2 or not codes.is_contiguous():
        raise ValueError("codes must be contiguous [N, M/2]")
    if out is None:
        out = torch.empty((Q, N), dtype=torch.uint16, device=codes.device)
    _dev(out, torch.uint16, "out")
    ldo = out.stride(0) if Q > 0 else N
    _check(fn(_ptr(codes), N, M, _ptr(luts_u8), Q, _ptr(out), max(ldo, N), _stream(stream)))
    return out


def bolt_scan_l2(codes, luts_u8, out=None, stream=None):
    """uint16 sums [Q, N] = sum_m luts[q, m, code(n, m)]."""
    return _scan(_lib.bolt_scan_l2, codes, luts_u8, out, stream)


def bolt_scan_dot(codes, luts_u8, out=None, stream=None):
    return _scan(_lib.bolt_scan_dot, codes, luts_u8, out, stream)


def bolt_topk(dists, k, largest=False, vals=None, idx=None, stream=None):
    """(vals uint16 [Q, k], idx int32 [Q, k]) of each row of dists [Q, N]."""
    _dev(dists, torch.uint16, "dists")
    Q, N, ldd = _rows(dists, "dists")
    if vals is None:
        vals = torch.empty((Q, k), dtype=torch.uint16, device=dists.device)
    if idx is None:
        idx = torch.empty((Q, k), dtype=torch.int32, device=dists.device)
    nws = _lib.bolt_topk_ws_bytes(Q, N, k)
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dists.device)
    _check(_lib.bolt_topk(_ptr(dists), Q, N, ldd, k, 1 if largest else 0, _ptr(vals), _ptr(idx),
                          _ptr(ws), nws, _stream(stream)))
    return vals, idx


def bolt_scan_f32(codes, luts_f32, out=None, stream=None):
    """Bolt No Quantize: fp32 sums [Q, N] of the float tables over the codes."""
    _dev(codes, torch.uint8, "codes")
    _dev(luts_f32, torch.float32, "luts_f32")
    N = codes.shape[0]
    Q, M = luts_f32.shape[0], luts_f32.shape[1]
    if out is None:
        out = torch.empty((Q, N), dtype=torch.float32, device=codes.device)
    _dev(out, torch.float32, "out")
    ldo = out.stride(0) if out.shape[0] > 0 else N
    _check(_lib.bolt_scan_f32(_ptr(codes), N, M, _ptr(luts_f32), Q, _ptr(out), ldo, _stream(stream)))
    return out


def bolt_topk_f32(dists, k, largest=False, vals=None, idx=None, stream=None):
    """(vals fp32 [Q, k], idx int32 [Q, k]) of each row of fp32 dists [Q, N]."""
    _dev(dists, torch.float32, "dists")
    Q, N, ldd = _rows(dists, "dists")
    if vals is None:
        vals = torch.empty((Q, k), dtype=torch.float32, device=dists.device)
    if idx is None:
        idx = torch.empty((Q, k), dtype=torch.int32, device=dists.device)
    _check(_lib.bolt_topk_f32(_ptr(dists), Q, N, ldd, k, 1 if largest else 0, _ptr(vals), _ptr(idx),
                              _stream(stream)))
    return vals, idx


def bolt_kmeans(X, M, iters, init_rows, centroids=None, stream=None):
    """Codebooks on the GPU: (centroids device fp32 [M, 16, J/M], objective numpy fp64 [iters + 1])."""
    _dev(X, torch.float32, "X")
    n, J, ldx = _rows(X, "X")
    init = np.ascontiguousarray(init_rows, dtype=np.int64)
    if init.shape != (16,):
        raise ValueError("init_rows must hold 16 row indices")
    if centroids is None:
        centroids = torch.empty((M, 16, J // M if M else 0), dtype=torch.float32, device=X.device)
    _dev(centroids, torch.float32, "centroids")
    nws = int(_lib.bolt_kmeans_ws_bytes(J, M, iters))
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=X.device)
    obj = np.zeros(max(iters + 1, 1), dtype=np.float64)
    _check(_lib.bolt_kmeans(_ptr(X), n, J, ldx, M, iters, init.ctypes.data, _ptr(centroids),
                            obj.ctypes.data, _ptr(ws), nws, _stream(stream)))
    return centroids, obj


def bolt_scan_topk_ws_bytes(N, M, Q, k):
    return int(_lib.bolt_scan_topk_ws_bytes(N, M, Q, k))


def bolt_scan_topk(codes, luts_u8, metric, k, vals=None, idx=None, ws=None, stream=None):
    """Fused scan + top-k: (vals, idx) as bolt_topk(bolt_scan(...)) with largest = dot."""
    _dev(codes, torch.uint8, "codes")
    _dev(luts_u8, torch.uint8, "luts_u8")
    N = codes.shape[0]
    Q, M = luts_u8.shape[0], luts_u8.shape[1]
    if vals is None:
        vals = torch.empty((Q, k), dtype=torch.uint16, device=codes.device)
    if idx is None:
        idx = torch.empty((Q, k), dtype=torch.int32, device=codes.device)
    nws = bolt_scan_topk_ws_bytes(N, M, Q, k)
    if ws is None:
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=codes.device)
    wsb = ws.numel() * ws.element_size()
    _check(_lib.bolt_scan_topk(_ptr(codes), N, M, _ptr(luts_u8), Q, metric_id(metric), k,
                               _ptr(vals), _ptr(idx), _ptr(ws), wsb, _stream(stream)))
    return vals, idx


def bolt_scan_topk_split_ws_bytes(N, M, Q, q_split, k):
    return int(_lib.bolt_scan_topk_split_ws_bytes(N, M, Q, q_split, k))


def bolt_scan_topk_split(codes, luts_u8, q_split, metric_lo, metric_hi, k, vals=None, idx=None, ws=None,
                         stream=None):
    """Scan + top-k of queries [0, q_split) under metric_lo and [q_split, Q) under
    metric_hi in one call: (vals, idx) as bolt_scan_topk gives each side."""
    _dev(codes, torch.uint8, "codes")
    _dev(luts_u8, torch.uint8, "luts_u8")
    N = codes.shape[0]
    Q, M = luts_u8.shape[0], luts_u8.shape[1]
    if vals is None:
        vals = torch.empty((Q, k), dtype=torch.uint16, device=codes.device)
    if idx is None:
        idx = torch.empty((Q, k), dtype=torch.int32, device=codes.device)
    nws = bolt_scan_topk_split_ws_bytes(N, M, Q, q_split, k)
    if ws is None:
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=codes.device)
    wsb = ws.numel() * ws.element_size()
    _check(_lib.bolt_scan_topk_split(_ptr(codes), N, M, _ptr(luts_u8), Q, q_split, metric_id(metric_lo),
                                     metric_id(metric_hi), k, _ptr(vals), _ptr(idx), _ptr(ws), wsb,
                                     _stream(stream)))
    return vals, idx


def bolt_scan_topk_ranges(codes, luts_u8, metric, k, ranges, vals=None, idx=None, stream=None):
    """Scan + top-k over the rows of `ranges` (host int64 [R, 2]: ascending,
    disjoint [start, end) pairs); row indices refer to the whole codes."""
    _dev(codes, torch.uint8, "codes")
    _dev(luts_u8, torch.uint8, "luts_u8")
    N = codes.shape[0]
    Q, M = luts_u8.shape[0], luts_u8.shape[1]
    rg = np.ascontiguousarray(np.asarray(ranges, dtype=np.int64).reshape(-1, 2))
    R = rg.shape[0]
    if vals is None:
        vals = torch.empty((Q, k), dtype=torch.uint16, device=codes.device)
    if idx is None:
        idx = torch.empty((Q, k), dtype=torch.int32, device=codes.device)
    nws = int(_lib.bolt_scan_topk_ranges_ws_bytes(rg.ctypes.data, R, M, Q, k))
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=codes.device)
    _check(_lib.bolt_scan_topk_ranges(_ptr(codes), N, M, _ptr(luts_u8), Q, metric_id(metric), k, rg.ctypes.data,
                                      R, _ptr(vals), _ptr(idx), _ptr(ws), nws, _stream(stream)))
    return vals, idx


def bolt_amm(codes, luts_u8, bias, scale, out=None, transpose=False, stream=None):
    """Approximate product: fp32 (S + bias) * scale, [K, N] or [N, K] if transpose."""
    _dev(codes, torch.uint8, "codes")
    _dev(luts_u8, torch.uint8, "luts_u8")
    N = codes.shape[0]
    K, M = luts_u8.shape[0], luts_u8.shape[1]
    if out is None:
        shape = (N, K) if transpose else (K, N)
        out = torch.empty(shape, dtype=torch.float32, device=codes.device)
    _dev(out, torch.float32, "out")
    ldo = out.stride(0) if out.shape[0] > 0 else (K if transpose else N)
    _check(_lib.bolt_amm(_ptr(codes), N, M, _ptr(luts_u8), K, float(bias), float(scale),
                         _ptr(out), ldo, 1 if transpose else 0, _stream(stream)))
    return out


# ------------------------------------------------------------------ host training

def _np_ptr(a):
    return _P(a.ctypes.data) if a is not None else _P(0)


def bolt_train_host(X, M, iters, init_rows, Qt, metric, alphas=ALPHAS):
    """Offline phase on the host: (centroids [M,16,J/M], a, offsets [M], alpha index)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Qt = np.ascontiguousarray(Qt, dtype=np.float32)
    init_rows = np.ascontiguousarray(init_rows, dtype=np.int64)
    alphas = np.ascontiguousarray(alphas, dtype=np.float64)
    n, J = X.shape
    C = np.zeros((M, 16, J // M), dtype=np.float32)
    a = np.zeros(1, dtype=np.float32)
    offs = np.zeros(M, dtype=np.float32)
    ai = np.zeros(1, dtype=np.int32)
    _check(_lib.bolt_train_host(_np_ptr(X), n, J, J, M, iters, _np_ptr(init_rows), _np_ptr(Qt),
                                Qt.shape[0], J, metric_id(metric), _np_ptr(alphas), len(alphas),
                                _np_ptr(C), _np_ptr(a), _np_ptr(offs), _np_ptr(ai)))
    return C, float(a[0]), offs, int(ai[0])


def bolt_learn_quantizer_host(Qt, codes, centroids, metric, alphas=ALPHAS):
    """Quantiser for existing codebooks: (a, offsets [M], alpha index)."""
    Qt = np.ascontiguousarray(Qt, dtype=np.float32)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    C = np.ascontiguousarray(centroids, dtype=np.float32)
    alphas = np.ascontiguousarray(alphas, dtype=np.float64)
    M = C.shape[0]
    J = Qt.shape[1]
    a = np.zeros(1, dtype=np.float32)
    offs = np.zeros(M, dtype=np.float32)
    ai = np.zeros(1, dtype=np.int32)
    _check(_lib.bolt_learn_quantizer_host(_np_ptr(Qt), Qt.shape[0], J, J, _np_ptr(codes),
                                          codes.shape[0], _np_ptr(C), M, metric_id(metric),
                                          _np_ptr(alphas), len(alphas), _np_ptr(a), _np_ptr(offs),
                                          _np_ptr(ai)))
    return float(a[0]), offs, int(ai[0])


def bolt_learn_quantizer(Qt, codes, centroids, metric, alphas=ALPHAS, stream=None):
    """The quantiser search on the GPU: Qt fp32 [nq, J], codes uint8 [n, M/2]
    and centroids fp32 [M, 16, J/M] on the device.  Returns (a, offsets fp32
    [M] on the device, alpha index, losses fp64 [len(alphas)])."""
    _dev(Qt, torch.float32, "Qt")
    _dev(codes, torch.uint8, "codes")
    _dev(centroids, torch.float32, "centroids")
    nq, J, ldq = _rows(Qt, "Qt")
    M = centroids.shape[0]
    alphas = np.ascontiguousarray(alphas, dtype=np.float64)
    nws = int(_lib.bolt_learn_quantizer_ws_bytes(nq, M, len(alphas)))
    if nws == 0:
        raise BoltError(BOLT_ERR_UNSUPPORTED, "unsupported quantiser search size (nq = %d)" % nq)
    ws = torch.empty(nws, dtype=torch.uint8, device=Qt.device)
    offs = torch.empty(M, dtype=torch.float32, device=Qt.device)
    a = np.zeros(1, dtype=np.float32)
    ai = np.zeros(1, dtype=np.int32)
    losses = np.zeros(len(alphas), dtype=np.float64)
    _check(_lib.bolt_learn_quantizer(_ptr(Qt), nq, J, ldq, _ptr(codes), codes.shape[0], _ptr(centroids), M,
                                     metric_id(metric), _np_ptr(alphas), len(alphas), _np_ptr(a), _ptr(offs),
                                     _np_ptr(ai), _np_ptr(losses), _ptr(ws), nws, _stream(stream)))
    return float(a[0]), offs, int(ai[0]), losses


def debug_force_unfused_topk(on: bool):
    """Test hook: route bolt_scan_topk through scan + bolt_topk."""
    _check(_lib.bolt_debug_force_unfused_topk(1 if on else 0))


def debug_force_fused_kind(kind: int):
    """Test hook: many-query fused kernel, -1 automatic, 2 grouped, 3 matrix cores."""
    _check(_lib.bolt_debug_force_fused_kind(kind))


def debug_speculation(mode: int):
    """Test hook: speculative bounds, -1 automatic, 0 off, 1 on, 2 on and failing."""
    _check(_lib.bolt_debug_speculation(mode))


def debug_sparse_mfma(on: bool):
    """Test hook: matrix-core tiles with the sparse (True, default) or the dense instruction."""
    _check(_lib.bolt_debug_sparse_mfma(1 if on else 0))


def debug_force_scan_kernel(kind: int):
    """Test hook: -1 automatic, 0 generic, 1 few-query, 2 grouped, 3 matrix cores."""
    _check(_lib.bolt_debug_force_scan_kernel(kind))


# ------------------------------------------------------------------ batched databases

class BatchDb(ctypes.Structure):
    _fields_ = [("codes", _P), ("N", _I64), ("M", _I32), ("metric", _I32), ("luts", _P),
                ("Q", _I32), ("k", _I32), ("vals", _P), ("idx", _P)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("rows_per_tile", _I32), ("few_max_q", _I32), ("blocks_per_cu", _I32)]


for _name, _args, _res in [
    ("bolt_batch_ws_bytes", [ctypes.POINTER(BatchDb), _I32, ctypes.POINTER(BatchTuning)], _SZ),
    ("bolt_batch_plan_create", [ctypes.POINTER(BatchDb), _I32, ctypes.POINTER(BatchTuning), _P, _SZ, _P,
                                ctypes.POINTER(_P)], ctypes.c_int),
    ("bolt_batch_run", [_P, _P], ctypes.c_int),
    ("bolt_batch_plan_info", [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)],
     ctypes.c_int),
    ("bolt_batch_plan_destroy", [_P], ctypes.c_int),
    ("bolt_batch_graph_create", [_P, ctypes.POINTER(_P)], ctypes.c_int),
    ("bolt_batch_graph_launch", [_P, _P], ctypes.c_int),
    ("bolt_batch_graph_destroy", [_P], ctypes.c_int),
]:
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


class BatchPlan:
    """A planned batched scan + top-k over many databases (bolt_batch_*).

    dbs: list of dicts with keys codes (uint8 [N, M/2]), luts (uint8 [Q, M, 16]),
    metric ("l2"/"dot"), k; outputs vals/idx are allocated here unless given.
    The plan keeps references to every tensor it points at.
    """

    def __init__(self, dbs, tuning=None, stream=None):
        self.dbs = []
        arr = (BatchDb * max(len(dbs), 1))()
        dev = None
        for i, d in enumerate(dbs):
            codes, luts = d["codes"], d["luts"]
            _dev(codes, torch.uint8, "codes")
            _dev(luts, torch.uint8, "luts")
            dev = codes.device
            Q, M = luts.shape[0], luts.shape[1]
            k = int(d.get("k", 100))
            vals = d.get("vals")
            idx = d.get("idx")
            if vals is None:
                vals = torch.empty((Q, k), dtype=torch.uint16, device=codes.device)
            if idx is None:
                idx = torch.empty((Q, k), dtype=torch.int32, device=codes.device)
            self.dbs.append({"codes": codes, "luts": luts, "vals": vals, "idx": idx, "k": k, "M": M,
                             "metric": metric_id(d.get("metric", "l2"))})
            arr[i] = BatchDb(_ptr(codes), codes.shape[0], M, metric_id(d.get("metric", "l2")),
                             _ptr(luts), Q, k, _ptr(vals), _ptr(idx))
        self._arr = arr
        self.tuning = BatchTuning(*(tuning or (0, 0, 0)))
        n = len(dbs)
        nbytes = int(_lib.bolt_batch_ws_bytes(arr, n, ctypes.byref(self.tuning)))
        if nbytes == 0:
            raise BoltError(BOLT_ERR_INVALID, last_error())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev or "cuda")
        self._plan = _P()
        _check(_lib.bolt_batch_plan_create(arr, n, ctypes.byref(self.tuning), _ptr(self.ws), nbytes,
                                           _stream(stream), ctypes.byref(self._plan)))
        self._graph = None

    def info(self):
        t, q, g = _I64(), _I64(), _I32()
        _check(_lib.bolt_batch_plan_info(self._plan, ctypes.byref(t), ctypes.byref(q), ctypes.byref(g)))
        return {"tiles": t.value, "queries": q.value, "grid": g.value}

    def run(self, stream=None):
        _check(_lib.bolt_batch_run(self._plan, _stream(stream)))

    def capture(self):
        """Capture one run in a HIP graph (replayed by launch_graph)."""
        if self._graph is None:
            g = _P()
            _check(_lib.bolt_batch_graph_create(self._plan, ctypes.byref(g)))
            self._graph = g
        return self._graph

    def launch_graph(self, stream=None):
        _check(_lib.bolt_batch_graph_launch(self.capture(), _stream(stream)))

    def results(self):
        return [(d["vals"], d["idx"]) for d in self.dbs]

    def close(self):
        if getattr(self, "_graph", None) is not None:
            _lib.bolt_batch_graph_destroy(self._graph)
            self._graph = None
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.bolt_batch_plan_destroy(self._plan)
            self._plan = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ kernel timing

_lib.bolt_prof_enable.argtypes = [_I32]
_lib.bolt_prof_enable.restype = ctypes.c_int
_lib.bolt_prof_only.argtypes = [ctypes.c_char_p]
_lib.bolt_prof_only.restype = ctypes.c_int
_lib.bolt_prof_read.argtypes = [ctypes.c_char_p, _SZ, _I32]
_lib.bolt_prof_read.restype = ctypes.c_int


def prof_enable(on: bool = True, only: str = ""):
    """Record HIP events around every library kernel launch (on its stream),
    or only around those whose name starts with `only`."""
    _lib.bolt_prof_only(only.encode())
    _lib.bolt_prof_enable(1 if on else 0)


def prof_read(reset: bool = True):
    """{kernel name: (launches, total ms)} of the launches timed so far."""
    buf = ctypes.create_string_buffer(1 << 16)
    _lib.bolt_prof_read(buf, len(buf), 1 if reset else 0)
    out = {}
    for item in buf.value.decode().split(";"):
        if not item:
            continue
        name, rest = item.split("=")
        n, ms = rest.split(":")
        out[name] = (int(n), float(ms))
    return out
