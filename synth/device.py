"""Device-side generation of the mixture inputs (see synth/gmm.hip)."""
import ctypes
import os

import torch

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError("synth/libsynth.so is not built (python -m synth.build)")
        _lib = ctypes.CDLL(_LIB)
        _lib.synth_gmm_rows.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p]
        _lib.synth_gmm_rows.restype = ctypes.c_int
    return _lib


def gmm_rows(mix_seed, draw_seed, row0, nrows, J, out=None, device="cuda"):
    """fp32 [nrows, J] tensor on the GPU, bit-identical to synth.gmm_rows."""
    if out is None:
        out = torch.empty((nrows, J), dtype=torch.float32, device=device)
    st = _load().synth_gmm_rows(mix_seed, draw_seed, row0, nrows, J, out.stride(0) if nrows else J,
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise RuntimeError("synth_gmm_rows failed (%d)" % st)
    return out
