"""Bolt (Blalock & Guttag, KDD 2017) hot path on MI355X (gfx950).

Encode vectors to 4-bit codes, build uint8 lookup tables for queries, scan
the codes and select the top k -- all in hand-written HIP kernels behind the
C ABI of include/bolt.h.  ``paper_1706_10283_amd.bolt`` is the binding; its
names are re-exported here on first use (importing them without a built
libbolt.so raises ImportError: there is no CPU fallback).
"""
import importlib


def __getattr__(name):
    if name.startswith("__") or name in ("build",):
        raise AttributeError(name)
    mod = importlib.import_module(__name__ + ".bolt")
    return getattr(mod, name)
