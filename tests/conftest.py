import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _ensure_built():
    """Build the HIP library, device generator and oracle if they are missing
    (the host-side tests load them; building needs no GPU)."""
    libs = [os.path.join(ROOT, "paper_1706_10283_amd", "libbolt.so"),
            os.path.join(ROOT, "synth", "libsynth.so")]
    if not all(os.path.exists(p) for p in libs):
        import __graft_entry__
        __graft_entry__.build()


def pytest_configure(config):
    _ensure_built()
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
