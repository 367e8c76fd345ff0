"""Host-side bookkeeping of bench.py: the measured HBM traffic of the dominant
kernel is reported only for the code it was measured on (comments and blank
lines do not count as code), and only for its workload."""
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@pytest.fixture()
def bench(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    import bench as b
    return b


def _copy_sources(bench, dst):
    for f in bench.TRAFFIC_SOURCES["scan_topk_mfma"]:
        src = os.path.normpath(os.path.join(ROOT, "paper_1706_10283_amd", "csrc", f))
        out = os.path.normpath(os.path.join(dst, "paper_1706_10283_amd", "csrc", f))
        os.makedirs(os.path.dirname(out), exist_ok=True)
        shutil.copy(src, out)


def test_code_hash_ignores_comments_not_code(bench, tmp_path, monkeypatch):
    _copy_sources(bench, str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.sources_sha256("scan_topk_mfma")
    fused = tmp_path / "paper_1706_10283_amd" / "csrc" / "fused.hip"
    text = fused.read_text()
    fused.write_text("// a new comment line\n\n" + text.replace("\n", "\n\n", 3) + "/* and a block */\n")
    assert bench.sources_sha256("scan_topk_mfma") == h0
    fused.write_text(text.replace("constexpr int kRowsPerBlock = 16384;", "constexpr int kRowsPerBlock = 8192;"))
    assert bench.sources_sha256("scan_topk_mfma") != h0
    build = tmp_path / "paper_1706_10283_amd" / "build.py"
    fused.write_text(text)
    build.write_text(build.read_text().replace('"-munsafe-fp-atomics"', '"-munsafe-fp-atomics", "-g"'))
    assert bench.sources_sha256("scan_topk_mfma") != h0


def test_traffic_only_for_its_workload_and_code(bench, monkeypatch):
    t = bench.TRAFFIC["scan_topk_mfma"]
    wl = dict(t["workload"])
    nbytes = bench.traffic_bytes("scan_topk_mfma", wl)
    assert nbytes == pytest.approx(1024.0 * (bench.FETCH_FACTOR * t["fetch_kib"]
                                             + bench.WRITE_FACTOR * t["write_kib"]))
    assert bench.traffic_bytes("scan_topk_mfma", dict(wl, Q=wl["Q"] + 1)) is None
    monkeypatch.setitem(bench.TRAFFIC["scan_topk_mfma"], "sources_sha256", "0" * 64)
    assert bench.traffic_bytes("scan_topk_mfma", wl) is None
