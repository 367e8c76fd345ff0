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
    # another source file in the build list is not a change of this kernel's code
    build.write_text(build.read_text().replace('"-munsafe-fp-atomics", "-g"', '"-munsafe-fp-atomics"')
                     .replace('"encode.hip",', '"encode.hip", "other.hip",'))
    assert bench.sources_sha256("scan_topk_mfma") == h0


def test_traffic_only_for_its_workload_and_code(bench, monkeypatch):
    t = bench.TRAFFIC["scan_topk_mfma"]
    monkeypatch.setitem(t, "sources_sha256", bench.sources_sha256("scan_topk_mfma"))
    wl = dict(t["workload"])
    nbytes = bench.traffic_bytes("scan_topk_mfma", wl)
    assert nbytes == pytest.approx(1024.0 * (bench.FETCH_FACTOR * t["fetch_kib"]
                                             + bench.WRITE_FACTOR * t["write_kib"]))
    assert bench.traffic_bytes("scan_topk_mfma", dict(wl, Q=wl["Q"] + 1)) is None
    monkeypatch.setitem(bench.TRAFFIC["scan_topk_mfma"], "sources_sha256", "0" * 64)
    assert bench.traffic_bytes("scan_topk_mfma", wl) is None


def test_roofline_counts_the_methods_work(bench):
    """frac is one lookup and one add per (query, vector, subspace) against the
    dense int8 peak; the matrix-core slots the one-hot form occupies are
    reported separately and cap the method's fraction at 1 / slots."""
    Q, N, M, ms = 1000, 1_000_000, 32, 0.4
    r = bench.scan_roofline("scan_topk_mfma", Q, N, M, ms)
    method = 2.0 * Q * N * M / (ms * 1e-3)
    assert r["frac"] == pytest.approx(method / 5.0e15, abs=1e-4)
    assert r["achieved"] == pytest.approx(method / 1e12, rel=1e-3)
    assert r["matrix_slots_per_lookup"] == pytest.approx(9.0)
    assert r["matrix_ceiling_frac"] == pytest.approx(9.0 * r["frac"], rel=1e-3)
    assert r["bound"] == "mfma" and r["peak"] == 5000.0
    g = bench.scan_roofline("scan_topk_grouped", Q, N, M, ms)
    assert g["frac"] == r["frac"] and "matrix_ceiling_frac" not in g


def test_matrix_slots_count_the_instruction_mix():
    """Per pass of 32 rows: two dense 32x32x32 steps for subspaces 0-3 and one
    sparse 32x32x64 step per further four subspaces, each 32 cycles; the
    dense form would take M / 2 steps of the same length."""
    import bench as b
    for M in (8, 16, 32, 64):
        steps = 2 + (M - 4) // 4
        assert b.matrix_slots_per_lookup(M) == pytest.approx(16.0 * steps / (M / 2))


def test_cpu_baseline_threads_give_the_oracle_result(bench):
    """The all-thread run of the oracle splits rows and queries among threads
    and must compute exactly what the one-thread run computes."""
    import numpy as np
    import oracle
    import synth
    X = synth.gmm_rows(5, 6, 0, 2000, 32)
    Qv = synth.gmm_rows(5, 7, 0, 37, 32)
    C, _ = oracle.kmeans(X, 8, 2, synth.permutation_prefix(8, 2000, 16))
    quant = {m: oracle.learn_quantizer(Qv[:10], oracle.encode(X, C, 8), C, m)[:2] for m in ("l2", "dot")}
    c1, r1 = bench._oracle_step(oracle, X, C, 8, quant, Qv, 10, 1)
    c4, r4 = bench._oracle_step(oracle, X, C, 8, quant, Qv, 10, 4)
    assert np.array_equal(c1, c4)
    for m in ("l2", "dot"):
        assert np.array_equal(r1[m][0], r4[m][0]) and np.array_equal(r1[m][1], r4[m][1])
    model, threads, ncpu = bench.host_cpu()
    assert isinstance(model, str) and 1 <= threads <= ncpu
