"""Host logic of bench.py: the algorithmic byte and operation counts behind
the roofline figures, the per-step percentiles, the lookup of measured HBM
traffic in the committed profile summaries, and the refusal of more than
one GPU.  No GPU is used."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N, M, K_MAX = 1 << 22, 85, 101


def test_algorithmic_bytes_headline():
    # the input read once (8 N), the float32 plane written once (4 M N) and
    # the template spectra read once (8 M L): 1461.0 MB at L = 2048
    assert bench.algorithmic_bytes(N, M, 2048) == 8 * N + 4 * M * N + 8 * M * 2048
    assert abs(bench.algorithmic_bytes(N, M, 2048) / 1e6 - 1461.0) < 0.05


@pytest.mark.parametrize("L,expect", [(1024, 2.343e10), (2048, 2.419e10), (4096, 2.546e10), (8192, 2.701e10)])
def test_nominal_operations(L, expect):
    # 5 L log2 L per transform (one forward per segment, one inverse per
    # segment and template), 6 per complex product, 3 per power, with the
    # minimal overlap V = L - (K_max - 1)
    got = bench.nominal_flops(N, M, L, K_MAX)
    assert abs(got / expect - 1) < 1e-3, (L, got)
    v = L - (K_MAX - 1)
    s = math.ceil(N / v)
    assert got == s * (M * (5 * L * math.log2(L) + 6 * L + 3 * v) + 5 * L * math.log2(L))


def test_percentiles_pick_order_statistics():
    xs = [float(v) for v in range(100, 0, -1)]      # 100 .. 1, unsorted input
    p = bench.percentiles(xs)
    assert p == {"p10": 11.0, "median": 51.0, "p90": 90.0}
    assert bench.percentiles([3.0]) == {"p10": 3.0, "median": 3.0, "p90": 3.0}


def test_measured_traffic_tracks_kernel_source(monkeypatch, tmp_path):
    # a summary carrying the current source hash is used; any other hash,
    # or no summary for the segment length, gives null
    f = tmp_path / "traffic.md"
    f.write_text(f"kernel_source_sha: {bench.kernel_source_hash()}\n\ntraffic_bytes_per_call: 1.488765e+09\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {(2048, 56): str(f)})
    assert bench.measured_traffic(2048, 56) == 1.488765e9
    assert bench.measured_traffic(2048, 0) is None          # another split
    assert bench.measured_traffic(1024, 56) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(2048, 56) is None


def test_direct_mfma_operations():
    # blocks of 8 in order of tap count; per 16 outputs a block issues
    # 3 x ceil(K_block / 16) products of 16 x 16 x 32 (2 x 8192 operations)
    lens = [17, 19, 33, 33, 40, 41, 48, 49, 80, 3]
    n = 100                                                # 7 tiles of 16
    per = 3 * 2 * 16 * 16 * 32
    # sorted: 3 17 19 33 33 40 41 48 | 49 80 -> blocks of 48 and 80 taps
    assert bench.direct_mfma_flops(n, lens, 10) == 7 * per * (3 + 5)
    assert bench.direct_mfma_flops(n, lens, 8) == 7 * per * 3
    assert bench.direct_mfma_flops(n, lens, 0) == 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_measured_counters_track_kernel_source_and_split(monkeypatch, tmp_path):
    f = tmp_path / "sq.md"
    f.write_text(f"kernel_source_sha: {bench.kernel_source_hash()}\n\n"
                 "valu_issue_per_cu_cycle[direct=0]: 0.967\nmfma_busy[direct=40]: 0.64\n"
                 "valu_issue_per_cu_cycle[direct=40]: 0.929\n")
    monkeypatch.setattr(bench, "SQ_COUNTER_FILES", {2048: str(f)})
    assert bench.measured_valu_issue(2048, 0) == 0.967
    assert bench.measured_valu_issue(2048, 40) == 0.929
    assert bench.measured_mfma_busy(2048, 40) == 0.64
    assert bench.measured_valu_issue(2048, 56) is None       # no line for that split
    assert bench.measured_mfma_busy(2048, 0) is None
    assert bench.measured_valu_issue(1024, 0) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_valu_issue(2048, 0) is None


def test_unpacked_fp32_peak_from_unit_counts():
    # one wave64 FMA instruction per CU per cycle: 256 CUs x 64 lanes x 2 x 2.4 GHz
    assert abs(256 * 64 * 2 * 2.4e9 / 1e12 - bench.FP32_UNPACKED_PEAK_TFLOPS) < 0.1
    assert abs(2 * bench.FP32_UNPACKED_PEAK_TFLOPS - bench.FP32_VECTOR_PEAK_TFLOPS) < 0.2


def test_kernel_hash_ignores_comments_only():
    # comments, trailing blanks and empty lines do not count; code does
    a = "int f(int x) {  // doubles\n    return 2 * x;   \n}\n\n/* note */\n"
    b = "// header\nint f(int x) {\n    return 2 * x;\n}\n"
    c = "int f(int x) {\n    return 3 * x;\n}\n"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)
