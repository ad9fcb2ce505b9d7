"""Host check of the float32 segment transform (seg_fft.h) at every segment
length, 1024 to 8192: the passes run on the CPU work-item by work-item in
the kernels' order equal the DFT by definition (forward) and the inverse DFT
of a permuted-order spectrum (inverse), and the index maps are bijections
inside their LDS buffers.  Builds tests/seg_fft_check.cpp with hipcc (host
code only)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_segment_transform_maps():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "seg_fft_check")
        cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-I", os.path.join(ROOT, "paper_1805_12280_amd", "csrc"),
               os.path.join(ROOT, "tests", "seg_fft_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
        print(r.stdout)
        assert r.returncode == 0 and r.stdout.rstrip().endswith("ok"), r.stdout[-3000:]
