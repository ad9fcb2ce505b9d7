"""Host check of the 16-bit inverse transform's index maps (mixed_fft.h):
the three matrix-core passes emulated lane by lane in double precision
equal the inverse DFT by definition, the maps are bijections into their
LDS buffers, and the kernel's LDS accesses are free of bank conflicts.
Builds tests/mixed_maps_check.cpp with hipcc (host code only)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_mixed_index_maps():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "mixed_maps_check")
        cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-I", os.path.join(ROOT, "paper_1805_12280_amd", "csrc"),
               os.path.join(ROOT, "tests", "mixed_maps_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout[-2000:]
