"""Host check of the C ABI's argument checks and batch geometry under the
sanitizers: tests/abi_args_check.cpp includes the library's own check code
(paper_1805_12280_amd/csrc/fdas_args.h, plain C++) and is built with g++
-fsanitize=address,undefined, so an out-of-bounds access, a use of freed
memory, signed overflow or a misaligned access on any NULL, size, range or
alignment path, or in the batch shape of random batches, fails it."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_abi_argument_checks_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "abi_args_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror", "-pthread",
               "-I", os.path.join(ROOT, "include"),
               "-I", os.path.join(ROOT, "paper_1805_12280_amd", "csrc"),
               os.path.join(ROOT, "tests", "abi_args_check.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ)
        # a preloaded library ahead of the ASan runtime is not an error of the code under test
        env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1"
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        print(r.stdout)
        assert r.returncode == 0 and r.stdout.rstrip().endswith("ok"), (r.stdout[-2000:], r.stderr[-3000:])
