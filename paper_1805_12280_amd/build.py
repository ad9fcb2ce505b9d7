"""Build libfdas.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfdas.so")
SOURCES = ["fdas_kernels.hip", "fdas_batched.hip", "fdas_mixed.hip", "fdas_direct.hip", "fdas_abi.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions stay off in every device compile.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc_cmd(out: str) -> list:
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
            + DEVICE_FLAGS
            + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out])


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the device feature flag; that warning is expected
    noise = [ln for ln in (res.stderr or "").splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "warning generated" not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + (res.stderr or ""))
    if verbose and noise:
        print("\n".join(noise), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
