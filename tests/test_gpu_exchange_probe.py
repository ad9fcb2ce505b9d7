"""The exchange probe (tests/exchange_probe.hip): one radix-pass exchange of
a 1024-point segment transform held by a wave, through LDS as the kernels
do it and with the gfx950 cross-lane swaps.  Both must move the data the
same way (checked against a numpy emulation of the exchange); their times
and instruction counts are what the design's choice of LDS rests on."""
import ctypes
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def probe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import probe_build
    if not os.path.exists(probe_build.LIB):
        probe_build.build()
    lib = ctypes.CDLL(probe_build.LIB)
    lib.exchange_probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p]
    lib.exchange_probe.restype = ctypes.c_int
    return torch, lib


def run(torch, lib, method, x, reps):
    """x: CUDA complex64 [waves, 16, 64] (register r, lane); returns the
    output of `reps` exchanges."""
    out = torch.empty_like(x)
    rc = lib.exchange_probe(method, x.data_ptr(), out.data_ptr(), x.shape[0], reps,
                            torch.cuda.current_stream().cuda_stream)
    assert rc == 0, rc
    return out


def emulate(v, reps):
    """numpy: lane (k1, p) takes into v[4 pp + g] what lane (k1, pp) held in
    v[4 p + g]; then 1 is added to v[0] (real part)."""
    w = v.copy()
    r = np.arange(16)
    lane = np.arange(64)
    k1, p = lane % 16, lane // 16
    for _ in range(reps):
        new = np.empty_like(w)
        for o in r:                               # output register o = 4 pp + g
            pp, g = o // 4, o % 4
            new[:, o, :] = w[:, 4 * p + g, k1 + 16 * pp]
        new[:, 0, :] += 1.0
        w = new
    return w


@pytest.mark.parametrize("reps", [1, 2, 5])
def test_both_methods_move_the_data_alike(probe, reps):
    torch, lib = probe
    rng = np.random.Generator(np.random.PCG64(7))
    v = (rng.standard_normal((40, 16, 64)) + 1j * rng.standard_normal((40, 16, 64))).astype(np.complex64)
    want = emulate(v, reps)
    x = torch.from_numpy(v).cuda()
    for method in (0, 1):
        got = run(torch, lib, method, x, reps).cpu().numpy()
        assert np.array_equal(got, want), (method, reps)


def test_exchange_times(probe):
    """Many waves, many exchanges: both methods give the same bits; prints
    the time per exchange and wave."""
    torch, lib = probe
    waves, reps = 16384, 512
    rng = np.random.Generator(np.random.PCG64(8))
    v = (rng.standard_normal((waves, 16, 64)) + 1j * rng.standard_normal((waves, 16, 64))).astype(np.complex64)
    x = torch.from_numpy(v).cuda()
    outs, ms = {}, {}
    for method in (0, 1):
        for _ in range(3):
            run(torch, lib, method, x, reps)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            outs[method] = run(torch, lib, method, x, reps)
        b.record()
        torch.cuda.synchronize()
        ms[method] = a.elapsed_time(b) / 5
    assert torch.equal(outs[0], outs[1])
    for method, name in ((0, "LDS"), (1, "cross-lane swaps")):
        _say(f"[exchange] {name}: {ms[method]:.3f} ms for {waves} waves x {reps} exchanges, "
             f"{ms[method] * 1e6 / (waves * reps) * 256:.1f} ns per exchange per CU-slot of 256 CUs")
