"""fdas_convolve_batched_static (the entry point that allocates nothing)
against fdas_convolve_batched on the same plan and arrays, through the C
ABI: the candidates are computed by the same kernels on the same grid, so
they must be identical, bit for bit.  Two calls in a row, the second with a
smaller input, for a float32 plan and an FP16 plan; an oversized batch is
refused without touching the output."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1805_12280_amd import datagen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import os
    import torch
    from paper_1805_12280_amd import fdas
    assert torch.cuda.is_available()
    if not os.path.exists(fdas.LIB_PATH):
        from paper_1805_12280_amd import build
        build.build()
    return torch, fdas, fdas.load_library()


def call_static(torch, fdas, lib, plan, xs, topk):
    out = torch.full((len(xs), topk, 3), -9, dtype=torch.int32, device="cuda")
    ptrs = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
    ns = (ctypes.c_int64 * len(xs))(*[int(x.shape[0]) for x in xs])
    rc = lib.fdas_convolve_batched_static(plan._h, ptrs, ns, len(xs), topk, ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_static_workspace_equals_caller_workspace(env, prec):
    torch, fdas, lib = env
    x_all, bank = datagen.random_case(77, 600000, 13, 61)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=600000, seg_fft=2048 if prec != "fp32" else 1024,
                     precision=prec)
    dev = torch.from_numpy(x_all).cuda()
    if prec != "fp32":
        dev = torch.view_as_real(dev).to(plan.input_dtype()).contiguous()
    calls = [[dev[:600000], dev[1000:250000], dev[5:70000]],        # first call
             [dev[:90000], dev[333:4000]]]                            # then a smaller input
    for k, xs in enumerate(calls):
        xs = [x.contiguous() for x in xs]
        _say(f"[static ws] {prec} call {k}: lengths {[int(x.shape[0]) for x in xs]}")
        want = plan.convolve_batched(xs, topk=16)
        rc, got = call_static(torch, fdas, lib, plan, xs, 16)
        torch.cuda.synchronize()
        assert rc == fdas.FDAS_OK, lib.fdas_last_error()
        assert torch.equal(got, want), k
        t, b, p = fdas.split_candidates(got)
        assert int(t.min()) >= 0 and float(p.min()) >= 0.0
    plan.close()


def test_static_workspace_refuses_oversized_batch(env):
    torch, fdas, lib = env
    _, bank = datagen.random_case(78, 4, 5, 33)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1 << 22, seg_fft=2048, precision="fp16")
    big = torch.zeros(((1 << 22), 2), dtype=torch.float16, device="cuda")
    need = plan.batched_workspace_bytes([1 << 22, 1 << 22], 16)
    assert need > fdas.STATIC_WORKSPACE_BYTES
    rc, out = call_static(torch, fdas, lib, plan, [big, big], 16)
    torch.cuda.synchronize()
    assert rc == fdas.FDAS_EINVAL
    assert b"static workspace" in lib.fdas_last_error()
    assert bool((out == -9).all())              # nothing was enqueued
    plan.close()
