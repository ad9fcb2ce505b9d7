"""The C ABI on the GPU: status codes for bad arguments (no crash, nothing
launched), plan info, the segment transform and the template spectra against
the oracle's definitions."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1805_12280_amd import datagen

pytestmark = pytest.mark.gpu


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


def _create(lib, taps, tap_len, m, k, n, L, flags=0):
    h = ctypes.c_void_p()
    tp = ctypes.c_void_p(taps.ctypes.data) if taps is not None else None
    lp = ctypes.c_void_p(tap_len.ctypes.data) if tap_len is not None else None
    rc = lib.fdas_plan_create(ctypes.byref(h), tp, lp, m, k, n, L, flags, None)
    return rc, h


def test_plan_create_errors(env):
    torch, fdas, lib = env
    _, bank = datagen.random_case(1, 4, 3, 33)
    taps, tl = bank.taps, bank.tap_len
    assert lib.fdas_plan_create(None, ctypes.c_void_p(taps.ctypes.data), None, 3, 33, 100, 1024, 0, None) == fdas.FDAS_EINVAL
    cases = [
        ((None, tl, 3, 33, 100, 1024), fdas.FDAS_EINVAL),
        ((taps, tl, 0, 33, 100, 1024), fdas.FDAS_EINVAL),
        ((taps, tl, 3, 0, 100, 1024), fdas.FDAS_EINVAL),
        ((taps, tl, 3, 33, 0, 1024), fdas.FDAS_EINVAL),
        ((taps, tl, 3, 33, 100, 512), fdas.FDAS_EINVAL),
        ((taps, tl, 3, 33, 100, 3000), fdas.FDAS_EINVAL),
        ((np.zeros((3, 600), np.complex64), None, 3, 600, 100, 1024), fdas.FDAS_EINVAL),
        ((taps, np.array([1, 34, 2], np.int32), 3, 33, 100, 1024), fdas.FDAS_EINVAL),
        ((taps, np.array([1, -1, 2], np.int32), 3, 33, 100, 1024), fdas.FDAS_EINVAL),
    ]
    for args, want in cases:
        rc, h = _create(lib, *args)
        assert rc == want, (args[2:], rc)
        assert not h.value
        assert lib.fdas_last_error().decode()
    rc, h = _create(lib, taps, tl, 3, 33, 100, 1024, flags=1 << 5)
    assert rc == fdas.FDAS_EUNSUPPORTED
    rc, h = _create(lib, taps, tl, 3, 33, 100, 0)   # default L = 2048
    assert rc == 0
    info = fdas.PlanInfo()
    assert lib.fdas_plan_info(h, ctypes.byref(info)) == 0
    assert info.seg_fft == 2048 and info.valid_per_seg == 2048 - 32 and info.k_max == 33
    assert info.num_segments == 1 and info.num_templates == 3 and info.threads_per_fft == 128
    assert lib.fdas_variant_name(info.variant).decode() != "unknown"
    lib.fdas_plan_destroy(h)
    lib.fdas_plan_destroy(None)
    with pytest.raises(fdas.FdasError):
        fdas.Plan(taps, tl, input_len=100, seg_fft=1024, precision="bf16")


def test_call_errors(env):
    torch, fdas, lib = env
    _, bank = datagen.random_case(2, 4, 2, 9)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1000, seg_fft=1024)
    x = torch.zeros(1000, dtype=torch.complex64, device="cuda")
    out = torch.zeros((2, 1000), dtype=torch.float32, device="cuda")
    xp, op = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())
    for fn in (lib.fdas_convolve, lib.fdas_tdfir):
        assert fn(None, xp, 10, op, 10, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, None, 10, op, 10, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, xp, 10, None, 10, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, xp, 0, op, 10, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, xp, 1001, op, 1001, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, xp, 100, op, 99, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, ctypes.c_void_p(x.data_ptr() + 4), 10, op, 10, None) == fdas.FDAS_EINVAL
        assert fn(plan._h, xp, 10, ctypes.c_void_p(out.data_ptr() + 2), 10, None) == fdas.FDAS_EINVAL
    seg = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
    sp = ctypes.c_void_p(seg.data_ptr())
    assert lib.fdas_segment_fft(plan._h, sp, sp, 2, -1, None) == fdas.FDAS_EINVAL   # overlap
    assert lib.fdas_segment_fft(plan._h, sp, op, 0, -1, None) == fdas.FDAS_EINVAL
    assert lib.fdas_segment_fft(plan._h, sp, op, 1, 2, None) == fdas.FDAS_EINVAL
    assert lib.fdas_plan_template_spectra(None, None) == fdas.FDAS_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0      # nothing was launched


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_segment_fft_against_dft(env, L):
    torch, fdas, _ = env
    _, bank = datagen.random_case(3, 4, 1, 9)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=L, seg_fft=L)
    rng = np.random.default_rng(L)
    xs = (rng.standard_normal((3, L)) + 1j * rng.standard_normal((3, L))).astype(np.complex64)
    xd = torch.from_numpy(xs).cuda()
    fwd = plan.segment_fft(xd, -1).cpu().numpy()
    inv = plan.segment_fft(xd, +1).cpu().numpy()
    for r in range(3):
        ref_f = oracle.dft(xs[r].astype(np.complex128), -1)
        ref_i = oracle.dft(xs[r].astype(np.complex128), +1)
        assert np.max(np.abs(fwd[r] - ref_f)) <= 2e-6 * np.max(np.abs(ref_f))
        assert np.max(np.abs(inv[r] - ref_i)) <= 2e-6 * np.max(np.abs(ref_i))
    # round trip returns L * x
    back = plan.segment_fft(plan.segment_fft(xd, -1), +1).cpu().numpy() / L
    assert np.max(np.abs(back - xs)) <= 2e-6 * np.max(np.abs(xs))


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_template_spectra_against_definition(env, L):
    torch, fdas, _ = env
    bank = datagen.make_bank(datagen.Z_SKA)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1 << 16, seg_fft=L)
    H = plan.template_spectra()
    for t in (0, 17, 42, 84):
        ref = oracle.template_spectrum(bank.taps[t, : bank.tap_len[t]], L)
        # float64 arithmetic rounded once to float32
        assert np.max(np.abs(H[t] - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_workgroups_per_cu_knob(env, precision):
    """The persistent grid's size changes which workgroup runs an item, not
    what it computes: planes and batched candidates are bitwise identical
    for every cap, and the cap is reported and validated."""
    torch, fdas, lib = env
    x, bank = datagen.random_case(61, 50011, 5, 40)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=x.shape[0], seg_fft=2048, precision=precision)
    xd = torch.from_numpy(x).cuda()
    if precision != "fp32":
        xd = torch.view_as_real(xd).to(torch.float16).contiguous()
    xs = [xd, xd[:7777].contiguous()]
    full = plan.info.wg_per_cu_max
    assert full >= 1 and plan.info.wg_per_cu == 0
    ref_plane = plan.convolve(xd)
    ref_cands = plan.convolve_batched(xs, topk=16)
    for cap in (1, max(1, full // 2), full + 3):
        plan.set_workgroups_per_cu(cap)
        assert plan.info.wg_per_cu == cap
        assert torch.equal(plan.convolve(xd), ref_plane), cap
        assert torch.equal(plan.convolve_batched(xs, topk=16), ref_cands), cap
    plan.set_workgroups_per_cu(0)
    assert lib.fdas_plan_set_workgroups_per_cu(plan._h, -1) == fdas.FDAS_EINVAL
    assert lib.fdas_plan_set_workgroups_per_cu(None, 1) == fdas.FDAS_EINVAL
    plan.close()
