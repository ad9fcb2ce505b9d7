"""GPU parity of the direct-convolution route of a float32 plan (Eq. (1) on
the matrix cores, binary16 high/low operands, three products, float32
accumulation) against the FP64 oracle, at every split of the bank between
direct convolution and overlap-save.

Bar: the float32 one, max |P_gpu - P_ref| / max P_ref <= 1e-4, no write past
n, and a template's row is bitwise the same whichever split runs it by the
same route."""
import sys

import numpy as np
import pytest

import oracle
from fdas_check import FP32_TOL, PlaneStats
from paper_1805_12280_amd import datagen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def fdas(torch_cuda):
    import os
    from paper_1805_12280_amd import fdas as f
    if not os.path.exists(f.LIB_PATH):
        from paper_1805_12280_amd import build
        build.build()
    f.load_library()
    return f


def plane(torch, plan, x_np, n=None, ld=None):
    n = x_np.shape[0] if n is None else n
    x = torch.from_numpy(np.ascontiguousarray(x_np[:n])).cuda()
    out = torch.full((plan.num_templates, n if ld is None else ld), -7.0, dtype=torch.float32, device="cuda")
    plan.convolve(x, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def against_oracle(P, x_np, bank, n):
    st = PlaneStats()
    m = bank.num_templates
    for r0 in range(0, m, 16):
        rows = list(range(r0, min(m, r0 + 16)))
        st.add(rows, P[rows, :n], oracle.power(x_np[:n], bank.taps, bank.tap_len, rows=rows))
    return st


def ragged_bank(seed, m, k_hi):
    """m templates with tap counts spread over 1..k_hi (every 16-tap step
    count of the direct kernel, and some past its 96-tap limit when k_hi is
    larger), unit-energy complex Gaussian taps."""
    _, bank = datagen.random_case(seed, 8, m, k_hi)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    tl = np.sort(rng.integers(1, k_hi + 1, size=m)).astype(np.int32)
    tl[-1] = k_hi
    rng.shuffle(tl)                     # plane rows not in tap order
    taps = np.zeros_like(bank.taps)
    for t in range(m):
        v = rng.standard_normal(2 * int(tl[t]))
        taps[t, :tl[t]] = (v[0::2] + 1j * v[1::2]) / np.sqrt(2.0 * tl[t])
    return datagen.Bank(np.zeros(m), taps, tl)


@pytest.mark.parametrize("split", [0, 8, 16, 24, "all"])
def test_every_split_against_oracle(torch_cuda, fdas, split):
    """29 templates of 1..120 taps (blocks of 1 to 6 steps of 16 taps, and
    templates past 96 taps that stay on overlap-save), 70001 points (137
    waves of 512 outputs and a ragged tail), n < input_len and ld > n."""
    bank = ragged_bank(11, 29, 120)
    n = 70001
    x, _ = datagen.random_case(12, n, 1, 1)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n + 100, seg_fft=1024)
    plan.set_direct_templates(bank.num_templates if split == "all" else split)
    md = plan.info.direct_templates
    _say(f"[direct] split={split} -> {md} direct of {bank.num_templates}")
    if split == "all":
        # the leading blocks of 8 (in order of tap count) whose longest
        # template has at most 96 taps
        lens = np.sort(bank.tap_len)
        nb = 0
        while 8 * nb < len(lens) and lens[8 * nb:8 * nb + 8].max() <= 96:
            nb += 1
        assert md == min(len(lens), 8 * nb) and 0 < md < bank.num_templates
    else:
        assert md == split
    P = plane(torch_cuda, plan, x, ld=n + 37)
    assert np.all(P[:, n:] == -7.0), "wrote past n"
    st = against_oracle(P, x, bank, n)
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    ok, bad = st.topk_agree()
    assert ok, bad
    plan.close()


def test_every_tap_count_against_oracle(torch_cuda, fdas):
    """One template of each tap count 1..100 (every padding of every step
    count 1..6 on the direct route; 97..100 stay on overlap-save), all that
    can go direct run directly, 20011 points."""
    m = 100
    _, bank = datagen.random_case(31, 8, m, m)
    rng = np.random.Generator(np.random.PCG64(32))
    tl = np.arange(1, m + 1, dtype=np.int32)
    rng.shuffle(tl)
    taps = np.zeros_like(bank.taps)
    for t in range(m):
        v = rng.standard_normal(2 * int(tl[t]))
        taps[t, :tl[t]] = (v[0::2] + 1j * v[1::2]) / np.sqrt(2.0 * tl[t])
    bank = datagen.Bank(np.zeros(m), taps, tl)
    n = 20011
    x, _ = datagen.random_case(33, n, 1, 1)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=1024)
    plan.set_direct_templates(m)
    assert plan.info.direct_templates == 96
    P = plane(torch_cuda, plan, x)
    st = against_oracle(P, x, bank, n)
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    # each row on its own peak as well: short templates have small powers
    ref = oracle.power(x, bank.taps, bank.tap_len)
    for t in range(m):
        assert np.abs(P[t] - ref[t]).max() <= FP32_TOL * ref[t].max(), (t, int(tl[t]))
    plan.close()


def test_rows_are_bitwise_stable_across_splits(torch_cuda, fdas):
    """A template's row depends only on the route that computes it: the first
    block is the same with 8 or 16 direct templates, and every template on
    overlap-save is the same with 0, 8 or 16 direct ones."""
    bank = ragged_bank(13, 24, 90)
    n = 20000
    x, _ = datagen.random_case(14, n, 1, 1)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=2048)
    order = np.argsort(bank.tap_len, kind="stable")
    P = {}
    for m in (0, 8, 16):
        plan.set_direct_templates(m)
        P[m] = plane(torch_cuda, plan, x)
    first, second, rest = order[:8], order[8:16], order[16:]
    # the plan's own order of equal tap counts may differ from this one; the
    # blocks are compared as sets of rows, each row by itself
    assert np.array_equal(P[8][first], P[16][first])
    assert np.array_equal(P[0][second], P[8][second])
    assert np.array_equal(P[0][rest], P[16][rest]) and np.array_equal(P[0][rest], P[8][rest])
    # and the two routes agree to the float32 bar
    assert np.max(np.abs(P[16] - P[0])) <= FP32_TOL * P[0].max()
    plan.close()


@pytest.mark.parametrize("n", [1, 15, 16, 17, 511, 512, 513, 2047, 2049])
def test_short_inputs(torch_cuda, fdas, n):
    """Inputs shorter than, equal to and just past one tile (16) and one
    wave's 512 outputs, all templates direct."""
    bank = ragged_bank(15, 11, 96)
    x, _ = datagen.random_case(16 + n, n, 1, 1)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=4096, seg_fft=1024)
    plan.set_direct_templates(bank.num_templates)
    assert plan.info.direct_templates == 11
    P = plane(torch_cuda, plan, x, ld=n + 3)
    assert np.all(P[:, n:] == -7.0)
    st = against_oracle(P, x, bank, n)
    assert st.norm_err <= FP32_TOL, (n, st.summary())
    plan.close()


def test_zero_template_and_impulse(torch_cuda, fdas):
    """A template with no taps gives an all-zero row, and a unit impulse
    gives each template's tap powers, on the direct route."""
    bank = ragged_bank(17, 8, 64)
    tl = bank.tap_len.copy()
    tl[3] = 0
    bank = datagen.Bank(bank.z, bank.taps, tl)
    n, j0 = 6000, 2222
    x = np.zeros(n, np.complex64)
    x[j0] = 1.0
    plan = fdas.Plan(bank.taps, tl, input_len=n, seg_fft=1024)
    plan.set_direct_templates(8)
    assert plan.info.direct_templates == 8
    P = plane(torch_cuda, plan, x)
    assert np.all(P[3] == 0.0)
    for t in range(8):
        k = int(tl[t])
        ref = np.zeros(n)
        ref[j0:j0 + k] = np.abs(bank.taps[t, :k].astype(np.complex128)) ** 2
        assert np.max(np.abs(P[t] - ref)) <= FP32_TOL * max(ref.max(), 1e-30), t
    plan.close()


def test_dynamic_range_per_wave_and_template(torch_cuda, fdas):
    """Each wave scales its inputs by its own power of two and each template
    its taps by its own: regions of the input at 2^24, 1, 2^-24 and 0, and
    templates at 2^16 and 2^-16 (powers from about 2^-80 to 2^80, inside
    float32's normal range), each compared with the oracle on its own peak
    (away from the region boundaries, where a wave's scale is set by the
    larger neighbour)."""
    bank = ragged_bank(19, 8, 80)
    taps = bank.taps.copy()
    taps[1] *= np.float32(2.0 ** 16)
    taps[5] *= np.float32(2.0 ** -16)
    bank = datagen.Bank(bank.z, taps, bank.tap_len)
    seg = 8192
    x, _ = datagen.random_case(20, 4 * seg, 1, 1)
    scale = [2.0 ** 24, 1.0, 2.0 ** -24, 0.0]
    for r, s in enumerate(scale):
        x[r * seg:(r + 1) * seg] *= np.float32(s)
    n = x.shape[0]
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=1024)
    plan.set_direct_templates(8)
    P = plane(torch_cuda, plan, x)
    ref = oracle.power(x, bank.taps, bank.tap_len)
    margin = 1024
    for r, s in enumerate(scale):
        a, b = r * seg + margin, (r + 1) * seg - margin
        for t in range(8):
            pk = ref[t, a:b].max()
            err = np.abs(P[t, a:b] - ref[t, a:b]).max()
            if s == 0.0:
                assert err == 0.0, (r, t)
            else:
                assert err <= FP32_TOL * pk, (r, t, err / pk)
    plan.close()


def test_toy_all_direct_matches_oracle(torch_cuda, fdas, toy):
    """The 9 x 2^16 toy workload with every template direct: oracle bar,
    identical top-16 and the chirp de-chirped by the template of drift -6."""
    plan = fdas.Plan(toy.bank.taps, toy.bank.tap_len, input_len=toy.n, seg_fft=1024)
    plan.set_direct_templates(toy.bank.num_templates)
    assert plan.info.direct_templates == 9
    P = plane(torch_cuda, plan, toy.x)
    st = against_oracle(P, toy.x, toy.bank, toy.n)
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    ok, bad = st.topk_agree()
    assert ok, bad
    assert toy.bank.z[st.topk("gpu")[0][0]] == -6
    plan.close()


def test_split_requests(torch_cuda, fdas):
    """m rounds down to whole blocks of 8, m >= M takes every eligible block,
    -1 restores the default, and 16-bit plans refuse any split."""
    bank = ragged_bank(21, 20, 100)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1000, seg_fft=1024)
    default = plan.info.direct_templates
    plan.set_direct_templates(13)
    assert plan.info.direct_templates == 8
    plan.set_direct_templates(0)
    assert plan.info.direct_templates == 0
    plan.set_direct_templates(-1)
    assert plan.info.direct_templates == default
    with pytest.raises(fdas.FdasError):
        plan.set_direct_templates(-2)
    plan.close()
    p16 = fdas.Plan(bank.taps, bank.tap_len, input_len=1000, seg_fft=2048, precision="fp16")
    assert p16.info.direct_templates == 0
    with pytest.raises(fdas.FdasError):
        p16.set_direct_templates(8)
    p16.close()


def test_split_call_in_a_graph(torch_cuda, fdas):
    """Both launches of a split call captured in a HIP graph: every replay
    (with eager calls on the plan between them) equals the eager plane bit
    for bit."""
    torch = torch_cuda
    bank = ragged_bank(23, 20, 110)
    n = 50000
    x_np, _ = datagen.random_case(24, n, 1, 1)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=1024)
    plan.set_direct_templates(16)
    assert plan.info.direct_templates == 16
    x = torch.from_numpy(x_np).cuda()
    eager = plan.convolve(x).clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.convolve(x, out=out)
    for rep in range(3):
        out.fill_(-1.0)
        _ = plan.convolve(x[: n // 2].contiguous())     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    plan.close()
