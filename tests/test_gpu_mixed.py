"""GPU parity of the 16-bit plans (FP16 / BF16 storage of the input and the
template spectra, inverse segment transforms on the matrix cores with FP32
accumulation) against the FP64 oracle.

Two comparisons per case, both against the oracle (Eq. (1) and the power of
Section 4.3 in float64):
- on the ORIGINAL complex64 input: the acceptance figure, which includes the
  rounding of the stored input;
- on the input AS STORED (rounded to 16 bits, upcast exactly): what remains
  is the kernel's own error.
Bars: the kernel's own error <= 2e-3 of the peak power for both formats.
FP16 also meets 2e-3 on the original input, with the same top-16 cells up to
the near-tie rule.  BF16 keeps 8 significant bits, and rounding the input
alone moves the power by more than 2e-3 of the peak on the headline input
(the CPU test tests/test_precision_floor.py pins that floor); its total is
held to that case's floor (the oracle on the stored input against the oracle
on the original) plus the 2e-3 kernel bar, which bounds it by the triangle
inequality."""
import sys

import numpy as np
import pytest

import oracle
from fdas_check import MIXED_TOL, PlaneStats
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


def to16(torch, x_np, prec):
    """complex64 numpy [n] -> contiguous CUDA [n, 2] in the plan's 16-bit type
    (round to nearest even, done by torch)."""
    dt = torch.float16 if prec == "fp16" else torch.bfloat16
    v = torch.from_numpy(np.ascontiguousarray(x_np, dtype=np.complex64).view(np.float32).reshape(-1, 2))
    return v.cuda().to(dt).contiguous()


def run16(torch, plan, x_np, prec, ld=None):
    x = to16(torch, x_np, prec)
    n = x.shape[0]
    out = torch.full((plan.num_templates, n if ld is None else ld), -7.0, dtype=torch.float32, device="cuda")
    plan.convolve(x, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def stored(torch, x_np, prec):
    """The input as a 16-bit plan stores it, upcast exactly to complex64."""
    v = to16(torch, x_np, prec).float().cpu().numpy()
    return (v[:, 0].astype(np.float64) + 1j * v[:, 1]).astype(np.complex64)


class Three:
    """GPU plane against the oracle on the original input (total), against
    the oracle on the stored input (the kernel's own error), and the two
    oracle planes against each other (the input-rounding floor)."""

    def __init__(self):
        self.total, self.own, self.floor = PlaneStats(), PlaneStats(), PlaneStats()

    def add(self, rows, P_rows, ref, ref_stored):
        self.total.add(rows, P_rows, ref)
        self.own.add(rows, P_rows, ref_stored)
        self.floor.add(rows, ref_stored, ref)

    def check(self, prec, label=""):
        t, o, f = self.total.norm_err, self.own.norm_err, self.floor.norm_err
        _say(f"  {label}{prec}: total {t:.3e} (rrmse {self.total.rrmse:.2e}), kernel's own {o:.3e}, "
             f"input-rounding floor {f:.3e}")
        assert o <= MIXED_TOL, ("kernel's own error", prec, o)
        ok, bad = self.own.topk_agree(MIXED_TOL)
        assert ok, bad
        bar = MIXED_TOL if prec == "fp16" else f + MIXED_TOL * self.own.max_ref / max(self.total.max_ref, 1e-300)
        assert t <= bar, ("total error", prec, t, bar)
        ok, bad = self.total.topk_agree(bar)
        assert ok, bad


def compare3(torch, P, x_np, prec, bank, n, rows_per_block=16):
    th = Three()
    xs = stored(torch, x_np[:n], prec)
    m = bank.num_templates
    for r0 in range(0, m, rows_per_block):
        rows = list(range(r0, min(m, r0 + rows_per_block)))
        ref = oracle.power(x_np[:n], bank.taps, bank.tap_len, rows=rows)
        ref_s = oracle.power(xs, bank.taps, bank.tap_len, rows=rows)
        th.add(rows, P[rows, :n], ref, ref_s)
    return th


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("seed,n,m,k_max", [
    (11, 1, 3, 17),           # a single output
    (12, 2016, 2, 33),        # n = V (D = 32)
    (13, 2015, 2, 33),        # n = V - 1
    (14, 2017, 2, 33),        # n = V + 1
    (15, 5000, 5, 1),         # one tap
    (16, 9001, 3, 1024),      # K_max = L / 2
    (17, 70001, 7, 77),       # ragged taps, many segments, ragged tail
])
def test_mixed_cases(torch_cuda, fdas, prec, seed, n, m, k_max):
    _say(f"[mixed] {prec} seed={seed} n={n} m={m} k_max={k_max}")
    x, bank = datagen.random_case(seed, n, m, k_max)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n + 5, seg_fft=2048, precision=prec)
    assert plan.seg_fft == 2048 and plan.variant == f"fused-ols-mfma-{prec}"
    P = run16(torch_cuda, plan, x, prec, ld=n + 3)
    assert np.all(P[:, n:] == -7.0), "wrote beyond n"
    compare3(torch_cuda, P, x, prec, bank, n).check(prec)
    plan.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_every_tap_count(torch_cuda, fdas, prec):
    """One template of every tap count 1..1024 (up to L / 2), 12007 points:
    each row against the oracle on the stored input, on its own peak (the
    template spectra share one power-of-two scale, so short templates meet
    the matrix cores with small operands)."""
    torch = torch_cuda
    m = 1024
    _, bank = datagen.random_case(51, 8, m, m)
    rng = np.random.Generator(np.random.PCG64(52))
    tl = np.arange(1, m + 1, dtype=np.int32)
    rng.shuffle(tl)
    taps = np.zeros_like(bank.taps)
    for t in range(m):
        v = rng.standard_normal(2 * int(tl[t]))
        taps[t, :tl[t]] = (v[0::2] + 1j * v[1::2]) / np.sqrt(2.0 * tl[t])
    bank = datagen.Bank(np.zeros(m), taps, tl)
    n = 12007
    x, _ = datagen.random_case(53, n, 1, 1)
    _say(f"[mixed every tap count] {prec}: 1024 templates of 1..1024 taps, n={n}")
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=2048, precision=prec)
    P = run16(torch, plan, x, prec)
    ref = oracle.power(stored(torch, x, prec), bank.taps, bank.tap_len)
    worst = max(float(np.abs(P[t] - ref[t]).max() / ref[t].max()) for t in range(m))
    _say(f"  worst row error / its peak {worst:.3e}")
    assert worst <= MIXED_TOL
    plan.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_toy(torch_cuda, fdas, toy, prec):
    _say(f"[mixed toy] 9 x 2^16 {prec}")
    plan = fdas.Plan(toy.bank.taps, toy.bank.tap_len, input_len=toy.n, seg_fft=2048, precision=prec)
    P = run16(torch_cuda, plan, toy.x, prec)
    th = compare3(torch_cuda, P, toy.x, prec, toy.bank, toy.n)
    th.check(prec)
    t_best, _, _ = th.total.topk("gpu")[0]
    assert toy.bank.z[t_best] == -6


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_ska_full_plane(torch_cuda, fdas, prec):
    """85 templates x 2^22 points, the launch the bench times for the 16-bit
    plans, against the oracle over the whole plane."""
    torch = torch_cuda
    w = datagen.ska_workload()
    _say(f"[mixed ska] {w.name} {prec}, full-plane oracle")
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=w.n, seg_fft=2048, precision=prec)
    x = to16(torch, w.x, prec)
    out = torch.empty((85, w.n), dtype=torch.float32, device="cuda")
    plan.convolve(x, out=out)
    torch.cuda.synchronize()
    th = Three()
    xs = stored(torch, w.x, prec)
    for r0 in range(0, 85, 17):
        rows = list(range(r0, r0 + 17))
        ref = oracle.power(w.x, w.bank.taps, w.bank.tap_len, rows=rows)
        ref_s = oracle.power(xs, w.bank.taps, w.bank.tap_len, rows=rows)
        th.add(rows, out[r0:r0 + 17].cpu().numpy(), ref, ref_s)
        _say(f"  rows {r0}..{r0 + 16}: total so far {th.total.norm_err:.3e}, own {th.own.norm_err:.3e}")
    th.check(prec, "full plane ")
    top = th.total.topk("gpu")
    for c in w.chirps:
        assert any(abs(i - c.r0) < 300 and abs(w.bank.z[t] + c.z0) <= 1.5 for t, i, _ in top), c
    plan.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_power_of_two_scaling_is_exact(torch_cuda, fdas, prec):
    """The per-segment scale is a power of two chosen from the data, so
    scaling the input by 2^k scales every power by exactly 4^k (for k that
    keep the stored input exact: binary16 has subnormals below 2^-14, so it
    is only scaled up)."""
    torch = torch_cuda
    x, bank = datagen.random_case(21, 30011, 4, 60)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=x.shape[0], seg_fft=2048, precision=prec)
    xa = to16(torch, x, prec)
    ks = (0, 5, 3) if prec == "fp16" else (0, 5, -6)
    outs = []
    for k in ks:
        out = torch.empty((4, x.shape[0]), dtype=torch.float32, device="cuda")
        plan.convolve((xa.float() * 2.0 ** k).to(xa.dtype).contiguous(), out=out)
        outs.append(out)
    torch.cuda.synchronize()
    assert torch.equal(outs[1], outs[0] * 4.0 ** ks[1])
    assert torch.equal(outs[2], outs[0] * 4.0 ** ks[2])
    plan.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_zero_input_and_determinism(torch_cuda, fdas, prec):
    torch = torch_cuda
    x, bank = datagen.random_case(22, 12345, 3, 40)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=x.shape[0], seg_fft=2048, precision=prec)
    z = torch.zeros((x.shape[0], 2), dtype=plan.input_dtype(), device="cuda")
    out = torch.full((3, x.shape[0]), 5.0, dtype=torch.float32, device="cuda")
    plan.convolve(z, out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    xa = to16(torch, x, prec)
    a = plan.convolve(xa)
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        b = plan.convolve(xa, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_fp16_and_bf16_plans_share_the_loop(torch_cuda, fdas):
    """The two plans differ only in the input format their forward launch
    reads: on an input whose components are exact in both formats
    (integers up to 255 times 2^-6), their planes and their batched top-16
    are bitwise equal."""
    torch = torch_cuda
    _, bank = datagen.random_case(24, 8, 10, 80)
    n = 30001
    rng = np.random.Generator(np.random.PCG64(25))
    v = rng.integers(-255, 256, size=(n, 2)).astype(np.float32) * np.float32(2.0 ** -6)
    xs = (v[:, 0] + 1j * v[:, 1]).astype(np.complex64)
    planes, cands = {}, {}
    for prec in ("fp16", "bf16"):
        plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=2048, precision=prec)
        xa = to16(torch, xs, prec)
        assert torch.equal(xa.float().cpu(), torch.from_numpy(v)), prec      # exact in the format
        planes[prec] = plan.convolve(xa)
        cands[prec] = plan.convolve_batched([xa, xa[:15000].contiguous()], topk=16)
        torch.cuda.synchronize()
        plan.close()
    assert torch.count_nonzero(planes["fp16"]).item() > 0
    assert torch.equal(planes["fp16"], planes["bf16"])
    assert torch.equal(cands["fp16"], cands["bf16"])


def test_mixed_plan_errors(torch_cuda, fdas):
    torch = torch_cuda
    x, bank = datagen.random_case(23, 4000, 2, 20)
    with pytest.raises(fdas.FdasError) as ei:
        fdas.Plan(bank.taps, bank.tap_len, input_len=4000, seg_fft=1024, precision="fp16")
    assert ei.value.code == fdas.FDAS_EUNSUPPORTED
    with pytest.raises(fdas.FdasError) as ei:
        fdas.Plan(bank.taps, bank.tap_len, input_len=4000, precision="fp8")
    assert ei.value.code == fdas.FDAS_EINVAL
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=4000, seg_fft=2048, precision="fp16")
    xa = to16(torch, x, "fp16")
    # float32 entry points refuse a 16-bit plan
    out = torch.empty((2, 4000), dtype=torch.float32, device="cuda")
    for call in (lambda: plan.tdfir(xa, out=out),
                 lambda: plan.segment_fft(torch.zeros((1, 2048), dtype=torch.complex64, device="cuda"))):
        with pytest.raises(fdas.FdasError) as ei:
            call()
        assert ei.value.code == fdas.FDAS_EUNSUPPORTED
    # input of the wrong 16-bit type or shape
    for bad in (to16(torch, x, "bf16"), torch.from_numpy(x).cuda(), xa[:, :1].contiguous()):
        with pytest.raises(fdas.FdasError) as ei:
            plan.convolve(bad, out=out)
        assert ei.value.code == fdas.FDAS_EINVAL
        with pytest.raises(fdas.FdasError) as ei:
            plan.convolve_batched([bad], topk=4)
        assert ei.value.code == fdas.FDAS_EINVAL
    plan.close()


# ---------------------------------------------------------------------------
# batched form of the 16-bit plans
# ---------------------------------------------------------------------------

def plane_topk(P, k):
    """Top-k cells of a float32 plane, ordered (P desc, t asc, bin asc)."""
    m, n = P.shape
    flat = P.reshape(-1)
    take = min(k, flat.size)
    idx = np.argpartition(-flat, take - 1)[:take] if flat.size > take else np.arange(flat.size)
    thr = flat[idx].min()
    idx = np.nonzero(flat >= thr)[0]                    # every cell tied with the k-th
    order = np.lexsort((idx % n, idx // n, -flat[idx]))[:take]
    idx = idx[order]
    return [(int(i // n), int(i % n), float(flat[i])) for i in idx]


BATCH_LENGTHS = [1, 2015, 2017, 5000, 30011, 70001]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_batched_equals_plane(torch_cuda, fdas, prec):
    """Every cell of the batched call is computed as the plane call computes
    it, so each array's top-16 is the top-16 of its 16-bit plane, exactly."""
    torch = torch_cuda
    x_all, bank = datagen.random_case(31, 140000, 5, 77)
    xs = [x_all[(37 * i) % 1000:(37 * i) % 1000 + n] for i, n in enumerate(BATCH_LENGTHS)]
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=max(BATCH_LENGTHS), seg_fft=2048, precision=prec)
    dev = [to16(torch, x, prec) for x in xs]
    raw = plan.convolve_batched(dev, topk=16)
    torch.cuda.synchronize()
    t, b, p = fdas.split_candidates(raw)
    t, b, p = t.cpu().numpy(), b.cpu().numpy(), p.cpu().numpy()
    for a, x in enumerate(dev):
        P = plan.convolve(x).cpu().numpy()
        want = plane_topk(P, 16)
        got = [(int(t[a, r]), int(b[a, r]), float(p[a, r])) for r in range(len(want))]
        _say(f"[mixed batched] {prec} array {a} n={x.shape[0]}: top {got[0]}")
        assert got == want, (a, got[:4], want[:4])
        if len(want) < 16:
            assert np.all(t[a, len(want):] == -1) and np.all(p[a, len(want):] == -1.0)
    plan.close()


def test_mixed_batched_long_array(torch_cuda, fdas):
    """FP16 plan, an array of 25 * 2^20 points (2.2e9 cells, bins past 2^24)
    beside a short one: each batched top-16 is exactly the top-16 of the
    array's 16-bit plane (per-row top-40 merged with the (P desc, t asc,
    bin asc) order), and every reported power is within the 16-bit bar of
    the oracle at that cell."""
    torch = torch_cuda
    w = datagen.ska_workload(25 << 20)
    n0, n1 = w.n, (1 << 20) + 777
    xs = [w.x, np.ascontiguousarray(w.x[:n1])]
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=n0, seg_fft=2048, precision="fp16")
    dev = [to16(torch, x, "fp16") for x in xs]
    raw = plan.convolve_batched(dev, topk=16)
    torch.cuda.synchronize()
    t, b, p = fdas.split_candidates(raw)
    t, b, p = t.cpu().numpy(), b.cpu().numpy(), p.cpu().numpy()
    out = torch.empty((85, n0), dtype=torch.float32, device="cuda")
    for a, x in enumerate(dev):
        n = x.shape[0]
        plan.convolve(x, out=out[:, :n])
        vals, idx = torch.topk(out[:, :n], 40, dim=1)
        want = sorted(((r, int(ii), float(vv)) for r in range(85) for vv, ii in zip(vals[r].tolist(), idx[r].tolist())),
                      key=lambda c: (-c[2], c[0], c[1]))[:16]
        got = [(int(t[a, r]), int(b[a, r]), float(p[a, r])) for r in range(16)]
        _say(f"[mixed long batch] array {a} n={n}: top {got[0]}")
        assert got == want, (a, got[:4], want[:4])
        ref = oracle.power_at(xs[a], w.bank.taps, w.bank.tap_len, t[a], b[a])
        assert np.max(np.abs(p[a] - ref)) <= MIXED_TOL * float(ref.max())
    assert any(int(bb) > (1 << 24) for bb in b[0])
    plan.close()


def test_mixed_batched_against_oracle(torch_cuda, fdas):
    """FP16 batched candidates against the oracle's whole plane of each array
    (original complex64 input), at the 16-bit tolerance."""
    from fdas_check import check_against_plane
    torch = torch_cuda
    x_all, bank = datagen.random_case(32, 140000, 4, 60)
    lengths = [3, 4000, 33333, 100000]
    xs = [x_all[:n] for n in lengths]
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=max(lengths), seg_fft=2048, precision="fp16")
    raw = plan.convolve_batched([to16(torch, x, "fp16") for x in xs], topk=16)
    torch.cuda.synchronize()
    t, b, p = fdas.split_candidates(raw)
    t, b, p = t.cpu().numpy(), b.cpu().numpy(), p.cpu().numpy()
    for a, x in enumerate(xs):
        ref = oracle.power(x, bank.taps, bank.tap_len)
        check_against_plane(t[a], b[a], p[a], ref, 16, tol=MIXED_TOL)
    plan.close()


def test_mixed_batched_graph_replays(torch_cuda, fdas):
    torch = torch_cuda
    x_all, bank = datagen.random_case(33, 90000, 6, 40)
    lengths = [9000, 45000, 90000]
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=max(lengths), seg_fft=2048, precision="bf16")
    dev = [to16(torch, x_all[:n], "bf16") for n in lengths]
    ws = torch.empty(plan.batched_workspace_bytes(lengths, 8), dtype=torch.uint8, device="cuda")
    out = torch.empty((3, 8, 3), dtype=torch.int32, device="cuda")
    eager = plan.convolve_batched(dev, topk=8, out=out, workspace=ws).clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.convolve_batched(dev, topk=8, out=out, workspace=ws)
    for r in range(3):
        out.fill_(-5)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        plan.convolve(dev[1])                     # eager work between replays
        torch.cuda.synchronize()
    plan.close()
