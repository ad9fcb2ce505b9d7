"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (float32 path): max |P_gpu - P_ref| / max P_ref <= 1e-4 per input array,
and the same top-16 (template, bin) cells up to the near-tie rule."""
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


def run_plane(torch, plan, x_np, method, n=None, ld=None):
    n = x_np.shape[0] if n is None else n
    x = torch.from_numpy(np.ascontiguousarray(x_np[:n])).cuda()
    ld = n if ld is None else ld
    out = torch.full((plan.num_templates, ld), -7.0, dtype=torch.float32, device="cuda")
    getattr(plan, method)(x, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def compare(P, x_np, bank, n, rows_per_block=16, threads=0):
    st = PlaneStats()
    m = bank.num_templates
    for r0 in range(0, m, rows_per_block):
        rows = list(range(r0, min(m, r0 + rows_per_block)))
        ref = oracle.power(x_np[:n], bank.taps, bank.tap_len, rows=rows, nthreads=threads)
        st.add(rows, P[rows, :n], ref)
    return st


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
@pytest.mark.parametrize("method", ["convolve", "tdfir"])
def test_toy_full_plane(torch_cuda, fdas, toy, L, method):
    _say(f"[toy] 9 x 2^16 L={L} {method}")
    plan = fdas.Plan(toy.bank.taps, toy.bank.tap_len, input_len=toy.n, seg_fft=L)
    P = run_plane(torch_cuda, plan, toy.x, method)
    st = compare(P, toy.x, toy.bank, toy.n)
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    ok, bad = st.topk_agree()
    assert ok, bad
    # the chirp (z0 = +6) is de-chirped by the template of drift -6
    t_best, i_best, _ = st.topk("gpu")[0]
    assert toy.bank.z[t_best] == -6


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
def test_ska_headline_full_plane(torch_cuda, fdas, L):
    """85 templates x 2^22 points at every segment length the bench's
    autotuner may pick: the launch the bench times, compared with the oracle
    over the whole plane."""
    w = datagen.ska_workload()
    _say(f"[ska] {w.name} L={L} convolve, full-plane oracle")
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=w.n, seg_fft=L)
    x = torch_cuda.from_numpy(w.x).cuda()
    out = torch_cuda.empty((85, w.n), dtype=torch_cuda.float32, device="cuda")
    plan.convolve(x, out=out)
    torch_cuda.cuda.synchronize()
    st = PlaneStats()
    for r0 in range(0, 85, 17):
        rows = list(range(r0, r0 + 17))
        gpu = out[r0:r0 + 17].cpu().numpy()
        ref = oracle.power(w.x, w.bank.taps, w.bank.tap_len, rows=rows)
        st.add(rows, gpu, ref)
        _say(f"  rows {r0}..{r0 + 16}: norm_err so far {st.norm_err:.3e}")
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    ok, bad = st.topk_agree()
    assert ok, bad
    # every injected chirp shows up among the candidates, de-chirped by the
    # template of opposite drift
    top = st.topk("gpu")
    for c in w.chirps:
        assert any(abs(i - c.r0) < 300 and abs(w.bank.z[t] + c.z0) <= 1.5 for t, i, _ in top), c


def test_ska_tdfir_full_plane(torch_cuda, fdas):
    """The direct TDFIR on the 85 x 2^22 workload over the whole plane: at
    this size its workgroups take the templates in groups of four (their taps
    staged together in LDS) and the last group holds one template."""
    w = datagen.ska_workload()
    _say(f"[ska] {w.name} tdfir, full-plane oracle")
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=w.n, seg_fft=2048)
    x = torch_cuda.from_numpy(w.x).cuda()
    out = torch_cuda.empty((85, w.n), dtype=torch_cuda.float32, device="cuda")
    plan.tdfir(x, out=out)
    torch_cuda.cuda.synchronize()
    st = PlaneStats()
    for r0 in range(0, 85, 17):
        rows = list(range(r0, r0 + 17))
        st.add(rows, out[r0:r0 + 17].cpu().numpy(), oracle.power(w.x, w.bank.taps, w.bank.tap_len, rows=rows))
    _say(st.summary())
    assert st.norm_err <= FP32_TOL
    ok, bad = st.topk_agree()
    assert ok, bad


@pytest.mark.parametrize("seed,n,m,k_max,L", [
    (1, 1, 3, 17, 1024),          # a single output
    (2, 924, 2, 101, 1024),       # n = V exactly
    (3, 923, 2, 101, 1024),       # n = V - 1
    (4, 925, 2, 101, 1024),       # n = V + 1
    (5, 5000, 5, 1, 2048),        # one tap: P = |h0|^2 |x|^2
    (6, 9001, 3, 1024, 2048),     # K_max = L / 2
    (7, 20011, 1, 64, 4096),      # M = 1, prime length
    (8, 70001, 7, 77, 2048),      # ragged taps, several segments, ragged tail
    (9, 30001, 3, 4096, 8192),    # K_max = L / 2 at the longest segment
    (10, 8000, 2, 33, 8192),      # n shorter than one segment
])
@pytest.mark.parametrize("method", ["convolve", "tdfir"])
def test_edge_cases(torch_cuda, fdas, seed, n, m, k_max, L, method):
    _say(f"[edge] seed={seed} n={n} m={m} k_max={k_max} L={L} {method}")
    x, bank = datagen.random_case(seed, n, m, k_max)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n + 17, seg_fft=L)
    P = run_plane(torch_cuda, plan, x, method, ld=n + 5)
    assert np.all(P[:, n:] == -7.0), "wrote past n"
    st = compare(P, x, bank, n)
    assert st.norm_err <= FP32_TOL, st.summary()


@pytest.mark.parametrize("method", ["convolve", "tdfir"])
def test_every_tap_count_up_to_half_the_segment(torch_cuda, fdas, method):
    """One template of every tap count 1..512 at L = 1024 (up to K_max =
    L / 2), the whole bank by overlap-save (direct route off) or by TDFIR,
    12007 points, each row against the oracle on its own peak."""
    m = 512
    _, bank = datagen.random_case(41, 8, m, m)
    rng = np.random.Generator(np.random.PCG64(42))
    tl = np.arange(1, m + 1, dtype=np.int32)
    rng.shuffle(tl)
    taps = np.zeros_like(bank.taps)
    for t in range(m):
        v = rng.standard_normal(2 * int(tl[t]))
        taps[t, :tl[t]] = (v[0::2] + 1j * v[1::2]) / np.sqrt(2.0 * tl[t])
    bank = datagen.Bank(np.zeros(m), taps, tl)
    n = 12007
    x, _ = datagen.random_case(43, n, 1, 1)
    _say(f"[every tap count] 512 templates of 1..512 taps, n={n}, L=1024, {method}")
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=1024)
    plan.set_direct_templates(0)
    P = run_plane(torch_cuda, plan, x, method)
    ref = oracle.power(x, bank.taps, bank.tap_len)
    worst = max(float(np.abs(P[t] - ref[t]).max() / ref[t].max()) for t in range(m))
    _say(f"  worst row error / its peak {worst:.3e}")
    assert worst <= FP32_TOL
    plan.close()


def test_prefix_length_and_zero_template(torch_cuda, fdas):
    """n < input_len, and a template with zero taps gives an all-zero row."""
    x, bank = datagen.random_case(9, 30000, 4, 40)
    tl = bank.tap_len.copy()
    tl[2] = 0
    plan = fdas.Plan(bank.taps, tl, input_len=30000, seg_fft=1024)
    for n in (12345, 30000):
        for method in ("convolve", "tdfir"):
            P = run_plane(torch_cuda, plan, x, method, n=n)
            assert np.all(P[2] == 0.0)
            st = compare(P, x, datagen.Bank(bank.z, bank.taps, tl), n)
            assert st.norm_err <= FP32_TOL


def test_impulse_gives_template_power(torch_cuda, fdas):
    _, bank = datagen.random_case(10, 8, 3, 50)
    n, j0 = 5000, 1777
    x = np.zeros(n, np.complex64)
    x[j0] = 1.0
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n, seg_fft=1024)
    for method in ("convolve", "tdfir"):
        P = run_plane(torch_cuda, plan, x, method)
        for t in range(3):
            kt = int(bank.tap_len[t])
            ref = np.zeros(n)
            ref[j0:j0 + kt] = np.abs(bank.taps[t, :kt].astype(np.complex128)) ** 2
            assert np.max(np.abs(P[t] - ref)) <= FP32_TOL * ref.max()


def test_deterministic_and_two_streams(torch_cuda, fdas, toy):
    torch = torch_cuda
    plan = fdas.Plan(toy.bank.taps, toy.bank.tap_len, input_len=toy.n, seg_fft=1024)
    x = torch.from_numpy(toy.x).cuda()
    a = plan.convolve(x)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        b = plan.convolve(x)
    with torch.cuda.stream(s2):
        c = plan.convolve(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_taps_on_device(torch_cuda, fdas, toy):
    torch = torch_cuda
    p_host = fdas.Plan(toy.bank.taps, toy.bank.tap_len, input_len=toy.n, seg_fft=2048)
    p_dev = fdas.Plan(torch.from_numpy(toy.bank.taps).cuda(), toy.bank.tap_len,
                      input_len=toy.n, seg_fft=2048)
    x = torch.from_numpy(toy.x).cuda()
    assert torch.equal(p_host.convolve(x), p_dev.convolve(x))
    assert np.array_equal(p_host.template_spectra(), p_dev.template_spectra())


@pytest.fixture(scope="module")
def large(torch_cuda):
    """85 templates x 25 * 2^20 points (a ragged number of segments at every
    L): the plane holds 2.2e9 elements (8.9 GB), so row offsets pass 2^31
    elements and 2^32 bytes.  Oracle windows at the start, the middle, the
    end and around each injected chirp, in rows spread over the bank and the
    chirps' de-chirping rows."""
    w = datagen.ska_workload(25 << 20)
    n, m = w.n, w.bank.num_templates
    assert m * n > 2 ** 31
    rows = sorted({0, 21, 42, 63, m - 1} | {int(np.argmin(np.abs(w.bank.z + c.z0))) for c in w.chirps})
    wins = [(0, 4096), (n // 2 - 2048, n // 2 + 2048), (n - 4096, n)]
    wins += [(max(0, int(c.r0) - 2048), min(n, int(c.r0) + 2048)) for c in w.chirps]
    refs = [oracle.power(w.x, w.bank.taps, w.bank.tap_len, rows=rows, i0=a, i1=b) for a, b in wins]
    peak = max(float(r.max()) for r in refs)
    x = torch_cuda.from_numpy(w.x).cuda()
    out = torch_cuda.empty((m, n), dtype=torch_cuda.float32, device="cuda")
    return w, rows, wins, refs, peak, x, out


@pytest.mark.parametrize("prec,method,L", [
    ("fp32", "convolve", 1024), ("fp32", "convolve", 2048), ("fp32", "convolve", 4096),
    ("fp32", "convolve", 8192), ("fp32", "tdfir", 2048), ("fp16", "convolve", 2048), ("bf16", "convolve", 2048)])
def test_plane_past_2g_elements_sampled(torch_cuda, fdas, large, prec, method, L):
    """The large plane's sampled windows against the oracle: float32 FDFIR at
    every segment length and TDFIR at the 1e-4 bar, the 16-bit plans at 2e-3
    against the oracle on the input as stored (their own error; the input's
    rounding to 16 bits is a property of the format, pinned on the CPU)."""
    from fdas_check import MIXED_TOL
    torch = torch_cuda
    w, rows, wins, refs, peak, x, out = large
    tol = {"fp32": FP32_TOL, "fp16": MIXED_TOL, "bf16": MIXED_TOL}[prec]
    _say(f"[large] 85 x {w.n} {prec} {method} L={L}")
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=w.n, seg_fft=L, precision=prec)
    xin = x if prec == "fp32" else torch.view_as_real(x).to(plan.input_dtype()).contiguous()
    out.fill_(-7.0)
    getattr(plan, method)(xin, out=out)
    torch.cuda.synchronize()
    if prec != "fp32":
        v = xin.float().cpu().numpy()
        xs = (v[:, 0].astype(np.float64) + 1j * v[:, 1]).astype(np.complex64)
        refs = [oracle.power(xs, w.bank.taps, w.bank.tap_len, rows=rows, i0=a, i1=b) for a, b in wins]
        peak = max(float(r.max()) for r in refs)
    err = max(float(np.abs(out[rows, a:b].cpu().numpy() - r).max()) for (a, b), r in zip(wins, refs))
    _say(f"  max err / sampled peak {err / peak:.3e}")
    assert err <= tol * peak, (prec, method, L, err / peak)
    plan.close()


def test_direct_rows_past_2g_elements_sampled(torch_cuda, fdas, large):
    """The direct-convolution route writing rows whose offsets pass 2^31
    elements: with the bank in order of decreasing tap count, the plan's
    shortest templates (the ones it runs directly) are its last rows."""
    torch = torch_cuda
    w, _, wins, _, _, x, out = large
    order = np.argsort(-w.bank.tap_len, kind="stable")
    taps, tl = np.ascontiguousarray(w.bank.taps[order]), np.ascontiguousarray(w.bank.tap_len[order])
    m, n = len(tl), w.n
    plan = fdas.Plan(taps, tl, input_len=n, seg_fft=2048)
    md = plan.info.direct_templates
    _say(f"[large] 85 x {n} fp32, rows by decreasing tap count, {md} direct")
    assert md > 0 and (m - 1) * n > 2 ** 31
    rows = sorted({0, m - md - 1, m - md, m - md // 2, m - 2, m - 1})
    refs = [oracle.power(w.x, taps, tl, rows=rows, i0=a, i1=b) for a, b in wins]
    peak = max(float(r.max()) for r in refs)
    out.fill_(-7.0)
    plan.convolve(x, out=out)
    torch.cuda.synchronize()
    err = max(float(np.abs(out[rows, a:b].cpu().numpy() - r).max()) for (a, b), r in zip(wins, refs))
    _say(f"  max err / sampled peak {err / peak:.3e}")
    assert err <= FP32_TOL * peak, err / peak
    plan.close()


@pytest.mark.parametrize("L", [1024, 2048])
def test_paper_shape_84_filters_421_taps(torch_cuda, fdas, L):
    """The paper's studied bank shape (84 complex filters of 421 taps,
    Section 3), full plane at 2^16 points, FDFIR and TDFIR."""
    x, bank = datagen.random_case(421, 1 << 16, 84, 421, ragged=False)
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1 << 16, seg_fft=L)
    for method in ("convolve", "tdfir"):
        _say(f"[84x421] L={L} {method}")
        P = run_plane(torch_cuda, plan, x, method)
        st = compare(P, x, bank, 1 << 16, rows_per_block=28)
        assert st.norm_err <= FP32_TOL, st.summary()
        ok, bad = st.topk_agree()
        assert ok, bad


@pytest.fixture(scope="module")
def paper_shape(torch_cuda):
    """The sweep's input: 84 filters of 421 random taps, one 2^22-point
    spectrum (the bench's fig. 8 leg slices it to 2^18..2^22 points)."""
    x, bank = datagen.random_case(421, 1 << 22, 84, 421, ragged=False)
    return x, bank, torch_cuda.from_numpy(x).cuda()


@pytest.mark.parametrize("method,L", [("convolve", 1024), ("convolve", 2048), ("tdfir", 2048)])
def test_paper_shape_84x421_at_swept_sizes(torch_cuda, fdas, paper_shape, method, L):
    """The paper's bank shape (84 x 421 taps) at the sizes the sweep times:
    the whole 84 x 2^18 plane against the oracle (with the top-16 rule), and
    the 84 x 2^22 plane in oracle windows at the start, the middle, the end
    and five random places, in rows spread over the bank (Section 6.3's
    experiment shape)."""
    torch = torch_cuda
    x, bank, xd = paper_shape
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1 << 22, seg_fft=L)
    n = 1 << 18
    _say(f"[84x421 swept] L={L} {method} n=2^18 full plane")
    out = torch.full((84, n), -7.0, dtype=torch.float32, device="cuda")
    getattr(plan, method)(xd[:n], out=out)
    torch.cuda.synchronize()
    st = compare(out.cpu().numpy(), x, bank, n, rows_per_block=28)
    _say(st.summary())
    assert st.norm_err <= FP32_TOL, st.summary()
    ok, bad = st.topk_agree()
    assert ok, bad
    del out
    n = 1 << 22
    _say(f"[84x421 swept] L={L} {method} n=2^22 sampled windows")
    out = torch.full((84, n), -7.0, dtype=torch.float32, device="cuda")
    getattr(plan, method)(xd, out=out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8421)
    rows = [0, 17, 41, 62, 83]
    wins = [(0, 4096), (n // 2 - 2048, n // 2 + 2048), (n - 4096, n)]
    wins += [(int(a), int(a) + 2048) for a in rng.integers(0, n - 2048, 5)]
    err, peak = 0.0, 0.0
    for a, b in wins:
        ref = oracle.power(x, bank.taps, bank.tap_len, rows=rows, i0=a, i1=b)
        got = out[rows, a:b].cpu().numpy()
        err = max(err, float(np.abs(got - ref).max()))
        peak = max(peak, float(ref.max()))
    _say(f"  max err / sampled peak {err / peak:.3e}")
    assert err <= FP32_TOL * peak
    plan.close()
