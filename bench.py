"""Throughput of the FT-convolution hot path on one MI355X.

One step = one fdas_convolve call: overlap-save FDFIR of one 2^22-point
complex64 spectrum against 85 templates (z = -42..42, 17..101 taps), segment
transform L = 2048, writing the 85 x 2^22 float32 power plane.  The input
and the output plane are resident in HBM before timing starts.

Prints one JSON line (rank 0).  Extra legs: the direct TDFIR baseline on the
same workload, the 16-bit (FP16/BF16) plans on the same workload, the batched
DM-trial form, the served loop, paper-shaped sweeps, and the FP64 CPU oracle
timed on a bounded sample of the same workload (which also gives a parity
figure for the sampled rows).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "template-samples/s (85 tpl x 2^22 pts) + HBM roofline frac; served p50/p99 ms"
HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3       # MI355X published FP32 vector: 256 CU x 64 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
# What the library's kernels can issue: packed FP32 is off in every device compile, so at
# most one wave64 VALU instruction per CU per cycle, i.e. 256 CU x 64 lanes x
# 2 (FMA) x 2.4 GHz.
FP32_UNPACKED_PEAK_TFLOPS = 78.6
FP16_MFMA_PEAK_TFLOPS = 2500.0        # MI355X published dense binary16 matrix-core peak
SQ_COUNTER_FILES = {2048: os.path.join(ROOT, "profiles", "fdas_convolve_ska-85x2^22_L2048_sq_counters.md")}
SUSTAINED_S = 1.5                     # back-to-back calls timed for the sustained rate
SETTLE_S = 0.3                        # untimed back-to-back calls before the timed steps
KERNEL_SOURCES = ("paper_1805_12280_amd/csrc/seg_fft.h", "paper_1805_12280_amd/csrc/fdas_internal.h",
                  "paper_1805_12280_amd/csrc/fdas_kernels.hip", "paper_1805_12280_amd/csrc/fdas_direct.hip")
# HBM traffic summaries of one fdas_convolve call, keyed by (segment length,
# direct templates): the call's launches summed
TRAFFIC_FILES = {(L, md): os.path.join(ROOT, "profiles", f"fdas_convolve_ska-85x2^22_L{L}_direct{md}_traffic.md")
                 for L in (1024, 2048, 4096) for md in range(0, 86, 8)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(text: str) -> str:
    """Source text with comments, trailing blanks and empty lines removed, so
    a comment-only edit leaves the kernel's hash unchanged."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_source_hash() -> str:
    """First 16 hex digits of sha256 over the float32 path's sources (code
    only): the committed counter summaries carry the value they were taken
    on."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(L, md=0):
    """HBM bytes per fdas_convolve call from the committed rocprofv3 PMC
    summary for this segment length and direct split, if it was taken on the
    current kernel source; else None."""
    path = TRAFFIC_FILES.get((L, md))
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"traffic_bytes_per_call:\s*([0-9.eE+]+)", text)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def _sq_line(L, key):
    """A `key: value` line of the committed SQ-counter summary for this
    segment length, if it was taken on the current kernel source; else None."""
    path = SQ_COUNTER_FILES.get(L)
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    m_val = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    if not (m_hash and m_val) or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def measured_valu_issue(L, md=0):
    """VALU issue rate (wave64 instructions per CU per cycle) of the
    overlap-save launch at this split, from the committed SQ counters."""
    return _sq_line(L, f"valu_issue_per_cu_cycle[direct={md}]")


def measured_mfma_busy(L, md):
    """Matrix-core busy fraction of the direct launch at this split, from the
    committed SQ counters."""
    return _sq_line(L, f"mfma_busy[direct={md}]")


def algorithmic_bytes(n, m, L):
    """Bytes the method itself must move: the input once, the power plane once
    and the pre-transformed templates once."""
    return 8 * n + 4 * m * n + 8 * m * L


def nominal_flops(n, m, L, k_max):
    """Algorithmic operations of overlap-save with the minimal overlap
    V = L - (K_max - 1): 5 L log2 L per transform (the paper's C = 5), 6 per
    complex product, 3 per power value; one forward transform per segment."""
    v = L - (k_max - 1)
    s = math.ceil(n / v)
    fft = 5 * L * math.log2(L)
    return s * (m * (fft + 6 * L + 3 * v) + fft)


def time_calls(torch, fn, steps, warmup, mark=None):
    """Mean ms per call over `steps` calls between two events, after `warmup`
    untimed calls; synchronised on both sides.  `mark` names a marker range
    around the timed calls (a profiler's marker trace picks them out)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    if mark:
        torch.cuda.nvtx.range_push(mark)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    if mark:
        torch.cuda.nvtx.range_pop()
    return start.elapsed_time(stop) / steps


def time_steps(torch, fn, steps, warmup):
    """Mean ms per call over `steps` back-to-back calls bracketed by
    synchronisations, and the per-call times (events between calls)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, per


def settle(torch, fn, seconds=SETTLE_S):
    """Back-to-back untimed calls for about `seconds`."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            fn()
        torch.cuda.synchronize()


def sustained(torch, fn, ms_hint, seconds=SUSTAINED_S):
    """Mean ms per call over about `seconds` of back-to-back calls (the clock
    the chip holds under sustained load), with the first and last tenth of
    the run timed on their own to show any drift."""
    calls = max(20, int(math.ceil(seconds * 1e3 / max(ms_hint, 1e-3))))
    tenth = max(1, calls // 10)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(calls):
        fn()
        if k + 1 == tenth:
            ev[1].record(stream)
        if k + 1 == calls - tenth:
            ev[2].record(stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    total = ev[0].elapsed_time(ev[3])
    return {"calls": calls, "seconds": total / 1e3, "ms_per_call": total / calls,
            "first_tenth_ms_per_call": ev[0].elapsed_time(ev[1]) / tenth,
            "last_tenth_ms_per_call": ev[2].elapsed_time(ev[3]) / tenth}


def percentiles(xs):
    ys = sorted(xs)
    pick = lambda q: ys[min(len(ys) - 1, int(round(q * (len(ys) - 1))))]   # noqa: E731
    return {"p10": pick(0.1), "median": pick(0.5), "p90": pick(0.9)}


def mall_evicted_ms(torch, fn, reps=5):
    """Each call timed alone after writing a 512 MB buffer, so the input and
    the template spectra are no longer in the 256 MB MALL."""
    junk = torch.empty(128 << 20, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    out = []
    for r in range(reps):
        junk.fill_(float(r))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    del junk
    return percentiles(out)


def copy_probe_gbs(torch):
    """Achievable HBM bandwidth: a plain 1 GiB device-to-device copy."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    ms = time_calls(torch, lambda: dst.copy_(src), 5, 2)
    del src, dst
    return 2 * 2 ** 30 / ms / 1e6


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(w, P_gpu_rows_fn, target_s: float):
    """FP64 oracle on all 85 templates over a prefix of the outputs, sized to
    take about target_s of wall time on the host's cores."""
    import numpy as np
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from fdas_check import PlaneStats
    threads = oracle.threads()
    m = w.bank.num_templates
    # calibrate on a short prefix
    t0 = time.perf_counter()
    cal = 1 << 14
    oracle.power(w.x, w.bank.taps, w.bank.tap_len, i1=cal)
    rate = m * cal / max(time.perf_counter() - t0, 1e-6)
    n_s = int(min(w.n, max(cal, (rate * target_s / m) // 4096 * 4096)))
    t0 = time.perf_counter()
    ref = oracle.power(w.x, w.bank.taps, w.bank.tap_len, i1=n_s)
    wall = time.perf_counter() - t0
    st = PlaneStats()
    st.add(list(range(m)), P_gpu_rows_fn(n_s), ref)
    # the toy workload (9 x 2^16) on one core, for scale
    from paper_1805_12280_amd import datagen
    toy = datagen.toy_workload()
    t0 = time.perf_counter()
    oracle.power(toy.x, toy.bank.taps, toy.bank.tap_len, nthreads=1)
    toy_s = time.perf_counter() - t0
    del np
    return {
        "value": m * n_s / wall, "unit": "template-samples/s", "cores": threads, "kind": "oracle",
        "sample": f"all {m} templates x first {n_s} of {w.n} outputs (FP64 direct, C + OpenMP), "
                  f"{wall:.1f} s wall",
        "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
        "toy_9x2^16_single_core_s": toy_s,
    }, {"rows": m, "outputs": n_s, "norm_err": st.norm_err, "rrmse": st.rrmse}


def direct_mfma_flops(n, tap_len, md):
    """Matrix-core operations the direct launch issues for the md shortest
    templates: per 16 outputs and block of 8 templates, 3 binary16 products
    (high x high, high x low, low x high) of 16 x 16 x 32 per 16 taps of the
    block's longest template."""
    lens = np.sort(np.asarray(tap_len))[:md]
    tiles = math.ceil(n / 16)
    ops = 0
    for b in range(0, md, 8):
        nk = max(1, math.ceil(int(lens[b:b + 8].max()) / 16))
        ops += tiles * 3 * nk * 2 * 16 * 16 * 32
    return ops


def split_legs(torch, fdas, w, x, L, md, steps, warmup):
    """Each launch of a split call timed on its own: the md shortest
    templates on a plan that runs them all directly, the rest on an
    overlap-save plan (same segment length), each writing its rows of a
    plane.  Their sum is close to the split call's time."""
    m, n = w.bank.num_templates, w.n
    if md == 0:
        return {"direct": None, "overlap_save": None}
    order = np.argsort(w.bank.tap_len, kind="stable")
    res = {}
    for name, idx in (("direct", order[:md]), ("overlap_save", order[md:])):
        if len(idx) == 0:
            res[name] = None
            continue
        p = fdas.Plan(np.ascontiguousarray(w.bank.taps[idx]), np.ascontiguousarray(w.bank.tap_len[idx]),
                      input_len=n, seg_fft=L)
        p.set_direct_templates(len(idx) if name == "direct" else 0)
        o = torch.empty((len(idx), n), dtype=torch.float32, device=x.device)
        t = time_calls(torch, lambda: p.convolve(x, out=o), steps, warmup, mark=f"split leg {name}")
        by = 8 * n + 4 * len(idx) * n
        ent = {"templates": len(idx), "ms": t, "hbm_gbs": by / (t * 1e-3) / 1e9,
               "hbm_frac": by / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if name == "direct":
            fl = direct_mfma_flops(n, w.bank.tap_len, len(idx))
            ent.update({"mfma_tflops": fl / (t * 1e-3) / 1e12, "mfma_peak_tflops": FP16_MFMA_PEAK_TFLOPS,
                        "mfma_frac": fl / (t * 1e-3) / 1e12 / FP16_MFMA_PEAK_TFLOPS,
                        "mfma_busy_counter": measured_mfma_busy(L, md)})
        else:
            fl = nominal_flops(n, len(idx), L, w.bank.k_max)
            ent.update({"tflops": fl / (t * 1e-3) / 1e12, "peak_tflops": FP32_UNPACKED_PEAK_TFLOPS,
                        "frac": fl / (t * 1e-3) / 1e12 / FP32_UNPACKED_PEAK_TFLOPS})
        res[name] = ent
        p.close()
    return res


def batched_leg(torch, fdas, steps, warmup):
    """64 DM-trial spectra (2^19..2^22 points) x 85 templates per step, top-16
    cells per array, the segment length picked by the autotuner, the call
    captured once in a HIP graph and replayed."""
    from paper_1805_12280_amd import autotune, datagen
    log("generating the 64-array DM-trial batch ...")
    batch = datagen.dm_trial_batch()
    bank = batch.bank
    dev = [torch.from_numpy(x).to("cuda:0") for x in batch.xs]
    best, wg, _, tuned = autotune.tune(bank, dev, mode="batched", topk=16, use_cache=False)
    log(f"autotune (ms per batch, L/workgroups per CU): {tuned} -> L = {best}, wg = {wg}")
    plan = fdas.Plan(bank.taps, bank.tap_len, input_len=max(batch.lengths), seg_fft=best)
    plan.set_workgroups_per_cu(wg)
    ws = torch.empty(plan.batched_workspace_bytes(batch.lengths, 16), dtype=torch.uint8, device="cuda:0")
    out = torch.empty((len(dev), 16, 3), dtype=torch.int32, device="cuda:0")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.convolve_batched(dev, topk=16, out=out, workspace=ws)
    settle(torch, g.replay)
    ms = time_calls(torch, g.replay, steps, warmup, mark="batched fp32 timed steps")
    m = bank.num_templates
    samples = m * sum(batch.lengths)
    flops = sum(nominal_flops(n, m, best, bank.k_max) for n in batch.lengths)
    tflops = flops / (ms * 1e-3) / 1e12
    plan.close()
    res = {"workload": batch.name, "arrays": len(dev), "points": sum(batch.lengths),
           "topk": 16, "seg_fft": best, "workgroups_per_cu": wg, "autotune_ms": tuned, "graph": True,
           "ms_per_step": ms, "value": samples / (ms * 1e-3), "unit": "template-samples/s",
           "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_UNPACKED_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": tflops / FP32_UNPACKED_PEAK_TFLOPS}}
    # the same batch on the 16-bit plans (L = 2048), also graph-replayed
    for prec in ("fp16", "bf16"):
        plan = fdas.Plan(bank.taps, bank.tap_len, input_len=max(batch.lengths), seg_fft=2048, precision=prec)
        dev16 = [torch.view_as_real(x).to(plan.input_dtype()).contiguous() for x in dev]
        ws = torch.empty(plan.batched_workspace_bytes(batch.lengths, 16), dtype=torch.uint8, device="cuda:0")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            plan.convolve_batched(dev16, topk=16, out=out, workspace=ws)
        settle(torch, g.replay)
        ms16 = time_calls(torch, g.replay, steps, warmup, mark=f"batched {prec} timed steps")
        res[prec] = {"ms_per_step": ms16, "value": samples / (ms16 * 1e-3), "speedup_vs_fp32": ms / ms16,
                     "workspace_bytes": int(ws.numel())}
        log(f"batched {prec}: {ms16:.3f} ms/step ({ms / ms16:.2f}x fp32)")
        plan.close()
        del ws, dev16
    return res


SERVED_BANKS = {"z10": tuple(range(-10, 11)), "z21": tuple(range(-21, 22)), "z42": tuple(range(-42, 43))}
SERVED_LENGTHS = ((1 << 18, 0.5), (1 << 20, 0.3), (1 << 22, 0.2))


def served_leg(torch, jobs_per_rate=240, rates=(0.5, 0.8, 0.95), seed=4, precision="fp32"):
    """Poisson arrivals of jobs (length 2^18/2^20/2^22 with p = 0.5/0.3/0.2,
    bank of 21/43/85 templates), continuous batching on resident plans,
    top-16 per job.  The saturated rate is measured first (all jobs present at
    t = 0); then arrivals at fractions of it.  Inputs are resident spectra (the
    stage before filtering runs on the device; for a 16-bit precision they are
    stored as 16-bit pairs)."""
    import numpy as np
    from paper_1805_12280_amd import datagen
    from paper_1805_12280_amd.serve import GpuExecutor, Job, Scheduler, latency_stats
    rng = np.random.default_rng(seed)
    banks = {k: datagen.make_bank(v) for k, v in SERVED_BANKS.items()}
    pool = {}
    noise_rng = np.random.default_rng(seed + 1)
    for n, _ in SERVED_LENGTHS:
        pool[n] = [torch.from_numpy(datagen.make_spectrum(n, (), noise_rng)).to("cuda:0") for _ in range(2)]
        if precision != "fp32":
            dt = torch.float16 if precision == "fp16" else torch.bfloat16
            pool[n] = [torch.view_as_real(v).to(dt).contiguous() for v in pool[n]]
    lens = [n for n, _ in SERVED_LENGTHS]
    probs = [p for _, p in SERVED_LENGTHS]
    ex = GpuExecutor(banks, input_len=1 << 22, topk=16, slots=3, precision=precision,
                     seg_fft={k: (1024 if precision == "fp32" else 2048) for k in banks})
    ex.reserve(16, max(lens))
    mfree, _ = torch.cuda.mem_get_info()
    budget = int(0.25 * mfree)

    def draw(count):
        out = []
        for i in range(count):
            n = int(rng.choice(lens, p=probs))
            bank = str(rng.choice(list(banks)))
            out.append((i, bank, n, pool[n][int(rng.integers(0, 2))]))
        return out

    def run(spec, gaps):
        # the host loop runs with Python's cyclic collector paused (collected
        # just before): a full collection inside a run stalled one scheduler
        # step by ~40 ms
        gc.collect()
        gc.disable()
        try:
            return run_inner(spec, gaps)
        finally:
            gc.enable()

    def run_inner(spec, gaps):
        sched = Scheduler(ex, budget, max_batch=16, max_wait_s=2e-3)
        t = time.perf_counter()
        jobs = []
        for (i, bank, n, x), g in zip(spec, gaps):
            t += g
            jobs.append(Job(i, bank, x, n, t))
        start = time.perf_counter()
        pending = list(jobs)
        while pending or not sched.idle:
            now = time.perf_counter()
            while pending and pending[0].arrival <= now:
                sched.submit(pending.pop(0))
            sched.step()
        end = time.perf_counter()
        samples = sum(j.n * banks[j.bank].num_templates for j in jobs)
        st = latency_stats(jobs)
        st.update({"makespan_s": end - start, "jobs_per_s": len(jobs) / (end - start),
                   "template_samples_per_s": samples / (end - start),
                   "mean_batch": float(np.mean(sched.batches))})
        return st

    warm = draw(16)
    run(warm, [0.0] * len(warm))
    spec = draw(jobs_per_rate)
    sat = run(spec, [0.0] * len(spec))
    lam = sat["jobs_per_s"]
    out = {"precision": precision, "saturated": sat, "rates": [], "slots": ex.slots, "max_batch": 16,
           "max_wait_ms": 2.0, "topk": 16,
           "budget_bytes": budget, "jobs_per_rate": jobs_per_rate}
    for r in rates:
        gaps = rng.exponential(1.0 / (r * lam), size=len(spec)).tolist()
        st = run(spec, gaps)
        st["offered_fraction"] = r
        st["offered_jobs_per_s"] = r * lam
        out["rates"].append(st)
    ex.close()
    return out


def mixed_leg(torch, fdas, w, x32, P32, steps, warmup, fp32_ms):
    """The 16-bit plans (FP16 and BF16 storage, matrix-core inverse FFT) on
    the same 85 x 2^22 workload: time per call, speedup over the float32
    path, and the peak-normalised deviation of the whole plane from the
    float32 path's plane P32 (whose own error against the FP64 oracle is
    below 1e-4; the 16-bit plans' parity with the oracle is in the tests)."""
    m, n = w.bank.num_templates, w.n
    out = torch.empty((m, n), dtype=torch.float32, device=x32.device)
    peak = P32.max()
    res = {}
    for prec in ("fp16", "bf16"):
        plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=n, seg_fft=2048, precision=prec)
        xh = torch.view_as_real(x32).to(plan.input_dtype()).contiguous()
        settle(torch, lambda: plan.convolve(xh, out=out))
        ms = time_calls(torch, lambda: plan.convolve(xh, out=out), steps, warmup, mark=f"mixed {prec} timed steps")
        dev = float(((out - P32).abs().max() / peak).item())
        rr = float((torch.linalg.vector_norm((out - P32).flatten().double())
                    / torch.linalg.vector_norm(P32.flatten().double())).item())
        res[prec] = {"ms_per_step": ms, "value": m * n / (ms * 1e-3), "unit": "template-samples/s",
                     "speedup_vs_fp32": fp32_ms / ms, "variant": plan.variant,
                     "resident_bytes": int(plan.info.resident_bytes),
                     "max_dev_vs_fp32_plane": dev, "rrmse_vs_fp32_plane": rr,
                     # the float32 plane is within 1e-6 of the FP64 oracle, so
                     # this is the 16-bit plan's deviation from the oracle to
                     # that accuracy; the bar for mixed precision is 2e-3
                     "within_2e-3_bar": dev <= 2e-3}
        log(f"{prec}: {ms:.4f} ms/step ({fp32_ms / ms:.2f}x fp32), peak-normalised deviation "
            f"from the float32 plane {dev:.2e}")
        plan.close()
    del out
    return res


def sweeps_leg(torch, fdas):
    """The paper's experiment shapes on this GPU.
    fig8: M = 84 filters of 421 taps, inputs 2^18..2^22, FDFIR + power; the
          paper reports the average latency per filter (3xAOLS-2048-P on one
          FPGA: 2.98 ms per filter at 2^22, Section 6.3).
    fig7: one filter of 64/128/256/421 taps on 2^22 points, TDFIR vs FDFIR
          (the paper's FPGA TD theoretical latency is 108-124 ms at 421 taps,
          Table 4)."""
    import numpy as np
    from paper_1805_12280_amd import datagen
    out = {"fig8": [], "fig7": []}
    x_all, bank = datagen.random_case(421, 1 << 22, 84, 421, ragged=False)
    x = torch.from_numpy(x_all).to("cuda:0")
    for L in (1024, 2048):
        plan = fdas.Plan(bank.taps, bank.tap_len, input_len=1 << 22, seg_fft=L)
        for lg in range(18, 23):
            n = 1 << lg
            o = torch.empty((84, n), dtype=torch.float32, device="cuda:0")
            ms = time_calls(torch, lambda: plan.convolve(x[:n], out=o), 5, 2)
            out["fig8"].append({"n": n, "seg_fft": L, "filters": 84, "taps": 421, "ms": ms,
                                "ms_per_filter": ms / 84, "template_samples_per_s": 84 * n / (ms * 1e-3)})
            del o
        plan.close()
    for k in (64, 128, 256, 421):
        h = bank.taps[:1, :k].copy()
        h /= np.sqrt(np.sum(np.abs(h.astype(np.complex128)) ** 2))
        plan = fdas.Plan(h, None, input_len=1 << 22, seg_fft=1024 if k <= 256 else 2048)
        o = torch.empty((1, 1 << 22), dtype=torch.float32, device="cuda:0")
        fd = time_calls(torch, lambda: plan.convolve(x, out=o), 10, 2)
        td = time_calls(torch, lambda: plan.tdfir(x, out=o), 5, 1)
        out["fig7"].append({"taps": k, "n": 1 << 22, "seg_fft": plan.seg_fft, "fdfir_ms": fd, "tdfir_ms": td,
                            "tdfir_gflops": 8.0 * k * (1 << 22) / (td * 1e-3) / 1e9})
        plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seg-fft", type=int, default=0,
                    help="segment length; 0 = pick with the autotuner among 1024/2048/4096")
    ap.add_argument("--direct", type=int, default=None,
                    help="templates run by direct convolution (whole blocks of 8; -1 = the plan's "
                         "default); default: the autotuner's pick, or the plan's default with --seg-fft")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: the plan, W warmup and K timed fdas_convolve calls, "
                         "nothing else (every direct and overlap-save launch is a headline call)")
    ap.add_argument("--counters-precision", choices=("fp32", "fp16", "bf16"), default="fp32",
                    help="with --counters: the plan's precision (16-bit plans at L = 2048)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tdfir", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-sweeps", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling PMC byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the FT convolution here has no multi-GPU path "
              "(a spectrum or a template group per GPU would need no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_12280_amd import datagen, fdas

    if not os.path.exists(fdas.LIB_PATH):
        from paper_1805_12280_amd import build
        build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)    # 1 GiB
        dst = torch.empty_like(src)
        ms = time_calls(torch, lambda: dst.copy_(src), 5, 2)
        log(f"copy probe: 1 GiB read + 1 GiB write, {ms:.3f} ms, {2 * 2**30 / ms / 1e6:.1f} GB/s")
        return

    log("generating the 85 x 2^22 workload ...")
    w = datagen.ska_workload()
    m, n, k_max = w.bank.num_templates, w.n, w.bank.k_max
    x = torch.from_numpy(w.x).to(dev)
    tuned = None
    if args.seg_fft:
        L = args.seg_fft
    else:
        from paper_1805_12280_amd import autotune
        L, wg, direct, tuned = autotune.tune(w.bank, [x], mode="plane", use_cache=False)
        log(f"autotune (ms per call, L/workgroups per CU/direct templates, 0 = full grid): {tuned} -> "
            f"L = {L}, wg = {wg}, direct = {direct}")
    plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=n, seg_fft=L)
    if not args.seg_fft:
        plan.set_workgroups_per_cu(wg)
        plan.set_direct_templates(direct)
    if args.direct is not None:
        plan.set_direct_templates(args.direct)
    out = torch.empty((m, n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"plan: {plan.info.as_dict()} variant={plan.variant}")

    # untimed back-to-back calls first, so the timed steps see the clock the
    # chip holds under load rather than the idle clock after the tuning;
    # then exactly K steps between two events, and the per-call spread in a
    # pass of its own (events between calls add a small gap to each call)
    if args.counters and args.counters_precision != "fp32":
        plan.close()
        plan = fdas.Plan(w.bank.taps, w.bank.tap_len, input_len=n, seg_fft=2048, precision=args.counters_precision)
        xh = torch.view_as_real(x).to(plan.input_dtype()).contiguous()
        ms = time_calls(torch, lambda: plan.convolve(xh, out=out), args.steps, args.warmup)
        log(f"counters run ({args.counters_precision}): {args.warmup} + {args.steps} calls, {ms:.4f} ms/call")
        print(json.dumps({"counters_run": True, "precision": args.counters_precision, "ms_per_step": ms}),
              flush=True)
        plan.close()
        return
    if args.counters:
        ms = time_calls(torch, lambda: plan.convolve(x, out=out), args.steps, args.warmup)
        log(f"counters run: {args.warmup} + {args.steps} calls, {ms:.4f} ms/call, "
            f"direct templates {plan.info.direct_templates}")
        print(json.dumps({"counters_run": True, "ms_per_step": ms, "seg_fft": L,
                          "direct_templates": plan.info.direct_templates}), flush=True)
        plan.close()
        return
    settle(torch, lambda: plan.convolve(x, out=out))
    ms = time_calls(torch, lambda: plan.convolve(x, out=out), args.steps, args.warmup,
                    mark="fdas_convolve timed steps")
    _, per_step = time_steps(torch, lambda: plan.convolve(x, out=out), args.steps, 0)
    value = m * n / (ms * 1e-3)
    abytes = algorithmic_bytes(n, m, L)
    achieved = abytes / (ms * 1e-3) / 1e9
    traffic = measured_traffic(L, plan.info.direct_templates)
    tflops = nominal_flops(n, m, L, k_max) / (ms * 1e-3) / 1e12
    log(f"fdas_convolve: {ms:.4f} ms/step, {value:.4e} template-samples/s, {achieved:.1f} GB/s")
    md = plan.info.direct_templates
    kernels = split_legs(torch, fdas, w, x, L, md, args.steps, args.warmup)
    log(f"launches: {kernels}")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "template-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded complex Gaussian noise + 3 chirps at amplitude-SNR 8; "
                "85 chirp templates z=-42..42)",
        "config": {"workload": w.name, "templates": m, "n": n, "k_max": k_max,
                   "taps_total": int(w.bank.tap_len.sum()), "seg_fft": L,
                   "workgroups_per_cu": plan.info.wg_per_cu, "direct_templates": md,
                   "autotune_ms": tuned,
                   "path": ("direct convolution of the %d shortest templates on the matrix cores + "
                            "overlap-save FDFIR of the other %d, |y|^2 in both launches" % (md, m - md)
                            if md else "overlap-save FDFIR + |y|^2, one fused launch")},
        # the metric's roofline: algorithmic bytes per launch (input once,
        # plane once, template spectra once) over the launch's mean duration
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": abytes},
        # the overlap-save launch priced as arithmetic: nominal FFT operations
        # of all templates against the FP32 FMA peak the kernels can issue (no
        # packed FP32), with the VALU issue rate read from the committed SQ
        # counters; with a direct split, the per-launch figures are in
        # "launches"
        "alu_roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_UNPACKED_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / FP32_UNPACKED_PEAK_TFLOPS,
                         "published_fp32_vector_peak": FP32_VECTOR_PEAK_TFLOPS,
                         "valu_issue_per_cu_cycle": measured_valu_issue(L, md)},
        "launches": kernels,
        "step_ms": percentiles(per_step),
    }
    sus = sustained(torch, lambda: plan.convolve(x, out=out), ms)
    sus["value"] = m * n / (sus["ms_per_call"] * 1e-3)
    sus["hbm_frac"] = abytes / (sus["ms_per_call"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    result["sustained"] = sus
    result["mall_evicted_ms"] = mall_evicted_ms(torch, lambda: plan.convolve(x, out=out))
    cp = copy_probe_gbs(torch)
    result["roofline"].update({"copy_probe_gbs": cp, "frac_of_copy_probe": achieved / cp})
    log(f"per step {result['step_ms']}, sustained {sus}, MALL evicted {result['mall_evicted_ms']}, "
        f"copy probe {cp:.0f} GB/s")

    if not args.no_tdfir:
        td_steps = max(2, min(args.steps, 5))
        td_ms = time_calls(torch, lambda: plan.tdfir(x, out=out), td_steps, 1)
        td_flops = 8.0 * int(w.bank.tap_len.sum()) * n
        result["tdfir"] = {"ms_per_step": td_ms, "value": m * n / (td_ms * 1e-3),
                           "unit": "template-samples/s",
                           "tflops": td_flops / (td_ms * 1e-3) / 1e12,
                           "frac_fp32_vector_peak": td_flops / (td_ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS}
        log(f"fdas_tdfir: {td_ms:.3f} ms/step")
        plan.convolve(x, out=out)          # leave the FDFIR plane in `out`
        torch.cuda.synchronize()

    if not args.no_mixed:
        plan.convolve(x, out=out)
        result["mixed"] = mixed_leg(torch, fdas, w, x, out, args.steps, args.warmup, ms)

    if not args.no_batch:
        result["batched"] = batched_leg(torch, fdas, max(3, args.steps // 4), 2)
        log(f"batched: {result['batched']['ms_per_step']:.3f} ms/step, "
            f"{result['batched']['value']:.3e} template-samples/s")

    if not args.no_served:
        for key, prec in (("served", "fp32"), ("served_fp16", "fp16")):
            result[key] = served_leg(torch, precision=prec)
            log(f"{key}: " + json.dumps({k: (round(v, 3) if isinstance(v, float) else v)
                                         for k, v in result[key]["saturated"].items()}))
            for st in result[key]["rates"]:
                log(f"  offered {st['offered_fraction']:.2f} x saturated: p50 {st['p50_ms']:.2f} ms, "
                    f"p99 {st['p99_ms']:.2f} ms, {st['jobs_per_s']:.0f} jobs/s")

    if not args.no_sweeps:
        result["sweeps"] = sweeps_leg(torch, fdas)
        for r in result["sweeps"]["fig8"]:
            log(f"fig8 84x421 n=2^{int(math.log2(r['n']))} L={r['seg_fft']}: {r['ms']:.3f} ms "
                f"({r['ms_per_filter'] * 1e3:.1f} us per filter)")
        for r in result["sweeps"]["fig7"]:
            log(f"fig7 1x{r['taps']} taps: FDFIR {r['fdfir_ms']:.3f} ms, TDFIR {r['tdfir_ms']:.3f} ms")

    if not args.no_cpu_baseline:
        log("CPU oracle leg ...")
        cpu, parity = cpu_baseline_leg(w, lambda ns: out[:, :ns].cpu().numpy(), args.cpu_seconds)
        result["cpu_baseline"] = cpu
        result["parity_sample"] = parity
        log(f"cpu oracle: {cpu['value']:.3e} template-samples/s on {cpu['cores']} threads; "
            f"parity on sample: {parity}")

    print(json.dumps(result), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
