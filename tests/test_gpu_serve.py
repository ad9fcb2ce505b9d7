"""The served loop on the GPU: jobs over three resident banks arrive while
others run, are admitted and batched continuously, and each job's top-16
equals the same job run alone; small jobs also match the FP64 oracle."""
import time

import numpy as np
import pytest

import oracle
from fdas_check import FP32_TOL, MIXED_TOL, OracleTopk
from paper_1805_12280_amd import datagen

pytestmark = pytest.mark.gpu

BANKS = {"z10": tuple(range(-10, 11)), "z21": tuple(range(-21, 22)), "z42": tuple(range(-42, 43))}


@pytest.fixture(scope="module")
def env():
    import os
    import torch
    from paper_1805_12280_amd import fdas
    assert torch.cuda.is_available()
    if not os.path.exists(fdas.LIB_PATH):
        from paper_1805_12280_amd import build
        build.build()
    return torch, fdas


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_mix_equals_alone(env, precision):
    torch, fdas = env
    tol = FP32_TOL if precision == "fp32" else MIXED_TOL
    from paper_1805_12280_amd.serve import GpuExecutor, Job, Scheduler, latency_stats
    banks = {k: datagen.make_bank(v) for k, v in BANKS.items()}
    rng = np.random.default_rng(4)
    lengths = [1 << 16, 1 << 17, 1 << 18]
    jobs_spec = []
    originals = {}
    for i in range(24):
        n = int(rng.choice(lengths, p=[0.5, 0.3, 0.2]))
        bank = str(rng.choice(list(banks)))
        gap = float(rng.exponential(2e-4))
        if i < 4:                   # an opening burst on one bank: batched however fast the device is
            bank, gap = "z21", 0.0
        x, _ = datagen.random_case(500 + i, n, 1, 1)
        originals[i] = x
        xd = torch.from_numpy(x).cuda()
        if precision == "fp16":
            xd = torch.view_as_real(xd).to(torch.float16).contiguous()
        jobs_spec.append((i, bank, xd, n, gap))
    seg = {"z10": 1024, "z21": 2048, "z42": 1024} if precision == "fp32" else {k: 2048 for k in banks}
    ex = GpuExecutor(banks, input_len=1 << 18, topk=16, slots=3, seg_fft=seg, precision=precision)
    sched = Scheduler(ex, budget_bytes=16 << 20, max_batch=6, max_wait_s=2e-3)
    t0 = time.perf_counter()
    arrivals, t = [], t0
    for i, bank, x, n, gap in jobs_spec:
        t += gap
        arrivals.append(Job(i, bank, x, n, t))
    pending = list(arrivals)
    while pending or not sched.idle:
        now = time.perf_counter()
        while pending and pending[0].arrival <= now:
            sched.submit(pending.pop(0))
        sched.step()
    torch.cuda.synchronize()
    assert len(sched.completed) == 24 and sched.peak_in_use <= 16 << 20
    assert max(sched.batches) > 1, sched.batches        # jobs were batched
    print(latency_stats(sched.completed), sched.batches, flush=True)
    for j in arrivals:
        solo = Scheduler(ex, budget_bytes=16 << 20)
        sj = Job(j.job_id, j.bank, j.x, j.n, time.perf_counter())
        solo.submit(sj)
        solo.drain()
        torch.cuda.synchronize()
        assert torch.equal(sj.result, j.result), j.job_id
    # oracle check of the smallest jobs: the full top-16 under the near-tie
    # rule, against the oracle on the original complex64 spectrum (for the
    # 16-bit executor too: its bar covers the rounding of the stored input)
    for j in [a for a in arrivals if a.n == 1 << 16][:3]:
        b = banks[j.bank]
        xh = originals[j.job_id]
        t_, bin_, p_ = fdas.split_candidates(j.result)
        OracleTopk(xh, b.taps, b.tap_len, k=16).check(xh, b.taps, b.tap_len, t_.cpu().numpy(),
                                                      bin_.cpu().numpy(), p_.cpu().numpy(), tol=tol)
    ex.close()


# Jobs of the served workload's own shapes: spectra of 2^18, 2^20 and 2^22
# points on the 21-, 43- and 85-template banks, two of each of the largest.
SHAPES = [("z42", 1 << 22), ("z42", 1 << 20), ("z21", 1 << 20), ("z10", 1 << 18), ("z42", 1 << 18),
          ("z21", 1 << 22), ("z10", 1 << 20), ("z42", 1 << 20), ("z42", 1 << 22), ("z21", 1 << 18)]


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_served_shapes_against_oracle(env, precision):
    """A burst of jobs at the served workload's shapes (up to 85 templates x
    2^22 points) through the continuous-batching loop, several batches in
    flight at once: each job's top-16 equals the same job run alone
    (bitwise) and the top-16 of the FP64 oracle's whole plane of its
    original complex64 spectrum (near-tie rule at the path's bar); the
    device timeline shows batches overlapping."""
    torch, fdas = env
    tol = FP32_TOL if precision == "fp32" else MIXED_TOL
    from paper_1805_12280_amd.serve import GpuExecutor, Job, Scheduler
    banks = {k: datagen.make_bank(v) for k, v in BANKS.items()}
    rng = np.random.default_rng(42)
    noise_rng = np.random.default_rng(43)
    originals, jobs = {}, []
    for i, (bank, n) in enumerate(SHAPES):
        chirps = []
        if i % 3 == 0:              # some jobs carry an injected chirp
            chirps = [datagen.Chirp(int(rng.integers(1000, n - 1000)), float(rng.uniform(-8, 8)),
                                    float(np.sqrt(128.0 / n)))]
        x = datagen.make_spectrum(n, tuple(chirps), noise_rng)
        originals[i] = x
        xd = torch.from_numpy(x).cuda()
        if precision == "fp16":
            xd = torch.view_as_real(xd).to(torch.float16).contiguous()
        jobs.append(Job(i, bank, xd, n, 0.0))
    seg = {k: 2048 for k in banks}
    ex = GpuExecutor(banks, input_len=1 << 22, topk=16, slots=3, seg_fft=seg, precision=precision,
                     timeline=True)
    ex.reserve(2, 1 << 22)
    sched = Scheduler(ex, budget_bytes=1 << 30, max_batch=2, max_wait_s=0.0)
    now = time.perf_counter()
    for j in jobs:
        j.arrival = now
        sched.submit(j)
    sched.drain()
    torch.cuda.synchronize()
    assert len(sched.completed) == len(jobs)
    spans = ex.intervals()
    print("batches (start ms, end ms, jobs):", [(round(a, 3), round(b, 3), ids) for a, b, ids in spans], flush=True)
    overlap = any(a0 < b1 and a1 < b0 for k, (a0, b0, _) in enumerate(spans) for (a1, b1, _) in spans[k + 1:])
    assert overlap, spans
    for j in jobs:
        solo = Scheduler(ex, budget_bytes=1 << 30)
        sj = Job(j.job_id, j.bank, j.x, j.n, time.perf_counter())
        solo.submit(sj)
        solo.drain()
        torch.cuda.synchronize()
        assert torch.equal(sj.result, j.result), j.job_id
        b = banks[j.bank]
        xh = originals[j.job_id]
        t_, bin_, p_ = fdas.split_candidates(j.result)
        err = OracleTopk(xh, b.taps, b.tap_len, k=16, rows_per_block=17).check(
            xh, b.taps, b.tap_len, t_.cpu().numpy(), bin_.cpu().numpy(), p_.cpu().numpy(), tol=tol)
        print(f"[served {precision}] job {j.job_id} {j.bank} n={j.n}: top-16 ok, power err/peak {err:.2e}",
              flush=True)
    ex.close()
