"""The served loop on the GPU: jobs over three resident banks arrive while
others run, are admitted and batched continuously, and each job's top-16
equals the same job run alone; small jobs also match the FP64 oracle."""
import time

import numpy as np
import pytest

import oracle
from fdas_check import FP32_TOL, MIXED_TOL
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
    for i in range(24):
        n = int(rng.choice(lengths, p=[0.5, 0.3, 0.2]))
        bank = str(rng.choice(list(banks)))
        gap = float(rng.exponential(2e-4))
        if i < 4:                   # an opening burst on one bank: batched however fast the device is
            bank, gap = "z21", 0.0
        x, _ = datagen.random_case(500 + i, n, 1, 1)
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
    # oracle check of the smallest jobs
    for j in [a for a in arrivals if a.n == 1 << 16][:3]:
        b = banks[j.bank]
        if precision == "fp32":
            xh = j.x.cpu().numpy()
        else:                                   # the stored 16-bit input, upcast exactly
            v = j.x.float().cpu().numpy()
            xh = (v[:, 0] + 1j * v[:, 1]).astype(np.complex64)
        P = oracle.power(xh, b.taps, b.tap_len)
        want = oracle.topk(P, 16)
        t_, bin_, p_ = fdas.split_candidates(j.result)
        got = list(zip(t_.tolist(), bin_.tolist()))
        assert got[0] == (want[0][0], want[0][1])
        for (tt, bb), pv in zip(got, p_.tolist()):
            assert abs(pv - P[tt, bb]) <= tol * P.max()
    ex.close()
