"""Scheduler of the served loop on the CPU, with a fake executor whose results
come from the FP64 oracle and whose batches finish after a simulated time."""
import numpy as np
import pytest

import oracle
from paper_1805_12280_amd import datagen
from paper_1805_12280_amd.serve import Job, Scheduler, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class OracleExecutor:
    """Runs each batch with the oracle; a batch of total n points 'takes'
    n * cost seconds of simulated time."""

    def __init__(self, banks, clock, slots=2, cost=1e-6, topk=4):
        self.banks = banks
        self.clock = clock
        self.slots = slots
        self.cost = cost
        self.topk = topk
        self.started = []

    def footprint(self, bank, n):
        return 8 * n + 1000

    def start(self, bank, jobs):
        self.started.append((bank, [j.job_id for j in jobs], self.clock()))
        return {"bank": bank, "jobs": jobs, "until": self.clock() + self.cost * sum(j.n for j in jobs)}

    def poll(self, token):
        return self.clock() >= token["until"]

    def finish(self, token):
        b = self.banks[token["bank"]]
        out = []
        for j in token["jobs"]:
            P = oracle.power(j.x, b.taps, b.tap_len)
            out.append(oracle.topk(P, self.topk))
        return out


def make_jobs(rng, banks, count, lengths=(200, 500, 1200)):
    jobs = []
    t = 0.0
    for i in range(count):
        t += rng.exponential(1e-4)
        n = int(rng.choice(lengths))
        bank = str(rng.choice(list(banks)))
        x, _ = datagen.random_case(1000 + i, n, 1, 1)
        jobs.append(Job(i, bank, x, n, t))
    return jobs


@pytest.fixture
def banks():
    return {"b3": datagen.random_case(1, 4, 3, 9)[1], "b5": datagen.random_case(2, 4, 5, 17)[1]}


def run(jobs, ex, sched, clock, dt=2e-5):
    pending = sorted(jobs, key=lambda j: j.arrival)
    while pending or not sched.idle:
        while pending and pending[0].arrival <= clock.t:
            sched.submit(pending.pop(0))
        sched.step()
        clock.t += dt


def test_budget_fifo_and_batching(banks):
    rng = np.random.default_rng(0)
    clock = FakeClock()
    ex = OracleExecutor(banks, clock, slots=2)
    budget = 20000
    sched = Scheduler(ex, budget, max_batch=3, clock=clock)
    jobs = make_jobs(rng, banks, 40)
    run(jobs, ex, sched, clock)
    assert len(sched.completed) == 40
    assert sched.peak_in_use <= budget and sched.in_use == 0
    assert max(sched.batches) <= 3
    # admission in arrival order
    adm = sorted(jobs, key=lambda j: j.admitted)
    assert [j.job_id for j in adm] == sorted(j.job_id for j in jobs)
    # one bank per batch, jobs of a bank started in arrival order
    by_id = {j.job_id: j for j in jobs}
    for bank, ids, _ in ex.started:
        assert all(by_id[i].bank == bank for i in ids)
    for bank in banks:
        order = [i for b, ids, _ in ex.started if b == bank for i in ids]
        assert order == sorted(order)


def test_continuous_batching_overlaps(banks):
    """A job arriving while a batch runs starts when a slot frees, before the
    earlier batch has finished."""
    clock = FakeClock()
    ex = OracleExecutor(banks, clock, slots=2, cost=1e-3)
    sched = Scheduler(ex, 10 ** 9, max_batch=8, clock=clock)
    x1, _ = datagen.random_case(5, 1000, 1, 1)
    x2, _ = datagen.random_case(6, 100, 1, 1)
    long_job = Job(0, "b3", x1, 1000, 0.0)
    short_job = Job(1, "b5", x2, 100, 0.01)
    run([long_job, short_job], ex, sched, clock, dt=1e-3)
    assert short_job.started < long_job.done
    assert short_job.done < long_job.done


def test_results_alone_and_in_mix(banks):
    rng = np.random.default_rng(1)
    jobs = make_jobs(rng, banks, 12)
    clock = FakeClock()
    ex = OracleExecutor(banks, clock)
    sched = Scheduler(ex, 50000, max_batch=4, clock=clock)
    run(jobs, ex, sched, clock)
    for j in jobs:
        clock2 = FakeClock()
        solo = Job(j.job_id, j.bank, j.x, j.n, 0.0)
        s2 = Scheduler(OracleExecutor(banks, clock2), 50000, clock=clock2)
        run([solo], None, s2, clock2)
        assert solo.result == j.result
        b = banks[j.bank]
        assert j.result == oracle.topk(oracle.power(j.x, b.taps, b.tap_len), 4)


def test_oversized_job_rejected(banks):
    clock = FakeClock()
    sched = Scheduler(OracleExecutor(banks, clock), 5000, clock=clock)
    x, _ = datagen.random_case(3, 1000, 1, 1)
    with pytest.raises(ValueError):
        sched.submit(Job(0, "b3", x, 1000, 0.0))


def test_latency_stats():
    js = [Job(i, "b", None, 1, 0.0, done=(i + 1) * 1e-3) for i in range(100)]
    st = latency_stats(js)
    assert st["count"] == 100 and abs(st["p50_ms"] - 50.5) < 1.0 and abs(st["p99_ms"] - 99.0) < 1.01


def test_hold_small_batches_while_busy(banks):
    """With max_wait, a small batch waits while the device is busy, so later
    arrivals join it; an idle device starts at once."""
    clock = FakeClock()
    ex = OracleExecutor(banks, clock, slots=3, cost=1e-3)
    sched = Scheduler(ex, 10 ** 9, max_batch=4, max_wait_s=0.05, clock=clock)
    xs = [datagen.random_case(40 + i, 100, 1, 1)[0] for i in range(4)]
    jobs = [Job(i, "b3", xs[i], 100, 0.001 * i) for i in range(4)]
    run(jobs, ex, sched, clock, dt=1e-3)
    assert sched.batches[0] == 1            # idle device: started at once
    assert sched.batches[1] == 3            # the rest waited for each other
