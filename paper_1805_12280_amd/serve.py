"""Served FT convolution: a continuous-batching request loop.

Jobs (one DM-trial spectrum each, against one of several resident template
banks) arrive over time; the server keeps one plan per bank resident on the
device, admits jobs while their device footprint fits a budget, and, whenever
an execution slot (a stream) is free, launches the oldest admitted jobs of
one bank as a single batched call (fdas_convolve_batched: one persistent
launch over all their segments and templates, each spectrum reduced to its
top-K cells).  Several slots run at once, so work admitted while other
batches are on the device overlaps with them; a batch's footprint is
released when its completion event has fired.

The scheduler is plain Python over a small executor interface, so its policy
(admission, batching, ordering, latency accounting) runs on the CPU against
any executor; GpuExecutor is the one that drives the library.  A
latency-sensitive loop should run with Python's cyclic garbage collector
paused (collecting between bursts): one full collection inside a run stalled
a scheduler step by about 40 ms.
"""
from __future__ import annotations

import collections
import dataclasses
import time


@dataclasses.dataclass
class Job:
    job_id: int
    bank: str
    x: object                   # the spectrum (for GpuExecutor: a CUDA complex64 tensor, or
                                #   [n, 2] 16-bit pairs for a 16-bit executor)
    n: int
    arrival: float              # scheduler clock time of arrival
    admitted: float | None = None
    started: float | None = None
    done: float | None = None
    result: object = None       # per-job candidates [topk, 3] (t, bin, p bits)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class Scheduler:
    """Continuous batching with admission by device footprint.

    executor: object with
        slots                       number of batches that may run at once
        footprint(bank, n) -> int   device bytes a job holds while admitted
        start(bank, jobs) -> token  launch one batched call (non-blocking)
        poll(token) -> bool         True once the call has finished
        finish(token) -> list       per-job results, in the order given
    budget_bytes: admitted jobs' footprints never exceed this.
    max_batch: jobs per batched call.
    max_wait_s: while other batches are running, a batch smaller than
        max_batch is held until its oldest job has waited this long, so light
        load does not fragment the device into many one-job launches (an idle
        device starts a batch at once).
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 16, max_wait_s: float = 0.0,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_wait = float(max_wait_s)
        self.clock = clock
        self.waiting = collections.deque()               # arrived, not admitted
        self.admitted = collections.OrderedDict()        # bank -> deque of jobs
        self.in_use = 0
        self.peak_in_use = 0
        self.running = []                                # (token, bank, jobs, bytes)
        self.completed = []
        self.batches = []                                # sizes of launched batches

    # -- intake ---------------------------------------------------------------
    def submit(self, job: Job):
        fp = self.ex.footprint(job.bank, job.n)
        if fp > self.budget:
            raise ValueError(f"job {job.job_id} needs {fp} bytes, budget is {self.budget}")
        self.waiting.append(job)

    def _admit(self):
        now = self.clock()
        while self.waiting:
            job = self.waiting[0]
            fp = self.ex.footprint(job.bank, job.n)
            if self.in_use + fp > self.budget:
                break                                    # FIFO: later jobs wait too
            self.waiting.popleft()
            self.in_use += fp
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            job.admitted = now
            self.admitted.setdefault(job.bank, collections.deque()).append(job)

    def _launch(self):
        while len(self.running) < self.ex.slots:
            # the bank whose oldest admitted job arrived first
            best = None
            for bank, q in self.admitted.items():
                if q and (best is None or q[0].arrival < self.admitted[best][0].arrival):
                    best = bank
            if best is None:
                return
            q = self.admitted[best]
            now = self.clock()
            if self.running and len(q) < self.max_batch and now - q[0].arrival < self.max_wait:
                return
            jobs = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
            for j in jobs:
                j.started = now
            token = self.ex.start(best, jobs)
            nbytes = sum(self.ex.footprint(best, j.n) for j in jobs)
            self.running.append((token, best, jobs, nbytes))
            self.batches.append(len(jobs))

    def _reap(self):
        still = []
        for token, bank, jobs, nbytes in self.running:
            if self.ex.poll(token):
                now = self.clock()
                for j, r in zip(jobs, self.ex.finish(token)):
                    j.result = r
                    j.done = now
                    self.completed.append(j)
                self.in_use -= nbytes
            else:
                still.append((token, bank, jobs, nbytes))
        self.running = still

    def step(self):
        """One scheduler pass: retire finished batches, admit, launch."""
        self._reap()
        self._admit()
        self._launch()

    @property
    def idle(self):
        return not (self.waiting or self.running or any(self.admitted.values()))

    def drain(self, sleep_s: float = 0.0):
        while not self.idle:
            self.step()
            if sleep_s:
                time.sleep(sleep_s)


def latency_stats(jobs):
    lat = sorted(j.latency for j in jobs if j.latency is not None)
    if not lat:
        return {"count": 0}
    pick = lambda q: lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]   # noqa: E731
    return {"count": len(lat), "p50_ms": 1e3 * pick(0.50), "p99_ms": 1e3 * pick(0.99),
            "mean_ms": 1e3 * sum(lat) / len(lat), "max_ms": 1e3 * lat[-1]}


class GpuExecutor:
    """Batched calls on `slots` streams, with one resident plan per bank."""

    def __init__(self, banks: dict, input_len: int, topk: int = 16, slots: int = 2,
                 seg_fft: dict | None = None, device: str = "cuda:0", precision: str = "fp32",
                 timeline: bool = False):
        import torch
        from . import fdas
        self.torch = torch
        # timeline: record timing events around every batch on its stream, so
        # the device-side interval each batch was in flight can be read back
        # (intervals()); off by default (events with timing cost a little)
        self.timeline = bool(timeline)
        self.spans = []
        self.origin = None
        self.fdas = fdas
        self.topk = int(topk)
        self.slots = int(slots)
        self.device = torch.device(device)
        self.precision = precision
        self.plans = {}
        for name, bank in banks.items():
            L = (seg_fft or {}).get(name, 2048)
            self.plans[name] = fdas.Plan(bank.taps, bank.tap_len, input_len=input_len, seg_fft=L,
                                         precision=precision)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        self.free_streams = list(range(self.slots))
        # per-stream workspace and candidate buffers, grown on demand and then
        # reused (each batch only allocates the small copy of its candidates)
        self.ws = [None] * self.slots
        self.outs = [None] * self.slots

    def reserve(self, max_batch: int, max_n: int):
        """Allocate every slot's workspace and candidate buffer for the
        largest batch up front, so no call allocates device memory (a first
        allocation waits for the device), and run one small call of every
        bank on every slot, so each stream's first use (which sets up its
        hardware queue) happens here rather than inside a measured run."""
        torch = self.torch
        need = max(p.batched_workspace_bytes([int(max_n)] * int(max_batch), self.topk) for p in self.plans.values())
        for sid, st in enumerate(self.streams):
            with torch.cuda.stream(st):
                if self.ws[sid] is None or self.ws[sid].numel() < need:
                    self.ws[sid] = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=self.device)
                if self.outs[sid] is None or self.outs[sid].shape[0] < max_batch:
                    self.outs[sid] = torch.empty((max(max_batch, 16), self.topk, 3), dtype=torch.int32,
                                                 device=self.device)
        if self.precision == "fp32":
            probe = torch.zeros(4096, dtype=torch.complex64, device=self.device)
        else:
            dt = torch.float16 if self.precision == "fp16" else torch.bfloat16
            probe = torch.zeros((4096, 2), dtype=dt, device=self.device)
        torch.cuda.synchronize(self.device)
        for sid, st in enumerate(self.streams):
            with torch.cuda.stream(st):
                for plan in self.plans.values():
                    plan.convolve_batched([probe], topk=self.topk, out=self.outs[sid][:1], workspace=self.ws[sid])
        torch.cuda.synchronize(self.device)

    def footprint(self, bank, n):
        # the spectrum while it is admitted, its share of the batch workspace
        # (bounded by one candidate list per workgroup, plus for a 16-bit plan
        # the staged spectra: 8 KB per segment of about 1900 points), and
        # its candidates
        if self.precision == "fp32":
            return 8 * int(n) + 64 * 1024 + 12 * self.topk
        return 4 * int(n) + 5 * int(n) + 80 * 1024 + 12 * self.topk

    def start(self, bank, jobs):
        torch = self.torch
        sid = self.free_streams.pop()
        st = self.streams[sid]
        plan = self.plans[bank]
        need = plan.batched_workspace_bytes([j.n for j in jobs], self.topk)
        st.wait_stream(torch.cuda.current_stream(self.device))
        if self.timeline and self.origin is None:
            self.origin = torch.cuda.Event(enable_timing=True)
            self.origin.record(torch.cuda.current_stream(self.device))
            st.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(st):
            if self.timeline:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(st)
            # allocated on the slot's own stream: a replaced buffer is only
            # reused in that stream's order
            if self.ws[sid] is None or self.ws[sid].numel() < need:
                self.ws[sid] = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=self.device)
            if self.outs[sid] is None or self.outs[sid].shape[0] < len(jobs):
                self.outs[sid] = torch.empty((max(len(jobs), 16), self.topk, 3), dtype=torch.int32,
                                             device=self.device)
            out = self.outs[sid][:len(jobs)]
            plan.convolve_batched([j.x for j in jobs], topk=self.topk, out=out, workspace=self.ws[sid])
            res = out.clone()
            ev = torch.cuda.Event(enable_timing=self.timeline)
            ev.record(st)
            if self.timeline:
                self.spans.append((ev0, ev, [j.job_id for j in jobs]))
        return (sid, ev, res, jobs)

    def intervals(self):
        """(start_ms, end_ms, job ids) of every batch on the device timeline,
        relative to the first batch's launch (timeline=True; call after the
        device is synchronised): start is when the batch's stream reached it,
        end when its results were copied out."""
        return [(self.origin.elapsed_time(a), self.origin.elapsed_time(b), ids) for a, b, ids in self.spans]

    def poll(self, token):
        return token[1].query()

    def finish(self, token):
        sid, ev, res, jobs = token
        self.free_streams.append(sid)
        return [res[i] for i in range(len(jobs))]

    def close(self):
        for p in self.plans.values():
            p.close()
