"""Segment-length and grid autotuner for the FT-convolution plans.

The segment transform length L trades the overlap discarded per segment
(D / L, Section 3.2.2) against the transform cost per point (log2 L); the
paper finds the best N_FT experimentally per device (Section 3.3, Fig. 7/8).
The persistent grid's size (workgroups per CU) trades latency hiding against
how many templates share each forward transform.  For a float32 power plane
a third choice is how many of the shortest templates run by direct
convolution on the matrix cores instead (the time- versus frequency-domain
crossover of Section 3.1 and Fig. 7, taken per template): every whole block
of 8 that the plan can run directly is a candidate, from none upwards.
Here every admissible L in {1024, 2048, 4096, 8192} (K_max <= L/2), each
with the full and the half grid and, for a plane, each direct split, is
timed on the device with the call shape that will be used (plane or
batched top-K), and the fastest setting is kept.  Results are cached in a
JSON file keyed by the device name, bank shape and length profile, so a
server or bench pays the search once per device and bank.
"""
from __future__ import annotations

import json
import os
import time

from . import fdas

CANDIDATES = (1024, 2048, 4096, 8192)


def cache_path() -> str:
    return os.environ.get("FDAS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fdas_tune.json"))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _key(torch, bank, lengths, mode, topk):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    prof = sorted(set(int(n) for n in lengths))
    return f"{dev}|M={bank.num_templates}|K={bank.k_max}|{mode}|k={topk}|n={prof}|count={len(lengths)}"


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def direct_splits(plan) -> list:
    """Direct-template counts a float32 plan can take: 0 and every whole
    block of 8 up to the plan's eligible maximum (whatever was set before
    is restored)."""
    keep = plan.info.direct_templates
    plan.set_direct_templates(plan.num_templates)
    top = plan.info.direct_templates
    plan.set_direct_templates(keep)
    return sorted({0, top} | set(range(8, top, 8)))


def tune(bank, arrays, mode: str = "batched", topk: int = 16, reps: int = 3,
         use_cache: bool = True, candidates=CANDIDATES):
    """Pick (L, workgroups per CU, direct templates) for `bank` on the
    current GPU.

    arrays: CUDA complex64 tensors shaped like the real inputs (their values
    do not matter).  mode: "batched" (top-K over the list; overlap-save
    only, direct = 0) or "plane" (the first array's full power plane, each
    direct split timed).  Returns (best_L, best_wg, best_direct,
    {"L/wg/direct": ms}) with best_wg = 0 meaning the full grid (pass it to
    Plan.set_workgroups_per_cu) and best_direct for
    Plan.set_direct_templates.
    """
    import torch
    path = cache_path()
    key = _key(torch, bank, [a.shape[0] for a in arrays], mode, topk)
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache and "wg" in cache[key] and "direct" in cache[key]:
        ent = cache[key]
        return int(ent["best"]), int(ent["wg"]), int(ent["direct"]), dict(ent["ms"])
    n_max = max(a.shape[0] for a in arrays)
    times = {}
    best = None
    for L in candidates:
        if bank.k_max > L // 2:
            continue
        plan = fdas.Plan(bank.taps, bank.tap_len, input_len=n_max, seg_fft=L)
        full = plan.info.wg_per_cu_max
        splits = direct_splits(plan) if mode == "plane" else [0]
        for wg in sorted({0, max(1, full // 2)}):
            plan.set_workgroups_per_cu(wg)
            for m in splits:
                if mode == "plane":
                    plan.set_direct_templates(m)
                if mode == "batched":
                    ws = torch.empty(plan.batched_workspace_bytes([a.shape[0] for a in arrays], topk),
                                     dtype=torch.uint8, device=arrays[0].device)
                    out = torch.empty((len(arrays), topk, 3), dtype=torch.int32, device=arrays[0].device)
                    fn = lambda: plan.convolve_batched(arrays, topk=topk, out=out, workspace=ws)   # noqa: E731
                else:
                    x = arrays[0]
                    out = torch.empty((bank.num_templates, x.shape[0]), dtype=torch.float32, device=x.device)
                    fn = lambda: plan.convolve(x, out=out)   # noqa: E731
                ms = _time(torch, fn, reps)
                times[f"{L}/{wg}/{m}"] = ms
                if best is None or ms < best[3]:
                    best = (L, wg, m, ms)
        plan.close()
    if best is None:
        raise fdas.FdasError(fdas.FDAS_EINVAL, "no segment length admits this bank")
    if use_cache:
        cache[key] = {"best": best[0], "wg": best[1], "direct": best[2], "ms": times,
                      "when": time.strftime("%Y-%m-%d %H:%M:%S")}
        _store_cache(path, cache)
    return best[0], best[1], best[2], times
