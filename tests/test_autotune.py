"""Host logic of the segment-length and grid autotuner
(paper_1805_12280_amd/autotune.py): which candidates it times, which one it
keeps, and its cache.  The plan and the timer are replaced by fakes, so no
GPU is used; the timings on a real device are exercised by bench.py."""
import json
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1805_12280_amd import autotune, datagen, fdas  # noqa: E402


class _Info:
    wg_per_cu_max = 4


class FakePlan:
    """Stands in for fdas.Plan: records its segment length and grid cap, and
    its calls tell the fake timer which (L, workgroups per CU) ran."""
    made = []

    def __init__(self, taps, tap_len, input_len, seg_fft):
        self.L, self.wg, self.info = seg_fft, 0, _Info()
        FakePlan.made.append(seg_fft)

    def set_workgroups_per_cu(self, wg):
        self.wg = wg

    def batched_workspace_bytes(self, lengths, topk):
        return 64

    def convolve_batched(self, arrays, topk, out, workspace):
        return (self.L, self.wg)

    def convolve(self, x, out):
        return (self.L, self.wg)

    def close(self):
        pass


# ms per (L, workgroups per CU): 2048 with the half grid is the fastest
TABLE = {(1024, 0): 5.0, (1024, 2): 6.0, (2048, 0): 4.5, (2048, 2): 4.0,
         (4096, 0): 4.8, (4096, 2): 7.0, (8192, 0): 9.0, (8192, 2): 9.5}


@pytest.fixture
def fake(monkeypatch, tmp_path):
    FakePlan.made = []
    monkeypatch.setattr(fdas, "Plan", FakePlan)
    monkeypatch.setattr(autotune, "_time", lambda torch_, fn, reps: TABLE[fn()])
    monkeypatch.setattr(autotune, "_key", lambda torch_, bank, lengths, mode, topk:
                        f"dev|M={bank.num_templates}|K={bank.k_max}|{mode}|k={topk}|n={sorted(set(lengths))}")
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(path))
    return path


def _bank(k_max):
    _, bank = datagen.random_case(5, 8, 3, k_max, ragged=False)
    return bank


def test_picks_fastest_pair_and_times_every_admissible_one(fake):
    arrays = [torch.zeros(1000, dtype=torch.complex64), torch.zeros(3000, dtype=torch.complex64)]
    L, wg, ms = autotune.tune(_bank(101), arrays, mode="batched")
    assert (L, wg) == (2048, 2)
    assert ms == {f"{l}/{w}": v for (l, w), v in TABLE.items()}
    assert FakePlan.made == [1024, 2048, 4096, 8192]


def test_skips_lengths_the_bank_does_not_fit(fake):
    # K_max = 1500 needs L >= 3000: only 4096 and 8192 are timed
    L, wg, ms = autotune.tune(_bank(1500), [torch.zeros(100, dtype=torch.complex64)], mode="plane")
    assert FakePlan.made == [4096, 8192]
    assert (L, wg) == (4096, 0) and set(ms) == {"4096/0", "4096/2", "8192/0", "8192/2"}


def test_no_admissible_length_raises(fake):
    with pytest.raises(fdas.FdasError):
        autotune.tune(_bank(4097), [torch.zeros(100, dtype=torch.complex64)], mode="plane")


def test_cache_is_written_and_reused(fake, monkeypatch):
    arrays = [torch.zeros(1000, dtype=torch.complex64)]
    first = autotune.tune(_bank(101), arrays)
    ent = json.loads(fake.read_text())
    (key, val), = ent.items()
    assert val["best"] == 2048 and val["wg"] == 2
    # a second call with the same shape does not build a plan
    FakePlan.made = []
    assert autotune.tune(_bank(101), arrays) == first
    assert FakePlan.made == []
    # another length profile is a new entry
    autotune.tune(_bank(101), [torch.zeros(2000, dtype=torch.complex64)])
    assert len(json.loads(fake.read_text())) == 2 and FakePlan.made == [1024, 2048, 4096, 8192]


def test_unreadable_cache_is_ignored(fake):
    fake.write_text("{not json")
    L, wg, _ = autotune.tune(_bank(101), [torch.zeros(10, dtype=torch.complex64)])
    assert (L, wg) == (2048, 2)
    assert json.loads(fake.read_text())            # rewritten whole


def test_use_cache_false_neither_reads_nor_writes(fake):
    autotune.tune(_bank(101), [torch.zeros(10, dtype=torch.complex64)], use_cache=False)
    assert not fake.exists()
    assert np.array_equal(np.array(FakePlan.made), np.array([1024, 2048, 4096, 8192]))
