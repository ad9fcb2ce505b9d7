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

    def __init__(self, plan):
        self._plan = plan

    @property
    def direct_templates(self):
        return self._plan.m


class FakePlan:
    """Stands in for fdas.Plan: records its segment length, grid cap and
    direct split, and its calls tell the fake timer which (L, workgroups per
    CU, direct templates) ran.  It can take up to 16 templates directly
    (two blocks of 8)."""
    made = []
    max_direct = 16

    def __init__(self, taps, tap_len, input_len, seg_fft):
        self.L, self.wg, self.m = seg_fft, 0, 0
        self.num_templates = len(tap_len)
        self.info = _Info(self)
        FakePlan.made.append(seg_fft)

    def set_workgroups_per_cu(self, wg):
        self.wg = wg

    def set_direct_templates(self, m):
        self.m = min(m, self.max_direct, self.num_templates)

    def batched_workspace_bytes(self, lengths, topk):
        return 64

    def convolve_batched(self, arrays, topk, out, workspace):
        return (self.L, self.wg, self.m)

    def convolve(self, x, out):
        return (self.L, self.wg, self.m)

    def close(self):
        pass


# ms per (L, workgroups per CU, direct templates): 2048 with the half grid
# is the fastest overlap-save setting, and 8 direct templates beat 0 and 16
TABLE = {(1024, 0): 5.0, (1024, 2): 6.0, (2048, 0): 4.5, (2048, 2): 4.0,
         (4096, 0): 4.8, (4096, 2): 7.0, (8192, 0): 9.0, (8192, 2): 9.5}
DIRECT = {0: 0.0, 8: -0.5, 16: 0.25}


def _ms(key):
    L, wg, m = key
    return TABLE[(L, wg)] + DIRECT[m]


@pytest.fixture
def fake(monkeypatch, tmp_path):
    FakePlan.made = []
    monkeypatch.setattr(fdas, "Plan", FakePlan)
    monkeypatch.setattr(autotune, "_time", lambda torch_, fn, reps: _ms(fn()))
    monkeypatch.setattr(autotune, "_key", lambda torch_, bank, lengths, mode, topk:
                        f"dev|M={bank.num_templates}|K={bank.k_max}|{mode}|k={topk}|n={sorted(set(lengths))}")
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(path))
    return path


def _bank(k_max):
    _, bank = datagen.random_case(5, 8, 20, k_max, ragged=False)
    return bank


def test_picks_fastest_pair_and_times_every_admissible_one(fake):
    arrays = [torch.zeros(1000, dtype=torch.complex64), torch.zeros(3000, dtype=torch.complex64)]
    L, wg, m, ms = autotune.tune(_bank(101), arrays, mode="batched")
    # batched calls are overlap-save only: no direct split is timed
    assert (L, wg, m) == (2048, 2, 0)
    assert ms == {f"{l}/{w}/0": v for (l, w), v in TABLE.items()}
    assert FakePlan.made == [1024, 2048, 4096, 8192]


def test_plane_times_every_direct_split(fake):
    L, wg, m, ms = autotune.tune(_bank(101), [torch.zeros(1000, dtype=torch.complex64)], mode="plane")
    assert (L, wg, m) == (2048, 2, 8)
    assert ms == {f"{l}/{w}/{d}": v + DIRECT[d] for (l, w), v in TABLE.items() for d in (0, 8, 16)}


def test_direct_splits_are_whole_blocks_up_to_the_eligible_maximum():
    p = FakePlan(None, [1] * 40, 10, 1024)
    p.max_direct = 24
    p.set_direct_templates(8)
    assert autotune.direct_splits(p) == [0, 8, 16, 24]
    assert p.m == 8                                   # the previous split is restored
    p.max_direct = 0
    assert autotune.direct_splits(p) == [0]
    # a bank of 5 templates all eligible: one partial block
    q = FakePlan(None, [1] * 5, 10, 1024)
    q.max_direct = 5
    assert autotune.direct_splits(q) == [0, 5]


def test_skips_lengths_the_bank_does_not_fit(fake):
    # K_max = 1500 needs L >= 3000: only 4096 and 8192 are timed
    L, wg, m, ms = autotune.tune(_bank(1500), [torch.zeros(100, dtype=torch.complex64)], mode="plane")
    assert FakePlan.made == [4096, 8192]
    assert (L, wg, m) == (4096, 0, 8)
    assert set(ms) == {f"{l}/{w}/{d}" for l in (4096, 8192) for w in (0, 2) for d in (0, 8, 16)}


def test_no_admissible_length_raises(fake):
    with pytest.raises(fdas.FdasError):
        autotune.tune(_bank(4097), [torch.zeros(100, dtype=torch.complex64)], mode="plane")


def test_cache_is_written_and_reused(fake, monkeypatch):
    arrays = [torch.zeros(1000, dtype=torch.complex64)]
    first = autotune.tune(_bank(101), arrays)
    ent = json.loads(fake.read_text())
    (key, val), = ent.items()
    assert val["best"] == 2048 and val["wg"] == 2 and val["direct"] == 0
    # a second call with the same shape does not build a plan
    FakePlan.made = []
    assert autotune.tune(_bank(101), arrays) == first
    assert FakePlan.made == []
    # another length profile is a new entry
    autotune.tune(_bank(101), [torch.zeros(2000, dtype=torch.complex64)])
    assert len(json.loads(fake.read_text())) == 2 and FakePlan.made == [1024, 2048, 4096, 8192]


def test_entry_without_direct_split_is_tuned_again(fake):
    arrays = [torch.zeros(1000, dtype=torch.complex64)]
    autotune.tune(_bank(101), arrays, mode="plane")
    ent = json.loads(fake.read_text())
    (key, val), = ent.items()
    del val["direct"]
    fake.write_text(json.dumps(ent))
    FakePlan.made = []
    assert autotune.tune(_bank(101), arrays, mode="plane")[:3] == (2048, 2, 8)
    assert FakePlan.made == [1024, 2048, 4096, 8192]


def test_unreadable_cache_is_ignored(fake):
    fake.write_text("{not json")
    L, wg, m, _ = autotune.tune(_bank(101), [torch.zeros(10, dtype=torch.complex64)])
    assert (L, wg, m) == (2048, 2, 0)
    assert json.loads(fake.read_text())            # rewritten whole


def test_use_cache_false_neither_reads_nor_writes(fake):
    autotune.tune(_bank(101), [torch.zeros(10, dtype=torch.complex64)], use_cache=False)
    assert not fake.exists()
    assert np.array_equal(np.array(FakePlan.made), np.array([1024, 2048, 4096, 8192]))
