"""CPU checks of the comparison helpers used by the GPU parity tests."""
import numpy as np

import oracle
from fdas_check import PlaneStats


def test_streamed_topk_matches_definition():
    rng = np.random.default_rng(7)
    ref = rng.random((13, 500)) * 10
    gpu = ref + rng.normal(0, 1e-7, ref.shape)
    st = PlaneStats(k=16)
    for r0 in range(0, 13, 4):
        rows = list(range(r0, min(13, r0 + 4)))
        st.add(rows, gpu[rows], ref[rows])
    want = oracle.topk(ref, 16)
    assert [(t, i) for t, i, _ in st.topk("ref")] == [(t, i) for t, i, _ in want]
    ok, bad = st.topk_agree()
    assert ok, bad
    assert st.norm_err < 1e-6


def test_topk_disagreement_detected():
    ref = np.zeros((2, 100))
    ref[0, 10] = 100.0
    ref[1, 20] = 50.0
    gpu = ref.copy()
    gpu[1, 20] = 0.0
    gpu[1, 30] = 60.0
    st = PlaneStats(k=2)
    st.add([0, 1], gpu, ref)
    ok, bad = st.topk_agree(tol=1e-4)
    assert not ok and bad
    assert st.norm_err == 0.6
