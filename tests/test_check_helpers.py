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


def _plane_topk_list(P, k):
    t, i = np.unravel_index(np.argsort(-P, axis=None, kind="stable"), P.shape)
    return [(int(a), int(b), float(P[a, b])) for a, b in zip(t[:k], i[:k])]


def test_oracle_topk_streamed_equals_whole_plane():
    """The block-streamed oracle top-k equals oracle.topk of the whole plane,
    whatever the block size, ties included; its check accepts the exact list
    and rejects a list with a cell dropped, reordered or mis-valued."""
    from paper_1805_12280_amd import datagen
    from fdas_check import OracleTopk
    import pytest
    x, bank = datagen.random_case(41, 3000, 7, 25)
    P = oracle.power(x, bank.taps, bank.tap_len)
    want = oracle.topk(P, 16)
    for rpb in (1, 3, 7):
        o = OracleTopk(x, bank.taps, bank.tap_len, k=16, rows_per_block=rpb)
        assert o.top == want and o.maxref == P.max()
    t = np.array([c[0] for c in want])
    b = np.array([c[1] for c in want])
    p = np.array([c[2] for c in want], dtype=np.float32)
    o.check(x, bank.taps, bank.tap_len, t, b, p)
    with pytest.raises(AssertionError):           # the 16th cell replaced by a weak one
        t2, b2, p2 = t.copy(), b.copy(), p.copy()
        weak = np.unravel_index(np.argmin(P), P.shape)
        t2[15], b2[15], p2[15] = weak[0], weak[1], P[weak]
        o.check(x, bank.taps, bank.tap_len, t2, b2, p2)
    with pytest.raises(AssertionError):           # two cells swapped out of order
        o.check(x, bank.taps, bank.tap_len, t[[1, 0] + list(range(2, 16))], b[[1, 0] + list(range(2, 16))],
                p[[1, 0] + list(range(2, 16))])
    with pytest.raises(AssertionError):           # a reported power off by 1e-3 of the peak
        p3 = p.copy()
        p3[4] += 1e-3 * P.max()
        o.check(x, bank.taps, bank.tap_len, t, b, p3)
    # ties: a plane of equal cells keeps (t asc, i asc) order
    xz = np.zeros(50, np.complex64)
    o = OracleTopk(xz, bank.taps[:3], bank.tap_len[:3], k=5, rows_per_block=2)
    assert o.top == [(0, i, 0.0) for i in range(5)]
    assert _plane_topk_list(np.zeros((3, 50)), 5) == [(0, i, 0.0) for i in range(5)]
