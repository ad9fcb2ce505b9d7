"""The seeded synthetic inputs: template bank shape and energy, determinism."""
import numpy as np

from paper_1805_12280_amd import datagen


def test_template_bank_shapes():
    bank = datagen.make_bank(datagen.Z_SKA)
    assert bank.num_templates == 85 and bank.k_max == 101
    assert int(bank.tap_len.sum()) == 5057
    for z, k in zip(bank.z, bank.tap_len):
        assert k == 2 * abs(int(z)) + 17 and k % 2 == 1
    energy = np.sum(np.abs(bank.taps.astype(np.complex128)) ** 2, axis=1)
    assert np.allclose(energy, 1.0, atol=1e-6)
    for t in range(85):
        assert np.all(bank.taps[t, bank.tap_len[t]:] == 0)


def test_zero_drift_template_is_delta_at_8():
    h = datagen.template_taps(0.0).astype(np.complex128)
    assert h.shape == (17,)
    assert abs(h[8] - 1) < 1e-7
    assert np.max(np.abs(np.delete(h, 8))) < 1e-7


def test_toy_workload_deterministic():
    a = datagen.toy_workload()
    b = datagen.toy_workload()
    assert a.x.dtype == np.complex64 and a.x.shape == (1 << 16,)
    assert np.array_equal(a.x, b.x)
    assert a.bank.digest() == b.bank.digest()
    assert list(a.bank.tap_len) == [33, 29, 25, 21, 17, 21, 25, 29, 33]
    assert a.seg_fft == 1024


def test_random_case_ragged():
    x, bank = datagen.random_case(5, 100, 6, 20)
    assert x.shape == (100,) and bank.taps.shape == (6, 20)
    assert bank.tap_len.max() == 20 and bank.tap_len.min() >= 1
