"""Seeded synthetic inputs for the FT-convolution (FDAS) workload.

This module only *makes inputs*: the complex spectrum that is filtered and
the bank of complex FIR templates.  It holds none of the filtering
arithmetic (no convolution, no segment transform, no power), so the CPU
oracle and the GPU library can both be fed from it without sharing any
step of the method.

Workload shape (paper, Section 3): one DM-trial spectrum of 2^22 complex
single-precision points is filtered by a bank of acceleration templates,
each a complex FIR filter; the FOP keeps one row per template.  The paper
does not say how templates are built, so the bank follows the usual
acceleration-search construction: template z is the DFT of a unit chirp
exp(i*pi*z*t^2) on t in [0, 1) sampled at 4096 points, cut to
2*ceil(|z|)+17 taps centred on its peak bin and scaled to unit energy.

Every array is produced in float64 and rounded once to complex64; those
complex64 arrays are the exact inputs both sides consume.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

SEED_BASE = 180512280
TEMPLATE_DFT_LEN = 4096


def template_len(z: float) -> int:
    """Tap count of template z: 2*ceil(|z|)+17 (always odd)."""
    return 2 * int(math.ceil(abs(z))) + 17


def template_taps(z: float) -> np.ndarray:
    """complex64 taps of the acceleration template for drift z.

    c_z[n] = exp(i*pi*z*(n/4096)^2), C_z = DFT_4096(c_z).  The peak bin b*
    is the first maximum of |C_z| scanning signed bins -2048..2047 in
    ascending order; the taps are C_z[(b* - (K-1)/2 + k) mod 4096], k < K,
    scaled so that sum |h|^2 = 1.
    """
    n = np.arange(TEMPLATE_DFT_LEN, dtype=np.float64)
    c = np.exp(1j * np.pi * z * (n / TEMPLATE_DFT_LEN) ** 2)
    spec = np.fft.fft(c)
    signed = np.arange(-TEMPLATE_DFT_LEN // 2, TEMPLATE_DFT_LEN // 2)
    mag = np.abs(spec[signed % TEMPLATE_DFT_LEN])
    b_star = int(signed[int(np.argmax(mag))])
    k_len = template_len(z)
    idx = (b_star - (k_len - 1) // 2 + np.arange(k_len)) % TEMPLATE_DFT_LEN
    h = spec[idx]
    h = h / np.sqrt(np.sum(np.abs(h) ** 2))
    return h.astype(np.complex64)


@dataclasses.dataclass(frozen=True)
class Bank:
    """A template bank: taps [M][K_max] complex64 (zero-padded), tap_len[M]."""

    z: np.ndarray          # float64 [M]
    taps: np.ndarray       # complex64 [M][K_max], zero beyond tap_len[t]
    tap_len: np.ndarray    # int32 [M]

    @property
    def num_templates(self) -> int:
        return int(self.taps.shape[0])

    @property
    def k_max(self) -> int:
        return int(self.taps.shape[1])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.taps).tobytes())
        h.update(np.ascontiguousarray(self.tap_len).tobytes())
        return h.hexdigest()[:16]


def make_bank(z_values) -> Bank:
    z = np.asarray(list(z_values), dtype=np.float64)
    rows = [template_taps(float(v)) for v in z]
    k_max = max(len(r) for r in rows)
    taps = np.zeros((len(rows), k_max), dtype=np.complex64)
    for t, r in enumerate(rows):
        taps[t, : len(r)] = r
    tap_len = np.array([len(r) for r in rows], dtype=np.int32)
    return Bank(z=z, taps=taps, tap_len=tap_len)


@dataclasses.dataclass(frozen=True)
class Chirp:
    r0: float      # starting Fourier bin
    z0: float      # drift in bins over the observation
    amp: float     # time-domain amplitude under the orthonormal DFT


def chirp_spectrum(n: int, chirp: Chirp) -> np.ndarray:
    """complex128 spectrum of a*exp(2*pi*i*r0*m/n + i*pi*z0*(m/n)^2), m < n,
    under the orthonormal DFT (input synthesis only)."""
    m = np.arange(n, dtype=np.float64)
    s = chirp.amp * np.exp(2j * np.pi * chirp.r0 * m / n + 1j * np.pi * chirp.z0 * (m / n) ** 2)
    return np.fft.fft(s, norm="ortho")


def make_spectrum(n: int, chirps, rng: np.random.Generator) -> np.ndarray:
    """complex64[n]: complex Gaussian noise (re, im i.i.d. N(0,1)) plus chirps."""
    w = rng.standard_normal(2 * n)
    x = w[0::2] + 1j * w[1::2]
    for c in chirps:
        x = x + chirp_spectrum(n, c)
    return x.astype(np.complex64)


def _streams(config_index: int):
    ss = np.random.SeedSequence(SEED_BASE + config_index)
    noise_ss, param_ss = ss.spawn(2)
    return np.random.Generator(np.random.PCG64(noise_ss)), np.random.Generator(np.random.PCG64(param_ss))


def _draw_chirps(rng: np.random.Generator, n: int, count: int, k_max: int, amp: float,
                 z_lo: float = -40.0, z_hi: float = 40.0, min_gap: int = 1024):
    lo, hi = 2 * k_max, n - 2 * k_max - 64
    bins: list[int] = []
    while len(bins) < count:
        r = int(rng.integers(lo, hi + 1))
        if all(abs(r - b) >= min_gap for b in bins):
            bins.append(r)
    return [Chirp(r0=float(b), z0=float(rng.uniform(z_lo, z_hi)), amp=amp) for b in bins]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    x: np.ndarray          # complex64 [N]
    bank: Bank
    seg_fft: int
    chirps: tuple

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


# Bank z ranges of the two single-array workloads.
Z_TOY = tuple(range(-8, 9, 2))        # 9 templates, K_t = 17..33
Z_SKA = tuple(range(-42, 43))         # 85 templates, K_t = 17..101


def toy_workload() -> Workload:
    """2^16 points, 9 templates (z=-8..8 step 2), one chirp r0=5000, z0=6, a=0.5,
    segment transform 1024."""
    n = 1 << 16
    noise_rng, _ = _streams(0)
    chirps = (Chirp(r0=5000.0, z0=6.0, amp=0.5),)
    x = make_spectrum(n, chirps, noise_rng)
    return Workload("toy-9x2^16", x, make_bank(Z_TOY), 1024, chirps)


def ska_workload(n: int = 1 << 22) -> Workload:
    """SKA-shaped single DM trial: 2^22 points, 85 templates (z=-42..42),
    three chirps at amplitude SNR 8 after a unit-energy matched filter
    (injected energy 8^2 * E|noise|^2 = 128), segment transform 2048."""
    noise_rng, param_rng = _streams(1)
    bank = make_bank(Z_SKA)
    amp = math.sqrt(128.0 / n)
    chirps = tuple(_draw_chirps(param_rng, n, 3, bank.k_max, amp))
    x = make_spectrum(n, chirps, noise_rng)
    return Workload(f"ska-85x2^{int(math.log2(n))}", x, bank, 2048, chirps)


def random_case(seed: int, n: int, m: int, k_max: int, ragged: bool = True):
    """Small random complex64 input and bank (unit-variance entries) for tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(2 * n)
    x = (w[0::2] + 1j * w[1::2]).astype(np.complex64)
    taps = np.zeros((m, k_max), dtype=np.complex64)
    if ragged:
        tap_len = rng.integers(1, k_max + 1, size=m).astype(np.int32)
        tap_len[int(rng.integers(0, m))] = k_max
    else:
        tap_len = np.full(m, k_max, dtype=np.int32)
    for t in range(m):
        v = rng.standard_normal(2 * int(tap_len[t]))
        taps[t, : tap_len[t]] = (v[0::2] + 1j * v[1::2]) / math.sqrt(2.0 * tap_len[t])
    return x, Bank(z=np.zeros(m), taps=taps, tap_len=tap_len)


@dataclasses.dataclass(frozen=True)
class Batch:
    name: str
    xs: tuple              # complex64 arrays of uneven lengths
    bank: Bank
    seg_fft: int
    chirps: tuple          # per array, a tuple of Chirp

    @property
    def lengths(self):
        return [int(x.shape[0]) for x in self.xs]


BATCH_LENGTHS = (1 << 19, 1 << 20, 1 << 21, 1 << 22)


def dm_trial_batch(count: int = 64, lengths=BATCH_LENGTHS, seed_index: int = 2,
                   bank: Bank | None = None) -> Batch:
    """A batch of DM-trial spectra: lengths drawn uniformly from `lengths`,
    complex Gaussian noise plus 0-2 chirps each (amplitude-SNR 8 as in the
    single-array workload, z0 uniform in [-40, 40]), the 85-template bank."""
    noise_rng, param_rng = _streams(seed_index)
    bank = make_bank(Z_SKA) if bank is None else bank
    xs, chirps = [], []
    for _ in range(count):
        n = int(lengths[int(param_rng.integers(0, len(lengths)))])
        nc = int(param_rng.integers(0, 3))
        amp = math.sqrt(128.0 / n)
        cs = tuple(_draw_chirps(param_rng, n, nc, bank.k_max, amp))
        xs.append(make_spectrum(n, cs, noise_rng))
        chirps.append(cs)
    return Batch(f"dm-batch-{count}x85", tuple(xs), bank, 2048, tuple(chirps))
