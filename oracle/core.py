"""FP64 CPU oracle for overlap-save FT convolution with a power plane.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the GPU library or its binding.

What the hot path computes has a plain definition, the causal direct
convolution of Section 3.1, Eq. (1), followed by the spectral power of
Section 4.3 (no square root):

    y_t[i] = sum_{k < K_t} x[i-k] h_t[k]   (x[j] = 0 for j < 0),   0 <= i < N
    P_t[i] = Re(y_t[i])^2 + Im(y_t[i])^2

`conv`, `power` and `power_at` evaluate exactly that, in float64, through
the plain C loops in direct.c.  The remaining functions restate the
paper's other routes to the same result so the tests can pin indexing:

* `dft`               -- the discrete Fourier transform by its definition;
* `template_spectrum` -- pre-transformed coefficients (Alg. 2, the FFT of h
                         taken once), scaled by 1/L;
* `ols_convolve`      -- Alg. 2 (overlap-save on the input), Section 3.2.2;
* `ola_convolve`      -- Alg. 1 (overlap-add on the taps), Section 3.1.2;
* `topk`              -- the k largest cells of a power plane.

Readings where the paper is not explicit (see the design notes): outputs
are causal and start at i = 0 (front padding of K-1 zeros, discard of the
first K-1 points of each chunk); a bank with ragged K_t uses one geometry
from K_max, which is the same as zero-padding every template to K_max.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        for name in ("oracle_conv", "oracle_power"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int64, dp, i32p, ctypes.c_int32, ctypes.c_int32,
                          i32p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_int]
            f.restype = ctypes.c_int
        lib.oracle_power_at.argtypes = [dp, ctypes.c_int64, dp, i32p, ctypes.c_int32,
                                        ctypes.c_int32, i32p, i64p, ctypes.c_int64, dp,
                                        ctypes.c_int]
        lib.oracle_power_at.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _prep(x, taps, tap_len):
    x = np.ascontiguousarray(np.asarray(x).astype(np.complex128).reshape(-1))
    taps = np.asarray(taps)
    if taps.ndim == 1:
        taps = taps[None, :]
    taps = np.ascontiguousarray(taps.astype(np.complex128))
    if tap_len is None:
        tap_len = np.full(taps.shape[0], taps.shape[1], dtype=np.int32)
    tap_len = np.ascontiguousarray(np.asarray(tap_len, dtype=np.int32).reshape(-1))
    if tap_len.shape[0] != taps.shape[0]:
        raise ValueError("tap_len must have one entry per template")
    return x, taps, tap_len


def threads(n: int = 0) -> int:
    """Threads the oracle will use (n > 0 sets it)."""
    return int(_load().oracle_threads(int(n)))


def conv(x, taps, tap_len=None, rows=None, i0: int = 0, i1: int | None = None,
         nthreads: int = 0) -> np.ndarray:
    """complex128 [len(rows)][i1-i0]: y_t[i] of Eq. (1) in float64.

    x, taps are upcast exactly from whatever precision they arrive in.
    Indices i >= N give the tail of the full linear convolution.
    """
    x, taps, tap_len = _prep(x, taps, tap_len)
    n = x.shape[0]
    i1 = n if i1 is None else int(i1)
    rows = np.arange(taps.shape[0], dtype=np.int32) if rows is None else \
        np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))
    out = np.empty((rows.shape[0], i1 - i0), dtype=np.complex128)
    rc = _load().oracle_conv(_ptr(x.view(np.float64), ctypes.c_double), n,
                             _ptr(taps.view(np.float64), ctypes.c_double),
                             _ptr(tap_len, ctypes.c_int32), taps.shape[0], taps.shape[1],
                             _ptr(rows, ctypes.c_int32), rows.shape[0], int(i0), i1,
                             _ptr(out.view(np.float64), ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_conv rejected its arguments (rc=%d)" % rc)
    return out


def power(x, taps, tap_len=None, rows=None, i0: int = 0, i1: int | None = None,
          nthreads: int = 0) -> np.ndarray:
    """float64 [len(rows)][i1-i0]: P_t[i] = |y_t[i]|^2 (Section 4.3, no square root)."""
    x, taps, tap_len = _prep(x, taps, tap_len)
    n = x.shape[0]
    i1 = n if i1 is None else int(i1)
    rows = np.arange(taps.shape[0], dtype=np.int32) if rows is None else \
        np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))
    out = np.empty((rows.shape[0], i1 - i0), dtype=np.float64)
    rc = _load().oracle_power(_ptr(x.view(np.float64), ctypes.c_double), n,
                              _ptr(taps.view(np.float64), ctypes.c_double),
                              _ptr(tap_len, ctypes.c_int32), taps.shape[0], taps.shape[1],
                              _ptr(rows, ctypes.c_int32), rows.shape[0], int(i0), i1,
                              _ptr(out, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_power failed (rc=%d)" % rc)
    return out


def power_at(x, taps, tap_len, t_idx, i_idx, nthreads: int = 0) -> np.ndarray:
    """float64 [npts]: P_{t_idx[p]}[i_idx[p]], each evaluated on its own."""
    x, taps, tap_len = _prep(x, taps, tap_len)
    t_idx = np.ascontiguousarray(np.asarray(t_idx, dtype=np.int32).reshape(-1))
    i_idx = np.ascontiguousarray(np.asarray(i_idx, dtype=np.int64).reshape(-1))
    if t_idx.shape != i_idx.shape:
        raise ValueError("t_idx and i_idx must have the same length")
    out = np.empty(t_idx.shape[0], dtype=np.float64)
    rc = _load().oracle_power_at(_ptr(x.view(np.float64), ctypes.c_double), x.shape[0],
                                 _ptr(taps.view(np.float64), ctypes.c_double),
                                 _ptr(tap_len, ctypes.c_int32), taps.shape[0], taps.shape[1],
                                 _ptr(t_idx, ctypes.c_int32), _ptr(i_idx, ctypes.c_int64),
                                 t_idx.shape[0], _ptr(out, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_power_at rejected its arguments (rc=%d)" % rc)
    return out


# ---------------------------------------------------------------------------
# Transforms by definition
# ---------------------------------------------------------------------------

def dft(x, sign: int = -1) -> np.ndarray:
    """X[q] = sum_n x[n] exp(sign * 2*pi*i * n*q / L), float64, by definition.

    The phase index n*q is reduced mod L in integers before the angle is
    formed, so every exponential is evaluated at an angle in [0, 2*pi).
    O(L^2): meant for single segments (L <= 8192) in tests.
    """
    x = np.asarray(x, dtype=np.complex128)
    L = x.shape[-1]
    n = np.arange(L, dtype=np.int64)
    ph = (np.outer(n, n) % L).astype(np.float64)
    w = np.exp(sign * 2j * np.pi * ph / L)
    return x @ w


def template_spectrum(h, L: int) -> np.ndarray:
    """H[q] = (1/L) sum_{k<K} h[k] exp(-2*pi*i*q*k/L): the coefficient array
    transformed once (Alg. 2) with the inverse transform's 1/L folded in."""
    h = np.asarray(h, dtype=np.complex128).reshape(-1)
    if h.shape[0] > L:
        raise ValueError("template longer than the segment")
    q = np.arange(L, dtype=np.int64)
    k = np.arange(h.shape[0], dtype=np.int64)
    ph = (np.outer(q, k) % L).astype(np.float64)
    return (np.exp(-2j * np.pi * ph / L) @ h) / L


# ---------------------------------------------------------------------------
# Alg. 2 and Alg. 1 (pins for the segment / tap-block indexing)
# ---------------------------------------------------------------------------

def ols_geometry(n: int, k_max: int, L: int):
    """(V, S): outputs kept per chunk, V = L - (K_max - 1), and chunks S = ceil(n / V).

    Successive chunks overlap by K_max - 1 points (Section 3.2.2); each keeps
    the L - (K_max - 1) points that follow its discarded front."""
    if L < k_max:
        raise ValueError("segment shorter than the filter")
    v = L - (k_max - 1)
    return v, (n + v - 1) // v


def ols_convolve(x, taps, tap_len=None, L: int = 1024) -> np.ndarray:
    """Alg. 2, overlap-save on the input, in float64 with numpy's FFT as the
    transform primitive.  Returns complex128 [M][N], the first N outputs.

    Steps, in the algorithm's order: pad K-1 zeros at the front of x; split
    into chunks of L that overlap by K-1; transform the coefficients once;
    per chunk transform, multiply element-wise, inverse transform, discard
    the first K-1 points and append the rest to the output.  K is the bank's
    K_max (ragged templates are zero-padded to it).
    """
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    taps = np.asarray(taps, dtype=np.complex128)
    if taps.ndim == 1:
        taps = taps[None, :]
    m, k_max = taps.shape
    if tap_len is not None:
        taps = taps.copy()
        for t in range(m):
            taps[t, int(tap_len[t]):] = 0
    n = x.shape[0]
    v, s_count = ols_geometry(n, k_max, L)
    padded = np.concatenate([np.zeros(k_max - 1, dtype=np.complex128), x,
                             np.zeros(s_count * v + L, dtype=np.complex128)])
    Fh = np.fft.fft(taps, n=L, axis=1)                 # transform of h, once
    y = np.zeros((m, s_count * v), dtype=np.complex128)
    for s in range(s_count):
        chunk = padded[s * v: s * v + L]               # overlaps the previous by K-1
        Fx = np.fft.fft(chunk)
        yi = np.fft.ifft(Fx[None, :] * Fh, axis=1)     # times, then inverse transform
        y[:, s * v:(s + 1) * v] = yi[:, k_max - 1:]    # discard the front K-1 points
    return y[:, :n]


def ola_convolve(x, h, k_sub: int) -> np.ndarray:
    """Alg. 1, overlap-add on the taps: h is split into R = ceil(K/K') disjoint
    blocks of K' taps (the last one zero-padded); each block is convolved with
    x in the time domain (numpy.convolve) and added in, shifted by r*K'.
    Returns complex128 [N], the first N outputs."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    h = np.asarray(h, dtype=np.complex128).reshape(-1)
    n = x.shape[0]
    r_count = -(-h.shape[0] // k_sub)
    hp = np.concatenate([h, np.zeros(r_count * k_sub - h.shape[0], dtype=np.complex128)])
    y = np.zeros(n + r_count * k_sub, dtype=np.complex128)
    for r in range(r_count):
        yr = np.convolve(x, hp[r * k_sub:(r + 1) * k_sub])
        y[r * k_sub: r * k_sub + yr.shape[0]] += yr
    return y[:n]


# ---------------------------------------------------------------------------
# Candidates
# ---------------------------------------------------------------------------

def topk(plane, k: int):
    """The k largest cells of a power plane [M][N] as (t, i, P) triples,
    ordered by power descending, then t ascending, then i ascending."""
    plane = np.asarray(plane)
    flat = plane.reshape(-1)
    k = min(k, flat.shape[0])
    if k == 0:
        return []
    kth = np.partition(flat, flat.shape[0] - k)[flat.shape[0] - k]
    cand = np.nonzero(flat >= kth)[0]
    order = sorted(cand.tolist(), key=lambda c: (-float(flat[c]), c))
    n = plane.shape[-1]
    return [(c // n, c % n, float(flat[c])) for c in order[:k]]
