"""A numpy model of the operand roundings of the 16-bit plans' inverse
transform, to weigh the hi/lo split-precision correction against the
binary16 operands the matrix-core kernel feeds.

The inverse of the overlap-save product (Alg. 2, Eq. (2)) at L = 2048 is
factored, with Z indexed q = k1 + 16 r + 256 s and the output
n = p + 8 q' + 128 m, into

    pass A (radix 8):   c[k1][p][r]  = sum_s W8^(p s) W128^(p r) Z[q]
    pass B (radix 16):  b[k1][p][q'] = W2048^((p + 8 q') k1) sum_r W16^(q' r) c[k1][p][r]
    pass C (radix 16):  y[n]         = sum_k1 W16^(m k1) b[k1][p][q']

(W_N = exp(+2 pi i / N)).  Each pass is a small complex matrix product whose
operands the kernel rounds to binary16; the products are exact and summed in
float32 (here in float64, whose extra bits change nothing at this scale).
The model rounds, per variant:

  binary16       both operands of every pass to binary16, the spectrum
                 product Z = X H and the pass-B twiddle in packed binary16
                 arithmetic: the FP16 plan as built;
  split_matrix   the DFT matrices as hi + lo binary16 pairs (two products);
  split_data     the data operands as hi + lo pairs (two products);
  split_both     both (three products, lo x lo dropped), Z and the twiddle in
                 float32: the correction the survey's mixed-precision row
                 names;
  split_both_f32h  the same with the template spectra held in float32 (as a
                 BF16 plan holds them);
  exact          no rounding: pins the factorisation itself.

The reference is the direct convolution (Eq. (1)) of the same binary16-
stored input in float64, so every figure is the kernel's own error, the
input's rounding excluded.  Run from the repository root as a script
(``PYTHONPATH=. python tests/test_mixed_pass_model.py 19``) it prints the
figures at 2^19 points.
"""
import sys

import numpy as np

from paper_1805_12280_amd import datagen

L, D = 2048, 128
V = L - D
VARIANTS = ("exact", "binary16", "split_matrix", "split_data", "split_both", "split_both_f32h")


def r16(a):
    """Each real component rounded to binary16 (nearest even), as float64."""
    if np.iscomplexobj(a):
        return r16(a.real) + 1j * r16(a.imag)
    return a.astype(np.float16).astype(np.float64)


def operand(a, how):
    """The binary16 operands standing for a: [(value, is_low_half)]."""
    if how == "exact":
        return [(a, False)]
    hi = r16(a)
    if how == "half":
        return [(hi, False)]
    return [(hi, False), (r16(a - hi), True)]


def matmul(W, X, how_w, how_x, spec):
    """Matrix-core product of constant W and data X: every pair of operand
    parts except low x low, summed."""
    out = 0.0
    for w, wlo in operand(W, how_w):
        for x, xlo in operand(X, how_x):
            if not (wlo and xlo):
                out = out + np.einsum(spec, w, x)
    return out


def cmul_packed16(a, b):
    """Complex product in packed binary16 arithmetic: t = a.re * b rounded,
    then (t.re - a.im b.im, t.im + a.im b.re) by one rounded fused multiply-add."""
    t_re, t_im = r16(a.real * b.real), r16(a.real * b.imag)
    return r16(t_re - a.imag * b.imag) + 1j * r16(t_im + a.imag * b.real)


def plane(x, taps, tap_len, variant):
    """Power plane of the 16-bit overlap-save path under the variant's
    roundings (template spectra stored as binary16, as in an FP16 plan)."""
    n, m_t = x.shape[0], taps.shape[0]
    S = -(-n // V)
    H = np.zeros((m_t, L), complex)
    for t in range(m_t):
        h = np.zeros(L, complex)
        h[:tap_len[t]] = taps[t, :tap_len[t]]
        H[t] = np.fft.fft(h) / L
    eh = -int(np.ceil(np.log2(np.abs(np.concatenate([H.real, H.imag])).max())))
    Hs = H * 2.0 ** eh                                   # max |component| <= 1
    xp = np.concatenate([np.zeros(D, complex), x, np.zeros(S * V + L - n, complex)])
    X = np.fft.fft(np.stack([xp[s * V:s * V + L] for s in range(S)]), axis=1)
    # per-segment power of two: 2 sigma max|X| <= 16
    ex = np.frexp(2.0 * np.maximum(np.abs(X.real), np.abs(X.imag)).max(axis=1))[1]
    sig = 2.0 ** (4 - ex)
    unscale = 2.0 ** (-2 * (4 - ex + eh))
    X = X * sig[:, None]

    e = np.arange(16)
    w = lambda num, den: np.exp(2j * np.pi * num / den)
    MA = w(16 * np.outer(e[:8], e[:8])[None] + e[:8][None, :, None] * e[:, None, None], 128)   # [r][p][s]
    MB = w(np.outer(e, e), 16)                                                                 # [q'][r]
    TW = w((e[:8][:, None] + 8 * e[None, :])[None] * e[:, None, None], L)                     # [k1][p][q']
    if variant == "exact":
        how_w = how_x = "exact"
    else:
        how_w = "split" if variant.startswith(("split_matrix", "split_both")) else "half"
        how_x = "split" if variant.startswith(("split_data", "split_both")) else "half"
    packed = variant in ("binary16", "split_matrix")
    P = np.zeros((m_t, S * V))
    for t in range(m_t):
        if variant in ("exact", "split_both_f32h"):
            Z = X * Hs[t][None]
        elif packed:
            Z = cmul_packed16(r16(X), r16(Hs[t])[None])
        else:
            Z = X * r16(Hs[t])[None]
        c = matmul(MA, Z.reshape(S, 8, 16, 16), how_w, how_x, "rps,bsrk->bkpr")
        if how_x == "half":
            c = r16(c)
        b = matmul(MB, c, how_w, how_x, "qr,bkpr->bkpq")
        b = cmul_packed16(r16(b), r16(TW)[None]) if packed else b * TW[None]
        y = matmul(MB, b, how_w, how_x, "mk,bkpq->bmqp").reshape(S, L)   # n = p + 8 q' + 128 m
        P[t] = (np.abs(y) ** 2 * unscale[:, None])[:, D:].reshape(-1)
    return P[:, :n]


def own_errors(log2n, rows=range(0, 85, 6)):
    """max |P - P_ref| / max P_ref per variant, on the headline bank's rows
    and the first 2^log2n points of its input, stored as binary16 pairs."""
    wl = datagen.ska_workload(n=1 << log2n)
    x = r16(wl.x.astype(np.complex128))
    rows = list(rows)
    taps = wl.bank.taps[rows].astype(np.complex128)
    tl = wl.bank.tap_len[rows]
    ref = np.stack([np.abs(np.convolve(x, taps[i, :tl[i]])[:x.shape[0]]) ** 2 for i in range(len(rows))])
    pk = ref.max()
    return {v: float(np.abs(plane(x, taps, tl, v) - ref).max() / pk) for v in VARIANTS}


def test_pass_model():
    err = own_errors(15)
    print(err)
    # the three-pass factorisation is the 2048-point inverse DFT
    assert err["exact"] <= 1e-12
    # binary16 operands alone stay inside the 2e-3 mixed-precision bar
    assert err["binary16"] <= 2e-3
    # the full split recovers most of the kernel's own error; what is left
    # comes from the binary16 template spectra
    assert err["split_both"] <= err["binary16"] / 3
    assert err["split_both_f32h"] <= 1e-6


if __name__ == "__main__":
    for k, v in own_errors(int(sys.argv[1]) if len(sys.argv) > 1 else 15).items():
        print(f"{k:16s} {v:.3e}")
