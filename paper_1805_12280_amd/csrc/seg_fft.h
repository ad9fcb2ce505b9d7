// seg_fft.h -- L-point complex FP32 segment transform for gfx950, split into
// per-work-item stages so that a workgroup of T = L/16 work-items holds one
// transform in registers (16 points each) and exchanges it through LDS.
//
// This is the FFT/IFFT engine role of Section 4.2 (one engine used for the
// forward round and the inverse round, as in AOLS-FD), recast for a GPU:
// a three-pass mixed-radix Cooley-Tukey transform, L = 16 * 16 * R2 with
// R2 = L / 256 in {4, 8, 16}.
//
// Forward (decimation in frequency), natural-order input, work-item tau:
//   pass 0  j = tau:            a[j][k1] = DFT16_m(w[j + T m]) * W_L^(j k1)
//   pass 1  tau = 16 p + k1:    c[k1][p][r] = DFT16_q(a[p + R2 q][k1]) * W_T^(p r)
//   pass 2  tau = 16 p + k1:    for g < G = 16/R2, r = p G + g:
//                               X[k1 + 16 r + 256 s] = DFT_R2,p'(c[k1][p'][r])
// so after pass 2 the work-item holds X at the 16 frequencies perm(tau, e),
// e = g R2 + s.  Like TOLS-FD, which multiplies in the FFT engine's own
// output order (Section 4.2.2), the pointwise product is taken right there:
// the template spectra are stored in the same permuted order, and the
// inverse transform runs the three passes backwards from that order to a
// natural-order output, so no reorder pass exists.
//
// Inverse (the transpose of the forward passes, conjugate twiddles):
//   pass 2' per g: c'[k1][p'][r] = IDFT_R2,s(Z[k1 + 16 r + 256 s])
//   pass 1'       b'[k1][p + R2 q] = IDFT16_r(c'[k1][p][r] * W_T^-(p r))
//   pass 0'       y[j + T m] = IDFT16_k1(b'[k1][j] * W_L^-(j k1))
// Each inverse twiddle is applied by the work-item that receives the value
// after an LDS exchange, so it is the conjugate of the forward twiddle that
// the same work-item applies: one register set of 2 x 16 twiddles serves
// both directions.
//
// LDS: both exchanges use rows of T + 1 elements (an odd pitch).  With k1 the
// fastest-varying index of the work-item in passes 1 and 2, every group of 16
// neighbouring lanes touches 16 different rows, so each 8-byte access of a
// wavefront is free of bank conflicts, and every address is a per-work-item
// base plus a compile-time offset.
//
// Every function is __host__ __device__ so the index maps can be executed on
// the CPU (one work-item after another between the barriers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FDAS_HD __host__ __device__ __forceinline__

namespace fdas {

struct c32 {
    float re, im;
};

FDAS_HD c32 mk(float r, float i) { c32 z; z.re = r; z.im = i; return z; }
FDAS_HD c32 add(c32 a, c32 b) { return mk(a.re + b.re, a.im + b.im); }
FDAS_HD c32 sub(c32 a, c32 b) { return mk(a.re - b.re, a.im - b.im); }
FDAS_HD c32 mul(c32 a, c32 b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
FDAS_HD c32 conj(c32 a) { return mk(a.re, -a.im); }
FDAS_HD float norm2(c32 a) { return a.re * a.re + a.im * a.im; }

// (S i) * a, S = -1 for the forward transform, +1 for the inverse.
template <int S> FDAS_HD c32 mul_si(c32 a) { return S < 0 ? mk(a.im, -a.re) : mk(-a.im, a.re); }

// exp(S * 2 pi i * E / 16) as constants (E in 0..15).
template <int S, int E> FDAS_HD c32 w16()
{
    constexpr double kC[16] = {1.0, 0.92387953251128673848, 0.70710678118654752440,
                               0.38268343236508978178, 0.0, -0.38268343236508978178,
                               -0.70710678118654752440, -0.92387953251128673848, -1.0,
                               -0.92387953251128673848, -0.70710678118654752440,
                               -0.38268343236508978178, 0.0, 0.38268343236508978178,
                               0.70710678118654752440, 0.92387953251128673848};
    // sin(2 pi E / 16) = cos(2 pi (E - 4) / 16)
    return mk((float)kC[E & 15], (float)(S * kC[(E + 12) & 15]));
}

// a * exp(S 2 pi i E / 16), with the trivial angles done without multiplies.
template <int S, int E> FDAS_HD c32 rot16(c32 a)
{
    constexpr int e = E & 15;
    if constexpr (e == 0) return a;
    else if constexpr (e == 4) return mul_si<S>(a);
    else if constexpr (e == 8) return mk(-a.re, -a.im);
    else if constexpr (e == 12) return mul_si<-S>(a);
    else return mul(a, w16<S, e>());
}

// ---- small in-register DFTs, natural order in and out ----------------------

template <int S> FDAS_HD void dft2(c32 *v)
{
    c32 a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}

template <int S> FDAS_HD void dft4(c32 &x0, c32 &x1, c32 &x2, c32 &x3)
{
    c32 t0 = add(x0, x2), t1 = sub(x0, x2), t2 = add(x1, x3), t3 = mul_si<S>(sub(x1, x3));
    x0 = add(t0, t2);
    x2 = sub(t0, t2);
    x1 = add(t1, t3);
    x3 = sub(t1, t3);
}

template <int S> FDAS_HD void dft4v(c32 *v) { dft4<S>(v[0], v[1], v[2], v[3]); }

// 8 = 2 x 4: n = 2 n1 + n2, k = k1 + 4 k2.
template <int S> FDAS_HD void dft8(c32 *v)
{
    c32 a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
    c32 b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
    dft4<S>(a0, a1, a2, a3);
    dft4<S>(b0, b1, b2, b3);
    b1 = rot16<S, 2>(b1);
    b2 = rot16<S, 4>(b2);
    b3 = rot16<S, 6>(b3);
    v[0] = add(a0, b0); v[4] = sub(a0, b0);
    v[1] = add(a1, b1); v[5] = sub(a1, b1);
    v[2] = add(a2, b2); v[6] = sub(a2, b2);
    v[3] = add(a3, b3); v[7] = sub(a3, b3);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <int S> FDAS_HD void dft16(c32 *v)
{
    c32 y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        c32 a = v[n2], b = v[4 + n2], c = v[8 + n2], d = v[12 + n2];
        dft4<S>(a, b, c, d);       // over n1 -> k1
        y[4 * n2 + 0] = a;
        y[4 * n2 + 1] = b;
        y[4 * n2 + 2] = c;
        y[4 * n2 + 3] = d;
    }
    // twiddle W16^(n2 k1); y[4 n2 + k1]
    y[5] = rot16<S, 1>(y[5]);   y[6] = rot16<S, 2>(y[6]);   y[7] = rot16<S, 3>(y[7]);
    y[9] = rot16<S, 2>(y[9]);   y[10] = rot16<S, 4>(y[10]); y[11] = rot16<S, 6>(y[11]);
    y[13] = rot16<S, 3>(y[13]); y[14] = rot16<S, 6>(y[14]); y[15] = rot16<S, 9>(y[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        c32 a = y[k1], b = y[4 + k1], c = y[8 + k1], d = y[12 + k1];
        dft4<S>(a, b, c, d);       // over n2 -> k2
        v[k1] = a;
        v[k1 + 4] = b;
        v[k1 + 8] = c;
        v[k1 + 12] = d;
    }
}

template <int R, int S> FDAS_HD void dft(c32 *v)
{
    if constexpr (R == 2) dft2<S>(v);
    else if constexpr (R == 4) dft4v<S>(v);
    else if constexpr (R == 8) dft8<S>(v);
    else { static_assert(R == 16, "radix"); dft16<S>(v); }
}

// ---- the three-pass segment transform -------------------------------------

template <int L> struct Seg {
    static constexpr int T = L / 16;       // work-items per transform
    static constexpr int R2 = L / 256;     // radix of the last forward pass
    static constexpr int G = 16 / R2;      // last-pass butterflies per work-item
    static constexpr int PAD = 1;          // LDS row padding (complex elements)
    static constexpr int ROW = T + PAD;
    static constexpr int LDS_ELEMS = 16 * ROW;
    static_assert(L == 1024 || L == 2048 || L == 4096, "segment length");

    // LDS slots of the two exchanges (one buffer, used one after the other)
    FDAS_HD static int a_slot(int k1, int j) { return k1 * ROW + j; }
    FDAS_HD static int c_slot(int k1, int r, int p) { return k1 * ROW + r * R2 + p; }

    FDAS_HD static int k1_of(int tau) { return tau & 15; }
    FDAS_HD static int p_of(int tau) { return tau >> 4; }

    // Frequency held by work-item tau in register e after the forward passes.
    FDAS_HD static int perm(int tau, int e)
    {
        int g = e / R2, s = e % R2;
        return k1_of(tau) + 16 * (p_of(tau) * G + g) + 256 * s;
    }

    // Per-work-item twiddles, held in registers for the life of a workgroup:
    //   tw0[k1] = W_L^(tau k1)   (pass 0, and conjugated in pass 0')
    //   tw1[r]  = W_T^(p r)      (pass 1, and conjugated in pass 1')
    // twL[e] = exp(-2 pi i e / L).  Index 0 is 1 and is never used.
    FDAS_HD static void twiddles(int tau, const c32 *twL, c32 *tw0, c32 *tw1)
    {
        const int p = p_of(tau);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            tw0[k] = twL[(tau * k) & (L - 1)];
            tw1[k] = twL[(16 * p * k) & (L - 1)];
        }
    }

    // -- forward --
    // v[m] = w[tau + T m] on entry.
    FDAS_HD static void fwd0(int tau, c32 *v, const c32 *tw0)
    {
        dft16<-1>(v);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = mul(v[k1], tw0[k1]);
    }
    FDAS_HD static void put_a(int tau, const c32 *v, c32 *lds)
    {
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) lds[a_slot(k1, tau)] = v[k1];
    }
    FDAS_HD static void fwd1(int tau, c32 *v, const c32 *lds, const c32 *tw1)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = lds[a_slot(k1, p + R2 * q)];
        dft16<-1>(v);
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = mul(v[r], tw1[r]);
    }
    FDAS_HD static void put_c(int tau, const c32 *v, c32 *lds)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[c_slot(k1, r, p)] = v[r];
    }
    // v[e] = X[perm(tau, e)] on exit.
    FDAS_HD static void fwd2(int tau, c32 *v, const c32 *lds)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            c32 d[R2];
#pragma unroll
            for (int pp = 0; pp < R2; ++pp) d[pp] = lds[c_slot(k1, p * G + g, pp)];
            dft<R2, -1>(d);
#pragma unroll
            for (int s = 0; s < R2; ++s) v[g * R2 + s] = d[s];
        }
    }

    // -- inverse --
    // v[e] = Z[perm(tau, e)] on entry; writes c' to LDS.
    FDAS_HD static void inv2(int tau, const c32 *v, c32 *lds)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            c32 d[R2];
#pragma unroll
            for (int s = 0; s < R2; ++s) d[s] = v[g * R2 + s];
            dft<R2, +1>(d);
#pragma unroll
            for (int pp = 0; pp < R2; ++pp) lds[c_slot(k1, p * G + g, pp)] = d[pp];
        }
    }
    FDAS_HD static void inv1(int tau, c32 *v, const c32 *lds, const c32 *tw1)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
        v[0] = lds[c_slot(k1, 0, p)];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = mul(lds[c_slot(k1, r, p)], conj(tw1[r]));
        dft16<+1>(v);
    }
    FDAS_HD static void put_a_inv(int tau, const c32 *v, c32 *lds)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int q = 0; q < 16; ++q) lds[a_slot(k1, p + R2 * q)] = v[q];
    }
    // v[m] = y[tau + T m] on exit.
    FDAS_HD static void inv0(int tau, c32 *v, const c32 *lds, const c32 *tw0)
    {
        v[0] = lds[a_slot(0, tau)];
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = mul(lds[a_slot(k1, tau)], conj(tw0[k1]));
        dft16<+1>(v);
    }
};

}  // namespace fdas
