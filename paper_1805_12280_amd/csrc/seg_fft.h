// seg_fft.h -- L-point complex FP32 segment transform for gfx950, split into
// per-work-item stages so that a workgroup of T = L/16 work-items holds one
// transform in registers (16 points each) and exchanges it through LDS.
//
// This is the FFT/IFFT engine role of Section 4.2 (one engine used for the
// forward round and the inverse round, as in AOLS-FD), recast for a GPU:
// a three-pass mixed-radix Cooley-Tukey transform, L = 16 * 16 * R2 with
// R2 = L / 256 in {4, 8, 16}; at L = 8192 the last pass (R2 = 32) is itself
// split, 32 = 16 x 2, with one more exchange (see Seg<8192> below).
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

// exp(S * 2 pi i * E / 32) (E in 0..15)
template <int S> FDAS_HD c32 w32(int E)
{
    constexpr double kC[16] = {1.0, 0.98078528040323044913, 0.92387953251128673848, 0.83146961230254523708,
                               0.70710678118654752440, 0.55557023301960222474, 0.38268343236508978178,
                               0.19509032201612826785, 0.0, -0.19509032201612826785, -0.38268343236508978178,
                               -0.55557023301960222474, -0.70710678118654752440, -0.83146961230254523708,
                               -0.92387953251128673848, -0.98078528040323044913};
    // sin(2 pi E / 32) = cos(2 pi (8 - E) / 32), E <= 8; = cos(2 pi (E - 8) / 32) mirrored above
    const double sn = E <= 8 ? kC[8 - E] : kC[E - 8];
    return mk((float)kC[E], (float)(S * sn));
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

// ---- FMA forms of the butterfly with a multiplied operand ------------------
// A radix-2 step with a multiplied operand, (A + w c, A - w c), takes four
// FMAs for A + w c and two for A - w c = 2 A - (A + w c), instead of a
// complex multiply (four) and a complex add and subtract (four).

// a * w, or a * conj(w) when CJ
template <bool CJ> FDAS_HD c32 cmul(c32 a, c32 w)
{
    const float wi = CJ ? -w.im : w.im;
    return mk(a.re * w.re - a.im * wi, a.re * wi + a.im * w.re);
}
// A + c * w, or A + c * conj(w) when CJ
template <bool CJ> FDAS_HD c32 cfma(c32 A, c32 w, c32 c)
{
    const float wi = CJ ? -w.im : w.im;
    return mk(fmaf(-c.im, wi, fmaf(c.re, w.re, A.re)), fmaf(c.re, wi, fmaf(c.im, w.re, A.im)));
}
// 2 A - t
FDAS_HD c32 twice_minus(c32 A, c32 t) { return mk(fmaf(2.f, A.re, -t.re), fmaf(2.f, A.im, -t.im)); }

// radix-2 step (A + w c, A - w c) for a constant w = exp(S 2 pi i E / 16)
template <int S, int E> FDAS_HD void rad2_const(c32 A, c32 c, c32 &sum, c32 &dif)
{
    constexpr int e = E & 15;
    if constexpr (e == 0) { sum = add(A, c); dif = sub(A, c); }
    else if constexpr (e == 4 || e == 8 || e == 12) { c32 r = rot16<S, e>(c); sum = add(A, r); dif = sub(A, r); }
    else { sum = cfma<false>(A, w16<S, e>(), c); dif = twice_minus(A, sum); }
}

// Outputs of a 4-point DFT from its two radix-2 halves:
// s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3.
template <int S> FDAS_HD void dft4_join(c32 s02, c32 d02, c32 s13, c32 d13, c32 &X0, c32 &X1, c32 &X2, c32 &X3)
{
    const c32 r = mul_si<S>(d13);
    X0 = add(s02, s13);
    X2 = sub(s02, s13);
    X1 = add(d02, r);
    X3 = sub(d02, r);
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
    dft4_join<S>(add(x0, x2), sub(x0, x2), add(x1, x3), sub(x1, x3), x0, x1, x2, x3);
}

template <int S> FDAS_HD void dft4v(c32 *v) { dft4<S>(v[0], v[1], v[2], v[3]); }

// 8 = 2 x 4: n = 2 n1 + n2, k = k1 + 4 k2.  Input: the radix-2 halves of the
// two 4-point DFTs over n1 (pairs n1 = {0, 2} and {1, 3}) for n2 = 0, 1.
template <int S> FDAS_HD void dft8_tail(const c32 *s, const c32 *d, c32 *v)
{
    // s[2 n2 + h], d[2 n2 + h]: h = 0 pairs (n1 0, 2), h = 1 pairs (n1 1, 3)
    c32 a0, a1, a2, a3, b0, b1, b2, b3;
    dft4_join<S>(s[0], d[0], s[1], d[1], a0, a1, a2, a3);
    dft4_join<S>(s[2], d[2], s[3], d[3], b0, b1, b2, b3);
    rad2_const<S, 0>(a0, b0, v[0], v[4]);
    rad2_const<S, 2>(a1, b1, v[1], v[5]);
    rad2_const<S, 4>(a2, b2, v[2], v[6]);
    rad2_const<S, 6>(a3, b3, v[3], v[7]);
}

template <int S> FDAS_HD void dft8(c32 *v)
{
    c32 s[4], d[4];
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s[2 * n2 + h] = add(v[2 * h + n2], v[2 * h + 4 + n2]);
            d[2 * n2 + h] = sub(v[2 * h + n2], v[2 * h + 4 + n2]);
        }
    dft8_tail<S>(s, d, v);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.  The second layer: y[4 n2 + k1]
// (first-layer outputs) times W16^(n2 k1), 4-point DFT over n2.
template <int S> FDAS_HD void dft16_layer2(const c32 *y, c32 *v)
{
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        c32 s02, d02, s13, d13, B;
        // pair (n2 = 0, n2 = 2): y[k1] + W^(2 k1) y[8 + k1]
        switch (k1) {
        case 0: rad2_const<S, 0>(y[0], y[8], s02, d02); break;
        case 1: rad2_const<S, 2>(y[1], y[9], s02, d02); break;
        case 2: rad2_const<S, 4>(y[2], y[10], s02, d02); break;
        default: rad2_const<S, 6>(y[3], y[11], s02, d02); break;
        }
        // pair (n2 = 1, n2 = 3): W^k1 y[4 + k1] + W^(3 k1) y[12 + k1]
        switch (k1) {
        case 0: rad2_const<S, 0>(y[4], y[12], s13, d13); break;
        case 1: B = rot16<S, 1>(y[5]);  rad2_const<S, 3>(B, y[13], s13, d13); break;
        case 2: B = rot16<S, 2>(y[6]);  rad2_const<S, 6>(B, y[14], s13, d13); break;
        default: B = rot16<S, 3>(y[7]); rad2_const<S, 9>(B, y[15], s13, d13); break;
        }
        dft4_join<S>(s02, d02, s13, d13, v[k1], v[k1 + 4], v[k1 + 8], v[k1 + 12]);
    }
}

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
    dft16_layer2<S>(y, v);
}

// 16-point DFT of v[k] * tw[k] (tw[0] taken as 1; conj(tw) when CJ).
template <int S, bool CJ> FDAS_HD void dft16_tw(c32 *v, const c32 *tw)
{
    c32 y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        const c32 A = n2 == 0 ? v[0] : cmul<CJ>(v[n2], tw[n2]);
        const c32 s02 = cfma<CJ>(A, tw[8 + n2], v[8 + n2]);
        const c32 d02 = twice_minus(A, s02);
        const c32 B = cmul<CJ>(v[4 + n2], tw[4 + n2]);
        const c32 s13 = cfma<CJ>(B, tw[12 + n2], v[12 + n2]);
        const c32 d13 = twice_minus(B, s13);
        dft4_join<S>(s02, d02, s13, d13, y[4 * n2], y[4 * n2 + 1], y[4 * n2 + 2], y[4 * n2 + 3]);
    }
    dft16_layer2<S>(y, v);
}

template <int R, int S> FDAS_HD void dft(c32 *v)
{
    if constexpr (R == 2) dft2<S>(v);
    else if constexpr (R == 4) dft4v<S>(v);
    else if constexpr (R == 8) dft8<S>(v);
    else { static_assert(R == 16, "radix"); dft16<S>(v); }
}

// R-point DFT of the products a[k] * b[k] (the pointwise product of Alg. 2
// folded into the first butterfly layer).
template <int R, int S> FDAS_HD void dft_prod(const c32 *a, const c32 *b, c32 *v)
{
    // radix-2 pairs (k, k + R/2): A + a' b' and 2 A - (A + a' b'), A = a b
    auto pair = [&](int i, int j, c32 &sum, c32 &dif) {
        const c32 A = cmul<false>(a[i], b[i]);
        sum = cfma<false>(A, b[j], a[j]);
        dif = twice_minus(A, sum);
    };
    if constexpr (R == 2) {
        pair(0, 1, v[0], v[1]);
    } else if constexpr (R == 4) {
        c32 s02, d02, s13, d13;
        pair(0, 2, s02, d02);
        pair(1, 3, s13, d13);
        dft4_join<S>(s02, d02, s13, d13, v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        c32 s[4], d[4];
#pragma unroll
        for (int n2 = 0; n2 < 2; ++n2)
#pragma unroll
            for (int h = 0; h < 2; ++h) pair(2 * h + n2, 2 * h + 4 + n2, s[2 * n2 + h], d[2 * n2 + h]);
        dft8_tail<S>(s, d, v);
    } else {
        static_assert(R == 16, "radix");
        c32 y[16];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            c32 s02, d02, s13, d13;
            pair(n2, 8 + n2, s02, d02);
            pair(4 + n2, 12 + n2, s13, d13);
            dft4_join<S>(s02, d02, s13, d13, y[4 * n2], y[4 * n2 + 1], y[4 * n2 + 2], y[4 * n2 + 3]);
        }
        dft16_layer2<S>(y, v);
    }
}

// ---- the three-pass segment transform -------------------------------------

template <int L> struct Seg {
    static constexpr int T = L / 16;       // work-items per transform
    static constexpr int R2 = L / 256;     // radix of the last forward pass
    static constexpr int G = R2 <= 16 ? 16 / R2 : 1;   // last-pass butterflies per work-item (R2 <= 16)
    static constexpr int PAD = 1;          // LDS row padding (complex elements)
    static constexpr int ROW = T + PAD;
    static constexpr int LDS_ELEMS = 16 * ROW;
    static_assert(L == 1024 || L == 2048 || L == 4096 || L == 8192, "segment length");

    // LDS slots of the two exchanges (one buffer, used one after the other)
    FDAS_HD static int a_slot(int k1, int j) { return k1 * ROW + j; }
    FDAS_HD static int c_slot(int k1, int r, int p) { return k1 * ROW + r * R2 + p; }

    FDAS_HD static int k1_of(int tau) { return tau & 15; }
    FDAS_HD static int p_of(int tau) { return tau >> 4; }

    // Frequency held by work-item tau in register e after the forward passes.
    FDAS_HD static int perm(int tau, int e)
    {
        if constexpr (L == 8192) {
            // pass 2b work-item (k1, r, h) = (tau % 16, tau / 16 % 16, tau / 256):
            // register e = s0' + 8 s1 holds s' = 8 h + s0' + 16 s1
            return k1_of(tau) + 16 * ((tau >> 4) & 15) + 256 * (8 * (tau >> 8) + (e & 7) + 16 * (e >> 3));
        } else {
            int g = e / R2, s = e % R2;
            return k1_of(tau) + 16 * (p_of(tau) * G + g) + 256 * s;
        }
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
    // v[e] = X[perm(tau, e)] on exit.  At L = 8192 the pass is split and
    // reuses lds for its own exchange, behind two barriers of its own.
    FDAS_HD static void fwd2(int tau, c32 *v, c32 *lds)
    {
        if constexpr (L == 8192) {
            c32 d[16];
            fwd2a(tau, d, lds);
            __syncthreads();
            put_e(tau, d, lds);
            __syncthreads();
            fwd2b(tau, v, lds);
        } else {
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
    }

    // -- inverse --
    // Z[perm(tau, e)] = X[e] * Hs[e] (the pointwise product, taken inside the
    // first butterfly layer); writes c' to LDS.  At L = 8192 the pass is
    // split and reuses lds for its own exchange (two barriers of its own).
    FDAS_HD static void inv2(int tau, const c32 *X, const c32 *Hs, c32 *lds)
    {
        if constexpr (L == 8192) {
            inv2b(tau, X, Hs, lds);
            __syncthreads();
            c32 d[16];
            inv2a(tau, d, lds);
            __syncthreads();
            put_c_inv(tau, d, lds);
        } else {
            const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                c32 d[R2];
                dft_prod<R2, +1>(X + g * R2, Hs + g * R2, d);
#pragma unroll
                for (int pp = 0; pp < R2; ++pp) lds[c_slot(k1, p * G + g, pp)] = d[pp];
            }
        }
    }

    // -- the split last pass at L = 8192 (32 = 16 x 2) --
    // With p = p0 + 2 p1 and s' = s0 + 16 s1 (p0, s1 < 2; p1, s0 < 16),
    //   X[k1 + 16 r + 256 s'] = sum_p0 W2^(p0 s1) W32^(p0 s0) sum_p1 W16^(p1 s0) c[k1][p][r].
    // Pass 2a, work-item (k1, r, p0) = (tau % 16, tau / 16 % 16, tau / 256):
    //   e[k1][p0][r][s0] = W32^(p0 s0) DFT16_p1(c[k1][p0 + 2 p1][r]);
    // pass 2b, work-item (k1, r, h): radix 2 over p0 for s0 = 8 h .. 8 h + 7.
    // p0 and h are uniform over a wavefront.  The inverse runs the transpose
    // (2b' with the product, then 2a' with conjugate twiddles).
    FDAS_HD static int e_slot(int k1, int r, int p0, int s0) { return k1 * ROW + 32 * r + 2 * s0 + p0; }
    FDAS_HD static void fwd2a(int tau, c32 *d, const c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, p0 = tau >> 8;
#pragma unroll
        for (int p1 = 0; p1 < 16; ++p1) d[p1] = lds[c_slot(k1, r, p0 + 2 * p1)];
        dft16<-1>(d);
        if (p0) {
#pragma unroll
            for (int s0 = 1; s0 < 16; ++s0) d[s0] = mul(d[s0], w32<-1>(s0));
        }
    }
    FDAS_HD static void put_e(int tau, const c32 *d, c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, p0 = tau >> 8;
#pragma unroll
        for (int s0 = 0; s0 < 16; ++s0) lds[e_slot(k1, r, p0, s0)] = d[s0];
    }
    FDAS_HD static void fwd2b(int tau, c32 *v, const c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, h = tau >> 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const c32 a = lds[e_slot(k1, r, 0, 8 * h + i)], b = lds[e_slot(k1, r, 1, 8 * h + i)];
            v[i] = add(a, b);
            v[i + 8] = sub(a, b);
        }
    }
    FDAS_HD static void inv2b(int tau, const c32 *X, const c32 *Hs, c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, h = tau >> 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const c32 a[2] = {X[i], X[i + 8]}, b[2] = {Hs[i], Hs[i + 8]};
            c32 d[2];
            dft_prod<2, +1>(a, b, d);
            lds[e_slot(k1, r, 0, 8 * h + i)] = d[0];
            lds[e_slot(k1, r, 1, 8 * h + i)] = d[1];
        }
    }
    FDAS_HD static void inv2a(int tau, c32 *d, const c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, p0 = tau >> 8;
#pragma unroll
        for (int s0 = 0; s0 < 16; ++s0) d[s0] = lds[e_slot(k1, r, p0, s0)];
        if (p0) {
            c32 tw[16];
#pragma unroll
            for (int s0 = 0; s0 < 16; ++s0) tw[s0] = w32<-1>(s0);     // conjugated inside: W32^(+s0)
            dft16_tw<+1, true>(d, tw);
        } else {
            dft16<+1>(d);
        }
    }
    FDAS_HD static void put_c_inv(int tau, const c32 *d, c32 *lds)
    {
        const int k1 = k1_of(tau), r = (tau >> 4) & 15, p0 = tau >> 8;
#pragma unroll
        for (int p1 = 0; p1 < 16; ++p1) lds[c_slot(k1, r, p0 + 2 * p1)] = d[p1];
    }
    FDAS_HD static void inv1(int tau, c32 *v, const c32 *lds, const c32 *tw1)
    {
        const int k1 = k1_of(tau), p = p_of(tau);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lds[c_slot(k1, r, p)];
        dft16_tw<+1, true>(v, tw1);
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
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds[a_slot(k1, tau)];
        dft16_tw<+1, true>(v, tw0);
    }
};

}  // namespace fdas
