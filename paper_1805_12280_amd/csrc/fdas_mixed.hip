// fdas_mixed.hip -- the overlap-save hot path with 16-bit storage of the
// input spectrum (binary16 or bfloat16) and the inverse segment transforms on
// the matrix cores (binary16 operands, FP32 accumulation).  L = 2048.
//
// Both plans feed the matrix cores binary16 operands: each segment is scaled
// by a power of two, so the 5 exponent bits of binary16 suffice and its 11
// significant bits keep 3 more than bfloat16's 8.  Both store the template
// spectra as binary16 and form Z = X H in packed binary16 arithmetic; they
// differ only in the input format the forward launch reads.
//
// Two launches per call.  Per segment (mixed_fwd_kernel, float32 VALU):
// gather the 16-bit input, forward FFT (seg_fft.h), redistribute the
// spectrum X into the lanes that feed pass A (mixed_fft.h), pick a
// power-of-two scale sigma from max |X| so the 16-bit operands stay well
// inside their range, and stage sigma X.  Per (segment, template)
// (fdfir_mixed_kernel): Z = sigma X H in packed binary16 arithmetic, passes
// A, B, C as matrix products, |y|^2 unscaled exactly by the powers of two,
// full-line streaming stores.  The batched form (mixed_fwd_batch_kernel,
// fdfir_mixed_topk_kernel) runs the same passes over many spectra and keeps
// each one's top-K cells instead of its plane.
#include "fdas_internal.h"
#include "mixed_fft.h"
#include "seg_fft.h"

namespace fdas {

typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Matrix-core operands and the elementwise products of the template loop:
// a complex value as a pair of IEEE binary16 numbers in one 32-bit word.
struct Half {
    __device__ static uint32_t pack(float re, float im)
    {
        // opaque to the compiler, so the arithmetic that produced re and im
        // stays in float32 instead of being fused into half-writing
        // mixed-precision FMAs (a slower, serialised form here)
        __asm__("" : "+v"(re), "+v"(im));
        h2v v = {(_Float16)re, (_Float16)im};   // round to nearest even
        return __builtin_bit_cast(uint32_t, v);
    }
    // the same rounding without the barrier, for matrix-core results (no
    // arithmetic precedes the conversion, and a barrier on two registers of
    // one result tuple costs a register copy)
    __device__ static uint32_t pack_acc(float re, float im)
    {
        h2v v = {(_Float16)re, (_Float16)im};
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static c32 unpack(uint32_t w)
    {
        const h2v v = __builtin_bit_cast(h2v, w);
        float re = (float)v.x, im = (float)v.y;
        __asm__("" : "+v"(re), "+v"(im));      // plain conversions, then float32 arithmetic
        return mk(re, im);
    }
    __device__ static f4v mma16(uint2 a, uint2 b, f4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4v, a), __builtin_bit_cast(h4v, b), c, 0, 0, 0);
    }
    __device__ static f4v mma32(uint4 a, uint4 b, f4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0, 0);
    }
    // Complex product of two packed binary16 values in packed binary16
    // arithmetic: t = (a.re b.re, a.re b.im) rounded, then
    // (t.re - a.im b.im, t.im + a.im b.re) by one fused multiply-add.
    __device__ static uint32_t cmulp(uint32_t a, uint32_t b)
    {
        const h2v av = __builtin_bit_cast(h2v, a), bv = __builtin_bit_cast(h2v, b);
        const h2v are = {av.x, av.x}, aim = {av.y, av.y}, bsw = {-bv.y, bv.x};
        const h2v z = __builtin_elementwise_fma(aim, bsw, are * bv);
        return __builtin_bit_cast(uint32_t, z);
    }
    // The scaled spectrum and the pass-B twiddles are held as packed
    // binary16 (the products Z = X H and b W run in packed arithmetic).
    __device__ static uint32_t zmul(uint32_t x, uint32_t h) { return cmulp(x, h); }
    __device__ static uint32_t twmul(float re, float im, uint32_t w) { return cmulp(pack_acc(re, im), w); }
};

// Input formats: a complex value as a pair of 16-bit numbers in one word.
template <bool BF> struct In16;
template <> struct In16<false> {
    __device__ static c32 unpack(uint32_t w) { return Half::unpack(w); }
};
template <> struct In16<true> {
    __device__ static c32 unpack(uint32_t w)
    {
        return mk(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
};

// Template spectra of one work-item for one template, in the order pass A
// consumes them (16 packed binary16 values).
struct HSpec {
    uint4 q[4];
    __device__ __forceinline__ uint32_t at(int v) const { return (&q[v >> 2].x)[v & 3]; }
};

// One real matrix entry of exp(2 pi i turns) for interleaved rows/columns.
__device__ __forceinline__ float wentry(int row, int k, double turns)
{
    double s, c;
    sincospi(2.0 * turns, &s, &c);
    switch (mix::entry_sel(row, k)) {
    case 0: return (float)c;
    case 1: return (float)-s;
    case 2: return (float)s;
    default: return (float)c;
    }
}


// ---------------------------------------------------------------------------
// template spectra in the lane layout of pass A, 16-bit, scaled by 2^eh
// ---------------------------------------------------------------------------

__global__ void tspec_mix_kernel(const c32 *__restrict__ taps, const int *__restrict__ tap_len, int kp, int M,
                                 float scale, uint32_t *__restrict__ H16)
{
    using namespace mix;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * L) return;
    const int t = (int)(idx / L);
    const int rem = (int)(idx - (int64_t)t * L);      // (w * 64 + l) * 16 + v
    const int v = rem & 15, wl = rem >> 4, w = wl >> 6, l = wl & 63;
    const int q = zq(w, l, v);
    const c32 *h = taps + (int64_t)t * kp;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < tap_len[t]; ++k) {
        const int r = (int)(((int64_t)q * k) & (L - 1));
        double s, c;
        sincospi(-2.0 * (double)r / (double)L, &s, &c);
        const double hr = h[k].re, hi = h[k].im;
        re += hr * c - hi * s;
        im += hr * s + hi * c;
    }
    H16[idx] = Half::pack((float)(re / L * scale), (float)(im / L * scale));
}

// ---------------------------------------------------------------------------
// fused kernel
// ---------------------------------------------------------------------------

// The DFT matrices in operand lane order, 16-bit:
//   MA[r * 64 + lane]  pass A for column set r (W128^(p r) folded in): 4 values (uint2)
//   MD[h * 64 + lane]  DFT16 of passes B and C, output half h: 8 values (uint4)
constexpr int MAT_A_UINT2 = 16 * 64;
constexpr int MAT_D = MAT_A_UINT2 / 2;         // in uint4 units
constexpr int MAT_UINT4 = MAT_D + 2 * 64;
constexpr size_t MAT_BYTES = MAT_UINT4 * sizeof(uint4);

__global__ void mat_table_kernel(uint4 *__restrict__ tab)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = idx & 63, i = l & 15, g = l >> 4;
    if (idx < MAT_A_UINT2) {
        const int r = idx >> 6;
        float e4[4];
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * g + e;
            e4[e] = wentry(i, k, mix::turns_A(r, i >> 1, k >> 1));
        }
        reinterpret_cast<uint2 *>(tab)[idx] = make_uint2(Half::pack(e4[0], e4[1]), Half::pack(e4[2], e4[3]));
    } else if (idx < MAT_A_UINT2 + 2 * 64) {
        const int h = (idx - MAT_A_UINT2) >> 6, out = 8 * h + (i >> 1);
        float e8[8];
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * g + e;
            e8[e] = wentry(i, k, mix::turns_D16(out, k >> 1));
        }
        tab[MAT_D + h * 64 + l] = make_uint4(Half::pack(e8[0], e8[1]), Half::pack(e8[2], e8[3]),
                                             Half::pack(e8[4], e8[5]), Half::pack(e8[6], e8[7]));
    }
}

// ---------------------------------------------------------------------------
// per segment: forward FFT (float32) and the power-of-two scale
// ---------------------------------------------------------------------------

// One workgroup transforms the segment of x16 starting at input point base
// and writes, as two packed binary16 complex values per work-item and step,
// out[v / 2][tau] = sigma X at the frequencies zq(w, l, v), zq(w, l, v + 1)
// that work-item tau = 64 w + l feeds to pass A (rounded once, as pass A
// takes them), and *ps = 2^-2(e + eh),
// which undoes both power-of-two scalings of |y|^2 (sigma = 2^e with
// 2 sigma max|X| <= 16, max over the components of the segment's spectrum).
template <bool BF>
__device__ __forceinline__ void forward_scaled(const uint32_t *__restrict__ x16, int64_t n, int64_t base,
                                               const c32 *__restrict__ twL, int eh, uint2 *__restrict__ out,
                                               float *__restrict__ ps)
{
    using SG = Seg<2048>;
    constexpr int L = mix::L, T = mix::T;
    // One LDS buffer serves both exchanges and the redistribution (2176
    // slots of 17 per 16 frequencies), one barrier more than two buffers but
    // half the LDS, so twice the workgroups fit a CU.
    constexpr int LDS_SLOTS = SG::LDS_ELEMS > L + L / 16 ? SG::LDS_ELEMS : L + L / 16;
    __shared__ c32 lds[LDS_SLOTS];
    __shared__ float s_max[2];
    c32 *const bufA = lds, *const bufC = lds;
    const int tau = threadIdx.x, w = tau >> 6, l = tau & 63, col = l & 15, g = l >> 4;

    c32 v[16];
    {
        const uint32_t *xs = x16 + base;
        const int lo = (int)max<int64_t>(0, -base), hi = (int)min<int64_t>(L, n - base);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int j = tau + T * m;
            v[m] = (j >= lo && j < hi) ? In16<BF>::unpack(xs[j]) : mk(0.f, 0.f);
        }
    }
    {
        c32 tw0[16], tw1[16];
        SG::twiddles(tau, twL, tw0, tw1);
        SG::fwd0(tau, v, tw0);
        SG::put_a(tau, v, bufA);
        __syncthreads();
        SG::fwd1(tau, v, bufA, tw1);
    }
    __syncthreads();                       // pass-1 reads done before bufC (the same buffer) is written
    SG::put_c(tau, v, bufC);
    __syncthreads();
    SG::fwd2(tau, v, bufC);
    __syncthreads();
    // redistribute X to the pass-A lanes through LDS, rows of 16 frequencies
    // padded to 17: slot(q) = q + q / 16.  Register e holds
    // q = k1 + 16 (2 p + e / 8) + 256 (e % 8) (R2 = 8, G = 2), so
    // slot = (k1 + 34 p) + 17 (e / 8) + 272 (e % 8).
    float mx = 0.f;
    {
        c32 *dst = lds + SG::k1_of(tau) + 34 * SG::p_of(tau);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            dst[17 * (e >> 3) + 272 * (e & 7)] = v[e];
            mx = fmaxf(mx, fmaxf(fabsf(v[e].re), fabsf(v[e].im)));
        }
    }
    // workgroup max of the component magnitudes
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (l == 0) s_max[w] = mx;
    __syncthreads();
    mx = fmaxf(s_max[0], s_max[1]);
    // sigma = 2^es with 2 sigma max|X| max|H16| <= 16 (max|H16| <= 1)
    int es = 0;
    if (mx > 0.f) {
        int ex;
        frexpf(2.f * mx, &ex);             // 2 mx < 2^ex
        es = 4 - ex;
    }
    const float sigma = ldexpf(1.f, es);
    if (tau == 0) *ps = ldexpf(1.f, -2 * (es + eh));
    // lane (w, l) takes q = zq(w, l, v): slot = (col + 136 w + 544 g)
    // + 17 (v / 2) + 272 (v % 2)
    const c32 *src = lds + col + 136 * w + 544 * g;
#pragma unroll
    for (int vp = 0; vp < 8; ++vp) {
        const c32 z0 = src[17 * vp], z1 = src[17 * vp + 272];
        out[vp * T + tau] = make_uint2(Half::pack(z0.re * sigma, z0.im * sigma), Half::pack(z1.re * sigma, z1.im * sigma));
    }
}

// Staging layout: segment s at Xs + s * L / 2 (uint2: two packed binary16
// complex values), its scale at ps[s].
template <bool BF>
__global__ __launch_bounds__(128) void mixed_fwd_kernel(const uint32_t *__restrict__ x16, int64_t n,
                                                        const c32 *__restrict__ twL, int D, int V, int eh,
                                                        uint2 *__restrict__ Xs, float *__restrict__ ps)
{
    const int64_t s = blockIdx.x;
    forward_scaled<BF>(x16, n, s * V - D, twL, eh, Xs + s * (mix::L / 2), ps + s);
}

// ---------------------------------------------------------------------------
// per (segment, template): Z = X H, inverse on the matrix cores
// ---------------------------------------------------------------------------

// What one work-item holds for the inverse passes of every item: its lanes
// of the 16-bit DFT matrices (pass A per column set r = 8 w + gam, with
// W128^(p r) folded in; the DFT16 of passes B and C) and the pass-B output
// twiddles W2048^(j k1).  Both template-loop kernels run the passes through
// these members, so they compute every cell identically.
struct MixLane {
    using HF = Half;
    uint2 aA[8];
    uint4 aD[2];
    uint32_t twc[4][2][2];

    __device__ __forceinline__ void init(const uint4 *__restrict__ mat, const c32 *__restrict__ twL, int w, int l)
    {
        const int col = l & 15, g = l >> 4;
#pragma unroll
        for (int gam = 0; gam < 8; ++gam) aA[gam] = reinterpret_cast<const uint2 *>(mat)[(8 * w + gam) * 64 + l];
        aD[0] = mat[MAT_D + l];
        aD[1] = mat[MAT_D + 64 + l];
#pragma unroll
        for (int gam = 0; gam < 4; ++gam)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int j = 4 * w + gam + 8 * (8 * h + 2 * g + i);
                    const c32 f = twL[(j * col) & (mix::L - 1)];        // exp(-2 pi i j k1 / L)
                    twc[gam][h][i] = HF::pack(f.re, -f.im);
                }
    }
    // pass A, column set r = 8w + gam: Z = X H (packed binary16), radix 8 over s;
    // returns c[2g][col][r] and c[2g + 1][col][r] packed
    __device__ __forceinline__ void pass_a(const uint32_t (&X)[16], const HSpec &Hn, int gam,
                                           uint32_t &c0, uint32_t &c1) const
    {
        const uint2 bop = make_uint2(HF::zmul(X[2 * gam], Hn.at(2 * gam)), HF::zmul(X[2 * gam + 1], Hn.at(2 * gam + 1)));
        const f4v d = HF::mma16(aA[gam], bop, f4v{0.f, 0.f, 0.f, 0.f});
        c0 = HF::pack_acc(d[0], d[1]);
        c1 = HF::pack_acc(d[2], d[3]);
    }
    // pass B: radix 16 over r for p = 4w + gam (reads cc), the twiddle, and
    // b[col][j], j = 4w + gam + 8 (8h + 2g + i), four consecutive j per store
    __device__ __forceinline__ void pass_b(const uint32_t *ccr, uint32_t *bbw) const
    {
        uint32_t pb[2][2][4];          // [h][i][gam]
#pragma unroll
        for (int gam = 0; gam < 4; ++gam) {
            const uint4 bop = *reinterpret_cast<const uint4 *>(ccr + 16 * gam);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f4v d = HF::mma32(aD[h], bop, f4v{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int i = 0; i < 2; ++i) pb[h][i][gam] = HF::twmul(d[2 * i], d[2 * i + 1], twc[gam][h][i]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                *reinterpret_cast<uint4 *>(bbw + (16 * h + 2 * i) * mix::BJ) =
                    make_uint4(pb[h][i][0], pb[h][i][1], pb[h][i][2], pb[h][i][3]);
    }
    // pass C, columns j = 16 (4w + gam) + col: radix 16 over k1.  The
    // operand is read from bb, then each half h of the outputs is one
    // product whose rows are outputs m = 8h + 2g + i (re, im)
    __device__ __forceinline__ uint4 pass_c_operand(const uint32_t *bbr, int gam) const
    {
        const uint32_t *src = bbr + 4 * gam * mix::BJ;
        return make_uint4(src[0], src[4], src[8], src[12]);
    }
    __device__ __forceinline__ f4v pass_c(int h, uint4 bop) const
    {
        return HF::mma32(aD[h], bop, f4v{0.f, 0.f, 0.f, 0.f});
    }
};

// per-lane LDS bases of the exchanges (the per-group offsets are constants)
struct MixBases {
    uint32_t *ccw;         // pass A writes c[2g + c][col][8w + 4a ..]
    const uint32_t *ccr;   // pass B reads c[4w + gam][col][4g ..]
    uint32_t *bbw;         // pass B writes b[col][4w + gam + 8 q']
    const uint32_t *bbr;   // pass C reads b[4g ..][16 (4w + gam) + col]
    __device__ __forceinline__ MixBases(uint32_t *cc, uint32_t *bb, int w, int l)
    {
        const int col = l & 15, g = l >> 4;
        ccw = cc + mix::cc_word(2 * g, col, 8 * w);
        ccr = cc + mix::cc_word(4 * w, col, 4 * g);
        bbw = bb + mix::bb_word(4 * w + 16 * g, col);
        bbr = bb + mix::bb_word(64 * w + col, 4 * g);
    }
    __device__ __forceinline__ void store_a(const uint32_t (&pa)[2][8]) const
    {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                *reinterpret_cast<uint4 *>(ccw + 16 * c + 4 * a) =
                    make_uint4(pa[c][4 * a], pa[c][4 * a + 1], pa[c][4 * a + 2], pa[c][4 * a + 3]);
    }
};

// template spectra of template t for work-item tau (its 16 values, contiguous)
__device__ __forceinline__ void load_h16(const void *__restrict__ H16, int t, int tau, HSpec &Hn)
{
    const uint4 *Ht = reinterpret_cast<const uint4 *>(H16) + ((int64_t)t * mix::L + tau * 16) / 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) Hn.q[k] = Ht[k];
}

// staged spectrum of global segment s for work-item tau
__device__ __forceinline__ void load_x16(const uint2 *__restrict__ Xs, int64_t s, int tau, uint32_t (&X)[16])
{
    const uint2 *src = Xs + s * (mix::L / 2) + tau;
#pragma unroll
    for (int vp = 0; vp < 8; ++vp) {
        const uint2 f = src[vp * mix::T];
        X[2 * vp] = f.x;
        X[2 * vp + 1] = f.y;
    }
}

// Items u = (segment s = u / M, template t = u % M), persistent: each
// workgroup takes one contiguous range.  They run as a software pipeline
// over the two exchange buffers: after pass B of item u (cc -> bb) and a
// barrier, pass C of item u (reads bb) and pass A of item u + 1 (writes cc)
// run interleaved in one phase, so the matrix products of one overlap the
// vector work of the other.
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void fdfir_mixed_kernel(
    const uint2 *__restrict__ Xs, const float *__restrict__ ps, int64_t n, const void *__restrict__ H16,
    const c32 *__restrict__ twL, const uint4 *__restrict__ mat, int M, int D, int V, int64_t items,
    float *__restrict__ P, int64_t ld)
{
    constexpr int L = mix::L;
    __shared__ __align__(16) uint32_t cc[mix::CC_WORDS];
    __shared__ __align__(16) uint32_t bb[mix::BB_WORDS];
    // Per-wave transpose of the powers: a wave's pass C yields outputs
    // n = 64 w + j' + 128 m (j' < 64, m < 16), lane (g, col) holding rows
    // m = 8 h + 2 g + i of column j' = 16 gam + col.  Each lane writes its
    // four rows of a column (2g, 2g + 1, 2g + 8, 2g + 9) as one 16-byte
    // chunk; lane j' then reads its column's four chunks and stores the 16
    // rows back as rows of 64 consecutive floats.  Chunk g of column j' sits
    // at mix::stage_word(j', g), rotated so that the 16-byte writes and
    // reads are free of bank conflicts (16-byte accesses are served 8 lanes
    // at a time: a rotation by j' / 4, distinct over 16 lanes of 64 banks
    // only, measured 16 more conflict cycles per wave and item).  The
    // staging reuses the wave's own rows of bb (its pass-C operands,
    // 16 x BJ >= 1024 words, dead once read).
    static_assert(16 * mix::BJ >= mix::STAGE_WORDS, "power staging does not fit the wave's rows of bb");

    const int tau = threadIdx.x, w = tau >> 6, l = tau & 63, col = l & 15, g = l >> 4;
    const MixBases xb(cc, bb, w, l);
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t u0 = items * b / nb, u1 = items * (b + 1) / nb;
    if (u0 >= u1) return;
    MixLane ml;
    ml.init(mat, twL, w, l);

    int64_t s = u0 / M;                // segment and template of item u
    int t = (int)(u0 - s * M);
    int64_t sa = s;                    // segment and template of the pass-A item
    int ta = t;
    HSpec Hn;                          // template spectra of the pass-A item
    uint32_t X[16];                    // sigma-scaled spectrum of segment sa at zq(w, l, v)
    // advance the pass-A item; its template spectra are in flight from here on
    auto next_a = [&]() {
        if (++ta == M) { ta = 0; ++sa; }
        load_h16(H16, ta, tau, Hn);
    };

    load_h16(H16, ta, tau, Hn);
    load_x16(Xs, sa, tau, X);
    float pscale = ps[s];              // 2^-2(e_s + eh) of the pass-A segment
    {
        uint32_t pa[2][8];
#pragma unroll
        for (int gam = 0; gam < 8; ++gam) ml.pass_a(X, Hn, gam, pa[0][gam], pa[1][gam]);
        next_a();
        xb.store_a(pa);
    }
    // Drain the prologue's loads here (matrices, twiddles, first spectra):
    // a load still outstanding at the loop entry would otherwise leave a
    // memory-counter wait inside the loop, which on every item would also
    // wait for the previous item's power stores.
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    for (int64_t u = u0; u < u1; ++u) {
        ml.pass_b(xb.ccr, xb.bbw);
        // the pass-A item u + 1 may start a new segment (past the last item
        // pass A runs on stale data and its result is never read)
        const float pscale_u = pscale;
        if (sa != s && u + 1 < u1) {
            load_x16(Xs, sa, tau, X);
            pscale = ps[sa];
        }
        __syncthreads();
        // ---- pass C of item u interleaved with pass A of item u + 1 ----
        // (cc is free: pass B of u read it before the barrier)
        // Power stores go through a buffer resource spanning this segment's
        // kept outputs P_t[sV, sV + hi - D): offsets are taken relative to
        // output D of the segment, so a discarded output (n < D) has a
        // negative offset, which wraps past the resource's range, and a store
        // beyond the input's end is past it too; the hardware drops both.
        const int64_t base = s * V - D;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            P + (int64_t)t * ld + s * V, 0, 4 * ((int)min<int64_t>(L, n - base) - D), kBufWord3);
        float *const otw = reinterpret_cast<float *>(bb) + 16 * w * mix::BJ;
        uint32_t pa[2][8];
        uint4 bops[4];
#pragma unroll
        for (int gam = 0; gam < 4; ++gam) bops[gam] = ml.pass_c_operand(xb.bbr, gam);
#pragma unroll
        for (int gam = 0; gam < 4; ++gam) {
            ml.pass_a(X, Hn, 2 * gam, pa[0][2 * gam], pa[1][2 * gam]);
            ml.pass_a(X, Hn, 2 * gam + 1, pa[0][2 * gam + 1], pa[1][2 * gam + 1]);
            const f4v d0 = ml.pass_c(0, bops[gam]), d1 = ml.pass_c(1, bops[gam]);
            const int jc = 16 * gam + col;
            *reinterpret_cast<float4 *>(otw + mix::stage_word(jc, g)) =
                make_float4((d0[0] * d0[0] + d0[1] * d0[1]) * pscale_u, (d0[2] * d0[2] + d0[3] * d0[3]) * pscale_u,
                            (d1[0] * d1[0] + d1[1] * d1[1]) * pscale_u, (d1[2] * d1[2] + d1[3] * d1[3]) * pscale_u);
        }
        // 16 rows of 64 consecutive outputs per wave (the wave's own region:
        // its LDS accesses are executed in order, so its pass-C reads above
        // are done before these rows are overwritten; no barrier needed)
        const int off0 = 4 * (64 * w + l - D);
        float4 pw[4];                  // pw[gq] = rows 2gq, 2gq + 1, 2gq + 8, 2gq + 9
#pragma unroll
        for (int gq = 0; gq < 4; ++gq)
            pw[gq] = *reinterpret_cast<const float4 *>(otw + mix::stage_word(l, gq));
#pragma unroll
        for (int m = 0; m < 16; ++m)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((&pw[(m >> 1) & 3].x)[2 * (m >> 3) + (m & 1)]), rs,
                                                  off0 + 512 * m, 0, kNonTemporal);
        next_a();
        xb.store_a(pa);
        __syncthreads();
        if (++t == M) { t = 0; ++s; }
    }
}

// ---------------------------------------------------------------------------
// batched form: many spectra, each reduced to its top-K cells
// ---------------------------------------------------------------------------

// Forward transforms of every segment of a batch: block sg is global segment
// sg; items are ordered (array, segment, template), so the global segment of
// item u is u / M and array a's segments start at item_begin[a] / M.
template <bool BF>
__global__ __launch_bounds__(128) void mixed_fwd_batch_kernel(BatchSet bs, int M, const c32 *__restrict__ twL,
                                                              int D, int V, int eh, uint2 *__restrict__ Xs,
                                                              float *__restrict__ ps)
{
    const int64_t sg = blockIdx.x;
    int a = 0;
    while (bs.item_begin[a + 1] <= sg * M) ++a;        // uniform: at most 128 steps
    const int64_t base = (sg - bs.item_begin[a] / M) * V - D;
    forward_scaled<BF>(reinterpret_cast<const uint32_t *>(bs.x[a]), bs.n[a], base, twL, eh,
                       Xs + sg * (mix::L / 2), ps + sg);
}

// The template loop of fdfir_mixed_kernel over the items of a batch, with
// the power plane replaced by an exact running top-K per array in LDS (the
// scheme of the float32 batched kernel: a uniform threshold, candidates
// appended to an LDS list, ranked into the kept list), written to the
// workspace as one list per array the workgroup touches.
// (3 waves per SIMD with a few spills outside the hot loop, which measured
// 5% faster than 2)
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void fdfir_mixed_topk_kernel(
    BatchSet bs, const uint2 *__restrict__ Xs, const float *__restrict__ ps, const void *__restrict__ H16,
    const c32 *__restrict__ twL, const uint4 *__restrict__ mat, int M, int D, int V, int K, int64_t items,
    Cand *__restrict__ stage, int2 *__restrict__ hdr, int *__restrict__ nslots, int max_slots)
{
    constexpr int L = mix::L, T = mix::T;
    __shared__ __align__(16) uint32_t cc[mix::CC_WORDS];
    // the B->C exchange, and after pass C the candidate list (up to L cells)
    __shared__ __align__(16) uint32_t bx[2 * L];
    static_assert(mix::BB_WORDS <= 2 * L, "LDS");
    __shared__ float keptP[2][TOPK_MAX];
    __shared__ int keptT[2][TOPK_MAX];
    __shared__ int keptI[2][TOPK_MAX];
    __shared__ float smax[T];
    __shared__ int s_cnt;
    __shared__ float s_thr;
    float2 *cand = reinterpret_cast<float2 *>(bx);

    const int tau = threadIdx.x, w = tau >> 6, l = tau & 63, col = l & 15, g = l >> 4;
    const MixBases xb(cc, bx, w, l);
    const int nbase = 64 * w + col + 256 * g;     // bin of this lane's value (gam, h, i) = 0 within a segment
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t u0 = items * b / nb, u1 = items * (b + 1) / nb;
    if (u0 >= u1) {
        if (tau == 0) nslots[b] = 0;
        return;
    }
    MixLane ml;
    ml.init(mat, twL, w, l);

    // item u: global segment gs = u / M, template t; array a; its segments
    // are the global segments [seg0, seg1)
    int64_t gs = u0 / M;
    int t = (int)(u0 - gs * M);
    int a = 0;
    while (bs.item_begin[a + 1] <= u0) ++a;
    int64_t seg0 = bs.item_begin[a] / M, seg1 = bs.item_begin[a + 1] / M;
    // the pass-A item u + 1 runs one phase ahead
    int64_t gsa = gs;
    int ta = t;
    HSpec Hn;
    uint32_t X[16];
    auto next_a = [&]() {
        if (++ta == M) { ta = 0; ++gsa; }
        load_h16(H16, ta, tau, Hn);
    };

    int par = 0, kc = 0, slot = 0;
    float thr = -1.f;
    auto flush = [&](int arr) {
        if (slot < max_slots) {
            Cand *dst = stage + ((int64_t)b * max_slots + slot) * K;
            if (tau < kc) {
                Cand c;
                c.t = keptT[par][tau];
                c.bin = keptI[par][tau];
                c.p = keptP[par][tau];
                dst[tau] = c;
            }
            if (tau == 0) hdr[(int64_t)b * max_slots + slot] = make_int2(arr, kc);
        }
        ++slot;
    };

    if (tau == 0) s_cnt = 0;
    load_h16(H16, ta, tau, Hn);
    load_x16(Xs, gsa, tau, X);
    float pscale = ps[gs];
    {
        uint32_t pa[2][8];
#pragma unroll
        for (int gam = 0; gam < 8; ++gam) ml.pass_a(X, Hn, gam, pa[0][gam], pa[1][gam]);
        next_a();
        xb.store_a(pa);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    for (int64_t u = u0; u < u1; ++u) {
        ml.pass_b(xb.ccr, xb.bbw);
        const float pscale_u = pscale;
        if (gsa != gs && u + 1 < u1) {
            load_x16(Xs, gsa, tau, X);
            pscale = ps[gsa];
        }
        __syncthreads();
        // ---- pass C of item u (powers kept in registers) with pass A of u + 1 ----
        const int64_t base = (gs - seg0) * V - D;
        const int hi = (int)min<int64_t>(L, bs.n[a] - base);
        float pw[4][2][2];
        uint32_t pa[2][8];
#pragma unroll
        for (int gam = 0; gam < 4; ++gam) {
            ml.pass_a(X, Hn, 2 * gam, pa[0][2 * gam], pa[1][2 * gam]);
            const uint4 bop = ml.pass_c_operand(xb.bbr, gam);
            ml.pass_a(X, Hn, 2 * gam + 1, pa[0][2 * gam + 1], pa[1][2 * gam + 1]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f4v d = ml.pass_c(h, bop);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int nn = nbase + 16 * gam + 1024 * h + 128 * i;
                    const float p = (d[2 * i] * d[2 * i] + d[2 * i + 1] * d[2 * i + 1]) * pscale_u;
                    pw[gam][h][i] = (nn >= D && nn < hi) ? p : -1.f;     // -1: not an output
                }
            }
        }
        next_a();
        xb.store_a(pa);
        // ---- top-K of item u's cells, merged into the workgroup's list ----
        float mx = -1.f;
#pragma unroll
        for (int gam = 0; gam < 4; ++gam)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 2; ++i) mx = fmaxf(mx, pw[gam][h][i]);
        float th = thr;
        if (kc < K) {
            // no full list yet: the K-th largest per-work-item maximum is a
            // lower bound of this item's K-th largest cell
            smax[tau] = mx;
            __syncthreads();
            int gt = 0, ge = 0;
            for (int q = 0; q < T; ++q) {
                const float o = smax[q];
                gt += o > mx;
                ge += o >= mx;
            }
            if (gt < K && ge >= K) s_thr = mx;
            __syncthreads();
            th = s_thr;
        }
        // some cell qualifies exactly when the item's maximum does
        const bool any = mx >= 0.f && mx >= th;
        // (also the barrier after pass C's reads of bx and pass A's writes of cc)
        if (__syncthreads_or(any)) {
#pragma unroll
            for (int gam = 0; gam < 4; ++gam)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        if (pw[gam][h][i] >= 0.f && pw[gam][h][i] >= th) {
                            const int c = atomicAdd(&s_cnt, 1);
                            cand[c] = make_float2(pw[gam][h][i],
                                                  __int_as_float(nbase + 16 * gam + 1024 * h + 128 * i));
                        }
            __syncthreads();
            const int cnt = s_cnt;
            const int total = kc + cnt;
            for (int e = tau; e < total; e += T) {
                float pe;
                int te, ie;
                if (e < kc) {
                    pe = keptP[par][e];
                    te = keptT[par][e];
                    ie = keptI[par][e];
                } else {
                    const float2 c = cand[e - kc];
                    pe = c.x;
                    te = t;
                    ie = (int)(base + __float_as_int(c.y));
                }
                int rank = 0;
                for (int f = 0; f < kc; ++f) rank += beats(keptP[par][f], keptT[par][f], keptI[par][f], pe, te, ie);
                for (int f = 0; f < cnt; ++f) {
                    const float2 c = cand[f];
                    rank += beats(c.x, t, (int)(base + __float_as_int(c.y)), pe, te, ie);
                }
                if (rank < K) {
                    keptP[par ^ 1][rank] = pe;
                    keptT[par ^ 1][rank] = te;
                    keptI[par ^ 1][rank] = ie;
                }
            }
            __syncthreads();
            par ^= 1;
            kc = min(K, total);
            thr = kc == K ? keptP[par][K - 1] : -1.f;
            if (tau == 0) s_cnt = 0;        // read again only after the next item's barriers
        }
        // ---- next item ----
        if (++t == M) {
            t = 0;
            if (++gs == seg1) {
                flush(a);
                kc = 0;
                thr = -1.f;
                if (++a < bs.count) {
                    seg0 = seg1;
                    seg1 = bs.item_begin[a + 1] / M;
                }
            }
        }
    }
    if (kc > 0) flush(a);
    if (tau == 0) nslots[b] = min(slot, max_slots);
}

// ---------------------------------------------------------------------------

size_t mixed_matrix_bytes() { return MAT_BYTES; }

hipError_t launch_mat_table(void *tab, hipStream_t st)
{
    const dim3 grid((MAT_A_UINT2 + 2 * 64 + 255) / 256), blk(256);
    hipLaunchKernelGGL(mat_table_kernel, grid, blk, 0, st, (uint4 *)tab);
    return hipGetLastError();
}

size_t mixed_spectra_bytes(int M) { return sizeof(uint32_t) * (size_t)M * mix::L; }

hipError_t launch_tspec_mix(const c32 *taps, const int *tap_len, int kp, int M, float scale, void *H16,
                            hipStream_t st)
{
    const int64_t total = (int64_t)M * mix::L;
    dim3 grid((unsigned)((total + 255) / 256)), blk(256);
    hipLaunchKernelGGL(tspec_mix_kernel, grid, blk, 0, st, taps, tap_len, kp, M, scale, (uint32_t *)H16);
    return hipGetLastError();
}

int mixed_blocks_per_cu()
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fdfir_mixed_kernel, 128, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int mixed_topk_blocks_per_cu()
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fdfir_mixed_topk_kernel, 128, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_mixed_topk(const MixedTopkArgs &a, hipStream_t st)
{
    uint2 *Xs = (uint2 *)a.xstage;
    float *ps = (float *)((char *)a.xstage + (size_t)a.segments * mix::L * sizeof(uint32_t));
    const dim3 gf((unsigned)a.segments), blk(128), gi((unsigned)a.grid);
    if (a.bf)
        hipLaunchKernelGGL(mixed_fwd_batch_kernel<true>, gf, blk, 0, st, *a.bs, a.M, a.twL, a.D, a.V, a.eh, Xs, ps);
    else
        hipLaunchKernelGGL(mixed_fwd_batch_kernel<false>, gf, blk, 0, st, *a.bs, a.M, a.twL, a.D, a.V, a.eh, Xs, ps);
    hipLaunchKernelGGL(fdfir_mixed_topk_kernel, gi, blk, 0, st, *a.bs, Xs, ps, a.H16, a.twL, (const uint4 *)a.mat,
                       a.M, a.D, a.V, a.K, a.items, (Cand *)a.stage, (int2 *)a.hdr, a.nslots, a.max_slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_topk_merge(a.stage, a.hdr, a.nslots, (int)a.grid, a.max_slots, a.K, a.bs->count, a.out, st);
}

static_assert(mix::L == MIXED_L, "staging size of the 16-bit plans (mixed_stage_bytes)");

hipError_t launch_mixed(const MixedArgs &a, hipStream_t st)
{
    // stage: [segments][L] packed binary16 complex, then [segments] float
    uint2 *Xs = (uint2 *)a.stage;
    float *ps = (float *)((char *)a.stage + (size_t)a.segments * mix::L * sizeof(uint32_t));
    const dim3 gf((unsigned)a.segments), blk(128), gi((unsigned)a.grid);
    if (a.bf)
        hipLaunchKernelGGL(mixed_fwd_kernel<true>, gf, blk, 0, st, (const uint32_t *)a.x, a.n, a.twL, a.D, a.V,
                           a.eh, Xs, ps);
    else
        hipLaunchKernelGGL(mixed_fwd_kernel<false>, gf, blk, 0, st, (const uint32_t *)a.x, a.n, a.twL, a.D, a.V,
                           a.eh, Xs, ps);
    hipLaunchKernelGGL(fdfir_mixed_kernel, gi, blk, 0, st, Xs, ps, a.n, a.H16, a.twL, (const uint4 *)a.mat, a.M,
                       a.D, a.V, a.items, a.P, a.ld);
    return hipGetLastError();
}

}  // namespace fdas
