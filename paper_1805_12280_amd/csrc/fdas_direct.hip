// fdas_direct.hip -- direct convolution (Section 3.1, Eq. (1)) of the
// shortest templates of a float32 plan on the matrix cores, with the power
// of Section 4.3, at float32-class accuracy.
//
// For a template of K taps, overlap-save costs one inverse FFT of L points
// per segment and template whatever K is, while direct convolution costs K
// complex products per output (the crossover the paper studies between its
// time- and frequency-domain kernels).  On the matrix cores the direct form
// is a dense product: rows are templates, columns are outputs, and the
// contraction runs over taps against a sliding window of the input.  A
// float32 plan routes its shortest templates here and the rest to the
// overlap-save kernel; both write the same plane.
//
// Product, per 16 outputs i0 + j (j < 16), 8 templates and 16 taps, one
// v_mfma_f32_16x16x32_f16 (K = 32 real values = 16 complex taps):
//   y_t[i] = sum_{k' < KP} x[i - KP + 1 + k'] h'_t[k'],   h'_t[k'] = h_t[KP - 1 - k']
// (the taps reversed and zero-padded to KP = 16 NK, so the operand is the
// window x[i - KP + 1 ..] read forward).  Complex values become real ones by
// interleaving re/im along K and along the rows: row 2tt of A gives Re y,
// row 2tt + 1 gives Im y, with the entries [hr, -hi] and [hi, hr] of the
// complex weight.  Lane layouts:
//   A[row][k]: lane row + 16 (k / 8), element k % 8
//   B[k][j]:   lane j + 16 (k / 8),   element k % 8
//   D[row][j]: lane j + 16 (row / 4), element row % 4
// so lane (j, g = l / 16) reads four consecutive complex inputs x[..+4g..]
// for its B operand, and holds Re/Im of templates 2g and 2g + 1 for output
// j.  A block's tap operands take 8 NK registers and a tile's accumulator
// 4, so a wave keeps them all in registers at 3 waves per SIMD.
//
// Float32-class accuracy from binary16 operands: every operand v (scaled by a
// power of two so |v| < 2^14) is split v = hi + lo with hi = fp16(v) and
// lo = fp16(v - hi) (v - hi is exact in float32), and each product is
// A_hi B_hi + A_hi B_lo + A_lo B_hi accumulated in float32: 22 significant
// bits per operand, the dropped A_lo B_lo term below 2^-22 of the product.
// The taps are split once at plan time (float64, on the host); the input is
// split by the wave that stages it.  The powers are unscaled exactly by
// ldexp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fdas_internal.h"
#include "seg_fft.h"

namespace fdas {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

namespace {
constexpr int kWaveOut = 512;                  // outputs per wave: 32 tiles of 16
constexpr int kWaves = 4;                      // waves per workgroup
constexpr int kMaxNK = DIRECT_MAX_NK;          // K steps of 16 taps: up to 96 taps
constexpr int kSpan = kWaveOut + 16 * kMaxNK;  // staged inputs per wave (>= 512 + KP - 1)
// LDS words between the two shifted copies of a plane: even (8-byte rows),
// 16 more than a multiple of 32, so the copies start 16 banks apart
constexpr int kCopy = (kSpan + 1) / 2 * 2 + ((16 - ((kSpan + 1) / 2 * 2) % 32) + 32) % 32;
static_assert(kCopy % 2 == 0 && kCopy % 32 == 16 && kCopy >= kSpan, "copy stride");
constexpr int kScaleExp = 14;                  // operands scaled into [2^13, 2^14)
// words per power staging row: 64 outputs plus 8, so the half-wave that
// writes rows 2g + s for g = 0, 1 (lanes 0..31) lands 2 x 72 = 144 = 16
// (mod 32) banks apart and fills all 32 banks once
constexpr int kRow = 72;

// round a float to binary16 and back (the high part of a split)
__device__ __forceinline__ float hi_part(float v) { return (float)(_Float16)v; }

__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    h2v v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ f4v mma(uint4 a, uint4 b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0, 0);
}

// One block of 8 templates with NK steps of 16 taps over the wave's 32
// tiles of 16 outputs.  Tile v at step k reads the window at staged offset
// 16 v + 16 k = 16 beta with beta = v + k, so one window read (beta) feeds
// the NK tiles beta - NK + 1 .. beta, one step each: the windows are read
// once each, in order, and the NK tiles they feed accumulate as independent
// chains in slots v % NK.  The sweep over the 32 + NK - 1 windows is fully
// unrolled, so every slot, tile and store position is a constant and the
// only scalar work left is the block's set-up.
// xh/xl: the wave's staged high and low planes (one word, a complex binary16
// pair, per element), each as two copies kCopy words apart, copy c shifted
// by c elements (word i of copy c is element i + c): a lane's four
// consecutive elements starting at element q are two aligned 8-byte words
// of copy q % 2.  Read 16 lanes at a time, the even lanes j of a half-wave
// take banks j, j + 1 of copy 0 and the odd ones banks 16 + j - 1, 16 + j of
// copy 1 (mod 32): all 32 banks once, for each of the two reads.
template <int NK>
__device__ __forceinline__ void run_block(const uint4 *__restrict__ A, const int *__restrict__ rows,
                                          const int *__restrict__ pexp, const uint32_t *xh, const uint32_t *xl,
                                          float *pw, int kpmax, int sx2, int64_t o0, int64_t n,
                                          float *__restrict__ P, int64_t ld, int l)
{
    constexpr int NT = kWaveOut / 16;                  // tiles per wave
    constexpr int NW = NT + NK - 1;                    // windows
    const int j = l & 15, g = l >> 4;
    // one buffer resource per plane row, based at the wave's first output
    // and spanning its outputs below n (a padding row, row < 0, spans
    // nothing), so a store needs only the lane's byte offset and the
    // hardware drops the tail
    const int span = (int)max<int64_t>(0, min<int64_t>(kWaveOut, n - o0));
    __amdgpu_buffer_rsrc_t rs[DIRECT_BLOCK];
#pragma unroll
    for (int tt = 0; tt < DIRECT_BLOCK; ++tt) {
        const int row = __builtin_amdgcn_readfirstlane(rows[tt]);
        rs[tt] = __builtin_amdgcn_make_buffer_rsrc(P + (int64_t)max(row, 0) * ld + o0, 0, row < 0 ? 0 : 4 * span,
                                                   kBufWord3);
    }
    uint4 ah[NK], al[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        ah[k] = A[(2 * k) * 64 + l];
        al[k] = A[(2 * k + 1) * 64 + l];
    }
    // power scale of this lane's 2 templates (tt = 2g + s)
    int pe[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) pe[s] = pexp[2 * g + s] - sx2;
    // staged index of this lane's first element at window 0 (windows move
    // by 16 elements, so its parity picks the copy for every window)
    const int qoff = kpmax - 16 * NK + j + 4 * g;
    const int cpy = qoff & 1;
    const uint2 *bh2 = reinterpret_cast<const uint2 *>(xh + cpy * kCopy + (qoff - cpy));
    const uint2 *bl2 = reinterpret_cast<const uint2 *>(xl + cpy * kCopy + (qoff - cpy));
    f4v acc[NK];
    const f4v zero = {};
    auto window = [&](int beta, uint4 &bh, uint4 &bl) {
        const uint2 h0 = bh2[8 * beta], h1 = bh2[8 * beta + 1];
        const uint2 l0 = bl2[8 * beta], l1 = bl2[8 * beta + 1];
        bh = make_uint4(h0.x, h0.y, h1.x, h1.y);
        bl = make_uint4(l0.x, l0.y, l1.x, l1.y);
    };
    uint4 nh, nl;
    window(0, nh, nl);
#pragma unroll
    for (int beta = 0; beta < NW; ++beta) {
        // this window's operands; the next window's are read now, one
        // window ahead of their use
        const uint4 bh = nh, bl = nl;
        if (beta + 1 < NW) window(beta + 1, nh, nl);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int v = beta - k;                    // tile fed at step k
            if (v < 0 || v >= NT) continue;
            f4v &c = acc[v % NK];
            c = mma(ah[k], bh, k == 0 ? zero : c);
            c = mma(ah[k], bl, c);
            c = mma(al[k], bh, c);
        }
        // tile beta - NK + 1 is complete: its powers go to the wave's
        // staging rows pw[tt][kRow] (outputs 16 (v % 4) + j); after every
        // fourth tile, each row's 64 outputs are written by one store
        // instruction (256 contiguous bytes of one plane row)
        const int v = beta - (NK - 1);
        if (v < 0) continue;
        const f4v &c = acc[v % NK];
#pragma unroll
        for (int s = 0; s < 2; ++s)
            pw[(2 * g + s) * kRow + 16 * (v & 3) + j] = ldexpf(c[2 * s] * c[2 * s] + c[2 * s + 1] * c[2 * s + 1], pe[s]);
        if ((v & 3) == 3) {
            float val[DIRECT_BLOCK];
#pragma unroll
            for (int tt = 0; tt < DIRECT_BLOCK; ++tt) val[tt] = pw[tt * kRow + l];
            const int off = 4 * (16 * (v - 3) + l);
#pragma unroll
            for (int tt = 0; tt < DIRECT_BLOCK; ++tt)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val[tt]), rs[tt], off, 0, kNonTemporal);
        }
    }
}

}  // namespace

// Grid: one wave per 512 outputs, kWaves waves per workgroup.  Each wave
// stages x[o0 - kpmax + 1, o0 + 512) (zero outside [0, n)) in its own LDS
// rows, scaled by 2^sx (so every component is below 2^14) and split into
// binary16 high and low parts, then runs every direct block over its 32
// tiles.  blocks: [nblk] steps of 16 taps; A: the blocks' split tap
// operands, block b at aoff[b] (uint4 units): for step k, 64 lanes of hi
// then 64 of lo; rows/pexp: [nblk][8] plane row (-1 for padding) and -2 x
// (the template's scale exponent).
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3))) void dconv_kernel(
    const c32 *__restrict__ x, int64_t n, const uint4 *__restrict__ A, const int *__restrict__ aoff,
    const int *__restrict__ nks, const int *__restrict__ rows, const int *__restrict__ pexp, int nblk, int kpmax,
    float *__restrict__ P, int64_t ld)
{
    // per wave: the staged elements' high plane and low plane, two shifted
    // copies each (see run_block)
    __shared__ __align__(16) uint32_t sh[kWaves][2][2 * kCopy];
    __shared__ float spw[kWaves][DIRECT_BLOCK * kRow];   // per wave: powers of four tiles
    // the wave index is uniform across the wave: every address and bound
    // derived from it below stays in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int64_t o0 = ((int64_t)blockIdx.x * kWaves + w) * kWaveOut;
    uint32_t *xh = sh[w][0], *xl = sh[w][1];
    const int span = kWaveOut + kpmax - 1;
    const int64_t org = o0 - kpmax + 1;

    // stage: load, scale by the wave's power of two, split
    constexpr int kPer = (kSpan + 63) / 64;
    c32 v[kPer];
    float mx = 0.f;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int q = l + 64 * r;
        const int64_t idx = org + q;
        v[r] = (q < span && idx >= 0 && idx < n) ? x[idx] : mk(0.f, 0.f);
        mx = fmaxf(mx, fmaxf(fabsf(v[r].re), fabsf(v[r].im)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    int sx = 0;
    if (mx > 0.f) {
        int ex;
        frexpf(mx, &ex);                   // mx < 2^ex
        sx = kScaleExp - ex;
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int q = l + 64 * r;
        if (q < kSpan) {
            const float re = ldexpf(v[r].re, sx), im = ldexpf(v[r].im, sx);
            const float hr = hi_part(re), hi = hi_part(im);
            const uint32_t wh = pack2(hr, hi), wl = pack2(re - hr, im - hi);
#pragma unroll
            for (int c = 0; c < 2; ++c)
                if (q >= c) {
                    xh[c * kCopy + q - c] = wh;
                    xl[c * kCopy + q - c] = wl;
                }
        }
    }
    __syncthreads();                       // (each wave reads only its own rows)
    if (o0 >= n) return;
    for (int b = 0; b < nblk; ++b) {
        const uint4 *Ab = A + aoff[b];
        const int *rb = rows + 8 * b, *pb = pexp + 8 * b;
        switch (nks[b]) {
#define FDAS_DCONV_CASE(K) \
    case K: run_block<K>(Ab, rb, pb, xh, xl, spw[w], kpmax, 2 * sx, o0, n, P, ld, l); break;
            FDAS_DCONV_CASE(1) FDAS_DCONV_CASE(2) FDAS_DCONV_CASE(3)
            FDAS_DCONV_CASE(4) FDAS_DCONV_CASE(5) FDAS_DCONV_CASE(6)
#undef FDAS_DCONV_CASE
        default: break;
        }
    }
}

static_assert(kMaxNK == 6, "one case per step count");

// ---------------------------------------------------------------------------
// plan-time tables (host, float64)
// ---------------------------------------------------------------------------

int direct_nk(int taps) { return std::max(1, (taps + 15) / 16); }

void build_direct_tables(const c32 *taps, const int *tap_len, int M, int kp, const std::vector<int> &order,
                         int nblk, DirectTables &out)
{
    constexpr int BT = DIRECT_BLOCK;
    out.nblk = nblk;
    out.nks.assign(nblk, 1);
    out.aoff.assign(nblk, 0);
    out.rows.assign(BT * (size_t)nblk, -1);
    out.pexp.assign(BT * (size_t)nblk, 0);
    out.A.clear();
    out.kpmax = 16;
    for (int b = 0; b < nblk; ++b) {
        int kmax = 0;
        for (int tt = 0; tt < BT && BT * b + tt < M; ++tt) kmax = std::max(kmax, tap_len[order[BT * b + tt]]);
        const int NK = direct_nk(kmax), KP = 16 * NK;
        out.nks[b] = NK;
        out.kpmax = std::max(out.kpmax, KP);
        out.aoff[b] = (int)out.A.size();
        // per template: scale 2^st so the largest component is below 2^14
        int st[BT] = {0};
        for (int tt = 0; tt < BT && BT * b + tt < M; ++tt) {
            const int t = order[BT * b + tt];
            double m = 0.0;
            for (int k = 0; k < tap_len[t]; ++k)
                m = std::max(m, std::max(std::fabs((double)taps[(size_t)t * kp + k].re),
                                         std::fabs((double)taps[(size_t)t * kp + k].im)));
            int e = 0;
            if (m > 0.0) std::frexp(m, &e);                // m < 2^e
            st[tt] = m > 0.0 ? 14 - e : 0;
            out.rows[BT * b + tt] = t;
            out.pexp[BT * b + tt] = -2 * st[tt];
        }
        for (int k = 0; k < NK; ++k)
            for (int part = 0; part < 2; ++part)
                for (int l = 0; l < 64; ++l) {
                    uint16_t e16[8];
                    for (int e = 0; e < 8; ++e) {
                        const int row = l & 15, kk = 8 * (l >> 4) + e;
                        const int tt = row >> 1, a = row & 1, c = kk & 1;
                        const int kr = 16 * k + (kk >> 1);             // reversed tap index k'
                        const int tap = KP - 1 - kr;                   // original tap index
                        double val = 0.0;
                        if (BT * b + tt < M) {
                            const int t = order[BT * b + tt];
                            if (tap >= 0 && tap < tap_len[t]) {
                                const c32 h = taps[(size_t)t * kp + tap];
                                const double hr = std::ldexp((double)h.re, st[tt]);
                                const double hi = std::ldexp((double)h.im, st[tt]);
                                val = a == 0 ? (c == 0 ? hr : -hi) : (c == 0 ? hi : hr);
                            }
                        }
                        const _Float16 vh = (_Float16)val;
                        const _Float16 vl = (_Float16)(val - (double)vh);
                        e16[e] = __builtin_bit_cast(uint16_t, part == 0 ? vh : vl);
                    }
                    uint4 u;
                    u.x = e16[0] | ((uint32_t)e16[1] << 16);
                    u.y = e16[2] | ((uint32_t)e16[3] << 16);
                    u.z = e16[4] | ((uint32_t)e16[5] << 16);
                    u.w = e16[6] | ((uint32_t)e16[7] << 16);
                    out.A.push_back(u);
                }
    }
}

hipError_t launch_dconv(const DconvArgs &a, hipStream_t st)
{
    const int64_t waves = (a.n + kWaveOut - 1) / kWaveOut;
    const int64_t grid = (waves + kWaves - 1) / kWaves;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dconv_kernel, dim3((unsigned)grid), dim3(64 * kWaves), 0, st, (const c32 *)a.x, a.n,
                       (const uint4 *)a.A, a.aoff, a.nks, a.rows, a.pexp, a.nblk, a.kpmax, a.P, a.ld);
    return hipGetLastError();
}

}  // namespace fdas
