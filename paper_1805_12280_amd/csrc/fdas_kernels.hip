// fdas_kernels.hip -- gfx950 kernels of the FT-convolution hot path and
// their launchers (host side, C++ linkage, used by fdas_abi.cpp only).
//
//   twiddle_kernel     W_L^e = exp(-2 pi i e / L), float64 -> complex64 table
//   tspec_kernel       pre-transformed templates (Alg. 2, FFT of h once), in
//                      float64 from the complex64 taps, 1/L folded in, stored
//                      in the segment transform's permuted frequency order
//   fdfir_fused_kernel the overlap-save hot path (Section 3.2.2, Alg. 2):
//                      segment gather with a K_max-1 halo, one forward FFT
//                      per segment shared by all templates (the AOLS
//                      amortisation, Section 4.2.1), pointwise product,
//                      inverse FFT, discard of the first K_max-1 points and
//                      |y|^2 (Section 4.3), all in one persistent launch
//   segfft_kernel      the segment transform alone, natural order in/out
//   tdfir_kernel       direct Eq. (1) with taps in blocks of 8 accumulated in
//                      registers (overlap-add on the taps, Alg. 1)
#include "fdas_internal.h"
#include "seg_fft.h"

namespace fdas {

// ---------------------------------------------------------------------------
// plan-time tables (float64 arithmetic, rounded once)
// ---------------------------------------------------------------------------

__global__ void twiddle_kernel(c32 *twL, int L)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= L) return;
    double s, c;
    sincospi(-2.0 * (double)e / (double)L, &s, &c);
    twL[e] = mk((float)c, (float)s);
}

template <int L>
__global__ void tspec_kernel(const c32 *__restrict__ taps, const int *__restrict__ tap_len,
                             int kp, int M, c32 *__restrict__ H)
{
    using SG = Seg<L>;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * L) return;
    const int t = (int)(idx / L);
    const int rem = (int)(idx - (int64_t)t * L);
    const int e = rem / SG::T, tau = rem - e * SG::T;
    const int q = SG::perm(tau, e);
    const c32 *h = taps + (int64_t)t * kp;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < tap_len[t]; ++k) {
        const int r = (int)(((int64_t)q * k) & (L - 1));     // exact phase reduction
        double s, c;
        sincospi(-2.0 * (double)r / (double)L, &s, &c);
        const double hr = h[k].re, hi = h[k].im;
        re += hr * c - hi * s;
        im += hr * s + hi * c;
    }
    H[(int64_t)t * L + rem] = mk((float)(re / L), (float)(im / L));
}

// ---------------------------------------------------------------------------
// fused overlap-save FDFIR + power
// ---------------------------------------------------------------------------

// Work item u in [0, S*M) is (segment s = u / M, template t = u % M).  Each
// workgroup takes one contiguous range of items, so it transforms a segment
// forward once and reuses the spectrum for every template of that segment
// in its range.
//
// Segment s covers input points [s V - D, s V - D + L); its points j >= D are
// outputs s V + j - D.  D >= K_max - 1 (the overlap of Alg. 2, rounded up to
// a multiple of 32 so each segment's outputs start on a 128-byte line) and
// V = L - D.  Two LDS buffers (one per exchange) need two barriers per
// inverse transform; the template spectra of the next item are loaded into
// registers while the current item is transformed.
//
// The loops are nested (segments outside, that segment's templates inside)
// so the spectrum X is invariant in the inner loop: with one flat loop over
// items and the forward transform under a branch, X is a loop-carried value
// and the compiler copies its 32 registers twice per item.
// The kernel runs M templates of the bank: template t's spectra are H[t] and
// its powers go to row rows[t] of the plane (the plan passes its rows routed
// to overlap-save, with their spectra in that order).
template <int L>
__global__ __launch_bounds__(L / 16, L == 8192 ? 1 : 2) void fdfir_fused_kernel(
    const c32 *__restrict__ x, int64_t n, const c32 *__restrict__ H, const c32 *__restrict__ twL,
    const int *__restrict__ rows, int M, int D, int V, int64_t items, float *__restrict__ P, int64_t ld)
{
    using SG = Seg<L>;
    constexpr int T = SG::T;
    __shared__ c32 bufA[SG::LDS_ELEMS];   // pass-0 <-> pass-1 exchange
    __shared__ c32 bufC[SG::LDS_ELEMS];   // pass-1 <-> pass-2 exchange
    const int tau = threadIdx.x;
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t u0 = items * b / nb, u1 = items * (b + 1) / nb;
    if (u0 >= u1) return;

    c32 tw0[16], tw1[16];
    SG::twiddles(tau, twL, tw0, tw1);

    int64_t s = u0 / M;
    int t = (int)(u0 - s * M);
    c32 Hn[16];                            // spectra of the template of item u
    {
        const c32 *Ht = H + (int64_t)t * L;
#pragma unroll
        for (int e = 0; e < 16; ++e) Hn[e] = Ht[e * T + tau];
    }
    for (int64_t u = u0; u < u1; ++s) {
        const int64_t base = s * V - D;        // input/output index of segment point 0
        const int hi = (int)min<int64_t>(L, n - base);
        c32 X[16];
        {
            const c32 *xs = x + base;           // uniform; read only inside [0, n)
            const int lo = (int)max<int64_t>(0, -base);
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = tau + T * m;
                X[m] = (j >= lo && j < hi) ? xs[j] : mk(0.f, 0.f);
            }
            SG::fwd0(tau, X, tw0);
            __syncthreads();                    // bufA/bufC free (previous item done)
            SG::put_a(tau, X, bufA);
            __syncthreads();
            SG::fwd1(tau, X, bufA, tw1);
            SG::put_c(tau, X, bufC);
            __syncthreads();
            SG::fwd2(tau, X, bufC);
            __syncthreads();                    // bufC reads done before inv2 rewrites it
        }
        // Power stores go through a buffer resource spanning the segment's
        // kept outputs P_t[sV, sV + hi - D): offsets are relative to segment
        // point D, so a discarded point (j < D) has a negative offset, which
        // wraps past the range, and a point past the input's end is past it
        // too; the hardware drops both.  Every store is then unconditional,
        // so the compiler counts all of them between the next template's
        // spectrum loads and their use, and waits for those loads only (with
        // predicated stores it could not, and each item waited for the
        // previous item's stores to complete).
        const int nkeep = hi - D;
        const int64_t u_end = min<int64_t>(u1, u + (M - t));     // this segment's items
        for (; u < u_end; ++u) {
            c32 v[16];
            SG::inv2(tau, X, Hn, bufC);
            // next item's template spectra, in flight during this transform
            // (after the last item this reads a valid row that is never used)
            const int tn = (t + 1 == M) ? 0 : t + 1;
            const int row = rows[t];
            {
                const c32 *Ht = H + (int64_t)tn * L;
#pragma unroll
                for (int e = 0; e < 16; ++e) Hn[e] = Ht[e * T + tau];
            }
            __syncthreads();
            SG::inv1(tau, v, bufC, tw1);
            SG::put_a_inv(tau, v, bufA);
            __syncthreads();
            SG::inv0(tau, v, bufA, tw0);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(P + (int64_t)row * ld + s * V, 0, 4 * nkeep, kBufWord3);
#pragma unroll
            for (int m = 0; m < 16; ++m)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(norm2(v[m])), rs, 4 * (tau + T * m - D), 0,
                                                      kNonTemporal);
            t = tn;
        }
    }
}

// ---------------------------------------------------------------------------
// stand-alone segment transform (natural order in and out)
// ---------------------------------------------------------------------------

template <int L, int DIR>
__global__ __launch_bounds__(L / 16) void segfft_kernel(const c32 *__restrict__ in,
                                                        c32 *__restrict__ out,
                                                        const c32 *__restrict__ twL)
{
    using SG = Seg<L>;
    constexpr int T = SG::T;
    __shared__ c32 lds[SG::LDS_ELEMS];
    const int tau = threadIdx.x;
    const c32 *src = in + (int64_t)blockIdx.x * L;
    c32 *dst = out + (int64_t)blockIdx.x * L;
    c32 v[16], tw0[16], tw1[16];
    SG::twiddles(tau, twL, tw0, tw1);
    if (DIR < 0) {
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = src[tau + T * m];
        SG::fwd0(tau, v, tw0);
        SG::put_a(tau, v, lds);
        __syncthreads();
        SG::fwd1(tau, v, lds, tw1);
        __syncthreads();
        SG::put_c(tau, v, lds);
        __syncthreads();
        SG::fwd2(tau, v, lds);
#pragma unroll
        for (int e = 0; e < 16; ++e) dst[SG::perm(tau, e)] = v[e];
    } else {
        c32 one[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            v[e] = src[SG::perm(tau, e)];
            one[e] = mk(1.f, 0.f);
        }
        SG::inv2(tau, v, one, lds);
        __syncthreads();
        SG::inv1(tau, v, lds, tw1);
        __syncthreads();
        SG::put_a_inv(tau, v, lds);
        __syncthreads();
        SG::inv0(tau, v, lds, tw0);
#pragma unroll
        for (int m = 0; m < 16; ++m) dst[tau + T * m] = v[m];
    }
}

// ---------------------------------------------------------------------------
// direct TDFIR baseline
// ---------------------------------------------------------------------------

// Tile of TD_TILE outputs per workgroup, TD_R consecutive outputs per
// work-item, for a group of tg templates (grid.y indexes the groups).  LDS
// holds x[i0 - kp .. i0 + TD_TILE) as two planes (real parts, then
// imaginary parts) with one pad slot every 8 elements: work-items 8 elements
// apart then read 4-byte words 9 apart, so the 64 lanes of a read touch 64
// different banks.  The taps of the group's templates follow the planes and
// are read as broadcasts (every lane the same tap).  Taps and tile are
// staged once, behind one barrier, so the template loop has no barrier; and
// taps in LDS rather than in scalar registers keep every wait of the block
// loop an in-order LDS wait (scalar loads complete out of order and share
// the same counter, so each wait for a window read would drain them too).
__device__ __forceinline__ int td_skew(int e) { return e + (e >> 3); }
__host__ __device__ __forceinline__ int td_plane(int span) { return (span + (span >> 3) + 1 + 3) & ~3; }

static_assert(TD_R == 8, "the window addressing assumes 8 outputs per work-item");

__global__ __launch_bounds__(TD_THREADS) void tdfir_kernel(
    const c32 *__restrict__ x, int64_t n, const c32 *__restrict__ taps,
    const int *__restrict__ tap_len, int M, int kp, int tg, float *__restrict__ P, int64_t ld)
{
    extern __shared__ __align__(16) float xsf[];
    const int tau = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * TD_TILE;
    const int64_t org = i0 - kp;
    const int span = TD_TILE + kp;
    const int plane = td_plane(span);         // a multiple of 4 floats: hs is 16-byte aligned
    float *const xr = xsf, *const xi = xsf + plane;
    c32 *const hs = reinterpret_cast<c32 *>(xsf + 2 * plane);
    const int t_beg = blockIdx.y * tg, t_end = min(M, t_beg + tg);
    for (int l = tau; l < span; l += TD_THREADS) {
        const int64_t i = org + l;
        const c32 v = (i >= 0 && i < n) ? x[i] : mk(0.f, 0.f);
        xr[td_skew(l)] = v.re;
        xi[td_skew(l)] = v.im;
    }
    const int ntaps = (t_end - t_beg) * kp;
    for (int k = tau; k < ntaps; k += TD_THREADS) hs[k] = taps[(int64_t)t_beg * kp + k];
    __syncthreads();
    // Window of work-item tau for the tap block starting at kb = 8 blk: tile
    // elements l0 + c, c < 15, l0 = TD_R tau + kp - kb - 7 = 8 q + 1 with
    // q = tau + kp / 8 - 1 - blk (kp is a multiple of 8), whose slots are
    // 9 q + 1 + c + (c + 1) / 8: a per-work-item base, 9 words lower per
    // block, plus compile-time offsets.  Consecutive windows overlap: element
    // c + 8 of block blk is element c of block blk - 1 (c < 7).  So each block
    // reads only its 8 new elements, and reads them one block ahead: three
    // 8-element buffers take the roles (this block's new elements, the
    // previous block's, the next block's) in turn, three blocks per loop
    // trip, so no register is copied.
    const int wb = 9 * (tau + kp / 8 - 1) + 1;
    auto load_new = [&](int blk, c32 (&dst)[8]) {
        const float *const wr = xr + wb - 9 * blk, *const wi = xi + wb - 9 * blk;
#pragma unroll
        for (int c = 0; c < 8; ++c) dst[c] = mk(wr[c + (c + 1) / 8], wi[c + (c + 1) / 8]);
    };
    for (int t = t_beg; t < t_end; ++t) {
        const c32 *const ht = hs + (t - t_beg) * kp;
        const int nblk = (tap_len[t] + 7) >> 3;
        c32 acc[TD_R];
#pragma unroll
        for (int r = 0; r < TD_R; ++r) acc[r] = mk(0.f, 0.f);
        // one block of 8 taps: y[i] += sum_{k in block} x[i-k] h[k], with the
        // window's elements c < 8 in cur and c >= 8 in prev; the next block's
        // new elements are read into nxt first (the last block re-reads its
        // own, unused)
        float4 hn[4];                       // the next block's 8 taps, two per 16-byte read
        auto load_taps = [&](int blk) {
#pragma unroll
            for (int e = 0; e < 4; ++e) hn[e] = reinterpret_cast<const float4 *>(ht)[4 * blk + e];
        };
        auto step = [&](const c32 (&cur)[8], const c32 (&prev)[8], c32 (&nxt)[8], int blk) {
            float4 h2[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) h2[e] = hn[e];
            const int nb = blk + 1 < nblk ? blk + 1 : blk;
            load_new(nb, nxt);
            load_taps(nb);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const c32 hk = (kk & 1) ? mk(h2[kk >> 1].z, h2[kk >> 1].w) : mk(h2[kk >> 1].x, h2[kk >> 1].y);
#pragma unroll
                for (int r = 0; r < TD_R; ++r) {
                    const int c = r - kk + 7;
                    const c32 xv = c < 8 ? cur[c] : prev[c - 8];
                    acc[r].re = fmaf(xv.re, hk.re, acc[r].re);
                    acc[r].re = fmaf(-xv.im, hk.im, acc[r].re);
                    acc[r].im = fmaf(xv.re, hk.im, acc[r].im);
                    acc[r].im = fmaf(xv.im, hk.re, acc[r].im);
                }
            }
        };
        c32 wa[8], wb8[8], wc[8];
        if (nblk > 0) {
            load_taps(0);
            load_new(0, wa);                // block 0: elements c < 8
            {                               // and c = 8..14 (the would-be block -1's new ones)
                const float *const wr = xr + wb, *const wi = xi + wb;
#pragma unroll
                for (int c = 8; c < 15; ++c) wc[c - 8] = mk(wr[c + (c + 1) / 8], wi[c + (c + 1) / 8]);
                wc[7] = mk(0.f, 0.f);
            }
        }
        int blk = 0;
        for (; blk + 3 <= nblk; blk += 3) {
            step(wa, wc, wb8, blk);
            step(wb8, wa, wc, blk + 1);
            step(wc, wb8, wa, blk + 2);
        }
        if (blk < nblk) {
            step(wa, wc, wb8, blk);
            if (blk + 1 < nblk) step(wb8, wa, wc, blk + 1);
        }
        float *Pt = P + (int64_t)t * ld;
        const int64_t ib = i0 + TD_R * tau;
#pragma unroll
        for (int r = 0; r < TD_R; ++r)
            if (ib + r < n) __builtin_nontemporal_store(norm2(acc[r]), Pt + ib + r);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_twiddles(c32 *twL, int L, hipStream_t st)
{
    hipLaunchKernelGGL(twiddle_kernel, dim3((L + 255) / 256), dim3(256), 0, st, twL, L);
    return hipGetLastError();
}

hipError_t launch_tspec(const c32 *taps, const int *tap_len, int kp, int M, int L, c32 *H,
                        hipStream_t st)
{
    const int64_t total = (int64_t)M * L;
    dim3 grid((unsigned)((total + 255) / 256)), blk(256);
    switch (L) {
    case 1024: hipLaunchKernelGGL(tspec_kernel<1024>, grid, blk, 0, st, taps, tap_len, kp, M, H); break;
    case 2048: hipLaunchKernelGGL(tspec_kernel<2048>, grid, blk, 0, st, taps, tap_len, kp, M, H); break;
    case 4096: hipLaunchKernelGGL(tspec_kernel<4096>, grid, blk, 0, st, taps, tap_len, kp, M, H); break;
    case 8192: hipLaunchKernelGGL(tspec_kernel<8192>, grid, blk, 0, st, taps, tap_len, kp, M, H); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L> static int blocks_per_cu_of()
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fdfir_fused_kernel<L>, L / 16, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int fused_blocks_per_cu(int L)
{
    switch (L) {
    case 1024: return blocks_per_cu_of<1024>();
    case 2048: return blocks_per_cu_of<2048>();
    case 4096: return blocks_per_cu_of<4096>();
    case 8192: return blocks_per_cu_of<8192>();
    default: return 1;
    }
}

template <int L> static void launch_fused_t(const FusedArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((fdfir_fused_kernel<L>), dim3((unsigned)a.grid), dim3(L / 16), 0, st,
                       (const c32 *)a.x, a.n, (const c32 *)a.H, (const c32 *)a.twL, a.rows, a.M, a.D,
                       a.V, a.items, a.P, a.ld);
}

hipError_t launch_fused(const FusedArgs &a, hipStream_t st)
{
    switch (a.L) {
    case 1024: launch_fused_t<1024>(a, st); break;
    case 2048: launch_fused_t<2048>(a, st); break;
    case 4096: launch_fused_t<4096>(a, st); break;
    case 8192: launch_fused_t<8192>(a, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_segfft(const void *in, void *out, int64_t count, int dir, int L, const c32 *twL,
                         hipStream_t st)
{
    dim3 grid((unsigned)count), blk(L / 16);
    const c32 *i = (const c32 *)in;
    c32 *o = (c32 *)out;
#define FDAS_SEGFFT_CASE(LL)                                                                   \
    case LL:                                                                                    \
        if (dir < 0) hipLaunchKernelGGL((segfft_kernel<LL, -1>), grid, blk, 0, st, i, o, twL);  \
        else hipLaunchKernelGGL((segfft_kernel<LL, 1>), grid, blk, 0, st, i, o, twL);           \
        break;
    switch (L) {
        FDAS_SEGFFT_CASE(1024)
        FDAS_SEGFFT_CASE(2048)
        FDAS_SEGFFT_CASE(4096)
        FDAS_SEGFFT_CASE(8192)
    default: return hipErrorInvalidValue;
    }
#undef FDAS_SEGFFT_CASE
    return hipGetLastError();
}

size_t tdfir_lds_bytes(int kp, int tg)
{
    // two planes of td_skew(span) + 1 floats (rounded up to 16 bytes), then
    // the taps of tg templates
    return 2 * sizeof(float) * (size_t)td_plane(TD_TILE + kp) + sizeof(c32) * (size_t)kp * tg;
}

size_t fused_lds_bytes(int L)
{
    // two exchange buffers of 16 rows of L / 16 + 1 complex values (the
    // batched kernel adds its candidate lists, 1 KB)
    return 2 * sizeof(c32) * 16 * (size_t)(L / 16 + 1) + 1024;
}

int tdfir_group(int kp, int M)
{
    // templates per workgroup: their taps within TD_TAP_BYTES of LDS
    const int g = TD_TAP_BYTES / (int)(sizeof(c32) * kp);
    return g < 1 ? 1 : (g > M ? M : g);
}

hipError_t launch_tdfir(const TdArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)a.tiles, (unsigned)a.groups), blk(TD_THREADS);
    hipLaunchKernelGGL(tdfir_kernel, grid, blk, tdfir_lds_bytes(a.kp, a.tg), st, (const c32 *)a.x, a.n,
                       (const c32 *)a.taps, a.tap_len, a.M, a.kp, a.tg, a.P, a.ld);
    return hipGetLastError();
}

}  // namespace fdas
