// fdas_batched.hip -- many DM-trial spectra in one persistent launch, each
// array's power plane reduced on the fly to its top-K cells.
//
// Section 3 of the paper: every beam has about 6000 DM-trial spectra, each
// filtered by the same template bank, and only the strongest cells of the
// filter-output plane matter to the candidate search that follows.  Here the
// overlap-save hot path of fdas_kernels.hip runs over the items
// (array, segment, template) of a whole batch; instead of storing |y|^2, each
// workgroup keeps an exact running top-K of the cells it has produced for the
// current array, and a second small kernel merges the per-workgroup lists of
// each array.
//
// Order of cells (Cand, beats in fdas_internal.h): power descending, then
// template ascending, then bin ascending.
#include <mutex>

#include "fdas_internal.h"
#include "seg_fft.h"

namespace fdas {

// Workspace of fdas_convolve_batched_static: a fixed device array, one per
// GPU the library runs on, held until the process ends.  Host code never
// passes `scratch` itself to a kernel or a copy (on the host it names a
// stand-in, not device memory): it uses the device address that
// static_workspace() looked up on that device.
static __device__ __align__(256) unsigned char scratch[FDAS_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_done[kMaxDevices];
}  // namespace

hipError_t static_workspace(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        // once per device, with that device current (the caller's contract)
        void *p = nullptr;
        g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_addr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
        g_scratch_done[device] = true;
    }
    *ptr = g_scratch_addr[device];
    return g_scratch_err[device];
}

// Work item u in [0, items) of the batch is (array a, segment s, template t),
// ordered by array, then segment, then template; bs.item_begin[a] is the
// first item of array a.  Each workgroup takes one contiguous range, so it
// touches each array in one contiguous run and writes one list per array
// it touches: stage[(b * max_slots + slot) * K + r], hdr[b * max_slots + slot]
// = (array, entries), nslots[b] = lists written.
template <int L>
__global__ __launch_bounds__(L / 16, L == 8192 ? 1 : 2) void fdfir_topk_kernel(
    BatchSet bs, const c32 *__restrict__ H, const c32 *__restrict__ twL, int M, int D, int V, int K,
    int64_t items, Cand *__restrict__ stage, int2 *__restrict__ hdr, int *__restrict__ nslots,
    int max_slots)
{
    using SG = Seg<L>;
    constexpr int T = SG::T;
    __shared__ c32 bufA[SG::LDS_ELEMS];   // exchange 0<->1; candidate list after pass 0'
    __shared__ c32 bufC[SG::LDS_ELEMS];   // exchange 1<->2; per-thread maxima
    __shared__ float keptP[2][TOPK_MAX];
    __shared__ int keptT[2][TOPK_MAX];
    __shared__ int keptI[2][TOPK_MAX];
    __shared__ int s_cnt;
    __shared__ float s_thr;

    const int tau = threadIdx.x;
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t u0 = items * b / nb, u1 = items * (b + 1) / nb;
    if (u0 >= u1) {
        if (tau == 0) nslots[b] = 0;
        return;
    }

    c32 tw0[16], tw1[16];
    SG::twiddles(tau, twL, tw0, tw1);

    int a = 0;
    while (bs.item_begin[a + 1] <= u0) ++a;
    int64_t s = (u0 - bs.item_begin[a]) / M;
    int t = (int)(u0 - bs.item_begin[a] - s * M);
    int64_t s_end = (bs.n[a] + V - 1) / V;

    c32 Hn[16];
    {
        const c32 *Ht = H + (int64_t)t * L;
#pragma unroll
        for (int e = 0; e < 16; ++e) Hn[e] = Ht[e * T + tau];
    }
    if (tau == 0) s_cnt = 0;

    int par = 0, kc = 0, slot = 0;
    float thr = -1.f;                       // a cell enters the list if P >= thr
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

    // Segments outside, that segment's templates inside, so the spectrum X
    // is invariant in the inner loop (no per-item register copies of it).
    for (int64_t u = u0; u < u1;) {
        const int64_t n = bs.n[a];
        const int64_t base = s * V - D;
        const int hi = (int)min<int64_t>(L, n - base);
        c32 X[16];
        {
            const c32 *xs = bs.x[a] + base;
            const int lo = (int)max<int64_t>(0, -base);
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = tau + T * m;
                X[m] = (j >= lo && j < hi) ? xs[j] : mk(0.f, 0.f);
            }
            SG::fwd0(tau, X, tw0);
            __syncthreads();
            SG::put_a(tau, X, bufA);
            __syncthreads();
            SG::fwd1(tau, X, bufA, tw1);
            SG::put_c(tau, X, bufC);
            __syncthreads();
            SG::fwd2(tau, X, bufC);
            __syncthreads();
        }
        const int64_t u_end = min<int64_t>(u1, u + (M - t));     // this segment's items
        for (; u < u_end; ++u) {
            c32 v[16];
            SG::inv2(tau, X, Hn, bufC);
            const int tn = (t + 1 == M) ? 0 : t + 1;
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

            // ---- top-K of this item's cells, merged into the workgroup's list ----
            float pw[16];
            float mx = -1.f;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = tau + T * m;
                pw[m] = (j >= D && j < hi) ? norm2(v[m]) : -1.f;   // -1: not an output
                mx = fmaxf(mx, pw[m]);
            }
            float th = thr;
            if (kc < K) {
                // No full list yet: the K-th largest per-work-item maximum is a
                // lower bound of this item's K-th largest cell, so no cell of the
                // true top-K is below it.
                float *smax = reinterpret_cast<float *>(bufC);      // free until the next inv2
                smax[tau] = mx;
                __syncthreads();
                int gt = 0, ge = 0;
                for (int q = 0; q < T; ++q) {
                    const float o = smax[q];
                    gt += o > mx;
                    ge += o >= mx;
                }
                if (gt < K && ge >= K) s_thr = mx;                   // every writer writes the same value
                __syncthreads();
                th = s_thr;
            }
            // some cell qualifies exactly when the item's maximum does: the
            // maximum is one of the cells whenever it is not negative
            const bool any = mx >= 0.f && mx >= th;
            if (__syncthreads_or(any)) {
                float2 *cand = reinterpret_cast<float2 *>(bufA);    // free: pass 0' reads are done
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    if (pw[m] >= 0.f && pw[m] >= th) {
                        const int c = atomicAdd(&s_cnt, 1);
                        cand[c] = make_float2(pw[m], __int_as_float(tau + T * m));
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

            t = tn;
        }
        // ---- next segment (t wrapped to 0 unless the range ended inside it) ----
        if (t == 0) {
            if (++s == s_end) {
                flush(a);
                kc = 0;
                thr = -1.f;
                s = 0;
                if (++a < bs.count) s_end = (bs.n[a] + V - 1) / V;
            }
        }
    }
    if (kc > 0) flush(a);
    if (tau == 0) nslots[b] = min(slot, max_slots);
}

// One workgroup per array: K-way merge of that array's per-workgroup lists
// (each sorted best first) by K rounds of a workgroup-wide argmax of the list
// heads.  Each of the nb workgroups of the first kernel wrote at most one
// list per array; work-item tid owns workgroups tid, tid + 256, ...
// (MERGE_THREADS, MERGE_Q: fdas_args.h; nb <= MERGE_MAX_LISTS)

__global__ __launch_bounds__(MERGE_THREADS) void topk_merge_kernel(
    const Cand *__restrict__ stage, const int2 *__restrict__ hdr, const int *__restrict__ nslots,
    int nb, int max_slots, int K, Cand *__restrict__ out)
{
    const int a = blockIdx.x, tid = threadIdx.x;
    const Cand *lst[MERGE_Q];
    int pos[MERGE_Q], len[MERGE_Q];
#pragma unroll
    for (int q = 0; q < MERGE_Q; ++q) {
        lst[q] = nullptr;
        pos[q] = 0;
        len[q] = 0;
        const int b = tid + MERGE_THREADS * q;
        if (b < nb) {
            const int ns = nslots[b];
            for (int sl = 0; sl < ns; ++sl) {
                const int2 h = hdr[(int64_t)b * max_slots + sl];
                if (h.x == a) {
                    lst[q] = stage + ((int64_t)b * max_slots + sl) * K;
                    len[q] = h.y;
                }
            }
        }
    }
    __shared__ float rp[MERGE_THREADS];
    __shared__ int rt[MERGE_THREADS], ri[MERGE_THREADS], ro[MERGE_THREADS];
    for (int r = 0; r < K; ++r) {
        float bp = -1.f;
        int bt = 0, bi = 0, bo = -1;
#pragma unroll
        for (int q = 0; q < MERGE_Q; ++q) {
            if (pos[q] < len[q]) {
                const Cand c = lst[q][pos[q]];
                if (bo < 0 || beats(c.p, c.t, c.bin, bp, bt, bi)) {
                    bp = c.p;
                    bt = c.t;
                    bi = c.bin;
                    bo = tid * MERGE_Q + q;
                }
            }
        }
        rp[tid] = bp;
        rt[tid] = bt;
        ri[tid] = bi;
        ro[tid] = bo;
        __syncthreads();
        for (int w = MERGE_THREADS / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const int o = tid + w;
                const bool take = ro[o] >= 0 && (ro[tid] < 0 || beats(rp[o], rt[o], ri[o], rp[tid], rt[tid], ri[tid]));
                if (take) {
                    rp[tid] = rp[o];
                    rt[tid] = rt[o];
                    ri[tid] = ri[o];
                    ro[tid] = ro[o];
                }
            }
            __syncthreads();
        }
        const int win = ro[0];
        if (tid == 0) {
            Cand c;
            if (win >= 0) {
                c.t = rt[0];
                c.bin = ri[0];
                c.p = rp[0];
            } else {
                c.t = -1;
                c.bin = -1;
                c.p = -1.f;
            }
            out[(int64_t)a * K + r] = c;
        }
        if (win >= 0 && win / MERGE_Q == tid) {
#pragma unroll
            for (int q = 0; q < MERGE_Q; ++q)
                if (q == win % MERGE_Q) ++pos[q];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------

template <int L> static int topk_blocks_per_cu_of()
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fdfir_topk_kernel<L>, L / 16, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

int topk_blocks_per_cu(int L)
{
    switch (L) {
    case 1024: return topk_blocks_per_cu_of<1024>();
    case 2048: return topk_blocks_per_cu_of<2048>();
    case 4096: return topk_blocks_per_cu_of<4096>();
    case 8192: return topk_blocks_per_cu_of<8192>();
    default: return 1;
    }
}

template <int L> static void launch_topk_t(const TopkArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((fdfir_topk_kernel<L>), dim3((unsigned)a.grid), dim3(L / 16), 0, st, *a.bs,
                       (const c32 *)a.H, (const c32 *)a.twL, a.M, a.D, a.V, a.K, a.items,
                       (Cand *)a.stage, (int2 *)a.hdr, a.nslots, a.max_slots);
}

hipError_t launch_topk(const TopkArgs &a, hipStream_t st)
{
    switch (a.L) {
    case 1024: launch_topk_t<1024>(a, st); break;
    case 2048: launch_topk_t<2048>(a, st); break;
    case 4096: launch_topk_t<4096>(a, st); break;
    case 8192: launch_topk_t<8192>(a, st); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_topk_merge(a.stage, a.hdr, a.nslots, (int)a.grid, a.max_slots, a.K, a.bs->count, a.out, st);
}

hipError_t launch_topk_merge(const void *stage, const void *hdr, const int *nslots, int nb, int max_slots,
                             int K, int count, void *out, hipStream_t st)
{
    if (nb > MERGE_MAX_LISTS) return hipErrorInvalidValue;   // excluded by batch_shape
    hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)count), dim3(MERGE_THREADS), 0, st,
                       (const Cand *)stage, (const int2 *)hdr, nslots, nb, max_slots, K, (Cand *)out);
    return hipGetLastError();
}

}  // namespace fdas
