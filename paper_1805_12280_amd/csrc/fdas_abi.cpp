// fdas_abi.cpp -- the C ABI of libfdas.so (declared in include/fdas.h):
// plan construction and the launches of the hot path.  Argument checks and
// launch geometry live in fdas_args.h (plain C++, also built on its own under
// the sanitizers); all arithmetic of the method runs in the kernels of
// fdas_kernels.hip, fdas_batched.hip and fdas_mixed.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fdas.h"
#include "fdas_args.h"
#include "fdas_internal.h"
#include "seg_fft.h"

#define FDAS_API extern "C" __attribute__((visibility("default")))

using fdas::c32;
using fdas::fail;

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FDAS_ENOMEM : FDAS_EHIP, "%s: %s (%d)", what,
                hipGetErrorString(e), (int)e);
}

constexpr int kVariantFusedPersistent = 1;
constexpr int kVariantMixedFp16 = 2;
constexpr int kVariantMixedBf16 = 3;

template <int L> int perm_of(int tau, int e) { return fdas::Seg<L>::perm(tau, e); }

int perm_dispatch(int L, int tau, int e)
{
    switch (L) {
    case 1024: return perm_of<1024>(tau, e);
    case 2048: return perm_of<2048>(tau, e);
    case 4096: return perm_of<4096>(tau, e);
    default: return perm_of<8192>(tau, e);
    }
}

// The last work a plan's calls enqueued on one stream (an event recorded
// after it), so that fdas_plan_destroy waits for the plan's own work only.
struct StreamMark {
    hipStream_t stream;
    hipEvent_t done;
};
constexpr size_t kMaxMarks = 64;

}  // namespace

struct fdas_plan {
    fdas::PlanGeom g;          // M, K_max, L, D, V, kp, input_len, precision, grid caps
    int device = 0;
    int lds_per_block = 0;     // LDS bytes one workgroup may use
    uint32_t flags = 0;
    int fused_per_cu = 1;
    int mixed_per_cu = 1;
    int eh = 0;                // template spectra scaled by 2^eh in 16-bit storage
    void *d_H16 = nullptr;     // [M][2048] template spectra, pass-A lane order (binary16 pairs)
    void *d_mat = nullptr;     // 16-bit DFT matrices of the inverse passes
    void *d_stage = nullptr;   // scaled segment spectra of one call (16-bit plans)
    hipEvent_t stage_free = nullptr;  // recorded after each call that used d_stage
    mutable std::mutex stage_mu;      // orders the enqueues of calls that share d_stage
    mutable hipStream_t stage_stream = nullptr;
    mutable bool stage_used = false;
    mutable std::mutex mark_mu;       // guards marks
    mutable std::vector<StreamMark> marks;
    c32 *d_H = nullptr;        // [M][L], permuted frequency order per template
    c32 *d_tw = nullptr;       // [L]
    c32 *d_taps = nullptr;     // [M][kp], zero beyond tap_len
    int *d_tap_len = nullptr;  // [M]
    int64_t resident_bytes = 0;
    void *static_ws = nullptr;        // this device's static workspace (fdas_convolve_batched_static)
    hipError_t static_ws_err = hipSuccess;
    // float32 plans: the bank's rows in order of tap count; the first
    // DIRECT_BLOCK * direct_blocks of them run on the matrix cores (direct
    // convolution), the rest by overlap-save
    std::vector<int> order;
    int *d_order = nullptr;           // [M]
    c32 *d_Hs = nullptr;              // [M][L]: d_H's rows in that order (the overlap-save launch)
    fdas::DirectTables dt;            // the leading blocks of 8 that direct convolution can take
    void *d_dA = nullptr;
    int *d_dmeta = nullptr;           // aoff [nblk], nks [nblk], rows [8 nblk], pexp [8 nblk]
    int direct_blocks = 0;            // blocks in use
};

namespace {

void free_plan(fdas_plan *p)
{
    if (!p) return;
    if (p->d_H) (void)hipFree(p->d_H);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_taps) (void)hipFree(p->d_taps);
    if (p->d_tap_len) (void)hipFree(p->d_tap_len);
    if (p->d_H16) (void)hipFree(p->d_H16);
    if (p->d_mat) (void)hipFree(p->d_mat);
    if (p->d_stage) (void)hipFree(p->d_stage);
    if (p->stage_free) (void)hipEventDestroy(p->stage_free);
    if (p->d_order) (void)hipFree(p->d_order);
    if (p->d_Hs) (void)hipFree(p->d_Hs);
    if (p->d_dA) (void)hipFree(p->d_dA);
    if (p->d_dmeta) (void)hipFree(p->d_dmeta);
    for (const StreamMark &m : p->marks) (void)hipEventDestroy(m.done);
    delete p;
}

// Record, on `st`, the end of the work a call just enqueued.  Skipped while
// `st` is being captured into a graph: the replays of such a graph are the
// caller's to finish before the plan is destroyed.  A failure here is
// reported like a launch failure (the work itself is already enqueued).
hipError_t mark_use(const fdas_plan *p, hipStream_t st)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cap);
    if (e != hipSuccess) return e;
    if (cap != hipStreamCaptureStatusNone) return hipSuccess;
    std::lock_guard<std::mutex> lock(p->mark_mu);
    StreamMark *slot = nullptr;
    for (StreamMark &m : p->marks)
        if (m.stream == st) { slot = &m; break; }
    if (!slot) {
        // reuse the mark of a stream whose recorded work has finished
        if (p->marks.size() >= kMaxMarks)
            for (StreamMark &m : p->marks)
                if (hipEventQuery(m.done) == hipSuccess) { slot = &m; slot->stream = st; break; }
        if (!slot) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
            p->marks.push_back({st, ev});
            slot = &p->marks.back();
        }
    }
    return hipEventRecord(slot->done, st);
}

// Default split of a float32 plan: the leading blocks of DIRECT_BLOCK
// templates (in order of tap count) run on the matrix cores while the
// block's direct cost stays below overlap-save's for its rows.  Per 16
// outputs and SIMD, a block of NK steps of 16 taps issues 3 NK binary16
// products of 16 cycles; overlap-save costs about 39 cycles per template
// and 16 outputs (36 VALU instructions per point at 4 cycles per wave64
// instruction and ~93% issue).  Taking the products at 80% of their issue
// rate, a full block goes direct up to NK = 5 (80 taps), the crossover
// measured on the 85-template bank; a short last block only while its few
// rows still pay for the block's products.
int default_direct_blocks(const fdas_plan *p)
{
    int nb = 0;
    for (int b = 0; b < p->dt.nblk; ++b) {
        const int rows = std::min(fdas::DIRECT_BLOCK, p->g.M - fdas::DIRECT_BLOCK * b);
        if (3 * p->dt.nks[b] * 16 > 39 * rows * 4 / 5) break;
        nb = b + 1;
    }
    return nb;
}

int direct_templates(const fdas_plan *p) { return std::min(p->g.M, fdas::DIRECT_BLOCK * p->direct_blocks); }

int64_t fused_grid(const fdas_plan *p, int64_t items)
{
    const int64_t resident = (int64_t)fdas::per_cu(p->g, p->fused_per_cu) * std::max(1, p->g.num_cu);
    return std::max<int64_t>(1, std::min(items, resident));
}

}  // namespace

FDAS_API int fdas_plan_create(fdas_plan **out, const void *taps, const int32_t *tap_len, int32_t M,
                              int32_t K_max, int64_t input_len, int32_t seg_fft, uint32_t flags,
                              void *hip_stream)
{
    fdas::last_error().clear();
    if (!out) return fail(FDAS_EINVAL, "out is NULL");
    *out = nullptr;
    fdas::PlanGeom geom;
    int rc = fdas::check_plan_args(taps, M, K_max, input_len, seg_fft, flags, geom);
    if (rc != FDAS_OK) return rc;
    const int L = geom.L, prec = geom.prec;
    const bool on_dev = (flags & FDAS_TAPS_ON_DEVICE) != 0;
    hipStream_t st = (hipStream_t)hip_stream;

    // tap lengths, validated on the host
    std::vector<int32_t> lens((size_t)M, K_max);
    if (tap_len) {
        if (on_dev) {
            hipError_t e = hipMemcpy(lens.data(), tap_len, sizeof(int32_t) * (size_t)M, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "copying tap_len");
        } else {
            std::memcpy(lens.data(), tap_len, sizeof(int32_t) * (size_t)M);
        }
    }
    rc = fdas::check_tap_lens(lens.data(), M, K_max);
    if (rc != FDAS_OK) return rc;

    fdas_plan *p = new (std::nothrow) fdas_plan();
    if (!p) return fail(FDAS_ENOMEM, "host allocation of the plan failed");
    p->g = geom;
    p->flags = flags;
    const int kp = geom.kp;

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipGetDevice"); }
    e = hipDeviceGetAttribute(&p->g.num_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&p->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    // the transform's two exchange buffers (L = 8192: 128 KB) must fit a workgroup's LDS
    if (fdas::fused_lds_bytes(L) > (size_t)p->lds_per_block) {
        free_plan(p);
        return fail(FDAS_EUNSUPPORTED, "seg_fft=%d needs %zu bytes of LDS per workgroup (device: %d)", L,
                    fdas::fused_lds_bytes(L), p->lds_per_block);
    }

    const size_t bytes_H = sizeof(c32) * (size_t)M * L;
    const size_t bytes_tw = sizeof(c32) * (size_t)L;
    const size_t bytes_taps = sizeof(c32) * (size_t)M * kp;
    const size_t bytes_len = sizeof(int) * (size_t)M;
    p->resident_bytes = (int64_t)(bytes_H + bytes_tw + bytes_taps + bytes_len);
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipMemGetInfo"); }
    if ((size_t)p->resident_bytes > free_b) {
        int64_t need = p->resident_bytes;
        free_plan(p);
        return fail(FDAS_ENOMEM, "plan needs %lld bytes, %zu free", (long long)need, free_b);
    }
    if ((e = hipMalloc((void **)&p->d_H, bytes_H)) != hipSuccess ||
        (e = hipMalloc((void **)&p->d_tw, bytes_tw)) != hipSuccess ||
        (e = hipMalloc((void **)&p->d_taps, bytes_taps)) != hipSuccess ||
        (e = hipMalloc((void **)&p->d_tap_len, bytes_len)) != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "hipMalloc");
    }

    // taps -> [M][kp] complex64, zero beyond tap_len[t]
    std::vector<c32> src((size_t)M * K_max);
    if (on_dev) {
        e = hipMemcpy(src.data(), taps, sizeof(c32) * src.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "copying device taps"); }
    } else {
        std::memcpy(src.data(), taps, sizeof(c32) * src.size());
    }
    std::vector<c32> h((size_t)M * kp, fdas::mk(0.f, 0.f));
    for (int t = 0; t < M; ++t)
        std::memcpy(&h[(size_t)t * kp], &src[(size_t)t * K_max], sizeof(c32) * (size_t)lens[t]);
    e = hipMemcpyAsync(p->d_taps, h.data(), bytes_taps, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_tap_len, lens.data(), bytes_len, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = fdas::launch_twiddles(p->d_tw, L, st);
    if (e == hipSuccess) e = fdas::launch_tspec(p->d_taps, p->d_tap_len, kp, M, L, p->d_H, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "building template spectra"); }

    // set-up of the static workspace on this device (looked up once per
    // device; a failure is reported by the calls that need it)
    p->static_ws_err = fdas::static_workspace(p->device, &p->static_ws);

    // rows by tap count, and the direct-convolution tables of the leading
    // blocks of 8 whose longest template the matrix-core kernel takes
    p->order.resize((size_t)M);
    for (int t = 0; t < M; ++t) p->order[t] = t;
    std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) { return lens[a] < lens[b]; });
    e = hipMalloc((void **)&p->d_order, sizeof(int) * (size_t)M);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_order, p->order.data(), sizeof(int) * (size_t)M, hipMemcpyHostToDevice);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "row order"); }
    p->resident_bytes += (int64_t)(sizeof(int) * (size_t)M);
    if (prec == 0) {
        e = hipMalloc((void **)&p->d_Hs, bytes_H);
        for (int t = 0; t < M && e == hipSuccess; ++t)
            e = hipMemcpy(p->d_Hs + (size_t)t * L, p->d_H + (size_t)p->order[t] * L, sizeof(c32) * (size_t)L,
                          hipMemcpyDeviceToDevice);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "spectra in row order"); }
        p->resident_bytes += (int64_t)bytes_H;
    }
    if (prec == 0) {
        int nblk = 0;
        constexpr int BT = fdas::DIRECT_BLOCK;
        while (BT * nblk < M) {
            int kmax = 0;
            for (int tt = 0; tt < BT && BT * nblk + tt < M; ++tt) kmax = std::max(kmax, lens[p->order[BT * nblk + tt]]);
            if (fdas::direct_nk(kmax) > fdas::DIRECT_MAX_NK) break;
            ++nblk;
        }
        if (nblk > 0) {
            fdas::build_direct_tables(h.data(), lens.data(), M, kp, p->order, nblk, p->dt);
            std::vector<int> meta;
            meta.insert(meta.end(), p->dt.aoff.begin(), p->dt.aoff.end());
            meta.insert(meta.end(), p->dt.nks.begin(), p->dt.nks.end());
            meta.insert(meta.end(), p->dt.rows.begin(), p->dt.rows.end());
            meta.insert(meta.end(), p->dt.pexp.begin(), p->dt.pexp.end());
            const size_t bytes_a = sizeof(uint4) * p->dt.A.size(), bytes_m = sizeof(int) * meta.size();
            e = hipMalloc(&p->d_dA, bytes_a);
            if (e == hipSuccess) e = hipMalloc((void **)&p->d_dmeta, bytes_m);
            if (e == hipSuccess) e = hipMemcpy(p->d_dA, p->dt.A.data(), bytes_a, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(p->d_dmeta, meta.data(), bytes_m, hipMemcpyHostToDevice);
            if (e != hipSuccess) { free_plan(p); return hip_fail(e, "direct-convolution tables"); }
            p->resident_bytes += (int64_t)(bytes_a + bytes_m);
            p->direct_blocks = default_direct_blocks(p);
        }
    }

    p->fused_per_cu = fdas::fused_blocks_per_cu(L);
    p->g.topk_fit = fdas::topk_blocks_per_cu(L);
    if (prec != 0) {
        // template spectra in the matrix-core lane order, scaled by 2^eh so
        // the largest component is in (1/2, 1] (binary16 pairs for an FP16
        // plan, float32 for a BF16 plan)
        std::vector<c32> hf((size_t)M * L);
        e = hipMemcpy(hf.data(), p->d_H, sizeof(c32) * hf.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "reading template spectra"); }
        float mx = 0.f;
        for (const c32 &z : hf) mx = std::max(mx, std::max(std::fabs(z.re), std::fabs(z.im)));
        int ex = 0;
        if (mx > 0.f) std::frexp(mx, &ex);           // mx < 2^ex
        p->eh = -ex;
        const size_t bytes16 = fdas::mixed_spectra_bytes(M);
        const size_t stage = fdas::mixed_stage_bytes(p->g.segments(input_len));
        e = hipMalloc((void **)&p->d_H16, bytes16);
        if (e == hipSuccess) e = hipMalloc(&p->d_mat, fdas::mixed_matrix_bytes());
        if (e == hipSuccess) e = hipMalloc(&p->d_stage, stage);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->stage_free, hipEventDisableTiming);
        if (e == hipSuccess) e = fdas::launch_mat_table(p->d_mat, st);
        if (e == hipSuccess)
            e = fdas::launch_tspec_mix(p->d_taps, p->d_tap_len, kp, M, std::ldexp(1.f, p->eh), p->d_H16, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "building 16-bit template spectra"); }
        p->resident_bytes += (int64_t)(bytes16 + fdas::mixed_matrix_bytes() + stage);
        p->mixed_per_cu = fdas::mixed_blocks_per_cu();
        p->g.topk_fit = fdas::mixed_topk_blocks_per_cu();
    }
    *out = p;
    return FDAS_OK;
}

FDAS_API int fdas_convolve(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
                           int64_t ld_power, void *hip_stream)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    int rc = fdas::check_io(plan->g, d_in, n, d_power, ld_power);
    if (rc != FDAS_OK) return rc;
    const fdas::PlanGeom &g = plan->g;
    hipStream_t st = (hipStream_t)hip_stream;
    if (g.prec != 0) {
        fdas::MixedArgs m;
        m.x = d_in;
        m.n = n;
        m.H16 = plan->d_H16;
        m.mat = plan->d_mat;
        m.twL = plan->d_tw;
        m.M = g.M;
        m.D = g.D;
        m.V = g.V;
        m.eh = plan->eh;
        m.bf = g.prec == 2;
        m.segments = g.segments(n);
        m.items = m.segments * g.M;
        m.grid = std::max<int64_t>(1, std::min<int64_t>(m.items, (int64_t)fdas::per_cu(g, plan->mixed_per_cu) *
                                                                  std::max(1, g.num_cu)));
        m.stage = plan->d_stage;
        m.P = d_power;
        m.ld = ld_power;
        // calls on one plan share its staging buffer: each call's work waits
        // for the previous call's (stream order already gives that when both
        // were enqueued on the same stream)
        std::lock_guard<std::mutex> lock(plan->stage_mu);
        hipError_t e = hipSuccess;
        if (plan->stage_used && plan->stage_stream != st) e = hipStreamWaitEvent(st, plan->stage_free, 0);
        if (e == hipSuccess) e = fdas::launch_mixed(m, st);
        if (e == hipSuccess) e = hipEventRecord(plan->stage_free, st);
        if (e == hipSuccess) e = mark_use(plan, st);
        if (e != hipSuccess) return hip_fail(e, "launching the 16-bit FDFIR kernels");
        plan->stage_used = true;
        plan->stage_stream = st;
        return FDAS_OK;
    }
    // the shortest templates by direct convolution on the matrix cores, the
    // rest by overlap-save; both write their rows of the same plane
    const int md = direct_templates(plan), mf = g.M - md;
    hipError_t e = hipSuccess;
    if (md > 0) {
        const int nb = plan->direct_blocks, nall = plan->dt.nblk;
        fdas::DconvArgs d;
        d.x = d_in;
        d.n = n;
        d.A = plan->d_dA;
        d.aoff = plan->d_dmeta;
        d.nks = plan->d_dmeta + nall;
        d.rows = plan->d_dmeta + 2 * nall;
        d.pexp = plan->d_dmeta + 2 * nall + fdas::DIRECT_BLOCK * nall;
        d.nblk = nb;
        d.kpmax = 16 * plan->dt.nks[nb - 1];         // blocks are in order of tap count
        d.P = d_power;
        d.ld = ld_power;
        e = fdas::launch_dconv(d, st);
        if (e != hipSuccess) return hip_fail(e, "launching the direct-convolution kernel");
    }
    if (mf > 0) {
        fdas::FusedArgs a;
        a.x = d_in;
        a.n = n;
        a.H = plan->d_Hs + (size_t)md * g.L;
        a.twL = plan->d_tw;
        a.rows = plan->d_order + md;
        a.M = mf;
        a.D = g.D;
        a.V = g.V;
        a.L = g.L;
        a.items = g.segments(n) * mf;
        a.grid = fused_grid(plan, a.items);
        a.P = d_power;
        a.ld = ld_power;
        e = fdas::launch_fused(a, st);
        if (e != hipSuccess) return hip_fail(e, "launching the fused FDFIR kernel");
    }
    e = mark_use(plan, st);
    if (e != hipSuccess) return hip_fail(e, "recording the call's completion");
    return FDAS_OK;
}

FDAS_API int fdas_tdfir(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
                        int64_t ld_power, void *hip_stream)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    int rc = fdas::check_io(plan->g, d_in, n, d_power, ld_power);
    if (rc != FDAS_OK) return rc;
    const fdas::PlanGeom &g = plan->g;
    if (g.prec != 0) return fail(FDAS_EUNSUPPORTED, "fdas_tdfir takes float32 plans only");
    fdas::TdArgs a;
    a.x = d_in;
    a.n = n;
    a.taps = plan->d_taps;
    a.tap_len = plan->d_tap_len;
    a.M = g.M;
    a.kp = g.kp;
    a.tiles = (n + fdas::TD_TILE - 1) / fdas::TD_TILE;
    // template groups: small enough that their taps fit the LDS set aside
    // for them, and numerous enough to cover the chip several times over
    const int64_t want_groups = std::max<int64_t>(1, (4LL * std::max(1, g.num_cu) + a.tiles - 1) / a.tiles);
    const int64_t groups = std::min<int64_t>(g.M, want_groups);
    a.tg = std::min((int)((g.M + groups - 1) / groups), fdas::tdfir_group(a.kp, g.M));
    a.groups = (g.M + a.tg - 1) / a.tg;
    const size_t lds = fdas::tdfir_lds_bytes(a.kp, a.tg);
    if (lds > (size_t)plan->lds_per_block)
        return fail(FDAS_EUNSUPPORTED, "fdas_tdfir: K_max=%d needs %zu bytes of LDS per workgroup (device: %d)",
                    g.k_max, lds, plan->lds_per_block);
    a.P = d_power;
    a.ld = ld_power;
    if (a.tiles > 0x7fffffffLL) return fail(FDAS_EINVAL, "n too large for one launch");
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = fdas::launch_tdfir(a, st);
    if (e == hipSuccess) e = mark_use(plan, st);
    if (e != hipSuccess) return hip_fail(e, "launching the TDFIR kernel");
    return FDAS_OK;
}

FDAS_API int fdas_batched_workspace_bytes(const fdas_plan *plan, const int64_t *n, int32_t count,
                                          int32_t topk, size_t *out)
{
    fdas::last_error().clear();
    if (!out) return fail(FDAS_EINVAL, "out is NULL");
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    fdas::BatchShape sh;
    int rc = fdas::batch_shape(plan->g, n, count, topk, sh);
    if (rc != FDAS_OK) return rc;
    *out = sh.bytes;
    return FDAS_OK;
}

namespace {

// The launches of one batched call over a checked shape and workspace.
int launch_batched(const fdas_plan *plan, const void *const *d_in, fdas::BatchShape &sh, int32_t topk,
                   fdas_cand *d_out, void *ws, hipStream_t st)
{
    const fdas::PlanGeom &g = plan->g;
    for (int a = 0; a < sh.bs.count; ++a) sh.bs.x[a] = (const c32 *)d_in[a];
    hipError_t e;
    if (g.prec) {
        fdas::MixedTopkArgs m;
        m.bs = &sh.bs;
        m.H16 = plan->d_H16;
        m.mat = plan->d_mat;
        m.twL = plan->d_tw;
        m.M = g.M;
        m.D = g.D;
        m.V = g.V;
        m.K = topk;
        m.eh = plan->eh;
        m.bf = g.prec == 2;
        m.items = sh.items;
        m.grid = sh.grid;
        m.segments = sh.segments;
        m.xstage = (char *)ws + sh.off_xstage;
        m.stage = ws;
        m.hdr = (char *)ws + sh.off_hdr;
        m.nslots = (int *)((char *)ws + sh.off_nslots);
        m.max_slots = sh.max_slots;
        m.out = d_out;
        e = fdas::launch_mixed_topk(m, st);
    } else {
        fdas::TopkArgs a;
        a.bs = &sh.bs;
        a.H = plan->d_H;
        a.twL = plan->d_tw;
        a.M = g.M;
        a.D = g.D;
        a.V = g.V;
        a.L = g.L;
        a.K = topk;
        a.items = sh.items;
        a.grid = sh.grid;
        a.stage = ws;
        a.hdr = (char *)ws + sh.off_hdr;
        a.nslots = (int *)((char *)ws + sh.off_nslots);
        a.max_slots = sh.max_slots;
        a.out = d_out;
        e = fdas::launch_topk(a, st);
    }
    if (e == hipSuccess) e = mark_use(plan, st);
    if (e != hipSuccess) return hip_fail(e, "launching the batched FDFIR kernels");
    return FDAS_OK;
}

}  // namespace

FDAS_API int fdas_convolve_batched(const fdas_plan *plan, const void *const *d_in, const int64_t *n,
                                   int32_t count, int32_t topk, fdas_cand *d_out, void *d_workspace,
                                   size_t workspace_bytes, void *hip_stream)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    fdas::BatchShape sh;
    int rc = fdas::batch_shape(plan->g, n, count, topk, sh);
    if (rc == FDAS_OK) rc = fdas::check_batched_ptrs(plan->g, d_in, count, d_out);
    if (rc == FDAS_OK) rc = fdas::check_workspace(sh, d_workspace, workspace_bytes);
    if (rc != FDAS_OK) return rc;
    return launch_batched(plan, d_in, sh, topk, d_out, d_workspace, (hipStream_t)hip_stream);
}

FDAS_API int fdas_convolve_batched_static(const fdas_plan *plan, const void *const *d_in, const int64_t *n,
                                          int32_t count, int32_t topk, fdas_cand *d_out, void *hip_stream)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    fdas::BatchShape sh;
    int rc = fdas::batch_shape(plan->g, n, count, topk, sh);
    if (rc == FDAS_OK) rc = fdas::check_batched_ptrs(plan->g, d_in, count, d_out);
    if (rc == FDAS_OK) rc = fdas::check_static_workspace(sh);
    if (rc != FDAS_OK) return rc;
    if (plan->static_ws_err != hipSuccess || !plan->static_ws)
        return hip_fail(plan->static_ws_err != hipSuccess ? plan->static_ws_err : hipErrorInvalidSymbol,
                        "looking up the static workspace");
    return launch_batched(plan, d_in, sh, topk, d_out, plan->static_ws, (hipStream_t)hip_stream);
}

FDAS_API int fdas_segment_fft(const fdas_plan *plan, const void *d_in, void *d_out, int64_t count,
                              int32_t direction, void *hip_stream)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (plan->g.prec != 0) return fail(FDAS_EUNSUPPORTED, "fdas_segment_fft takes float32 plans only");
    if (!d_in || !d_out) return fail(FDAS_EINVAL, "NULL buffer");
    if (count < 1 || count > 0x7fffffffLL) return fail(FDAS_EINVAL, "count=%lld out of range", (long long)count);
    if (direction != -1 && direction != 1) return fail(FDAS_EINVAL, "direction=%d not -1 or +1", direction);
    if (((uintptr_t)d_in) % 8 || ((uintptr_t)d_out) % 8) return fail(FDAS_EINVAL, "buffers not 8-byte aligned");
    const char *a = (const char *)d_in, *b = (const char *)d_out;
    const size_t bytes = sizeof(c32) * (size_t)plan->g.L * (size_t)count;
    if (a < b + bytes && b < a + bytes) return fail(FDAS_EINVAL, "d_in and d_out overlap");
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = fdas::launch_segfft(d_in, d_out, count, direction, plan->g.L, plan->d_tw, st);
    if (e == hipSuccess) e = mark_use(plan, st);
    if (e != hipSuccess) return hip_fail(e, "launching the segment transform");
    return FDAS_OK;
}

FDAS_API int fdas_plan_template_spectra(const fdas_plan *plan, void *host_out)
{
    fdas::last_error().clear();
    if (!plan || !host_out) return fail(FDAS_EINVAL, "NULL argument");
    const int L = plan->g.L, T = L / 16, M = plan->g.M;
    std::vector<c32> tmp((size_t)M * L);
    hipError_t e = hipMemcpy(tmp.data(), plan->d_H, sizeof(c32) * tmp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copying template spectra");
    c32 *dst = (c32 *)host_out;
    for (int t = 0; t < M; ++t)
        for (int e16 = 0; e16 < 16; ++e16)
            for (int tau = 0; tau < T; ++tau)
                dst[(size_t)t * L + perm_dispatch(L, tau, e16)] = tmp[(size_t)t * L + (size_t)e16 * T + tau];
    return FDAS_OK;
}

FDAS_API int fdas_plan_set_workgroups_per_cu(fdas_plan *plan, int32_t per_cu_cap)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (per_cu_cap < 0) return fail(FDAS_EINVAL, "per_cu=%d < 0", per_cu_cap);
    plan->g.wg_cap = per_cu_cap;
    return FDAS_OK;
}

FDAS_API int fdas_plan_set_direct_templates(fdas_plan *plan, int32_t m)
{
    fdas::last_error().clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (m < -1) return fail(FDAS_EINVAL, "m=%d < -1", m);
    if (plan->g.prec != 0) return fail(FDAS_EUNSUPPORTED, "direct convolution is built for float32 plans only");
    if (m == -1) {
        plan->direct_blocks = default_direct_blocks(plan);
        return FDAS_OK;
    }
    constexpr int BT = fdas::DIRECT_BLOCK;
    const int want = m >= plan->g.M ? (plan->g.M + BT - 1) / BT : m / BT;
    plan->direct_blocks = std::min(want, plan->dt.nblk);
    return FDAS_OK;
}

FDAS_API int fdas_plan_info(const fdas_plan *plan, fdas_plan_info_t *out)
{
    fdas::last_error().clear();
    if (!plan || !out) return fail(FDAS_EINVAL, "NULL argument");
    const fdas::PlanGeom &g = plan->g;
    std::memset(out, 0, sizeof *out);
    out->seg_fft = g.L;
    out->valid_per_seg = g.V;
    out->num_segments = g.segments(g.input_len);
    out->k_max = g.k_max;
    out->num_templates = g.M;
    out->input_len = g.input_len;
    out->resident_bytes = plan->resident_bytes;
    out->threads_per_fft = g.L / 16;
    out->fused_grid = (int32_t)fused_grid(plan, out->num_segments * g.M);
    out->variant = g.prec == 1 ? kVariantMixedFp16 : g.prec == 2 ? kVariantMixedBf16 : kVariantFusedPersistent;
    out->device = plan->device;
    out->wg_per_cu_max = g.prec ? plan->mixed_per_cu : plan->fused_per_cu;
    out->wg_per_cu = g.wg_cap;
    out->direct_templates = direct_templates(plan);
    return FDAS_OK;
}

FDAS_API void fdas_plan_destroy(fdas_plan *plan)
{
    if (!plan) return;
    const int dev = plan->device;
    int cur = dev;
    if (hipGetDevice(&cur) == hipSuccess && cur != dev) (void)hipSetDevice(dev);
    // wait for the last work each stream was given by a call on this plan
    // (other work on the device is not waited for)
    {
        std::lock_guard<std::mutex> lock(plan->mark_mu);
        for (const StreamMark &m : plan->marks) (void)hipEventSynchronize(m.done);
    }
    if (plan->stage_free) (void)hipEventSynchronize(plan->stage_free);
    free_plan(plan);
    if (cur != dev) (void)hipSetDevice(cur);
}

FDAS_API const char *fdas_strerror(int status)
{
    switch (status) {
    case FDAS_OK: return "ok";
    case FDAS_EINVAL: return "invalid argument";
    case FDAS_ENOMEM: return "out of device memory";
    case FDAS_EHIP: return "HIP runtime error";
    case FDAS_EUNSUPPORTED: return "unsupported flag or precision";
    default: return "unknown status";
    }
}

FDAS_API const char *fdas_last_error(void) { return fdas::last_error().c_str(); }

FDAS_API const char *fdas_variant_name(int32_t variant)
{
    switch (variant) {
    case kVariantFusedPersistent: return "fused-ols-persistent-fp32";
    case kVariantMixedFp16: return "fused-ols-mfma-fp16";
    case kVariantMixedBf16: return "fused-ols-mfma-bf16";
    default: return "unknown";
    }
}
