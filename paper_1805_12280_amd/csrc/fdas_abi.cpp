// fdas_abi.cpp -- the C ABI of libfdas.so (declared in include/fdas.h):
// argument checks, plan construction and the launches of the hot path.
// All arithmetic of the method runs in the kernels of fdas_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fdas.h"
#include "fdas_internal.h"
#include "seg_fft.h"

#define FDAS_API extern "C" __attribute__((visibility("default")))

using fdas::c32;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FDAS_ENOMEM : FDAS_EHIP, "%s: %s (%d)", what,
                hipGetErrorString(e), (int)e);
}

constexpr int kVariantFusedPersistent = 1;
constexpr int kVariantMixedFp16 = 2;
constexpr int kVariantMixedBf16 = 3;

bool supported_l(int L) { return L == 1024 || L == 2048 || L == 4096 || L == 8192; }

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

}  // namespace

struct fdas_plan {
    int device = 0;
    int num_cu = 0;
    int lds_per_block = 0;     // LDS bytes one workgroup may use
    int32_t M = 0, k_max = 0, L = 0, D = 0, V = 0, kp = 0;
    int64_t input_len = 0;
    uint32_t flags = 0;
    int fused_per_cu = 1;
    int topk_per_cu = 1;
    int prec = 0;              // 0 float32, 1 binary16, 2 bfloat16
    int mixed_per_cu = 1;
    int mixed_topk_per_cu = 1;
    int wg_cap = 0;            // fdas_plan_set_workgroups_per_cu, 0 = none
    int eh = 0;                // template spectra scaled by 2^eh in 16-bit storage
    uint32_t *d_H16 = nullptr; // [M][2048] packed 16-bit pairs, pass-A lane order
    void *d_mat = nullptr;     // 16-bit DFT matrices of the inverse passes
    void *d_stage = nullptr;   // scaled segment spectra of one call (16-bit plans)
    hipEvent_t stage_free = nullptr;  // recorded after each call that used d_stage
    mutable std::mutex stage_mu;      // orders the enqueues of calls that share d_stage
    mutable hipStream_t stage_stream = nullptr;
    mutable bool stage_used = false;
    c32 *d_H = nullptr;        // [M][L], permuted frequency order per template
    c32 *d_tw = nullptr;       // [L]
    c32 *d_taps = nullptr;     // [M][kp], zero beyond tap_len
    int *d_tap_len = nullptr;  // [M]
    int64_t resident_bytes = 0;
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
    delete p;
}

int check_io(const fdas_plan *plan, const void *d_in, int64_t n, const float *d_power,
             int64_t ld_power)
{
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (!d_in) return fail(FDAS_EINVAL, "d_in is NULL");
    if (!d_power) return fail(FDAS_EINVAL, "d_power is NULL");
    if (n < 1 || n > plan->input_len)
        return fail(FDAS_EINVAL, "n=%lld outside [1, input_len=%lld]", (long long)n,
                    (long long)plan->input_len);
    if (ld_power < n) return fail(FDAS_EINVAL, "ld_power=%lld < n=%lld", (long long)ld_power, (long long)n);
    if (((uintptr_t)d_in) % (plan->prec ? 4 : 8) != 0) return fail(FDAS_EINVAL, "d_in is misaligned");
    if (((uintptr_t)d_power) % 4 != 0) return fail(FDAS_EINVAL, "d_power is not 4-byte aligned");
    return FDAS_OK;
}

}  // namespace

FDAS_API int fdas_plan_create(fdas_plan **out, const void *taps, const int32_t *tap_len, int32_t M,
                              int32_t K_max, int64_t input_len, int32_t seg_fft, uint32_t flags,
                              void *hip_stream)
{
    g_last_error.clear();
    if (!out) return fail(FDAS_EINVAL, "out is NULL");
    *out = nullptr;
    if ((flags & ~(FDAS_TAPS_ON_DEVICE | FDAS_FP16 | FDAS_BF16)) != 0 ||
        ((flags & FDAS_FP16) && (flags & FDAS_BF16)))
        return fail(FDAS_EUNSUPPORTED, "unsupported flags 0x%x", flags);
    const int prec = (flags & FDAS_FP16) ? 1 : (flags & FDAS_BF16) ? 2 : 0;
    if (prec != 0 && seg_fft != 0 && seg_fft != 2048)
        return fail(FDAS_EUNSUPPORTED, "16-bit plans are built for seg_fft = 2048 only");
    if (!taps) return fail(FDAS_EINVAL, "taps is NULL");
    if (M < 1) return fail(FDAS_EINVAL, "M=%d < 1", M);
    if (K_max < 1) return fail(FDAS_EINVAL, "K_max=%d < 1", K_max);
    if (input_len < 1) return fail(FDAS_EINVAL, "input_len=%lld < 1", (long long)input_len);
    const int L = seg_fft == 0 ? 2048 : seg_fft;
    if (!supported_l(L)) return fail(FDAS_EINVAL, "seg_fft=%d not in {1024, 2048, 4096, 8192}", seg_fft);
    if (K_max > L / 2) return fail(FDAS_EINVAL, "K_max=%d > seg_fft/2=%d", K_max, L / 2);
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
    for (int t = 0; t < M; ++t)
        if (lens[t] < 0 || lens[t] > K_max)
            return fail(FDAS_EINVAL, "tap_len[%d]=%d outside [0, K_max=%d]", t, lens[t], K_max);

    fdas_plan *p = new (std::nothrow) fdas_plan();
    if (!p) return fail(FDAS_ENOMEM, "host allocation of the plan failed");
    p->M = M;
    p->k_max = K_max;
    p->L = L;
    // discard D >= K_max - 1 points per segment, rounded up to 32 outputs so
    // every segment's kept outputs start on a 128-byte line
    p->D = (K_max - 1 + 31) / 32 * 32;
    p->V = L - p->D;
    p->kp = (K_max + 7) / 8 * 8;
    p->input_len = input_len;
    p->flags = flags;
    p->prec = prec;

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipGetDevice"); }
    e = hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, p->device);
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
    const size_t bytes_taps = sizeof(c32) * (size_t)M * p->kp;
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
    std::vector<c32> h((size_t)M * p->kp, fdas::mk(0.f, 0.f));
    for (int t = 0; t < M; ++t)
        std::memcpy(&h[(size_t)t * p->kp], &src[(size_t)t * K_max], sizeof(c32) * (size_t)lens[t]);
    e = hipMemcpyAsync(p->d_taps, h.data(), bytes_taps, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_tap_len, lens.data(), bytes_len, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = fdas::launch_twiddles(p->d_tw, L, st);
    if (e == hipSuccess) e = fdas::launch_tspec(p->d_taps, p->d_tap_len, p->kp, M, L, p->d_H, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "building template spectra"); }

    p->fused_per_cu = fdas::fused_blocks_per_cu(L);
    p->topk_per_cu = fdas::topk_blocks_per_cu(L);
    if (prec != 0) {
        // 16-bit spectra in the matrix-core lane order, scaled by 2^eh so the
        // largest component is in (1/2, 1]
        std::vector<c32> hf((size_t)M * L);
        e = hipMemcpy(hf.data(), p->d_H, sizeof(c32) * hf.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "reading template spectra"); }
        float mx = 0.f;
        for (const c32 &z : hf) mx = std::max(mx, std::max(std::fabs(z.re), std::fabs(z.im)));
        int ex = 0;
        if (mx > 0.f) std::frexp(mx, &ex);           // mx < 2^ex
        p->eh = -ex;
        const size_t bytes16 = sizeof(uint32_t) * (size_t)M * L;
        const size_t stage = fdas::mixed_stage_bytes((input_len + p->V - 1) / p->V);
        e = hipMalloc((void **)&p->d_H16, bytes16);
        if (e == hipSuccess) e = hipMalloc(&p->d_mat, fdas::mixed_matrix_bytes());
        if (e == hipSuccess) e = hipMalloc(&p->d_stage, stage);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->stage_free, hipEventDisableTiming);
        if (e == hipSuccess) e = fdas::launch_mat_table(prec == 2, p->d_mat, st);
        if (e == hipSuccess)
            e = fdas::launch_tspec_mix(p->d_taps, p->d_tap_len, p->kp, M, std::ldexp(1.f, p->eh), prec == 2,
                                       p->d_H16, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "building 16-bit template spectra"); }
        p->resident_bytes += (int64_t)(bytes16 + fdas::mixed_matrix_bytes() + stage);
        p->mixed_per_cu = fdas::mixed_blocks_per_cu(prec == 2);
        p->mixed_topk_per_cu = fdas::mixed_topk_blocks_per_cu(prec == 2);
    }
    *out = p;
    return FDAS_OK;
}

namespace {

// persistent workgroups per CU: what fits, capped by the plan's setting
int per_cu(const fdas_plan *p, int fit) { return p->wg_cap > 0 ? std::min(fit, p->wg_cap) : fit; }

int64_t fused_grid(const fdas_plan *p, int64_t items)
{
    const int64_t resident = (int64_t)per_cu(p, p->fused_per_cu) * std::max(1, p->num_cu);
    return std::max<int64_t>(1, std::min(items, resident));
}

}  // namespace

FDAS_API int fdas_convolve(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
                           int64_t ld_power, void *hip_stream)
{
    g_last_error.clear();
    int rc = check_io(plan, d_in, n, d_power, ld_power);
    if (rc != FDAS_OK) return rc;
    if (plan->prec != 0) {
        fdas::MixedArgs m;
        m.x = d_in;
        m.n = n;
        m.H16 = plan->d_H16;
        m.mat = plan->d_mat;
        m.twL = plan->d_tw;
        m.M = plan->M;
        m.D = plan->D;
        m.V = plan->V;
        m.eh = plan->eh;
        m.bf = plan->prec == 2;
        m.segments = (n + plan->V - 1) / plan->V;
        m.items = m.segments * plan->M;
        m.grid = std::max<int64_t>(1, std::min<int64_t>(m.items, (int64_t)per_cu(plan, plan->mixed_per_cu) *
                                                                  std::max(1, plan->num_cu)));
        m.stage = plan->d_stage;
        m.P = d_power;
        m.ld = ld_power;
        // calls on one plan share its staging buffer: each call's work waits
        // for the previous call's (stream order already gives that when both
        // were enqueued on the same stream)
        hipStream_t st = (hipStream_t)hip_stream;
        std::lock_guard<std::mutex> lock(plan->stage_mu);
        hipError_t e = hipSuccess;
        if (plan->stage_used && plan->stage_stream != st) e = hipStreamWaitEvent(st, plan->stage_free, 0);
        if (e == hipSuccess) e = fdas::launch_mixed(m, st);
        if (e == hipSuccess) e = hipEventRecord(plan->stage_free, st);
        if (e != hipSuccess) return hip_fail(e, "launching the 16-bit FDFIR kernels");
        plan->stage_used = true;
        plan->stage_stream = st;
        return FDAS_OK;
    }
    fdas::FusedArgs a;
    a.x = d_in;
    a.n = n;
    a.H = plan->d_H;
    a.twL = plan->d_tw;
    a.M = plan->M;
    a.D = plan->D;
    a.V = plan->V;
    a.L = plan->L;
    a.items = (n + plan->V - 1) / plan->V * plan->M;
    a.grid = fused_grid(plan, a.items);
    a.P = d_power;
    a.ld = ld_power;
    hipError_t e = fdas::launch_fused(a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "launching the fused FDFIR kernel");
    return FDAS_OK;
}

FDAS_API int fdas_tdfir(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
                        int64_t ld_power, void *hip_stream)
{
    g_last_error.clear();
    int rc = check_io(plan, d_in, n, d_power, ld_power);
    if (rc != FDAS_OK) return rc;
    if (plan->prec != 0) return fail(FDAS_EUNSUPPORTED, "fdas_tdfir takes float32 plans only");
    fdas::TdArgs a;
    a.x = d_in;
    a.n = n;
    a.taps = plan->d_taps;
    a.tap_len = plan->d_tap_len;
    a.M = plan->M;
    a.kp = plan->kp;
    a.tiles = (n + fdas::TD_TILE - 1) / fdas::TD_TILE;
    // template groups: small enough that their taps fit the LDS set aside
    // for them, and numerous enough to cover the chip several times over
    const int64_t want_groups = std::max<int64_t>(1, (4LL * std::max(1, plan->num_cu) + a.tiles - 1) / a.tiles);
    const int64_t groups = std::min<int64_t>(plan->M, want_groups);
    a.tg = std::min((int)((plan->M + groups - 1) / groups), fdas::tdfir_group(a.kp, plan->M));
    a.groups = (plan->M + a.tg - 1) / a.tg;
    const size_t lds = fdas::tdfir_lds_bytes(a.kp, a.tg);
    if (lds > (size_t)plan->lds_per_block)
        return fail(FDAS_EUNSUPPORTED, "fdas_tdfir: K_max=%d needs %zu bytes of LDS per workgroup (device: %d)",
                    plan->k_max, lds, plan->lds_per_block);
    a.P = d_power;
    a.ld = ld_power;
    if (a.tiles > 0x7fffffffLL) return fail(FDAS_EINVAL, "n too large for one launch");
    hipError_t e = fdas::launch_tdfir(a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "launching the TDFIR kernel");
    return FDAS_OK;
}

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Shape of one batched launch, computed on the host from the lengths alone.
struct BatchShape {
    fdas::BatchSet bs;
    int64_t items = 0, grid = 0;
    int max_slots = 0;
    size_t off_hdr = 0, off_nslots = 0, off_xstage = 0, bytes = 0;
    int64_t segments = 0;
};

int batch_shape(const fdas_plan *plan, const int64_t *n, int32_t count, int32_t topk, BatchShape &sh)
{
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (!n) return fail(FDAS_EINVAL, "n is NULL");
    if (count < 1 || count > FDAS_MAX_BATCH)
        return fail(FDAS_EINVAL, "count=%d outside [1, %d]", count, FDAS_MAX_BATCH);
    if (topk < 1 || topk > FDAS_MAX_TOPK) return fail(FDAS_EINVAL, "topk=%d outside [1, %d]", topk, FDAS_MAX_TOPK);
    std::memset(&sh.bs, 0, sizeof sh.bs);
    sh.bs.count = count;
    int64_t acc = 0;
    for (int a = 0; a < count; ++a) {
        if (n[a] < 1 || n[a] > plan->input_len || n[a] >= (int64_t(1) << 31))
            return fail(FDAS_EINVAL, "n[%d]=%lld outside [1, input_len=%lld]", a, (long long)n[a],
                        (long long)plan->input_len);
        sh.bs.n[a] = n[a];
        sh.bs.item_begin[a] = acc;
        acc += (n[a] + plan->V - 1) / plan->V * plan->M;
    }
    sh.bs.item_begin[count] = acc;
    sh.items = acc;
    const int fit = plan->prec ? plan->mixed_topk_per_cu : plan->topk_per_cu;
    const int64_t resident = (int64_t)per_cu(plan, fit) * std::max(1, plan->num_cu);
    sh.grid = std::max<int64_t>(1, std::min(acc, resident));
    // most arrays any workgroup's contiguous item range touches
    int ms = 1, a0 = 0;
    for (int64_t b = 0; b < sh.grid; ++b) {
        const int64_t u0 = acc * b / sh.grid, u1 = acc * (b + 1) / sh.grid;
        if (u0 >= u1) continue;
        while (sh.bs.item_begin[a0 + 1] <= u0) ++a0;
        int a1 = a0;
        while (sh.bs.item_begin[a1 + 1] <= u1 - 1) ++a1;
        ms = std::max(ms, a1 - a0 + 1);
    }
    sh.max_slots = ms;
    const size_t lists = (size_t)sh.grid * ms;
    sh.off_hdr = align_up(lists * topk * sizeof(fdas_cand));
    sh.off_nslots = sh.off_hdr + align_up(lists * 2 * sizeof(int));
    sh.bytes = sh.off_nslots + align_up((size_t)sh.grid * sizeof(int));
    sh.segments = acc / plan->M;
    if (plan->prec) {
        // 16-bit plans: the scaled spectra of every segment of the batch
        sh.off_xstage = sh.bytes;
        sh.bytes += align_up(fdas::mixed_stage_bytes(sh.segments));
    }
    return FDAS_OK;
}

}  // namespace

FDAS_API int fdas_batched_workspace_bytes(const fdas_plan *plan, const int64_t *n, int32_t count,
                                          int32_t topk, size_t *out)
{
    g_last_error.clear();
    if (!out) return fail(FDAS_EINVAL, "out is NULL");
    BatchShape sh;
    int rc = batch_shape(plan, n, count, topk, sh);
    if (rc != FDAS_OK) return rc;
    *out = sh.bytes;
    return FDAS_OK;
}

FDAS_API int fdas_convolve_batched(const fdas_plan *plan, const void *const *d_in, const int64_t *n,
                                   int32_t count, int32_t topk, fdas_cand *d_out, void *d_workspace,
                                   size_t workspace_bytes, void *hip_stream)
{
    g_last_error.clear();
    BatchShape sh;
    int rc = batch_shape(plan, n, count, topk, sh);
    if (rc != FDAS_OK) return rc;
    if (!d_in) return fail(FDAS_EINVAL, "d_in is NULL");
    if (!d_out || ((uintptr_t)d_out) % 4) return fail(FDAS_EINVAL, "d_out is NULL or not 4-byte aligned");
    if (!d_workspace || ((uintptr_t)d_workspace) % kAlign)
        return fail(FDAS_EINVAL, "d_workspace is NULL or not %zu-byte aligned", kAlign);
    if (workspace_bytes < sh.bytes)
        return fail(FDAS_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, sh.bytes);
    for (int a = 0; a < count; ++a) {
        if (!d_in[a] || ((uintptr_t)d_in[a]) % (plan->prec ? 4 : 8))
            return fail(FDAS_EINVAL, "d_in[%d] is NULL or misaligned", a);
        sh.bs.x[a] = (const c32 *)d_in[a];
    }
    if (plan->prec) {
        fdas::MixedTopkArgs m;
        m.bs = &sh.bs;
        m.H16 = plan->d_H16;
        m.mat = plan->d_mat;
        m.twL = plan->d_tw;
        m.M = plan->M;
        m.D = plan->D;
        m.V = plan->V;
        m.K = topk;
        m.eh = plan->eh;
        m.bf = plan->prec == 2;
        m.items = sh.items;
        m.grid = sh.grid;
        m.segments = sh.segments;
        m.xstage = (char *)d_workspace + sh.off_xstage;
        m.stage = d_workspace;
        m.hdr = (char *)d_workspace + sh.off_hdr;
        m.nslots = (int *)((char *)d_workspace + sh.off_nslots);
        m.max_slots = sh.max_slots;
        m.out = d_out;
        hipError_t e = fdas::launch_mixed_topk(m, (hipStream_t)hip_stream);
        if (e != hipSuccess) return hip_fail(e, "launching the 16-bit batched FDFIR kernels");
        return FDAS_OK;
    }
    fdas::TopkArgs a;
    a.bs = &sh.bs;
    a.H = plan->d_H;
    a.twL = plan->d_tw;
    a.M = plan->M;
    a.D = plan->D;
    a.V = plan->V;
    a.L = plan->L;
    a.K = topk;
    a.items = sh.items;
    a.grid = sh.grid;
    a.stage = d_workspace;
    a.hdr = (char *)d_workspace + sh.off_hdr;
    a.nslots = (int *)((char *)d_workspace + sh.off_nslots);
    a.max_slots = sh.max_slots;
    a.out = d_out;
    hipError_t e = fdas::launch_topk(a, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "launching the batched FDFIR kernels");
    return FDAS_OK;
}

FDAS_API int fdas_segment_fft(const fdas_plan *plan, const void *d_in, void *d_out, int64_t count,
                              int32_t direction, void *hip_stream)
{
    g_last_error.clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (plan->prec != 0) return fail(FDAS_EUNSUPPORTED, "fdas_segment_fft takes float32 plans only");
    if (!d_in || !d_out) return fail(FDAS_EINVAL, "NULL buffer");
    if (count < 1 || count > 0x7fffffffLL) return fail(FDAS_EINVAL, "count=%lld out of range", (long long)count);
    if (direction != -1 && direction != 1) return fail(FDAS_EINVAL, "direction=%d not -1 or +1", direction);
    if (((uintptr_t)d_in) % 8 || ((uintptr_t)d_out) % 8) return fail(FDAS_EINVAL, "buffers not 8-byte aligned");
    const char *a = (const char *)d_in, *b = (const char *)d_out;
    const size_t bytes = sizeof(c32) * (size_t)plan->L * (size_t)count;
    if (a < b + bytes && b < a + bytes) return fail(FDAS_EINVAL, "d_in and d_out overlap");
    hipError_t e = fdas::launch_segfft(d_in, d_out, count, direction, plan->L, plan->d_tw,
                                       (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "launching the segment transform");
    return FDAS_OK;
}

FDAS_API int fdas_plan_template_spectra(const fdas_plan *plan, void *host_out)
{
    g_last_error.clear();
    if (!plan || !host_out) return fail(FDAS_EINVAL, "NULL argument");
    const int L = plan->L, T = L / 16;
    std::vector<c32> tmp((size_t)plan->M * L);
    hipError_t e = hipMemcpy(tmp.data(), plan->d_H, sizeof(c32) * tmp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copying template spectra");
    c32 *dst = (c32 *)host_out;
    for (int t = 0; t < plan->M; ++t)
        for (int e16 = 0; e16 < 16; ++e16)
            for (int tau = 0; tau < T; ++tau)
                dst[(size_t)t * L + perm_dispatch(L, tau, e16)] = tmp[(size_t)t * L + (size_t)e16 * T + tau];
    return FDAS_OK;
}

FDAS_API int fdas_plan_set_workgroups_per_cu(fdas_plan *plan, int32_t per_cu_cap)
{
    g_last_error.clear();
    if (!plan) return fail(FDAS_EINVAL, "plan is NULL");
    if (per_cu_cap < 0) return fail(FDAS_EINVAL, "per_cu=%d < 0", per_cu_cap);
    plan->wg_cap = per_cu_cap;
    return FDAS_OK;
}

FDAS_API int fdas_plan_info(const fdas_plan *plan, fdas_plan_info_t *out)
{
    g_last_error.clear();
    if (!plan || !out) return fail(FDAS_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof *out);
    out->seg_fft = plan->L;
    out->valid_per_seg = plan->V;
    out->num_segments = (plan->input_len + plan->V - 1) / plan->V;
    out->k_max = plan->k_max;
    out->num_templates = plan->M;
    out->input_len = plan->input_len;
    out->resident_bytes = plan->resident_bytes;
    out->threads_per_fft = plan->L / 16;
    out->fused_grid = (int32_t)fused_grid(plan, out->num_segments * plan->M);
    out->variant = plan->prec == 1 ? kVariantMixedFp16 : plan->prec == 2 ? kVariantMixedBf16 : kVariantFusedPersistent;
    out->device = plan->device;
    out->wg_per_cu_max = plan->prec ? plan->mixed_per_cu : plan->fused_per_cu;
    out->wg_per_cu = plan->wg_cap;
    return FDAS_OK;
}

FDAS_API void fdas_plan_destroy(fdas_plan *plan)
{
    if (!plan) return;
    const int dev = plan->device;
    int cur = dev;
    if (hipGetDevice(&cur) == hipSuccess && cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
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

FDAS_API const char *fdas_last_error(void) { return g_last_error.c_str(); }

FDAS_API const char *fdas_variant_name(int32_t variant)
{
    switch (variant) {
    case kVariantFusedPersistent: return "fused-ols-persistent-fp32";
    case kVariantMixedFp16: return "fused-ols-mfma-fp16";
    case kVariantMixedBf16: return "fused-ols-mfma-bf16";
    default: return "unknown";
    }
}
