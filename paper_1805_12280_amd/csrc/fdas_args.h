// fdas_args.h -- host-side argument checks and launch geometry of the C ABI
// (include/fdas.h), in plain C++ with no HIP dependency, so that the same
// code serves libfdas.so and a host-only build under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Not installed; not part of the ABI.
//
// Geometry (Section 3.2.2, Alg. 2): a segment of L points keeps V = L - D
// outputs after discarding D >= K_max - 1 points; D is K_max - 1 rounded up to
// 32 so that every segment's outputs start on a 128-byte line.  A call over n
// points runs S = ceil(n / V) segments, and S * M (segment, template) items.
#pragma once
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "fdas.h"

namespace fdas {

struct c32;

constexpr int MAX_BATCH = 128;              // FDAS_MAX_BATCH
constexpr int TOPK_MAX = 32;                // FDAS_MAX_TOPK
constexpr int MERGE_THREADS = 256;          // work-items of the candidate-merge kernel
constexpr int MERGE_Q = 8;                  // candidate lists per merge work-item
constexpr int MERGE_MAX_LISTS = MERGE_THREADS * MERGE_Q;   // workgroups one merge can take
constexpr int MIXED_L = 2048;               // segment length of the 16-bit plans
constexpr size_t kWorkspaceAlign = 256;

// Detail text of the last failing call on this thread (fdas_last_error).
inline std::string &last_error()
{
    static thread_local std::string s;
    return s;
}

inline int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error() = buf;
    return status;
}

inline bool supported_seg_fft(int L) { return L == 1024 || L == 2048 || L == 4096 || L == 8192; }
inline int discard_of(int k_max) { return (k_max - 1 + 31) / 32 * 32; }

// Bytes a 16-bit plan stages per call: the scaled forward spectrum of every
// segment (complex float32) and its power scale.
inline size_t mixed_stage_bytes(int64_t segments) { return (size_t)segments * (MIXED_L * 4 + sizeof(float)); }

// What the checks need to know of a plan.
struct PlanGeom {
    int32_t M = 0, k_max = 0, L = 0, D = 0, V = 0, kp = 0;
    int64_t input_len = 0;
    int prec = 0;              // 0 float32, 1 binary16, 2 bfloat16
    int num_cu = 0;
    int topk_fit = 1;          // persistent workgroups per CU of the batched kernel
    int wg_cap = 0;            // fdas_plan_set_workgroups_per_cu, 0 = none
    int64_t segments(int64_t n) const { return (n + V - 1) / V; }
};

// Scalar arguments of fdas_plan_create, checked before anything is read or
// allocated.  On success fills g's geometry fields.
inline int check_plan_args(const void *taps, int32_t M, int32_t K_max, int64_t input_len, int32_t seg_fft,
                           uint32_t flags, PlanGeom &g)
{
    if ((flags & ~(uint32_t)(FDAS_TAPS_ON_DEVICE | FDAS_FP16 | FDAS_BF16)) != 0 ||
        ((flags & FDAS_FP16) && (flags & FDAS_BF16)))
        return fail(FDAS_EUNSUPPORTED, "unsupported flags 0x%x", flags);
    const int prec = (flags & FDAS_FP16) ? 1 : (flags & FDAS_BF16) ? 2 : 0;
    if (prec != 0 && seg_fft != 0 && seg_fft != MIXED_L)
        return fail(FDAS_EUNSUPPORTED, "16-bit plans are built for seg_fft = 2048 only");
    if (!taps) return fail(FDAS_EINVAL, "taps is NULL");
    if (M < 1) return fail(FDAS_EINVAL, "M=%d < 1", M);
    if (K_max < 1) return fail(FDAS_EINVAL, "K_max=%d < 1", K_max);
    if (input_len < 1) return fail(FDAS_EINVAL, "input_len=%lld < 1", (long long)input_len);
    const int L = seg_fft == 0 ? 2048 : seg_fft;
    if (!supported_seg_fft(L)) return fail(FDAS_EINVAL, "seg_fft=%d not in {1024, 2048, 4096, 8192}", seg_fft);
    if (K_max > L / 2) return fail(FDAS_EINVAL, "K_max=%d > seg_fft/2=%d", K_max, L / 2);
    g.M = M;
    g.k_max = K_max;
    g.L = L;
    g.D = discard_of(K_max);
    g.V = L - g.D;
    g.kp = (K_max + 7) / 8 * 8;
    g.input_len = input_len;
    g.prec = prec;
    return FDAS_OK;
}

// Tap lengths (a host copy, M entries), each in [0, K_max].
inline int check_tap_lens(const int32_t *lens, int32_t M, int32_t K_max)
{
    for (int t = 0; t < M; ++t)
        if (lens[t] < 0 || lens[t] > K_max)
            return fail(FDAS_EINVAL, "tap_len[%d]=%d outside [0, K_max=%d]", t, lens[t], K_max);
    return FDAS_OK;
}

// Buffers and sizes of fdas_convolve / fdas_tdfir.
inline int check_io(const PlanGeom &g, const void *d_in, int64_t n, const float *d_power, int64_t ld_power)
{
    if (!d_in) return fail(FDAS_EINVAL, "d_in is NULL");
    if (!d_power) return fail(FDAS_EINVAL, "d_power is NULL");
    if (n < 1 || n > g.input_len)
        return fail(FDAS_EINVAL, "n=%lld outside [1, input_len=%lld]", (long long)n, (long long)g.input_len);
    if (ld_power < n) return fail(FDAS_EINVAL, "ld_power=%lld < n=%lld", (long long)ld_power, (long long)n);
    if (((uintptr_t)d_in) % (g.prec ? 4 : 8) != 0) return fail(FDAS_EINVAL, "d_in is misaligned");
    if (((uintptr_t)d_power) % 4 != 0) return fail(FDAS_EINVAL, "d_power is not 4-byte aligned");
    return FDAS_OK;
}

// Arrays of one batched call, passed by value as a kernel argument (so a
// captured graph holds it without any copy node).
struct BatchSet {
    const c32 *x[MAX_BATCH];
    int64_t n[MAX_BATCH];
    int64_t item_begin[MAX_BATCH + 1];    // first item of each array; [count] = total
    int count;
};

// Shape of one batched launch, computed from the lengths alone.  The
// workspace holds, in order: the per-workgroup candidate lists
// [grid][max_slots][topk], their headers [grid][max_slots] (array, entries),
// the list counts [grid], and for a 16-bit plan the staged spectra of every
// segment of the batch.
struct BatchShape {
    BatchSet bs;
    int64_t items = 0, grid = 0;
    int max_slots = 0;
    size_t off_hdr = 0, off_nslots = 0, off_xstage = 0, bytes = 0;
    int64_t segments = 0;
};

inline size_t align_ws(size_t v) { return (v + kWorkspaceAlign - 1) / kWorkspaceAlign * kWorkspaceAlign; }

// Persistent workgroups per CU: what fits, capped by the plan's setting.
inline int per_cu(const PlanGeom &g, int fit) { return g.wg_cap > 0 ? std::min(fit, g.wg_cap) : fit; }

inline int batch_shape(const PlanGeom &g, const int64_t *n, int32_t count, int32_t topk, BatchShape &sh)
{
    if (!n) return fail(FDAS_EINVAL, "n is NULL");
    if (count < 1 || count > FDAS_MAX_BATCH)
        return fail(FDAS_EINVAL, "count=%d outside [1, %d]", count, FDAS_MAX_BATCH);
    if (topk < 1 || topk > FDAS_MAX_TOPK) return fail(FDAS_EINVAL, "topk=%d outside [1, %d]", topk, FDAS_MAX_TOPK);
    std::memset(&sh.bs, 0, sizeof sh.bs);
    sh.bs.count = count;
    int64_t acc = 0;
    for (int a = 0; a < count; ++a) {
        if (n[a] < 1 || n[a] > g.input_len || n[a] >= (int64_t(1) << 31))
            return fail(FDAS_EINVAL, "n[%d]=%lld outside [1, input_len=%lld]", a, (long long)n[a],
                        (long long)g.input_len);
        sh.bs.n[a] = n[a];
        sh.bs.item_begin[a] = acc;
        acc += g.segments(n[a]) * g.M;
    }
    sh.bs.item_begin[count] = acc;
    sh.items = acc;
    // persistent grid: what fits the device, and never more workgroups than
    // the merge kernel takes lists from, so a valid call is never refused
    // after part of its work was enqueued
    const int64_t resident = (int64_t)per_cu(g, g.topk_fit) * std::max(1, g.num_cu);
    sh.grid = std::max<int64_t>(1, std::min<int64_t>({acc, resident, (int64_t)MERGE_MAX_LISTS}));
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
    sh.off_hdr = align_ws(lists * topk * sizeof(fdas_cand));
    sh.off_nslots = sh.off_hdr + align_ws(lists * 2 * sizeof(int));
    sh.bytes = sh.off_nslots + align_ws((size_t)sh.grid * sizeof(int));
    sh.segments = acc / g.M;
    if (g.prec) {
        sh.off_xstage = sh.bytes;
        sh.bytes += align_ws(mixed_stage_bytes(sh.segments));
    }
    return FDAS_OK;
}

// Pointers of fdas_convolve_batched (the workspace size is checked by the
// caller of this function, which knows where the workspace comes from).
inline int check_batched_ptrs(const PlanGeom &g, const void *const *d_in, int32_t count, const void *d_out)
{
    if (!d_in) return fail(FDAS_EINVAL, "d_in is NULL");
    if (!d_out || ((uintptr_t)d_out) % 4) return fail(FDAS_EINVAL, "d_out is NULL or not 4-byte aligned");
    for (int a = 0; a < count; ++a)
        if (!d_in[a] || ((uintptr_t)d_in[a]) % (g.prec ? 4 : 8))
            return fail(FDAS_EINVAL, "d_in[%d] is NULL or misaligned", a);
    return FDAS_OK;
}

inline int check_workspace(const BatchShape &sh, const void *d_workspace, size_t workspace_bytes)
{
    if (!d_workspace || ((uintptr_t)d_workspace) % kWorkspaceAlign)
        return fail(FDAS_EINVAL, "d_workspace is NULL or not %zu-byte aligned", kWorkspaceAlign);
    if (workspace_bytes < sh.bytes)
        return fail(FDAS_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, sh.bytes);
    return FDAS_OK;
}

// A batch for fdas_convolve_batched_static: its workspace must fit the
// library's static array.
inline int check_static_workspace(const BatchShape &sh)
{
    if (sh.bytes > FDAS_STATIC_WORKSPACE_BYTES)
        return fail(FDAS_EINVAL, "batch needs %zu bytes of workspace; the static workspace holds %zu", sh.bytes,
                    (size_t)FDAS_STATIC_WORKSPACE_BYTES);
    return FDAS_OK;
}

}  // namespace fdas
