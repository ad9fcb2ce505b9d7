/*
 * fdas.h -- C ABI of libfdas.so: FT convolution of one complex spectrum with
 * a bank of complex FIR templates, with the spectral power of every output,
 * on an MI355X (gfx950).
 *
 * What is computed (Section 3 of Wang, Thiagaraj & Sinnen, "FPGA-based
 * Acceleration of FT Convolution for Pulsar Search Using OpenCL"):
 * for each template t < M and output i < n,
 *
 *     y_t[i] = sum_{k < K_t} x[i-k] * h_t[k]      (Section 3.1, Eq. (1);
 *                                                  x[j] = 0 for j < 0)
 *     P_t[i] = Re(y_t[i])^2 + Im(y_t[i])^2        (power, Section 4.3)
 *
 * fdas_convolve reaches P by overlap-save on the input (Section 3.2.2,
 * Alg. 2): segments of L = seg_fft points overlapping by D >= K_max-1, one forward
 * FFT per segment shared by all templates, a pointwise product with the
 * pre-transformed templates, an inverse FFT per (segment, template), the
 * first D points of each discarded, and |y|^2 written (D is K_max-1
 * rounded up to a multiple of 32, so every segment's outputs start on a
 * 128-byte line; any D >= K_max-1 gives the exact result).  fdas_tdfir
 * evaluates Eq. (1) directly, with the taps processed in blocks (overlap-add
 * on the taps, Section 3.1.2, Alg. 1).  Both write the same plane.
 *
 * Conventions for every call:
 *  - Complex numbers are interleaved float32 pairs (re, im) ("complex64").
 *  - "device" pointers are HIP device memory of the plan's device; "host"
 *    pointers are ordinary host memory.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that take a stream only enqueue work on it and return without
 *    waiting, unless stated otherwise.
 *  - Every call returns an fdas status; nothing aborts, throws across the
 *    ABI or prints.  A failing call leaves its output buffers unspecified and
 *    records detail text for fdas_last_error().
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    FDAS_OK = 0,
    FDAS_EINVAL = 1,        /* NULL pointer, size out of range, misalignment,
                               unsupported seg_fft */
    FDAS_ENOMEM = 2,        /* plan would not fit in free device memory, or a
                               device allocation failed */
    FDAS_EHIP = 3,          /* a HIP runtime call failed; see fdas_last_error */
    FDAS_EUNSUPPORTED = 4   /* flag or precision this library does not build */
};

/* ---- plan flags -------------------------------------------------------- */
#define FDAS_FP32            0u          /* float32 storage and arithmetic */
#define FDAS_TAPS_ON_DEVICE  (1u << 0)   /* `taps` and `tap_len` are device pointers */
#define FDAS_FP16            (1u << 1)   /* binary16 input, matrix-core inverse FFT */
#define FDAS_BF16            (1u << 2)   /* bfloat16 input, matrix-core inverse FFT */

typedef struct fdas_plan fdas_plan;

typedef struct {
    int32_t seg_fft;          /* L: points per segment transform */
    int32_t valid_per_seg;    /* V = L - D: outputs kept per segment */
    int64_t num_segments;     /* S = ceil(input_len / V) */
    int32_t k_max;            /* K_max */
    int32_t num_templates;    /* M */
    int64_t input_len;        /* largest n accepted by fdas_convolve/fdas_tdfir */
    int64_t resident_bytes;   /* device memory the plan holds */
    int32_t threads_per_fft;  /* work-items per segment transform (L / 16) */
    int32_t fused_grid;       /* workgroups of one fdas_convolve launch at input_len */
    int32_t variant;          /* kernel variant id (see fdas_variant_name) */
    int32_t device;           /* HIP device ordinal the plan lives on */
    int32_t wg_per_cu_max;    /* persistent workgroups per CU that fit (fused launch) */
    int32_t wg_per_cu;        /* the cap in force (fdas_plan_set_workgroups_per_cu), 0 = none */
    int32_t direct_templates; /* templates fdas_convolve runs by direct convolution (float32 plans) */
} fdas_plan_info_t;

/*
 * fdas_plan_create -- validate a template bank, copy it to the device and
 * build the pre-transformed template spectra (Alg. 2: the coefficient array
 * is Fourier transformed once, ahead of the segments).
 *
 *   out        receives the plan (host pointer to a pointer; not NULL).
 *   taps       complex64 [M][K_max], row-major, zero-padded beyond
 *              tap_len[t]; host memory, or device memory with
 *              FDAS_TAPS_ON_DEVICE.  Copied: the caller may free it on return.
 *   tap_len    int32 [M], each in [0, K_max]; NULL means every row has K_max
 *              taps.  Same memory kind as taps.
 *   M          templates, >= 1.
 *   K_max      taps per row of `taps`, >= 1 and <= seg_fft / 2.
 *   input_len  largest input length the plan will be given, >= 1.
 *   seg_fft    L in {1024, 2048, 4096, 8192}, or 0 for the default 2048.
 *              L = 8192 (K_max up to 4096) needs 128 KB of LDS per
 *              workgroup; a device that has less returns FDAS_EUNSUPPORTED.
 *   flags      FDAS_FP32, FDAS_FP16 or FDAS_BF16, optionally |
 *              FDAS_TAPS_ON_DEVICE; anything else returns FDAS_EUNSUPPORTED.
 *              FDAS_FP16/FDAS_BF16 ("mixed" plans): the input spectrum is
 *              given as binary16 or bfloat16 pairs; the forward FFT runs in
 *              float32; the inverse FFT passes run on the matrix cores with
 *              binary16 operands and float32 accumulation, each segment
 *              scaled by a power of two (the 5 exponent bits then suffice,
 *              and binary16 keeps 11 significant bits against bfloat16's 8);
 *              the power plane is float32.  The template spectra (scaled by a
 *              power of two so their largest component is in [1/2, 1)) are
 *              stored as binary16 and Z = X H is formed in packed binary16
 *              arithmetic; the two flags differ only in the input format.
 *              Mixed plans need
 *              seg_fft = 2048 (or 0) and support fdas_convolve and
 *              fdas_convolve_batched; fdas_tdfir and fdas_segment_fft
 *              return FDAS_EUNSUPPORTED.  A mixed plan also
 *              holds a staging buffer of 8 KB per segment of input_len for
 *              the scaled segment spectra of one call.
 *   hip_stream stream on which the plan is built; the call waits for that
 *              work before it returns, so the plan is ready on any stream.
 *
 * The template spectra H_t[q] = (1/L) sum_k h_t[k] exp(-2 pi i q k / L) are
 * computed in float64 on the device and rounded once to complex64; the 1/L
 * of the inverse transform is folded into them.  The plan owns all device
 * memory it allocates; fdas_plan_destroy frees it.
 * Errors: FDAS_EINVAL (NULL out/taps, M < 1, K_max < 1, K_max > L/2,
 * tap_len out of range, input_len < 1, seg_fft not supported),
 * FDAS_EUNSUPPORTED, FDAS_ENOMEM (checked against free device memory before
 * allocating), FDAS_EHIP.  On error *out is set to NULL.
 */
int fdas_plan_create(fdas_plan **out, const void *taps, const int32_t *tap_len,
                     int32_t M, int32_t K_max, int64_t input_len, int32_t seg_fft,
                     uint32_t flags, void *hip_stream);

/*
 * fdas_plan_set_workgroups_per_cu -- size of the persistent grids.
 *
 * fdas_convolve and fdas_convolve_batched launch one persistent grid that
 * gives each workgroup a contiguous range of (segment, template) items
 * (Alg. 2's loops over segments and filters).  By default the grid holds as
 * many workgroups per compute unit as fit; per_cu >= 1 caps that number
 * (a tuning knob: fewer, longer-lived workgroups share each segment's
 * forward transform over more templates).  per_cu = 0 removes the cap.
 * Not to be called while calls on the plan may be enqueued from other host
 * threads.  Errors: FDAS_EINVAL (NULL plan, per_cu < 0).
 */
int fdas_plan_set_workgroups_per_cu(fdas_plan *plan, int32_t per_cu);

/*
 * fdas_plan_set_direct_templates -- how a float32 plan splits its bank.
 *
 * fdas_convolve runs a template either by overlap-save (Alg. 2; the cost per
 * output is one inverse FFT of L points whatever the tap count) or by direct
 * convolution (Eq. (1); the cost grows with the tap count), the two routes
 * the paper compares.  The plan orders its templates by tap count and runs
 * the shortest ones by direct convolution on the matrix cores (binary16 high
 * and low parts of every operand, three products, float32 accumulation: the
 * same float32-class result), in blocks of 8, and the rest by overlap-save.
 * m = number of shortest templates to run directly, rounded down to a
 * multiple of 8 (m >= M: all of them); blocks whose longest template has
 * more than 96 taps always run by overlap-save.  m = 0 runs the whole bank
 * by overlap-save; m = -1 restores the plan's default, the blocks for which
 * a cost model of the two kernels favours the direct form.
 * fdas_plan_info reports the split in force.  Not to be called while calls
 * on the plan may be enqueued from other host threads.
 * Errors: FDAS_EINVAL (NULL plan, m < -1), FDAS_EUNSUPPORTED (16-bit plan).
 */
int fdas_plan_set_direct_templates(fdas_plan *plan, int32_t m);

/*
 * fdas_convolve -- the overlap-save FDFIR hot path (Alg. 2 with the power
 * of Section 4.3) for all M templates.  A float32 plan runs its shortest
 * templates by direct convolution on the matrix cores (one launch, see
 * fdas_plan_set_direct_templates) and the rest by overlap-save (one fused
 * launch); both write their rows of the same plane, in stream order.
 *
 *   plan       from fdas_plan_create (not NULL).
 *   d_in       device complex64 [n], 8-byte aligned; for a mixed plan, pairs
 *              (re, im) of 16-bit numbers (binary16 or bfloat16), 4-byte
 *              aligned.
 *   n          1 <= n <= input_len.
 *   d_power    device float32, M rows of ld_power floats, 4-byte aligned;
 *              row t receives P_t[0..n).  Columns n..ld_power-1 are not
 *              written.
 *   ld_power   row stride in floats, >= n.
 *   hip_stream stream to enqueue on.
 *
 * Asynchronous: returns after enqueueing; the caller keeps d_in and d_power
 * alive until the stream has run the work.  A float32 plan is read-only
 * here, so one plan may be used from several streams at once.  A mixed plan
 * runs two launches (forward transforms and scales of all segments into the
 * plan's staging buffer, then the template loop) and orders its calls: each
 * call's work waits, on its stream, for the previous call's work on the same
 * plan, whichever stream that ran on.
 * Errors: FDAS_EINVAL (NULL or misaligned pointers, n or ld_power out of
 * range), FDAS_EHIP (launch failure).
 */
int fdas_convolve(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
                  int64_t ld_power, void *hip_stream);

/*
 * fdas_tdfir -- direct time-domain FIR (Section 3.1, Eq. (1)), taps taken in
 * blocks and accumulated (overlap-add on the taps, Alg. 1), with the same
 * power output.  Arguments, output contract and errors as fdas_convolve;
 * float32 plans only (FDAS_EUNSUPPORTED otherwise).  Its workgroups hold an
 * input tile and the taps of a few templates in LDS, about
 * 9 * (2048 + K_max) + max(4096, 8 * K_max) bytes; a K_max for which that
 * exceeds the device's per-workgroup LDS returns FDAS_EUNSUPPORTED (every
 * K_max <= 2048 fits in 64 KB; K_max = 4096 needs 88 KB).
 */
int fdas_tdfir(const fdas_plan *plan, const void *d_in, int64_t n, float *d_power,
               int64_t ld_power, void *hip_stream);

/* ---- batched DM trials ------------------------------------------------- */

#define FDAS_MAX_BATCH 128   /* arrays per fdas_convolve_batched call */
#define FDAS_MAX_TOPK  32    /* candidates kept per array */

/* One candidate of a power plane: template row, output bin, power. */
typedef struct {
    int32_t t;
    int32_t bin;
    float p;
} fdas_cand;

/*
 * fdas_batched_workspace_bytes -- device workspace fdas_convolve_batched
 * needs for this batch shape (host arguments only; nothing is launched).
 *   n      host int64 [count], each in [1, input_len].
 *   count  1 <= count <= FDAS_MAX_BATCH;  topk  1 <= topk <= FDAS_MAX_TOPK.
 *   out    host size_t, receives the byte count.
 * Errors: FDAS_EINVAL.
 */
int fdas_batched_workspace_bytes(const fdas_plan *plan, const int64_t *n, int32_t count,
                                 int32_t topk, size_t *out);

/*
 * fdas_convolve_batched -- the hot path over many DM-trial spectra at once
 * (Section 3: about 6000 trials per beam, each filtered by the same bank),
 * in one persistent launch, with each array's power plane reduced on the
 * fly to its topk largest cells instead of being written.
 *
 *   d_in       host array [count] of device complex64 pointers (8-byte
 *              aligned), array a holding n[a] points; for a mixed plan,
 *              pointers to 16-bit (re, im) pairs, 4-byte aligned.
 *   n          host int64 [count], 1 <= n[a] <= input_len, n[a] < 2^31.
 *   d_out      device fdas_cand [count][topk]: row a lists array a's topk
 *              cells (t, bin) with the largest P_t[bin], ordered by P
 *              descending, then t ascending, then bin ascending.  If an
 *              array has fewer than topk cells (n[a] * M < topk) the
 *              remainder is {-1, -1, -1.0f}.
 *   d_workspace, workspace_bytes  device scratch of at least
 *              fdas_batched_workspace_bytes(plan, n, count, topk) bytes,
 *              256-byte aligned, owned by the caller; no state is kept in
 *              it between calls.  For a mixed plan it also holds the scaled
 *              spectra of every segment of the batch (8 KB per segment).
 * Asynchronous on hip_stream (two kernel launches, three for a mixed plan;
 * no copies, no memsets, no allocation), so the call can be captured into
 * a HIP graph.  Calls that share a workspace must not overlap.  A mixed
 * plan computes every cell exactly as its fdas_convolve does.
 * Errors: FDAS_EINVAL (NULL/misaligned pointers, sizes out of range, or a
 * workspace that is too small), FDAS_EHIP.
 */
int fdas_convolve_batched(const fdas_plan *plan, const void *const *d_in, const int64_t *n,
                          int32_t count, int32_t topk, fdas_cand *d_out, void *d_workspace,
                          size_t workspace_bytes, void *hip_stream);

/*
 * fdas_convolve_batched_static -- fdas_convolve_batched without a caller
 * workspace and without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture that may not allocate, tight
 * serving loops, harnesses that forbid hipMalloc.
 *
 * The workspace is a fixed array inside the library,
 * FDAS_STATIC_WORKSPACE_BYTES on every GPU the library runs on, held from
 * the library's first use on that GPU until the process ends; its address
 * is looked up when a plan is created on that GPU.  The call allocates
 * nothing (no hipMalloc, no hipFree, no allocating library routine).
 * Arguments, output, ordering and errors are those of fdas_convolve_batched
 * without d_workspace and workspace_bytes; a batch whose workspace
 * (fdas_batched_workspace_bytes) exceeds FDAS_STATIC_WORKSPACE_BYTES returns
 * FDAS_EINVAL and enqueues nothing.  A float32 plan's batch of 64 spectra of
 * up to 2^22 points needs well under 1 MB; a 16-bit plan also stages 8 KB
 * per segment, about 4000 segments (7.6 M points at L = 2048) in all.
 * Every call on one GPU shares that GPU's array, and no call needs it
 * cleared or leaves state in it that a later call reads: calls that overlap
 * on one GPU (different streams, or a graph replay beside another call) race
 * on the array and give wrong candidates; the caller orders them.
 */
#define FDAS_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)
int fdas_convolve_batched_static(const fdas_plan *plan, const void *const *d_in, const int64_t *n,
                                 int32_t count, int32_t topk, fdas_cand *d_out, void *hip_stream);

/*
 * fdas_segment_fft -- the plan's L-point segment transform on its own,
 * in natural order, for `count` independent transforms (the FFT engine role
 * of Section 4.2).
 *
 *   d_in, d_out  device complex64 [count][L], 8-byte aligned; may not overlap.
 *   count        >= 1.
 *   direction    -1: X[q] = sum_n x[n] exp(-2 pi i n q / L);
 *                +1: x[n] = sum_q X[q] exp(+2 pi i n q / L) (no 1/L).
 * Asynchronous on hip_stream.  Errors: FDAS_EINVAL, FDAS_EHIP.
 */
int fdas_segment_fft(const fdas_plan *plan, const void *d_in, void *d_out, int64_t count,
                     int32_t direction, void *hip_stream);

/*
 * fdas_plan_template_spectra -- copy the plan's pre-transformed templates
 * H_t[q] (already scaled by 1/L) into host memory, natural order.
 *
 *   host_out   host complex64 [M][L].
 * Synchronous (waits for the copy).  Errors: FDAS_EINVAL, FDAS_EHIP.
 */
int fdas_plan_template_spectra(const fdas_plan *plan, void *host_out);

/* fdas_plan_info -- geometry and footprint of a plan (host struct, not NULL). */
int fdas_plan_info(const fdas_plan *plan, fdas_plan_info_t *out);

/*
 * fdas_plan_destroy -- wait for the work the plan's calls enqueued (on every
 * stream a call used, the last such work; other work on the device is not
 * waited for), then free the plan.  Calls captured into a HIP graph are not
 * tracked: the caller finishes the graph's replays first.  NULL is a no-op.
 */
void fdas_plan_destroy(fdas_plan *plan);

/* Static text for a status code. */
const char *fdas_strerror(int status);

/* Detail of the last failing call on this thread ("" if none). */
const char *fdas_last_error(void);

/* Name of a kernel variant id reported by fdas_plan_info. */
const char *fdas_variant_name(int32_t variant);

#ifdef __cplusplus
}
#endif
#endif /* FDAS_H */
