// fdas_internal.h -- interface between the C ABI (fdas_abi.cpp) and the
// kernel launchers (fdas_kernels.hip).  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "fdas_args.h"

namespace fdas {

struct c32;

constexpr int TD_THREADS = 256;              // work-items per TDFIR workgroup
constexpr int TD_R = 8;                      // consecutive outputs per work-item
constexpr int TD_TILE = TD_THREADS * TD_R;   // outputs per TDFIR workgroup
constexpr int TD_TAP_BYTES = 4096;           // LDS for the taps of one TDFIR template group

// Buffer resource word 3 of the gfx9 family (32-bit data format; offsets are
// range-checked against num_records and out-of-range stores are dropped),
// and the cache-policy bit of a streaming (non-temporal) store.
constexpr int kBufWord3 = 0x00020000;
constexpr int kNonTemporal = 2;
// s_waitcnt operand: vmcnt(0), expcnt and lgkmcnt at their maxima (gfx9 encoding)
constexpr int kWaitVmcnt0 = 0x0F70;

struct FusedArgs {
    const void *x;        // complex64 [n]
    int64_t n;
    const void *H;        // complex64 [M][L], permuted order: the spectra of the templates run
    const c32 *twL;       // complex64 [L]
    const int *rows;      // [M]: plane row of each template run
    int M, D, V, L;       // D: discarded points per segment, V = L - D kept
    int64_t items;        // S * M
    int64_t grid;         // workgroups
    float *P;
    int64_t ld;
};

struct TdArgs {
    const void *x;
    int64_t n;
    const void *taps;     // complex64 [M][kp]
    const int *tap_len;
    int M, kp, tg;
    int64_t tiles, groups;
    float *P;
    int64_t ld;
};

// One candidate cell (same layout as fdas_cand) and the order of cells:
// power descending, then template ascending, then bin ascending (a strict
// total order, since (template, bin) is unique).
struct Cand {
    int t;
    int bin;
    float p;
};

__device__ __forceinline__ bool beats(float pa, int ta, int ia, float pb, int tb, int ib)
{
    return pa > pb || (pa == pb && (ta < tb || (ta == tb && ia < ib)));
}

struct TopkArgs {
    const BatchSet *bs;
    const void *H;
    const c32 *twL;
    int M, D, V, L, K;
    int64_t items, grid;
    void *stage;          // Cand [grid][max_slots][K]
    void *hdr;            // int2 [grid][max_slots]
    int *nslots;          // int [grid]
    int max_slots;
    void *out;            // fdas_cand [count][K]
};

struct MixedArgs {
    const void *x;        // 16-bit complex [n]
    int64_t n;
    const void *H16;      // template spectra [M][2048], pass-A lane order (mixed_spectra_bytes)
    const void *mat;      // DFT matrices of the three passes (mixed_matrix_bytes())
    const c32 *twL;
    int M, D, V, eh;
    bool bf;              // input pairs are bfloat16 (else binary16)
    int64_t items, grid;
    int64_t segments;     // ceil(n / V)
    void *stage;          // mixed_stage_bytes(segments): scaled spectra and power scales
    float *P;
    int64_t ld;
};

hipError_t launch_twiddles(c32 *twL, int L, hipStream_t st);
hipError_t launch_tspec(const c32 *taps, const int *tap_len, int kp, int M, int L, c32 *H,
                        hipStream_t st);
int fused_blocks_per_cu(int L);
hipError_t launch_fused(const FusedArgs &a, hipStream_t st);
hipError_t launch_segfft(const void *in, void *out, int64_t count, int dir, int L, const c32 *twL,
                         hipStream_t st);
size_t tdfir_lds_bytes(int kp, int tg);
size_t fused_lds_bytes(int L);              // LDS of the float32 template-loop kernels at segment length L
int tdfir_group(int kp, int M);              // largest template group whose taps fit TD_TAP_BYTES
int topk_blocks_per_cu(int L);
hipError_t launch_tspec_mix(const c32 *taps, const int *tap_len, int kp, int M, float scale, void *H16,
                            hipStream_t st);
size_t mixed_spectra_bytes(int M);           // template spectra of a 16-bit plan (binary16)
int mixed_blocks_per_cu();
size_t mixed_matrix_bytes();
hipError_t launch_mat_table(void *tab, hipStream_t st);
hipError_t launch_mixed(const MixedArgs &a, hipStream_t st);
hipError_t launch_topk(const TopkArgs &a, hipStream_t st);
// merge of the per-workgroup candidate lists of each array (second kernel
// of both batched forms); nb = workgroups of the first kernel
hipError_t launch_topk_merge(const void *stage, const void *hdr, const int *nslots, int nb, int max_slots,
                             int K, int count, void *out, hipStream_t st);

struct MixedTopkArgs {
    const BatchSet *bs;   // x[] hold 16-bit pairs
    const void *H16, *mat;
    const c32 *twL;
    int M, D, V, K, eh;
    bool bf;              // input pairs are bfloat16 (else binary16)
    int64_t items, grid, segments;
    void *xstage;         // mixed_stage_bytes(segments)
    void *stage, *hdr;
    int *nslots;
    int max_slots;
    void *out;
};
int mixed_topk_blocks_per_cu();
hipError_t launch_mixed_topk(const MixedTopkArgs &a, hipStream_t st);
hipError_t launch_tdfir(const TdArgs &a, hipStream_t st);

// Direct convolution on the matrix cores (fdas_direct.hip) for the plan's
// shortest templates: blocks of DIRECT_BLOCK templates (in order of tap
// count), each with NK <= DIRECT_MAX_NK steps of 16 taps.
constexpr int DIRECT_BLOCK = 8;
constexpr int DIRECT_MAX_NK = 6;
struct DirectTables {
    int nblk = 0;
    int kpmax = 16;                // 16 * the largest NK of the blocks
    std::vector<int> nks;          // [nblk]
    std::vector<int> aoff;         // [nblk] first uint4 of each block's operands in A
    std::vector<int> rows;         // [nblk][DIRECT_BLOCK] plane row of each template, -1 = padding
    std::vector<int> pexp;         // [nblk][DIRECT_BLOCK] -2 x the template's scale exponent
    std::vector<uint4> A;          // split tap operands, per block and step: 64 lanes hi, 64 lanes lo
};
int direct_nk(int taps);
// order: the bank's rows by tap count; block b takes order[DIRECT_BLOCK b ..)
void build_direct_tables(const c32 *taps, const int *tap_len, int M, int kp, const std::vector<int> &order,
                         int nblk, DirectTables &out);
struct DconvArgs {
    const void *x;
    int64_t n;
    const void *A;
    const int *aoff, *nks, *rows, *pexp;
    int nblk, kpmax;
    float *P;
    int64_t ld;
};
hipError_t launch_dconv(const DconvArgs &a, hipStream_t st);
// Device address of the static workspace on `device` (which must be the
// current device); looked up once per device, the same result after that.
hipError_t static_workspace(int device, void **ptr);

}  // namespace fdas
