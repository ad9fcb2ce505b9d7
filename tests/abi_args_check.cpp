// Host check of the C ABI's argument checks and batch geometry
// (paper_1805_12280_amd/csrc/fdas_args.h), built with g++ under
// -fsanitize=address,undefined: every NULL, size, range and alignment path of
// plan creation, fdas_convolve / fdas_tdfir and fdas_convolve_batched returns
// its status without touching memory it should not, and the batch shape's
// persistent grid, candidate-list slots and workspace layout are checked
// against a brute-force walk of the workgroups' item ranges on random batches.
// Prints "ok" on success; any failed check prints its line and exits 1.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <string>
#include <thread>
#include <vector>

#include "fdas.h"
#include "fdas_args.h"

static int g_checks = 0;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        ++g_checks;                                                                  \
        if (!(cond)) {                                                               \
            fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", __LINE__, #cond, \
                    fdas::last_error().c_str());                                     \
            exit(1);                                                                 \
        }                                                                            \
    } while (0)

using fdas::PlanGeom;

static void plan_args()
{
    int dummy = 0;
    const void *taps = &dummy;
    PlanGeom g;
    CHECK(fdas::check_plan_args(taps, 4, 33, 1000, 1024, 1u << 7, g) == FDAS_EUNSUPPORTED);
    CHECK(fdas::check_plan_args(taps, 4, 33, 1000, 1024, FDAS_FP16 | FDAS_BF16, g) == FDAS_EUNSUPPORTED);
    CHECK(fdas::check_plan_args(taps, 4, 33, 1000, 1024, FDAS_FP16, g) == FDAS_EUNSUPPORTED);
    CHECK(fdas::check_plan_args(nullptr, 4, 33, 1000, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 0, 33, 1000, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, -5, 33, 1000, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 0, 1000, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 33, 0, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 33, 1000, 3000, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 33, 1000, 512, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 513, 1000, 1024, 0, g) == FDAS_EINVAL);
    CHECK(fdas::check_plan_args(taps, 4, 512, 1000, 1024, FDAS_TAPS_ON_DEVICE, g) == FDAS_OK);
    CHECK(g.L == 1024 && g.D == 512 && g.V == 512 && g.kp == 512 && g.prec == 0);
    CHECK(fdas::check_plan_args(taps, 85, 101, 1 << 22, 0, FDAS_BF16, g) == FDAS_OK);
    CHECK(g.L == 2048 && g.D == 128 && g.V == 1920 && g.kp == 104 && g.prec == 2 && g.M == 85);
    CHECK(g.segments(1 << 22) == 2185);
    for (int k = 1; k <= 4096; ++k) {
        CHECK(fdas::discard_of(k) >= k - 1 && fdas::discard_of(k) % 32 == 0 && fdas::discard_of(k) < k + 31);
    }
    std::vector<int32_t> lens = {0, 5, 33, 17};
    CHECK(fdas::check_tap_lens(lens.data(), 4, 33) == FDAS_OK);
    lens[2] = 34;
    CHECK(fdas::check_tap_lens(lens.data(), 4, 33) == FDAS_EINVAL);
    lens[2] = -1;
    CHECK(fdas::check_tap_lens(lens.data(), 4, 33) == FDAS_EINVAL);
}

static void io_args()
{
    PlanGeom g;
    g.input_len = 1000;
    g.prec = 0;
    alignas(16) static char buf[64];
    const float *pw = reinterpret_cast<const float *>(buf);
    CHECK(fdas::check_io(g, nullptr, 10, pw, 10) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf, 10, nullptr, 10) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf, 0, pw, 10) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf, -3, pw, 10) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf, 1001, pw, 2000) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf, 10, pw, 9) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf + 4, 10, pw, 10) == FDAS_EINVAL);          // float32 input: 8-byte pairs
    CHECK(fdas::check_io(g, buf, 10, reinterpret_cast<const float *>(buf + 2), 10) == FDAS_EINVAL);
    CHECK(fdas::check_io(g, buf + 8, 1000, pw, 1000) == FDAS_OK);
    g.prec = 1;                                                              // 16-bit pairs: 4 bytes
    CHECK(fdas::check_io(g, buf + 4, 10, pw, 10) == FDAS_OK);
    CHECK(fdas::check_io(g, buf + 2, 10, pw, 10) == FDAS_EINVAL);
}

// Brute force: for each workgroup b of `grid`, the arrays its item range
// [items*b/grid, items*(b+1)/grid) touches.
static int brute_max_slots(const std::vector<int64_t> &begin, int64_t items, int64_t grid)
{
    int ms = 1;
    const int count = (int)begin.size() - 1;
    for (int64_t b = 0; b < grid; ++b) {
        const int64_t u0 = items * b / grid, u1 = items * (b + 1) / grid;
        int touched = 0;
        for (int a = 0; a < count; ++a)
            if (begin[a] < u1 && begin[a + 1] > u0 && begin[a + 1] > begin[a]) ++touched;
        ms = touched > ms ? touched : ms;
    }
    return ms;
}

static void batch_args()
{
    PlanGeom g;
    int dummy = 0;
    CHECK(fdas::check_plan_args(&dummy, 85, 101, 1 << 22, 1024, 0, g) == FDAS_OK);
    g.num_cu = 256;
    g.topk_fit = 2;
    fdas::BatchShape sh;
    std::vector<int64_t> n = {1 << 22, 5, 1 << 19};
    CHECK(fdas::batch_shape(g, nullptr, 3, 16, sh) == FDAS_EINVAL);
    CHECK(fdas::batch_shape(g, n.data(), 0, 16, sh) == FDAS_EINVAL);
    CHECK(fdas::batch_shape(g, n.data(), FDAS_MAX_BATCH + 1, 16, sh) == FDAS_EINVAL);
    CHECK(fdas::batch_shape(g, n.data(), 3, 0, sh) == FDAS_EINVAL);
    CHECK(fdas::batch_shape(g, n.data(), 3, FDAS_MAX_TOPK + 1, sh) == FDAS_EINVAL);
    n[1] = 0;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_EINVAL);
    n[1] = (1 << 22) + 1;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_EINVAL);
    g.input_len = int64_t(1) << 33;
    n[1] = int64_t(1) << 31;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_EINVAL);
    n[1] = 5;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_OK);
    CHECK(sh.items == (g.segments(1 << 22) + 1 + g.segments(1 << 19)) * 85);
    CHECK(sh.bs.item_begin[0] == 0 && sh.bs.item_begin[3] == sh.items && sh.bs.count == 3);
    CHECK(sh.grid == 512);

    // the grid never exceeds what the merge kernel takes, whatever fits
    g.topk_fit = 16;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_OK);
    CHECK(sh.grid == fdas::MERGE_MAX_LISTS);
    g.wg_cap = 1;
    CHECK(fdas::batch_shape(g, n.data(), 3, 16, sh) == FDAS_OK);
    CHECK(sh.grid == 256);
    g.wg_cap = 0;

    // pointers and workspace
    alignas(256) static char ws[4096];
    const void *ptrs[3] = {ws, ws + 8, ws + 16};
    CHECK(fdas::check_batched_ptrs(g, nullptr, 3, ws) == FDAS_EINVAL);
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, nullptr) == FDAS_EINVAL);
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, ws + 2) == FDAS_EINVAL);
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, ws) == FDAS_OK);
    ptrs[2] = nullptr;
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, ws) == FDAS_EINVAL);
    ptrs[2] = ws + 4;
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, ws) == FDAS_EINVAL);
    g.prec = 1;
    CHECK(fdas::check_batched_ptrs(g, ptrs, 3, ws) == FDAS_OK);
    g.prec = 0;
    CHECK(fdas::check_workspace(sh, nullptr, 1 << 30) == FDAS_EINVAL);
    CHECK(fdas::check_workspace(sh, ws + 128, 1 << 30) == FDAS_EINVAL);
    CHECK(fdas::check_workspace(sh, ws, sh.bytes - 1) == FDAS_EINVAL);
    CHECK(fdas::check_workspace(sh, ws, sh.bytes) == FDAS_OK);

    // random batches: geometry against a brute-force walk of the item ranges
    std::mt19937_64 rng(20180512);
    for (int trial = 0; trial < 300; ++trial) {
        PlanGeom h;
        const int Ls[4] = {1024, 2048, 4096, 8192};
        const int L = Ls[rng() % 4];
        const int kmax = 1 + (int)(rng() % (L / 2));
        const int M = 1 + (int)(rng() % 96);
        const bool mixed = (trial % 5 == 0);
        CHECK(fdas::check_plan_args(&dummy, M, mixed ? std::min(kmax, 1024) : kmax, int64_t(1) << 24,
                                    mixed ? 2048 : L, mixed ? FDAS_FP16 : 0, h) == FDAS_OK);
        h.num_cu = 1 + (int)(rng() % 300);
        h.topk_fit = 1 + (int)(rng() % 12);
        h.wg_cap = (int)(rng() % 4);
        const int count = 1 + (int)(rng() % FDAS_MAX_BATCH);
        const int topk = 1 + (int)(rng() % FDAS_MAX_TOPK);
        std::vector<int64_t> lens(count);
        for (int a = 0; a < count; ++a) {
            const int kind = (int)(rng() % 4);
            lens[a] = kind == 0 ? 1 + (int64_t)(rng() % 64)
                    : kind == 1 ? 1 + (int64_t)(rng() % 100000)
                    : kind == 2 ? (int64_t(1) << (19 + rng() % 4))
                                : 1 + (int64_t)(rng() % (int64_t(1) << 24));
        }
        fdas::BatchShape s;
        CHECK(fdas::batch_shape(h, lens.data(), count, topk, s) == FDAS_OK);
        std::vector<int64_t> begin(count + 1);
        int64_t acc = 0;
        for (int a = 0; a < count; ++a) {
            begin[a] = acc;
            CHECK(s.bs.item_begin[a] == acc && s.bs.n[a] == lens[a]);
            acc += (lens[a] + h.V - 1) / h.V * h.M;
        }
        begin[count] = acc;
        CHECK(s.items == acc && s.bs.item_begin[count] == acc && s.segments * h.M == acc);
        const int64_t fit = (int64_t)fdas::per_cu(h, h.topk_fit) * h.num_cu;
        CHECK(s.grid >= 1 && s.grid <= acc && s.grid <= fit && s.grid <= fdas::MERGE_MAX_LISTS);
        CHECK(s.grid == std::min<int64_t>({acc, fit, (int64_t)fdas::MERGE_MAX_LISTS}));
        CHECK(s.max_slots == brute_max_slots(begin, acc, s.grid));
        const size_t lists = (size_t)s.grid * s.max_slots;
        CHECK(s.off_hdr % fdas::kWorkspaceAlign == 0 && s.off_hdr >= lists * topk * sizeof(fdas_cand));
        CHECK(s.off_nslots % fdas::kWorkspaceAlign == 0 && s.off_nslots - s.off_hdr >= lists * 2 * sizeof(int));
        CHECK(s.bytes - s.off_nslots >= (size_t)s.grid * sizeof(int) || mixed);
        if (mixed) {
            CHECK(s.off_xstage % fdas::kWorkspaceAlign == 0 && s.off_xstage >= s.off_nslots + s.grid * sizeof(int));
            CHECK(s.bytes - s.off_xstage >= fdas::mixed_stage_bytes(s.segments));
        } else {
            CHECK(s.bytes - s.off_nslots >= (size_t)s.grid * sizeof(int));
        }
        CHECK(fdas::check_workspace(s, ws, s.bytes) == FDAS_OK);
        CHECK(fdas::check_workspace(s, ws, s.bytes - 1) == FDAS_EINVAL);
        CHECK(fdas::check_static_workspace(s) == (s.bytes <= FDAS_STATIC_WORKSPACE_BYTES ? FDAS_OK : FDAS_EINVAL));
    }
    // the static workspace: a float32 DM-trial batch fits, a 16-bit batch of
    // two 2^22-point spectra (4370 staged segments of 8 KB) does not
    {
        PlanGeom h;
        CHECK(fdas::check_plan_args(&dummy, 85, 101, int64_t(1) << 22, 2048, 0, h) == FDAS_OK);
        h.num_cu = 256;
        h.topk_fit = 2;
        std::vector<int64_t> big(64, int64_t(1) << 22);
        fdas::BatchShape s;
        CHECK(fdas::batch_shape(h, big.data(), 64, 16, s) == FDAS_OK);
        CHECK(s.bytes < (size_t(1) << 20) && fdas::check_static_workspace(s) == FDAS_OK);
        CHECK(fdas::check_plan_args(&dummy, 85, 101, int64_t(1) << 22, 2048, FDAS_FP16, h) == FDAS_OK);
        CHECK(fdas::batch_shape(h, big.data(), 1, 16, s) == FDAS_OK);
        CHECK(fdas::check_static_workspace(s) == FDAS_OK);
        CHECK(fdas::batch_shape(h, big.data(), 2, 16, s) == FDAS_OK);
        CHECK(fdas::check_static_workspace(s) == FDAS_EINVAL);
        std::vector<int64_t> small(2, 1 << 20);
        CHECK(fdas::batch_shape(h, small.data(), 2, 16, s) == FDAS_OK);
        CHECK(fdas::check_static_workspace(s) == FDAS_OK);
    }
}

static void error_text()
{
    // a detail longer than the message buffer is truncated, not overrun
    std::string big(3000, 'x');
    CHECK(fdas::fail(FDAS_EINVAL, "%s", big.c_str()) == FDAS_EINVAL);
    CHECK(fdas::last_error().size() == 511);
    // the detail is per thread
    std::string seen = "unset";
    std::thread th([&] { seen = fdas::last_error(); });
    th.join();
    CHECK(seen.empty());
    fdas::last_error().clear();
}

int main()
{
    plan_args();
    io_args();
    batch_args();
    error_text();
    printf("%d checks\nok\n", g_checks);
    return 0;
}
