// Host check of the index maps of the 16-bit inverse transform
// (paper_1805_12280_amd/csrc/mixed_fft.h), built and run by
// tests/test_mixed_maps.py.  It emulates, in double precision, the three
// matrix-core passes lane by lane as the kernel arranges them (operand lane
// layouts of v_mfma_f32_16x16x{16,32}, LDS words of the two exchanges,
// twiddles) and compares the result with the inverse DFT by definition.  It
// also checks that the maps are bijections into their buffers and that the
// kernel's LDS accesses are free of bank conflicts (64 banks of 4 bytes).
// Prints "ok" and returns 0 on success.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "mixed_fft.h"

using namespace fdas::mix;
using cd = std::complex<double>;

static int failures = 0;
#define CHECK(c, ...)                                                    \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);             \
            std::printf(__VA_ARGS__);                                    \
            std::printf("\n");                                           \
            if (++failures > 20) std::exit(1);                           \
        }                                                                \
    } while (0)

static double entry(int row, int k, double turns)
{
    const double a = 2.0 * M_PI * turns;
    switch (entry_sel(row, k)) {
    case 0: return std::cos(a);
    case 1: return -std::sin(a);
    case 2: return std::sin(a);
    default: return std::cos(a);
    }
}

// D = A B for one 16 x 16 x K product given per-lane operands:
// A[i][k] is lane i + 16 (k / KPL) element k % KPL, B[k][j] lane j + 16 (k / KPL)
// element k % KPL, D[i][j] lane j + 16 (i / 4) element i % 4 (KPL = K / 4).
static void mma(int K, const std::vector<std::vector<double>> &alane, const std::vector<std::vector<double>> &blane,
                std::vector<std::vector<double>> &dlane)
{
    const int kpl = K / 4;
    dlane.assign(64, std::vector<double>(4, 0.0));
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += alane[i + 16 * (k / kpl)][k % kpl] * blane[j + 16 * (k / kpl)][k % kpl];
            dlane[j + 16 * (i / 4)][i % 4] = acc;
        }
}

int main()
{
    // ---- bijections ----
    {
        std::set<int> seen;
        for (int w = 0; w < 2; ++w)
            for (int l = 0; l < 64; ++l)
                for (int v = 0; v < 16; ++v) {
                    const int q = zq(w, l, v);
                    CHECK(q >= 0 && q < L, "zq out of range");
                    // q = k1 + 16 r + 256 s with k1 = col, r = 8 w + v / 2, s = 2 g + v % 2
                    CHECK(q == (l & 15) + 16 * (8 * w + v / 2) + 256 * (2 * (l >> 4) + (v & 1)), "zq form");
                    seen.insert(q);
                }
        CHECK((int)seen.size() == L, "zq is not a bijection (%zu)", seen.size());
        std::set<int> cw, bw;
        for (int p = 0; p < 8; ++p)
            for (int k1 = 0; k1 < 16; ++k1)
                for (int r = 0; r < 16; ++r) {
                    const int a = cc_word(p, k1, r);
                    CHECK(a >= 0 && a < CC_WORDS, "cc_word out of range");
                    cw.insert(a);
                }
        for (int j = 0; j < 128; ++j)
            for (int k1 = 0; k1 < 16; ++k1) {
                const int a = bb_word(j, k1);
                CHECK(a >= 0 && a < BB_WORDS, "bb_word out of range");
                bw.insert(a);
            }
        CHECK((int)cw.size() == 2048 && (int)bw.size() == 2048, "exchange maps are not injective");
    }

    // ---- the three passes, emulated lane by lane ----
    std::mt19937_64 rng(180512280);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<cd> Z(L), y(L, cd(0, 0)), ref(L);
    for (auto &z : Z) z = cd(nd(rng), nd(rng));
    std::vector<cd> cc(CC_WORDS), bb(BB_WORDS);
    std::vector<std::vector<double>> al(64, std::vector<double>(8)), bl(64, std::vector<double>(8)), dl;
    for (int w = 0; w < 2; ++w)            // pass A: one 16x16x16 product per (w, gam), r = 8 w + gam
        for (int gam = 0; gam < 8; ++gam) {
            const int r = 8 * w + gam;
            for (int l = 0; l < 64; ++l) {
                const int i = l & 15, g = l >> 4;
                al[l].assign(4, 0.0);
                bl[l].assign(4, 0.0);
                for (int e = 0; e < 4; ++e) {
                    const int k = 4 * g + e;
                    al[l][e] = entry(i, k, turns_A(r, i >> 1, k >> 1));
                }
                for (int ii = 0; ii < 2; ++ii) {
                    const cd z = Z[zq(w, l, 2 * gam + ii)];
                    bl[l][2 * ii] = z.real();
                    bl[l][2 * ii + 1] = z.imag();
                }
            }
            mma(16, al, bl, dl);
            for (int l = 0; l < 64; ++l) {
                const int col = l & 15, g = l >> 4;
                cc[cc_word(2 * g, col, r)] = cd(dl[l][0], dl[l][1]);
                cc[cc_word(2 * g + 1, col, r)] = cd(dl[l][2], dl[l][3]);
            }
        }
    for (int w = 0; w < 2; ++w)            // pass B: two 16x16x32 products per (w, gam), p = 4 w + gam
        for (int gam = 0; gam < 4; ++gam) {
            const int p = 4 * w + gam;
            for (int h = 0; h < 2; ++h) {
                for (int l = 0; l < 64; ++l) {
                    const int i = l & 15, g = l >> 4, col = l & 15;
                    al[l].assign(8, 0.0);
                    bl[l].assign(8, 0.0);
                    for (int e = 0; e < 8; ++e) {
                        const int k = 8 * g + e;
                        al[l][e] = entry(i, k, turns_D16(8 * h + (i >> 1), k >> 1));
                    }
                    for (int e = 0; e < 4; ++e) {
                        const cd c = cc[cc_word(p, col, 4 * g + e)];
                        bl[l][2 * e] = c.real();
                        bl[l][2 * e + 1] = c.imag();
                    }
                }
                mma(32, al, bl, dl);
                for (int l = 0; l < 64; ++l) {
                    const int col = l & 15, g = l >> 4;
                    for (int ii = 0; ii < 2; ++ii) {
                        const int j = p + 8 * (8 * h + 2 * g + ii);
                        const double a = 2.0 * M_PI * (double)((j * col) & (L - 1)) / L;
                        bb[bb_word(j, col)] = cd(dl[l][2 * ii], dl[l][2 * ii + 1]) * cd(std::cos(a), std::sin(a));
                    }
                }
            }
        }
    for (int w = 0; w < 2; ++w)            // pass C: two 16x16x32 products per (w, gam), j = 16 (4 w + gam) + col
        for (int gam = 0; gam < 4; ++gam)
            for (int h = 0; h < 2; ++h) {
                for (int l = 0; l < 64; ++l) {
                    const int i = l & 15, g = l >> 4, col = l & 15;
                    const int j = 16 * (4 * w + gam) + col;
                    al[l].assign(8, 0.0);
                    bl[l].assign(8, 0.0);
                    for (int e = 0; e < 8; ++e) {
                        const int k = 8 * g + e;
                        al[l][e] = entry(i, k, turns_D16(8 * h + (i >> 1), k >> 1));
                    }
                    for (int e = 0; e < 4; ++e) {
                        const cd b = bb[bb_word(j, 4 * g + e)];
                        bl[l][2 * e] = b.real();
                        bl[l][2 * e + 1] = b.imag();
                    }
                }
                mma(32, al, bl, dl);
                for (int l = 0; l < 64; ++l) {
                    const int col = l & 15, g = l >> 4;
                    const int j = 16 * (4 * w + gam) + col;
                    for (int ii = 0; ii < 2; ++ii) y[j + 128 * (8 * h + 2 * g + ii)] = cd(dl[l][2 * ii], dl[l][2 * ii + 1]);
                }
            }
    double err = 0.0, mx = 0.0;
    for (int n = 0; n < L; ++n) {
        cd s(0, 0);
        for (int q = 0; q < L; ++q) {
            const double a = 2.0 * M_PI * (double)(((long)q * n) & (L - 1)) / L;
            s += Z[q] * cd(std::cos(a), std::sin(a));
        }
        err = std::fmax(err, std::abs(s - y[n]));
        mx = std::fmax(mx, std::abs(s));
    }
    CHECK(err <= 1e-9 * mx, "passes differ from the inverse DFT: %g (max %g)", err, mx);

    // ---- LDS bank conflicts of the kernel's accesses ----
    // An access of W words per lane over B banks of 4 bytes is served B / W
    // lanes at a time; it is conflict-free when each group of lanes covers
    // distinct banks.  Every access is checked with 64 banks; the 16-byte
    // ones also with 32 (16-byte accesses measure as 8 lanes at a time).
    auto conflict_free_b = [](const int *addr, int W, int B) {
        const int G = B / W;
        for (int g0 = 0; g0 < 64; g0 += G) {
            std::set<int> banks;
            for (int l = g0; l < g0 + G; ++l)
                for (int k = 0; k < W; ++k) banks.insert((addr[l] + k) % B);
            if ((int)banks.size() != G * W) return false;
        }
        return true;
    };
    auto conflict_free = [&](const int *addr, int W) {
        return conflict_free_b(addr, W, 64) && (W != 4 || conflict_free_b(addr, W, 32));
    };
    int addr[64];
    for (int w = 0; w < 2; ++w) {
        for (int c = 0; c < 2; ++c)            // pass A stores: 4 consecutive r per lane
            for (int a = 0; a < 2; ++a) {
                for (int l = 0; l < 64; ++l) addr[l] = cc_word(2 * (l >> 4) + c, l & 15, 8 * w + 4 * a);
                CHECK(conflict_free(addr, 4), "pass A store w=%d c=%d a=%d", w, c, a);
            }
        for (int gam = 0; gam < 4; ++gam) {    // pass B loads
            for (int l = 0; l < 64; ++l) addr[l] = cc_word(4 * w + gam, l & 15, 4 * (l >> 4));
            CHECK(conflict_free(addr, 4), "pass B load w=%d gam=%d", w, gam);
        }
        for (int h = 0; h < 2; ++h)            // pass B stores: 4 consecutive j per lane
            for (int i = 0; i < 2; ++i) {
                for (int l = 0; l < 64; ++l) addr[l] = bb_word(4 * w + 16 * (l >> 4) + 64 * h + 8 * i, l & 15);
                CHECK(conflict_free(addr, 4), "pass B store w=%d h=%d i=%d", w, h, i);
            }
        for (int gam = 0; gam < 4; ++gam)      // pass C loads: 4 single words, k1 = 4g + e
            for (int e = 0; e < 4; ++e) {
                for (int l = 0; l < 64; ++l) addr[l] = bb_word(16 * (4 * w + gam) + (l & 15), 4 * (l >> 4) + e);
                CHECK(conflict_free(addr, 1), "pass C load w=%d gam=%d e=%d", w, gam, e);
            }
    }
    // ---- power staging (16 floats per column, chunks of 4) ----
    {
        std::set<int> words;
        for (int j = 0; j < 64; ++j)
            for (int g = 0; g < 4; ++g) {
                const int a = stage_word(j, g);
                CHECK(a >= 0 && a + 4 <= STAGE_WORDS && a % 4 == 0, "stage_word out of range or misaligned");
                for (int k = 0; k < 4; ++k) words.insert(a + k);
            }
        CHECK((int)words.size() == STAGE_WORDS, "stage_word is not a bijection");
        CHECK(16 * BJ >= STAGE_WORDS, "staging does not fit a wave's rows of bb");
        for (int gam = 0; gam < 4; ++gam) {    // writes: lane (g, col) -> column 16 gam + col, chunk g
            for (int l = 0; l < 64; ++l) addr[l] = stage_word(16 * gam + (l & 15), l >> 4);
            CHECK(conflict_free(addr, 4), "staging write gam=%d", gam);
        }
        for (int g = 0; g < 4; ++g) {          // reads: lane j' -> its column, chunk g
            for (int l = 0; l < 64; ++l) addr[l] = stage_word(l, g);
            CHECK(conflict_free(addr, 4), "staging read g=%d", g);
        }
    }
    if (failures) return 1;
    std::printf("ok max|err| %.3g of %.3g\n", err, mx);
    return 0;
}
