// Host check of the float32 segment transform (paper_1805_12280_amd/csrc/
// seg_fft.h), built and run by tests/test_seg_fft_maps.py.  For every
// segment length it runs the passes on the CPU one work-item after another
// between the barriers, exactly as the kernels sequence them (one LDS buffer
// per exchange, the split last pass at L = 8192 reusing its buffer), and
// compares the forward result with the DFT by definition (sign -1) and the
// inverse of a permuted-order spectrum with the inverse DFT (sign +1, no
// 1/L).  It also checks that perm is a bijection onto the frequencies and
// that every LDS slot lies inside the buffer, one slot per value.
// Prints "ok" and returns 0 on success.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "seg_fft.h"

using namespace fdas;
using cd = std::complex<double>;

static int failures = 0;
#define CHECK(c, ...)                                                    \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);             \
            std::printf(__VA_ARGS__);                                    \
            std::printf("\n");                                           \
            ++failures;                                                  \
        }                                                                \
    } while (0)

template <int L> void run()
{
    using SG = Seg<L>;
    constexpr int T = SG::T;
    std::vector<c32> twL(L);
    for (int e = 0; e < L; ++e) twL[e] = mk((float)std::cos(-2.0 * M_PI * e / L), (float)std::sin(-2.0 * M_PI * e / L));
    std::vector<c32> tw0(T * 16), tw1(T * 16);
    for (int t = 0; t < T; ++t) SG::twiddles(t, twL.data(), &tw0[t * 16], &tw1[t * 16]);

    // perm: a bijection onto [0, L)
    {
        std::set<int> seen;
        for (int t = 0; t < T; ++t)
            for (int e = 0; e < 16; ++e) {
                const int q = SG::perm(t, e);
                CHECK(q >= 0 && q < L, "L=%d perm out of range", L);
                seen.insert(q);
            }
        CHECK((int)seen.size() == L, "L=%d perm is not a bijection", L);
    }
    // LDS slots: inside the buffer and one per value
    {
        std::set<int> a, c;
        for (int k1 = 0; k1 < 16; ++k1)
            for (int j = 0; j < T; ++j) a.insert(SG::a_slot(k1, j));
        for (int k1 = 0; k1 < 16; ++k1)
            for (int r = 0; r < 16; ++r)
                for (int p = 0; p < SG::R2; ++p) c.insert(SG::c_slot(k1, r, p));   // p < T / 16 = R2
        CHECK((int)a.size() == L && *a.rbegin() < SG::LDS_ELEMS && *a.begin() >= 0, "L=%d a_slot", L);
        CHECK((int)c.size() == L && *c.rbegin() < SG::LDS_ELEMS && *c.begin() >= 0, "L=%d c_slot", L);
        if constexpr (L == 8192) {
            std::set<int> e;
            for (int k1 = 0; k1 < 16; ++k1)
                for (int r = 0; r < 16; ++r)
                    for (int p0 = 0; p0 < 2; ++p0)
                        for (int s0 = 0; s0 < 16; ++s0) e.insert(SG::e_slot(k1, r, p0, s0));
            CHECK((int)e.size() == L && *e.rbegin() < SG::LDS_ELEMS && *e.begin() >= 0, "L=%d e_slot", L);
        }
    }

    std::mt19937_64 rng(1805 + L);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<c32> A(SG::LDS_ELEMS), C(SG::LDS_ELEMS), regs(T * 16), d(T * 16);

    // ---- forward ----
    std::vector<cd> w(L);
    for (auto &z : w) z = cd(nd(rng), nd(rng));
    for (int t = 0; t < T; ++t)
        for (int m = 0; m < 16; ++m) regs[t * 16 + m] = mk((float)w[t + T * m].real(), (float)w[t + T * m].imag());
    for (int t = 0; t < T; ++t) SG::fwd0(t, &regs[t * 16], &tw0[t * 16]);
    for (int t = 0; t < T; ++t) SG::put_a(t, &regs[t * 16], A.data());
    for (int t = 0; t < T; ++t) SG::fwd1(t, &regs[t * 16], A.data(), &tw1[t * 16]);
    for (int t = 0; t < T; ++t) SG::put_c(t, &regs[t * 16], C.data());
    if constexpr (L == 8192) {
        for (int t = 0; t < T; ++t) SG::fwd2a(t, &d[t * 16], C.data());
        for (int t = 0; t < T; ++t) SG::put_e(t, &d[t * 16], C.data());
        for (int t = 0; t < T; ++t) SG::fwd2b(t, &regs[t * 16], C.data());
    } else {
        for (int t = 0; t < T; ++t) SG::fwd2(t, &regs[t * 16], C.data());
    }
    double err = 0.0, mx = 0.0;
    for (int t = 0; t < T; ++t)
        for (int e = 0; e < 16; ++e) {
            const int q = SG::perm(t, e);
            cd s(0, 0);
            for (int n = 0; n < L; ++n) {
                const double a = -2.0 * M_PI * (double)(((long)q * n) % L) / L;
                s += w[n] * cd(std::cos(a), std::sin(a));
            }
            const cd got(regs[t * 16 + e].re, regs[t * 16 + e].im);
            err = std::fmax(err, std::abs(got - s));
            mx = std::fmax(mx, std::abs(s));
        }
    CHECK(err <= 2e-5 * mx, "L=%d forward differs from the DFT: %g of %g", L, err, mx);
    std::printf("L=%d forward max|err| %.3g of %.3g\n", L, err, mx);

    // ---- inverse of a spectrum held in permuted order ----
    std::vector<cd> Z(L);
    for (auto &z : Z) z = cd(nd(rng), nd(rng));
    std::vector<c32> X(T * 16), one(16, mk(1.f, 0.f));
    for (int t = 0; t < T; ++t)
        for (int e = 0; e < 16; ++e) {
            const cd z = Z[SG::perm(t, e)];
            X[t * 16 + e] = mk((float)z.real(), (float)z.imag());
        }
    if constexpr (L == 8192) {
        for (int t = 0; t < T; ++t) SG::inv2b(t, &X[t * 16], one.data(), C.data());
        for (int t = 0; t < T; ++t) SG::inv2a(t, &d[t * 16], C.data());
        for (int t = 0; t < T; ++t) SG::put_c_inv(t, &d[t * 16], C.data());
    } else {
        for (int t = 0; t < T; ++t) SG::inv2(t, &X[t * 16], one.data(), C.data());
    }
    for (int t = 0; t < T; ++t) SG::inv1(t, &regs[t * 16], C.data(), &tw1[t * 16]);
    for (int t = 0; t < T; ++t) SG::put_a_inv(t, &regs[t * 16], A.data());
    for (int t = 0; t < T; ++t) SG::inv0(t, &regs[t * 16], A.data(), &tw0[t * 16]);
    err = 0.0;
    mx = 0.0;
    for (int t = 0; t < T; t += (L >= 4096 ? 3 : 1))       // a sample of outputs at the large lengths
        for (int m = 0; m < 16; ++m) {
            const int n = t + T * m;
            cd s(0, 0);
            for (int q = 0; q < L; ++q) {
                const double a = 2.0 * M_PI * (double)(((long)q * n) % L) / L;
                s += Z[q] * cd(std::cos(a), std::sin(a));
            }
            const cd got(regs[t * 16 + m].re, regs[t * 16 + m].im);
            err = std::fmax(err, std::abs(got - s));
            mx = std::fmax(mx, std::abs(s));
        }
    CHECK(err <= 2e-5 * mx, "L=%d inverse differs from the inverse DFT: %g of %g", L, err, mx);
    std::printf("L=%d inverse max|err| %.3g of %.3g\n", L, err, mx);
}

int main()
{
    run<1024>();
    run<2048>();
    run<4096>();
    run<8192>();
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
