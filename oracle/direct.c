/*
 * CPU oracle for the FT-convolution hot path -- TEST INFRASTRUCTURE ONLY.
 * Only the tests, the smoke check and the bench's CPU-baseline leg may load
 * this library; the GPU library never links or calls it.
 *
 * It is the plain definition of what the filter bank computes, written out
 * in float64 (Section 3.1, Eq. (1), and the power of Section 4.3):
 *
 *     y_t[i] = sum_{k=0}^{K_t-1} x[i-k] * h_t[k],   x[j] = 0 for j < 0,
 *     P_t[i] = Re(y_t[i])^2 + Im(y_t[i])^2,
 *
 * for every template t and output index i in [0, n).  The taps of a row are
 * summed in increasing k.  There is no segmentation, no transform and no
 * reordering: overlap-save (Alg. 2) reaches this same result, and the tests
 * pin that separately.
 *
 * Complex arrays are interleaved (re, im) float64.  Threads (OpenMP) split
 * the output into (row, chunk) pieces; every output is still the same
 * k-ordered sum, so the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CHUNK 4096

/* y[i - i0] for i in [i0, i1) of template row `t` (taps h, length K). */
static void conv_chunk(const double *x, int64_t n, const double *h, int32_t K,
                       int64_t i0, int64_t i1, double *y /* 2*(i1-i0) */)
{
    int64_t len = i1 - i0;
    memset(y, 0, sizeof(double) * 2 * (size_t)len);
    for (int32_t k = 0; k < K; ++k) {
        double hr = h[2 * k], hi = h[2 * k + 1];
        /* outputs i with 0 <= i - k < n contribute x[i-k] * h[k] */
        int64_t lo = i0 > k ? i0 : k;
        int64_t hiend = i1 < n + k ? i1 : n + k;
        for (int64_t i = lo; i < hiend; ++i) {
            double xr = x[2 * (i - k)], xi = x[2 * (i - k) + 1];
            double *o = y + 2 * (i - i0);
            o[0] += xr * hr - xi * hi;
            o[1] += xr * hi + xi * hr;
        }
    }
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Number of threads the next parallel region would use. */
int oracle_threads(int nthreads) { return set_threads(nthreads); }

/*
 * Complex outputs y_t[i], i in [i0, i1), for the templates listed in rows[].
 * taps: [M][K_max] interleaved complex; tap_len[t] <= K_max.
 * out:  [nrows][i1-i0] interleaved complex.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_conv(const double *x, int64_t n, const double *taps, const int32_t *tap_len,
                int32_t M, int32_t K_max, const int32_t *rows, int32_t nrows,
                int64_t i0, int64_t i1, double *out, int nthreads)
{
    if (!x || !taps || !tap_len || !rows || !out || n < 0 || i0 < 0 || i1 < i0 || K_max < 1)
        return -1;
    for (int32_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= M || tap_len[rows[r]] < 0 || tap_len[rows[r]] > K_max)
            return -1;
    set_threads(nthreads);
    int64_t len = i1 - i0;
    int64_t nchunks = (len + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    int64_t total = nchunks * (int64_t)nrows;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < total; ++w) {
        int32_t r = (int32_t)(w / nchunks);
        int64_t c = w % nchunks;
        int64_t a = i0 + c * ORACLE_CHUNK;
        int64_t b = a + ORACLE_CHUNK < i1 ? a + ORACLE_CHUNK : i1;
        int32_t t = rows[r];
        conv_chunk(x, n, taps + 2 * (int64_t)t * K_max, tap_len[t], a, b,
                   out + 2 * ((int64_t)r * len + (a - i0)));
    }
    return 0;
}

/*
 * Power P_t[i] = |y_t[i]|^2 for i in [i0, i1) of the listed templates.
 * out: [nrows][i1-i0] float64.
 */
int oracle_power(const double *x, int64_t n, const double *taps, const int32_t *tap_len,
                 int32_t M, int32_t K_max, const int32_t *rows, int32_t nrows,
                 int64_t i0, int64_t i1, double *out, int nthreads)
{
    if (!x || !taps || !tap_len || !rows || !out || n < 0 || i0 < 0 || i1 < i0 || K_max < 1)
        return -1;
    for (int32_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= M || tap_len[rows[r]] < 0 || tap_len[rows[r]] > K_max)
            return -1;
    set_threads(nthreads);
    int64_t len = i1 - i0;
    int64_t nchunks = (len + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    int64_t total = nchunks * (int64_t)nrows;
    int err = 0;
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * 2 * ORACLE_CHUNK);
        if (!y) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t w = 0; w < total; ++w) {
            if (!y) continue;
            int32_t r = (int32_t)(w / nchunks);
            int64_t c = w % nchunks;
            int64_t a = i0 + c * ORACLE_CHUNK;
            int64_t b = a + ORACLE_CHUNK < i1 ? a + ORACLE_CHUNK : i1;
            int32_t t = rows[r];
            conv_chunk(x, n, taps + 2 * (int64_t)t * K_max, tap_len[t], a, b, y);
            double *o = out + (int64_t)r * len + (a - i0);
            for (int64_t i = 0; i < b - a; ++i)
                o[i] = y[2 * i] * y[2 * i] + y[2 * i + 1] * y[2 * i + 1];
        }
        free(y);
    }
    return err;
}

/*
 * Power at individual points: out[p] = P_{t[p]}[i[p]], each one its own
 * k-ordered sum.  For sampled checks at sizes where whole rows are not needed.
 */
int oracle_power_at(const double *x, int64_t n, const double *taps, const int32_t *tap_len,
                    int32_t M, int32_t K_max, const int32_t *t_idx, const int64_t *i_idx,
                    int64_t npts, double *out, int nthreads)
{
    if (!x || !taps || !tap_len || !t_idx || !i_idx || !out || n < 0 || K_max < 1) return -1;
    for (int64_t p = 0; p < npts; ++p)
        if (t_idx[p] < 0 || t_idx[p] >= M || i_idx[p] < 0 || tap_len[t_idx[p]] < 0 ||
            tap_len[t_idx[p]] > K_max)
            return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        const double *h = taps + 2 * (int64_t)t_idx[p] * K_max;
        int64_t i = i_idx[p];
        double yr = 0.0, yi = 0.0;
        for (int32_t k = 0; k < tap_len[t_idx[p]]; ++k) {
            if (i - k < 0 || i - k >= n) continue;
            double xr = x[2 * (i - k)], xi = x[2 * (i - k) + 1];
            yr += xr * h[2 * k] - xi * h[2 * k + 1];
            yi += xr * h[2 * k + 1] + xi * h[2 * k];
        }
        out[p] = yr * yr + yi * yi;
    }
    return 0;
}
