/*
 * The oracle's C code run under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by the CPU tests with gcc together with oracle.c): the direct sum
 * (O1), the recursion (O2) and Bluestein (O3) on every length up to 300 and a
 * few larger ones, both signs, agree with each other; the separable
 * multi-dimensional driver agrees with the direct multi-dimensional sum; a
 * strided, negative-stride, in-place problem runs on several threads.  Any
 * memory error or undefined behaviour aborts the run (sanitizer report);
 * disagreement exits 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int64_t n, is, os; } oracle_iodim;
int oracle_dft(int rank, const oracle_iodim *dims, int vrank, const oracle_iodim *vdims,
               const double *in, double *out, int sign, int method, int nthreads);
void oracle_dft_direct_1d(int64_t n, int sign, const double *x, int64_t xs, double *y, int64_t ys);
void oracle_fft_rec_1d(int64_t n, int sign, const double *x, int64_t xs, double *y);
void oracle_fft_bluestein_1d(int64_t n, int sign, const double *x, int64_t xs, double *y);

static uint64_t state = 88172645463325252ull;
static double urand(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static double rel_diff(const double *a, const double *b, int64_t count)
{
    double num = 0, den = 0;
    for (int64_t i = 0; i < 2 * count; ++i) {
        num += (a[i] - b[i]) * (a[i] - b[i]);
        den += b[i] * b[i];
    }
    return den > 0 ? sqrt(num / den) : sqrt(num);
}

int main(void)
{
    int bad = 0;
    const int64_t extra[] = {512, 1000, 1009, 2187, 4096};
    for (int64_t t = 1; t <= 300 + 5; ++t) {
        const int64_t n = t <= 300 ? t : extra[t - 301];
        double *x = malloc(sizeof(double) * 2 * n);
        double *y1 = malloc(sizeof(double) * 2 * n);
        double *y2 = malloc(sizeof(double) * 2 * n);
        double *y3 = malloc(sizeof(double) * 2 * n);
        for (int64_t i = 0; i < 2 * n; ++i) x[i] = urand();
        for (int sign = -1; sign <= 1; sign += 2) {
            oracle_dft_direct_1d(n, sign, x, 1, y1, 1);
            oracle_fft_rec_1d(n, sign, x, 1, y2);
            oracle_fft_bluestein_1d(n, sign, x, 1, y3);
            const double e2 = rel_diff(y2, y1, n), e3 = rel_diff(y3, y1, n);
            if (e2 > 1e-14 || e3 > 1e-13) {
                printf("n=%lld sign=%d: O2 %.3e O3 %.3e\n", (long long)n, sign, e2, e3);
                bad = 1;
            }
        }
        free(x);
        free(y1);
        free(y2);
        free(y3);
    }
    /* multi-dimensional: separable driver vs the direct sum, 2 x 3 x 5, batch 2 */
    {
        oracle_iodim d[3] = {{2, 15, 15}, {3, 5, 5}, {5, 1, 1}};
        oracle_iodim v[1] = {{2, 30, 30}};
        double x[120], a[120], b[120];
        for (int i = 0; i < 120; ++i) x[i] = urand();
        if (oracle_dft(3, d, 1, v, x, a, -1, 0, 3) || oracle_dft(3, d, 1, v, x, b, -1, 4, 1)) bad = 1;
        if (rel_diff(a, b, 60) > 1e-14) {
            printf("multi-dimensional mismatch %.3e\n", rel_diff(a, b, 60));
            bad = 1;
        }
    }
    /* in place, negative and transposing strides, four threads: 16 x 24 */
    {
        const int64_t R = 16, C = 24;
        oracle_iodim d[1] = {{C, -1, R}};
        oracle_iodim v[1] = {{R, C, 1}};
        double *buf = malloc(sizeof(double) * 2 * R * C), *ref = malloc(sizeof(double) * 2 * R * C);
        for (int64_t i = 0; i < 2 * R * C; ++i) buf[i] = urand();
        /* reference: each row reversed, transformed, written as a column */
        for (int64_t r = 0; r < R; ++r) {
            double line[48], outl[48];
            for (int64_t k = 0; k < C; ++k) {
                line[2 * k] = buf[2 * (r * C + C - 1 - k)];
                line[2 * k + 1] = buf[2 * (r * C + C - 1 - k) + 1];
            }
            oracle_dft_direct_1d(C, 1, line, 1, outl, 1);
            for (int64_t k = 0; k < C; ++k) {
                ref[2 * (r + k * R)] = outl[2 * k];
                ref[2 * (r + k * R) + 1] = outl[2 * k + 1];
            }
        }
        /* element (0) of the input tensor is the last of row 0 */
        if (oracle_dft(1, d, 1, v, buf + 2 * (C - 1), buf, 1, 0, 4)) bad = 1;
        if (rel_diff(buf, ref, R * C) > 1e-14) {
            printf("strided in-place mismatch %.3e\n", rel_diff(buf, ref, R * C));
            bad = 1;
        }
        free(buf);
        free(ref);
    }
    printf(bad ? "oracle sanitizer check FAILED\n" : "oracle sanitizer check ok\n");
    return bad;
}
