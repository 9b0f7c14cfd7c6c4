/* Drives the FP64 oracle (oracle/planes.c, included as one translation unit) on small random
 * inputs under AddressSanitizer / UBSan: full planes for several width sets, look-ahead and
 * short rows, point evaluation and single boxcars, including widths that do not fit. */
#include "../../oracle/planes.c"

#include <stdio.h>

static float frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (float)((*s >> 8) & 0xffff) / 32768.0f - 1.0f;
}

int main(void) {
    unsigned seed = 1;
    const int n_dm = 3, n_in = 700, ld = 703;
    float *x = (float *)malloc(sizeof(float) * n_dm * ld);
    for (int i = 0; i < n_dm * ld; ++i) x[i] = frand(&seed);
    float mean[3] = {0.1f, -0.2f, 0.0f}, sigma[3] = {1.0f, 0.5f, 2.0f};
    const int outs[] = {700, 333, 1};
    for (int oi = 0; oi < 3; ++oi) {
        const int n_out = outs[oi];
        /* levels: k = 0 widths 1..9, k = 2 widths 12, 20, 64 (some do not fit near the end) */
        int32_t level_k[2] = {0, 2}, wptr[3] = {0, 9, 12};
        int32_t widths[12] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 20, 64};
        int64_t plane_off[2];
        int64_t s0 = n_out, s1 = (n_out + 3) / 4;
        plane_off[0] = 0;
        plane_off[1] = s0 * n_dm;
        int64_t tot = (s0 + s1) * n_dm;
        double *Y = (double *)malloc(sizeof(double) * tot), *gap = (double *)malloc(sizeof(double) * tot);
        int32_t *W = (int32_t *)malloc(sizeof(int32_t) * tot);
        oracle_planes(x, ld, n_dm, n_in, n_out, mean, sigma, 2, level_k, wptr, widths, plane_off,
                      Y, W, gap, NULL, 0);
        /* per-row sigma of each width */
        double *wsig = (double *)malloc(sizeof(double) * n_dm * 65);
        for (int i = 0; i < n_dm * 65; ++i) wsig[i] = 1.0 + 0.01 * (i % 65);
        oracle_planes(x, ld, n_dm, n_in, n_out, mean, sigma, 2, level_k, wptr, widths, plane_off,
                      Y, W, gap, wsig, 65);
        free(Y); free(gap); free(W); free(wsig);
    }
    {
        int32_t rows[4] = {0, 1, 2, 2}, lev[4] = {0, 1, 0, 1};
        int64_t slot[4] = {0, 10, 699, 174};
        int32_t level_k[2] = {0, 2}, wptr[3] = {0, 3, 5}, widths[5] = {1, 8, 700, 4, 696};
        double Y[4], gap[4];
        int32_t W[4];
        oracle_points(x, ld, n_in, mean, sigma, level_k, wptr, widths, 4, rows, lev, slot, Y, W, gap);
    }
    {
        int64_t starts[5] = {0, 10, 699, 700, -1};
        int32_t wl[5] = {1, 690, 1, 1, 3}, rows[5] = {0, 1, 2, 0, 1};
        double out[5];
        oracle_snr(x, ld, n_in, mean, sigma, 5, rows, starts, wl, out);
    }
#ifdef PLANT_OVERFLOW
    /* a read one past the input, to show that the build catches such mistakes */
    printf("%f\n", (double)x[n_dm * ld]);
#endif
    free(x);
    printf("oracle driver done\n");
    return 0;
}
