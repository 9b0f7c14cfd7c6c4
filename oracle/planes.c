/*
 * FP64 reference of the boxcar single-pulse search.  TEST INFRASTRUCTURE ONLY: linked by the
 * tests, by the smoke check and by the CPU-baseline leg of the benchmark, never by the library.
 *
 * What is computed (Section 2, eqs. "boxcar", "SNR", "SNRlong" and the white-noise scaling,
 * and the per-iteration output equation of Section 3):
 *
 *   X_L[s]      = sum_{j=0}^{L-1} x[s+j]
 *   SNR(s, L)   = (X_L[s] - L mu) / (sqrt(L) sigma)
 *   Y_k[m]      = max over the widths L of level k with s + L <= n_in of SNR(s, L),  s = m 2^k
 *   W_k[m]      = the smallest width attaining Y_k[m]
 *   gap_k[m]    = Y_k[m] minus the largest SNR among the other valid widths of the level
 *                 (+inf when only one width is valid)
 *   no valid width at s:  Y = -inf, W = 0, gap = +inf
 *
 * Level k has ceil(n_out / 2^k) slots per DM row.  Sums use the FP64 prefix sum of (x - mu),
 * whose differences equal X_L[s] - L mu.  Plain loops, no blocking; OpenMP only splits rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* wsig: NULL for the white-noise scaling sqrt(L) sigma, else the row's sigma of every width L
 * at wsig[L] (a measured standard-deviation table, Section 4.6). */
static void one_slot(const double *P, int64_t s, int32_t n_in, double sigma, const double *wsig,
                     const int32_t *w, int32_t nw, double *Y, int32_t *W, double *gap)
{
    double best = -INFINITY, second = -INFINITY;
    int32_t bw = 0;
    for (int32_t j = 0; j < nw; ++j) {
        int64_t L = w[j];
        if (s + L > n_in) continue;                       /* valid-only boundary */
        double snr = (P[s + L] - P[s]) / (wsig ? wsig[L] : sqrt((double)L) * sigma);
        if (snr > best) {                                 /* ascending widths: ties keep the smaller */
            second = best;
            best = snr;
            bw = (int32_t)L;
        } else if (snr > second) {
            second = snr;
        }
    }
    *Y = best;
    *W = bw;
    *gap = (bw == 0 || second == -INFINITY) ? INFINITY : best - second;
}

/*
 * x: [n_dm][ld] float32; mean, sigma: [n_dm].
 * Levels: level_k[i] = k of level i; widths of level i are widths[wptr[i] .. wptr[i+1]).
 * Outputs for level i start at element plane_off[i]; row d, slot m at plane_off[i] + d*slots_i + m
 * with slots_i = ceil(n_out / 2^k).
 */
void oracle_planes(const float *x, int64_t ld, int32_t n_dm, int32_t n_in, int32_t n_out,
                   const float *mean, const float *sigma, int32_t n_levels,
                   const int32_t *level_k, const int32_t *wptr, const int32_t *widths,
                   const int64_t *plane_off, double *Y, int32_t *W, double *gap,
                   const double *wsig, int64_t wsig_ld)
{
#pragma omp parallel
    {
        double *P = (double *)malloc(sizeof(double) * ((size_t)n_in + 1));
#pragma omp for schedule(dynamic, 1)
        for (int32_t d = 0; d < n_dm; ++d) {
            const float *row = x + (int64_t)d * ld;
            double mu = mean[d], sg = sigma[d];
            P[0] = 0.0;
            for (int32_t t = 0; t < n_in; ++t) P[t + 1] = P[t] + ((double)row[t] - mu);
            for (int32_t i = 0; i < n_levels; ++i) {
                int64_t stride = (int64_t)1 << level_k[i];
                int64_t slots = ((int64_t)n_out + stride - 1) / stride;
                int64_t base = plane_off[i] + (int64_t)d * slots;
                for (int64_t m = 0; m < slots; ++m)
                    one_slot(P, m * stride, n_in, sg, wsig ? wsig + (int64_t)d * wsig_ld : NULL,
                             widths + wptr[i], wptr[i + 1] - wptr[i],
                             Y + base + m, W + base + m, gap + base + m);
            }
        }
        free(P);
    }
}

/*
 * The same quantities at selected points only, by direct summation (no prefix sums), for
 * inputs too large for the full planes.  Point p: DM row rows[p], level index lev[p], slot
 * slot[p].  Widths as in oracle_planes.
 */
void oracle_points(const float *x, int64_t ld, int32_t n_in, const float *mean,
                   const float *sigma, const int32_t *level_k, const int32_t *wptr,
                   const int32_t *widths, int64_t n_points, const int32_t *rows,
                   const int32_t *lev, const int64_t *slot, double *Y, int32_t *W, double *gap)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n_points; ++p) {
        const float *row = x + (int64_t)rows[p] * ld;
        double mu = mean[rows[p]], sg = sigma[rows[p]];
        int32_t i = lev[p];
        int64_t s = slot[p] << level_k[i];
        const int32_t *w = widths + wptr[i];
        int32_t nw = wptr[i + 1] - wptr[i];
        double best = -INFINITY, second = -INFINITY, X = 0.0;
        int32_t bw = 0;
        int64_t summed = 0;
        for (int32_t j = 0; j < nw; ++j) {
            int64_t L = w[j];
            if (s + L > n_in) break;                      /* widths ascend: the rest are invalid too */
            for (; summed < L; ++summed) X += (double)row[s + summed] - mu;
            double snr = X / (sqrt((double)L) * sg);
            if (snr > best) {
                second = best;
                best = snr;
                bw = (int32_t)L;
            } else if (snr > second) {
                second = snr;
            }
        }
        Y[p] = best;
        W[p] = bw;
        gap[p] = (bw == 0 || second == -INFINITY) ? INFINITY : best - second;
    }
}

/* SNR(s, L) of single (row, start, width) triples by direct summation; -inf if s + L > n_in. */
void oracle_snr(const float *x, int64_t ld, int32_t n_in, const float *mean, const float *sigma,
                int64_t n, const int32_t *rows, const int64_t *starts, const int32_t *widths,
                double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; ++p) {
        int64_t s = starts[p], L = widths[p];
        if (L < 1 || s < 0 || s + L > n_in) {
            out[p] = -INFINITY;
            continue;
        }
        const float *row = x + (int64_t)rows[p] * ld;
        double mu = mean[rows[p]], X = 0.0;
        for (int64_t j = 0; j < L; ++j) X += (double)row[s + j] - mu;
        out[p] = X / (sqrt((double)L) * sigma[rows[p]]);
    }
}
