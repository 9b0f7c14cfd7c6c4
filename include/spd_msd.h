/*
 * spd_msd.h -- noise mean and standard deviation (MSD) per DM trial, with outlier rejection and
 * the standard deviation of every power-of-two decimation (C ABI, gfx950).
 *
 * Section 4.6 of Adamek & Armour (arXiv:1910.08324): the statistics of the base-level noise are
 * estimated with a numerically stable streaming algorithm (Chan, Golub & LeVeque 1983: partial
 * counts, means and sums of squared deviations combined pairwise) and point-wise outlier
 * rejection repeated until it converges; the standard deviation is computed for the series
 * decimated by powers of two (boxcar widths 2^k) and interpolated for the widths in between.
 *
 * Definitions used here (the paper gives no formulas):
 *   level k series   y_k[i] = sum of x[d][t] over t in [i 2^k, (i+1) 2^k), i < n_in >> k;
 *   estimate         mean and standard deviation (n - 1 denominator) of the kept values; the
 *                    first pass keeps every value, each later pass keeps |y - mean| <= tau sd of
 *                    the previous pass; stop after max_iter passes or when the kept count does
 *                    not change;
 *   rho[d][k]        sd_k / (sqrt(2^k) sd_0): 1 for white noise;
 *   sigma of width L sqrt(L) sd_0 rho(L), rho linear in log2 L between adjacent levels and held
 *                    at the last level's value above it (SPD_SIGMA_TABLE in spd_search).
 * All arithmetic is FP64; results are rounded to FP32 once.
 */
#ifndef SPD_MSD_H
#define SPD_MSD_H

#include <stdint.h>

#include "spd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* HOST *bytes of device workspace spd_msd needs. */
int spd_msd_workspace(int32_t n_dm, int32_t n_in, int32_t levels, int64_t *bytes);

/*
 * spd_msd: x [n_dm][ld] float (ld >= n_in); levels 1..SPD_MAX_LEVELS with n_in >> (levels-1)
 * >= 2; tau > 0; max_iter >= 0.  Outputs (device): mean[n_dm], sigma[n_dm] (float, level 0,
 * ready for spd_search), and, if not NULL, rho[n_dm][levels] and level_sd[n_dm][levels] (float)
 * and passes[n_dm] (int32: estimate passes, 1 + the most rejection passes any level took, at most
 * 1 + max_iter).  The first pass reads the row's samples and lists, per level 0..5, the values
 * beyond a band around a pre-estimate of the mean (from a few tiles of the row); while the
 * current limit covers that band, a rejection pass needs only the listed values, otherwise it
 * reads the row again and lists anew.  The kept sets, counts and passes are those of passes that
 * read every value; only the order of the FP64 sums differs, and it is fixed (results do not vary
 * from run to run).  The workspace holds, per row, the decimated values of levels 6 and up (fewer
 * than n_in / 32) and room for the lists (1/16 of the values of each level 0..5); its size
 * depends on n_in only.  One work-group per row; asynchronous on the stream.  SPD_EINVAL for bad
 * sizes or NULL mean / sigma, SPD_EWORKSPACE / SPD_EALIGN for a short or unaligned (256-byte)
 * workspace, SPD_EHIP for a failed launch.
 */
int spd_msd(const float *x, int64_t ld, int32_t n_dm, int32_t n_in, int32_t levels, float tau,
            int32_t max_iter, float *mean, float *sigma, float *rho, float *level_sd,
            int32_t *passes, void *workspace, int64_t workspace_bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SPD_MSD_H */
