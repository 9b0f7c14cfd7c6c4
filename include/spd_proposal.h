/*
 * spd_proposal.h -- learned tile proposal for the boxcar single-pulse search (C ABI, gfx950).
 *
 * Not part of Adamek & Armour (arXiv:1910.08324): a small network that reads the pure
 * decimated series y_k of the IGRID/DIT level cascade (Section 3.2; levels k = 4..8) of a tile
 * of 64 DM rows x 4096 samples and scores how likely the exhaustive boxcar set (Section 3.1)
 * finds a pulse there that the lossy sets miss by more than a margin (the signal-loss figures
 * of Section 4 and Appendix A).  Flagged tiles get the exhaustive search; the others keep the
 * lossy result.  Training runs on the GPU with these kernels (bfloat16 MFMA, FP32 accumulation)
 * on tiles generated on the GPU and labelled by the library's own exhaustive and lossy searches.
 *
 * Features of a row (normalised samples z = (x - mean) / sigma, 4096 per row):
 *     y_k[i] = sum of z over [i 2^k, (i+1) 2^k),  k = 4..8, divided by 2^(k/2);
 * laid out as P = 256 positions (level-4 resolution) by 8 channels (channel c < 5 holds level
 * 4 + c at position p >> c; channels 5..7 are zero), bfloat16, with two zero positions before
 * and four after each row: feat[row][SPD_PROP_ROW_POS][8], data at positions 2 .. 257.
 *
 * Network (per row): three 5-tap convolutions with 32 output channels, ReLU after each, zero
 * padding; a 1x1 read-out s[p] = bh + wh . a3[p]; tile logit = log(mean over the tile's
 * 64 x 256 positions of exp(s)).  Training loss: mean logistic loss over tiles.
 *
 * Parameters: one FP32 array of SPD_PROP_NPARAMS values (device), at the offsets below:
 *     W1[32][5][8] (entries with input channel >= 5 must be zero), b1[32], W2[32][5][32], b2[32],
 *     W3[32][5][32], b3[32], wh[32], bh, then 3 unused values.
 * W[co][t][ci] multiplies input channel ci at position p + t - 2 for output channel co at p.
 *
 * Conventions as in spd.h: every call returns SPD_OK or a negative status, is asynchronous on
 * the given HIP stream, never allocates and never synchronises; all pointers are device
 * pointers unless marked HOST.  Workspace alignment: 256 bytes.
 */
#ifndef SPD_PROPOSAL_H
#define SPD_PROPOSAL_H

#include <stdint.h>

#include "spd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SPD_PROP_TILE_ROWS 64
#define SPD_PROP_TILE_LEN 4096
#define SPD_PROP_POS 256
#define SPD_PROP_ROW_POS 262      /* positions per row in feature/activation buffers (pads) */
#define SPD_PROP_FEAT_CH 8
#define SPD_PROP_CH 32
#define SPD_PROP_TAPS 5

#define SPD_PROP_OFF_W1 0
#define SPD_PROP_OFF_B1 1280
#define SPD_PROP_OFF_W2 1312
#define SPD_PROP_OFF_B2 6432
#define SPD_PROP_OFF_W3 6464
#define SPD_PROP_OFF_B3 11584
#define SPD_PROP_OFF_WH 11616
#define SPD_PROP_OFF_BH 11648
#define SPD_PROP_NPARAMS 11652

/*
 * spd_tiles_generate: synthetic training/evaluation tiles, generated on the GPU.
 *   x  float [n_tiles * 64][4096]: tile t (absolute index first_tile + i) fills rows 64 i ..
 *      64 i + 63.  White N(0, 1) noise from Philox4x32-10 (Salmon et al., SC 2011; counter
 *      (block, row, t low, t high), key = seed) through the Box-Muller transform, plus 0, 1 or
 *      2 rectangular pulses of width 1..64 and SNR 6..30 (amplitude snr / sqrt(width)) drawn
 *      from counters (j, 0xffffffff, t low, t high).  The recipe is documented in synth/philox.py.
 * Returns SPD_EINVAL for n_tiles < 1, first_tile < 0 or x NULL.
 */
int spd_tiles_generate(uint64_t seed, int64_t first_tile, int32_t n_tiles, float *x,
                       void *hip_stream);

/*
 * spd_prop_features: DIT-level features of n_rows rows of 4096 samples.
 *   x [n_rows][ld] float (ld >= 4096, ld % 4 == 0, 16-byte aligned rows), mean/sigma [n_rows];
 *   feat bfloat16 (uint16 storage) [n_rows][SPD_PROP_ROW_POS][8], pads written as zero.
 */
int spd_prop_features(const float *x, int64_t ld, int32_t n_rows, const float *mean,
                      const float *sigma, uint16_t *feat, void *hip_stream);

/* Workspace bytes (HOST *bytes) that spd_prop_forward / spd_prop_backward need for n_tiles. */
int spd_prop_workspace(int32_t n_tiles, int64_t *bytes);

/*
 * spd_prop_forward: tile logits [n_tiles] (float) of the features of n_tiles tiles
 * (64 n_tiles rows).  Inference.
 */
int spd_prop_forward(const float *params, const uint16_t *feat, int32_t n_tiles, float *logits,
                     void *workspace, int64_t workspace_bytes, void *hip_stream);

/*
 * spd_prop_backward: forward pass, mean logistic loss against labels [n_tiles] (0 or 1, float)
 * written to loss[0], logits [n_tiles] (may be NULL) and the gradient of the loss with respect
 * to every parameter written to grads[SPD_PROP_NPARAMS] (the unused entries get 0).
 * Deterministic: partial sums are reduced in a fixed order.
 */
int spd_prop_backward(const float *params, const uint16_t *feat, const float *labels,
                      int32_t n_tiles, float *logits, float *grads, float *loss,
                      void *workspace, int64_t workspace_bytes, void *hip_stream);

/*
 * spd_prop_adam: one Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected; step >= 1) on params with the first/second moment arrays m, v (FP32,
 * SPD_PROP_NPARAMS each, zero before step 1).
 */
int spd_prop_adam(float *params, const float *grads, float *m, float *v, int32_t step, float lr,
                  void *hip_stream);

/*
 * spd_tile_max: maximum SNR of each tile of rows_per_tile consecutive DM rows over every level
 * plane of a search laid out as `info` describes (HOST pointer, from spd_plan for the same
 * parameters and sizes).  snr as written by spd_search; tile_max [n_dm / rows_per_tile] float.
 * n_dm must be a multiple of rows_per_tile.
 */
int spd_tile_max(const float *snr, const spd_plan_info *info, int32_t n_dm, int32_t rows_per_tile,
                 float *tile_max, void *hip_stream);

/*
 * spd_prop_labels: label[t] = 1 if exh_max[t] > threshold and exh_max[t] > (1 + margin)
 * lossy_max[t] (both products and comparisons in FP32), else 0.
 */
int spd_prop_labels(const float *exh_max, const float *lossy_max, int32_t n_tiles,
                    float threshold, float margin, float *labels, void *hip_stream);

/*
 * spd_prop_flags: the tile flag map of spd_search_gated (spd.h) from the logits of a grid of
 * n_row_tiles x n_col_tiles tiles.  logits [n_col_tiles * n_row_tiles] hold tile (r, c) at
 * c n_row_tiles + r (the order of spd_prop_features run on one column of tiles after another);
 * flags [n_row_tiles][n_col_tiles] (uint8) get 1 where the logit is above logit_threshold.
 */
int spd_prop_flags(const float *logits, int32_t n_row_tiles, int32_t n_col_tiles,
                   float logit_threshold, uint8_t *flags, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SPD_PROPOSAL_H */
