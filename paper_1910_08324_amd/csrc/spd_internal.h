// Internal types shared by the C-ABI layer (spd_api.cpp) and the gfx950 kernels
// (spd_kernels.hip).  Plain structs passed by value as kernel arguments.
#pragma once

#include <stdint.h>

#include "spd.h"

namespace spd {

constexpr int kMaxLevels = SPD_MAX_LEVELS;
constexpr int kMaxLevelWidths = SPD_MAX_LEVEL_WIDTHS;
constexpr int kStepMaxLevels = 6;     // levels handled by one launch of the cascade kernel
constexpr int kStepThreads = 256;     // threads per tile work-group
constexpr int kSmallStepThreads = 128; // threads per IG(1) work-group on short tiles
constexpr int kSmallTileMax = 3072;    // longest tile (units) run on kSmallStepThreads
constexpr int kGroup = 4;             // consecutive slots evaluated together by one thread
constexpr int kExhSlots = 256;        // output slots per exhaustive work item (64 lanes x 4)
constexpr int kExhBlock = 512;        // widths per LDS window refill in the exhaustive kernel
constexpr int kExhGroup = 64;         // most widths per max-only group (argmax recovered afterwards)
constexpr int kExhSmallGroupMax = 4096;  // largest L_end searched in groups of 16 widths
constexpr int kSlabCap = 64;          // pre-candidates kept per (level, row, tile): one per lane
constexpr int kExhSlabCap = 16;       // pre-candidates kept per exhaustive work item
constexpr int kExhItemsPerWave = 4;   // work items per wave when every width fits one block
constexpr int kPeakWaves = 8192;      // waves of the peak-finder passes

// One level of a cascade step.  The step's input series is y_{k0} (for the first step the
// normalised samples); level j of the step is the absolute level k = k0 + j, whose unit n is
// the sum of 2^k samples starting at n 2^k + base (BoxDIT: base = off_k, the width of the
// carried prefix; IGRID: 0).  Level j is made from level j-1 as
//     y_j[n] = y_{j-1}[2n + cshift] + y_{j-1}[2n + cshift + 1].
// The boxcars of the level at slot m are  carry[m] + sum_{u < U} y_j[m + u]  for every unit
// count U with bit (U-1) of `evalmask` set (BoxDIT adds the carried prefix; IGRID has none).
struct StepLevel {
    int32_t k;               // absolute level index = log2 of the boxcar separation
    int32_t cshift;          // cascade shift in units of level j-1
    int32_t n_units;         // units of this level formed in a tile (LDS buffer length)
    int32_t lds_y;           // LDS offset (floats) of the unit buffer
    int32_t lds_c;           // LDS offset (floats) of the carry buffer (BoxDIT)
    int32_t umax;            // widest unit count evaluated (0: output-only level)
    int32_t ufull;           // units in the carry handed to level j+1 (BoxDIT)
    int32_t base;            // raw width offset of the level
    int32_t slots;           // plane slots per row = ceil(n_out / 2^k)
    int32_t pattern;         // 1, 2: the family's compiled-in width pattern; 0: generic
    uint64_t evalmask;       // bit U-1: U units is one of the level's widths
    int64_t plane_off;       // element offset of the level's plane
    int64_t pitch;           // elements between rows of the plane
    int64_t slab_base;       // first pre-candidate slab of the level
    int64_t cnt_off;         // pre-candidate count of (row d, tile t) at cnt_off + (d n_tiles + t) J
    int64_t mask_off;        // candidates only: first word of the level's above-threshold bits
    int32_t mask_wps;        // words of above-threshold group bits per (row, tile) slab
    int32_t pad1;
};

// What the peak finder needs to form any slot of a cascade step again, bit for bit, when the
// planes are not written (candidates only): the step's input series and the constants of its
// levels.  Written into the workspace by the step's first work-group.
struct RecLevel {
    int32_t k, cshift, umax, ufull, base, slots;
    uint64_t evalmask;
    float rt[kMaxLevelWidths];        // the level's 1/sqrt(L) at [U-1]
};

struct RecStep {
    const float *in;          // step input series (raw samples for the first step)
    const float *cin;         // carried prefixes of the first level (BoxDIT, later steps), or null
    const float *mean;
    const float *sigma;
    const float *rho;         // sigma-table ratios, or null
    int64_t ld_in, ld_cin, ld_rho;
    int32_t n_rho, in_len, n_in, normalise, carry, J;
    RecLevel lv[kStepMaxLevels];
};

struct StepArgs {
    const float *in;          // step input series [n_dm][ld_in] (raw samples for the first step)
    const float *cin;         // carried prefixes of the first level [n_dm][ld_cin] (BoxDIT, k0 > 0)
    float *out;               // series for the next step [n_dm][ld_out], or null
    float *cout;              // carried prefixes for the next step, or null
    const float *mean;
    const float *sigma;
    float *Y;                 // planes (caller's or workspace)
    uint16_t *W;
    uint32_t *slab_cnt;
    uint32_t *slab_ent;
    int64_t ld_in, ld_cin, ld_out;
    int32_t n_dm;
    int32_t n_in;             // raw samples per row (valid-only boundary)
    int32_t in_len;           // units of the input series available per row
    int32_t T;                // tile length in units of the input series
    int32_t n_tiles;          // tiles per row
    int32_t J;                // bank levels in this step
    int32_t has_out;          // produce level J for the next step
    int32_t normalise;        // first step: z = (x - mean) / sigma on load
    int32_t carry;            // BoxDIT
    int32_t vec_ok;           // rows of `in` are 16-byte aligned
    int32_t want_cand;
    float threshold;
    const float *rho;         // per-row sigma-table ratios [n_dm][ld_rho] at widths 2^0.. (or null)
    int64_t ld_rho;
    int32_t n_rho;
    int32_t lds_sc;           // LDS offset (floats) of the per-row width scales (rho != null)
    int32_t write_planes;     // store the planes (else the peak finder recomputes what it reads)
    int32_t nth;              // threads per work-group (the planner's choice; single-beam launches)
    RecStep *rec;             // where the first work-group records the step, or null
    uint32_t *amask;          // above-threshold bits of the slots (candidates only), or null
    StepLevel lv[kStepMaxLevels + 1];
    float rtab[kStepMaxLevels][kMaxLevelWidths];   // 1/sqrt(base + U 2^k) at [j][U-1]
};

// The buffers and sizes of one beam in a cascade launch (a beam is a block of DM rows with its
// own length; the levels, width patterns and tile length are shared by the launch).
struct BeamView {
    const float *in;
    const float *cin;
    float *out;
    float *cout;
    const float *mean;
    const float *sigma;
    float *Y;
    uint16_t *W;
    uint32_t *slab_cnt;
    uint32_t *slab_ent;
    int64_t ld_in, ld_cin, ld_out;
    int32_t n_dm, n_in, in_len, n_tiles, vec_ok, pad0;
    RecStep *rec;               // the beam's record of this step (candidates only), or null
    uint32_t *amask;            // the beam's above-threshold bits (candidates only), or null
    int64_t mask_off[kStepMaxLevels];
    int64_t cnt_off[kStepMaxLevels];
    int64_t plane_off[kStepMaxLevels];
    int64_t pitch[kStepMaxLevels];
    int64_t slab_base[kStepMaxLevels];
    int32_t slots[kStepMaxLevels];
};

struct StepBatchArgs {
    StepArgs s;                 // shared fields (the per-beam ones are unused)
    const BeamView *beams;      // [n_beams], device
    const int64_t *item_base;   // [n_beams + 1], device: first work item of each beam
    int64_t n_items;
    int32_t n_beams;
};

struct ExhArgs {
    const float *x;
    int64_t ld;
    const float *mean;
    const float *sigma;
    float *Y;
    uint16_t *W;
    const float *scale;       // 1/sqrt(L) (or 1/sigma-table ratio), L = 1..l_end at index L-1
    int64_t scale_ld;         // 0: one table for every row; else row d's table at d * scale_ld
    const uint32_t *evalmask; // bit (L-1) set if width L is evaluated (list mode only)
    uint32_t *slab_cnt;
    uint32_t *slab_ent;
    int64_t pitch;
    int32_t n_dm, n_in, n_out, l_end;
    int32_t n_seg;
    int32_t segs_per_wave;    // consecutive work items per wave (> 1 only when l_end <= kExhBlock)
    int32_t vec_ok;
    int32_t want_cand;
    float threshold;
    // tile-gated search: only work items in tiles whose flag is set are searched (the others
    // record no pre-candidates and leave the planes untouched); null = every item
    const uint8_t *tile_flag;   // [n_row_tiles][n_col_tiles]
    int32_t tile_rows, tile_len, n_col_tiles;
};

struct ScaleArgs {
    float *scale;             // 1/sqrt(L) for L = 1..n at index L-1 (exhaustive search)
    int32_t n;
    int32_t n_rows;           // rho != null: one table per row, row d at d * row_ld
    int64_t row_ld;
    const float *rho;         // [n_rows][ld_rho]: scale = 1 / (sqrt(L) rho_d(L))
    int64_t ld_rho;
    int32_t n_rho;
};

struct MaskArgs {
    uint32_t *evalmask;
    int32_t n_words;
    uint32_t bits[SPD_MAX_LIST_LEND / 32];
};

// Pre-candidate slabs: one per (level, row, tile); the slabs of level k start at slab_base[k]
// and are ordered by row, then tile.  Tile t of level k covers slots
// [t tile_slots[k], min((t+1) tile_slots[k], slots[k])).
struct PeakArgs {
    const float *Y;
    const uint16_t *W;
    uint32_t *slab_cnt;
    uint32_t *slab_ent;       // sorted in place by the count pass
    uint32_t *surv;           // survivors per slab
    uint64_t *mask;           // survivor bitmask per slab (entries mode)
    int64_t *wave_tot;
    int64_t *wave_off;
    spd_candidate *cand;
    int64_t cand_cap;
    int64_t *cand_count;
    int64_t t0;
    int64_t n_slabs;
    int64_t slabs_per_wave;
    int32_t n_waves;
    int32_t slab_cap;
    int32_t n_levels, n_dm;
    float threshold;
    int32_t level_shift[kMaxLevels];
    int32_t level_slots[kMaxLevels];
    int32_t tiles_per_row[kMaxLevels];
    int32_t tile_slots[kMaxLevels];
    int64_t slab_base[kMaxLevels + 1];
    int64_t level_pitch[kMaxLevels];
    int64_t level_off[kMaxLevels];
    // the count of slab s = slab_base[k] + r (r = d tiles_per_row[k] + t) is slab_cnt[cnt_off[k] +
    // r cnt_stride[k]]: a cascade launch writes the counts of its levels for one tile together
    int64_t cnt_off[kMaxLevels];
    int32_t cnt_stride[kMaxLevels];
    // planes not written (lossy, candidates only): slot values are formed again from the
    // records of the cascade steps; level k is level level_j[k] of step level_step[k]
    const RecStep *rec;
    int8_t level_step[kMaxLevels];
    int8_t level_j[kMaxLevels];
    // bit g % 32 of word mask_off[k] + (d tiles_per_row[k] + t) mask_wps[k] + g / 32, with
    // g = (m - t tile_slots[k]) / kGroup: some slot of that group of level k in row d is above
    // the threshold (candidates only)
    const uint32_t *amask;
    int64_t mask_off[kMaxLevels];
    int32_t mask_wps[kMaxLevels];
    // tile gating: flag_mode 0 = every slot; 1 = candidates only in tiles whose flag is clear
    // (the planes are complete); 2 = only in tiles whose flag is set, where the plane exists
    // (neighbours in other tiles are absent).  Tile of (d, sample s): (d / tile_rows, s / tile_len).
    const uint8_t *tile_flag;
    int32_t flag_mode, tile_rows, tile_len, n_col_tiles;
    const int64_t *base_count;  // candidates already in the list (written before it), or null
};

// Launchers (spd_kernels.hip).  Return hipError_t as int.
int launch_scales(const ScaleArgs &a, void *stream);
int launch_evalmask(const MaskArgs &a, void *stream);
int launch_step(const StepArgs &a, int fam, int lds_bytes, void *stream);
int launch_step_batch(const StepBatchArgs &a, int fam, int lds_bytes, int grid, void *stream);
// unit-count mask of a family's compiled-in pattern (1 or 2); families: 1-3 IG(1..3),
// 4-6 BD-8/16/32, 7 DIT, 0 none
uint64_t family_mask(int fam, int pattern);
int launch_exhaustive(const ExhArgs &a, bool dense, void *stream);
int launch_peaks(const PeakArgs &a, void *stream);
// p[0 .. n) = v (a kernel, so that graph capture records no memset node)
int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, void *stream);

// the peak finder over every beam of a batch: a device table of PeakArgs (16-byte aligned) and
// the first global wave index of each beam (n_beams + 1 entries)
struct PeakBatchArgs {
    const PeakArgs *tab;
    const int64_t *wave_base;
    int64_t n_waves;
    int32_t n_beams;
};
int launch_peaks_batch(const PeakBatchArgs &a, void *stream);
const char *hip_error_text(int err);

}  // namespace spd
