// Internal types shared by the C-ABI layer (spd_api.cpp) and the gfx950 kernels
// (spd_kernels.hip).  Plain structs passed by value as kernel arguments.
#pragma once

#include <stdint.h>

#include "spd.h"

namespace spd {

constexpr int kMaxLevels = SPD_MAX_LEVELS;
constexpr int kMaxLevelWidths = SPD_MAX_LEVEL_WIDTHS;
constexpr int kLossyChunk = 1024;    // input samples streamed per step of the cascade kernel
constexpr int kExhSlots = 256;       // output slots per exhaustive work item (64 lanes x 4)
constexpr int kExhBlock = 512;       // widths per LDS window refill in the exhaustive kernel
constexpr int kExhGroup = 64;        // widths per max-only group (argmax recovered afterwards)
constexpr int kSlabCap = 64;         // pre-candidates kept per (level, row, segment), lossy
constexpr int kExhSlabCap = 16;      // pre-candidates kept per exhaustive work item
constexpr int kPeakWaves = 4096;     // waves of the peak-finder pass (slab ranges per wave)

// One separation level of a BoxDIT / IGRID search (boxcars every 2^k samples).
// Level k works on the decimated series y_k: unit n of y_k is the sum of the 2^k raw samples
// starting at n 2^k + base (relative to the work item's first sample).  It is made from level
// k-1 as y_k[n] = y_{k-1}[2n + cshift] + y_{k-1}[2n + cshift + 1].
// Widths of the level: base + units[j] 2^k, j < nw (ascending).  For BoxDIT every boxcar of the
// level also includes the carried sum of its first `base` samples (the previous iteration's
// longest boxcar).
struct LevelDesc {
    int32_t cshift;          // cascade shift in units of level k-1 (BoxDIT: L^{k-1}_max)
    int32_t nw;              // widths evaluated at this level
    int32_t umax;            // units[nw-1]
    int32_t ufull;           // units summed for the carry handed to level k+1 (BoxDIT)
    int32_t base;            // raw offset of unit 0 (BoxDIT: sum_{j<k} 2^j L^j_max)
    int32_t cap;             // LDS capacity (floats) of this level's window
    int32_t lds_y;           // LDS offset (floats) of the y_k window
    int32_t lds_c;           // LDS offset (floats) of the carry window (BoxDIT)
    int32_t scale_off;       // offset of this level's 1/sqrt(L) table in the scale buffer
    int32_t slots;           // ceil(n_out / 2^k)
    int64_t plane_off;       // element offset of this level's plane
    int64_t pitch;           // elements between rows
    uint8_t units[kMaxLevelWidths];
};

struct LossyArgs {
    const float *x;
    int64_t ld;
    const float *mean;
    const float *sigma;
    float *Y;                 // planes (caller's or workspace)
    uint16_t *W;
    uint32_t *slab_cnt;       // [n_levels][n_dm][n_seg]
    uint32_t *slab_ent;       // [...][kSlabCap]
    int32_t n_dm, n_in, n_out, n_levels;
    int32_t seg, n_seg;       // samples per work item, work items per row
    int32_t max_chunks;       // hard bound on streamed chunks per work item
    int32_t vec_ok;           // x rows are 16-byte aligned (float4 loads)
    int32_t want_cand;
    int32_t n_scale;          // widths over all levels (1/sqrt(L) table in LDS)
    int32_t lds_scale;        // LDS offset (floats) of that table
    float threshold;
    LevelDesc lv[kMaxLevels];
};

struct ExhArgs {
    const float *x;
    int64_t ld;
    const float *mean;
    const float *sigma;
    float *Y;
    uint16_t *W;
    const float *scale;       // 1/sqrt(L), L = 1..l_end at index L-1
    const uint32_t *evalmask; // bit (L-1) set if width L is evaluated (list mode only)
    uint32_t *slab_cnt;
    uint32_t *slab_ent;
    int64_t pitch;
    int32_t n_dm, n_in, n_out, l_end;
    int32_t n_seg;
    int32_t vec_ok;
    int32_t want_cand;
    float threshold;
};

struct ScaleArgs {
    float *scale;             // 1/sqrt(L) for L = 1..n at index L-1 (exhaustive search)
    int32_t n;
};

struct MaskArgs {
    uint32_t *evalmask;
    int32_t n_words;
    uint32_t bits[SPD_MAX_LIST_LEND / 32];
};

struct PeakArgs {
    const float *Y;
    const uint16_t *W;
    const uint32_t *slab_cnt;
    const uint32_t *slab_ent;
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
    int32_t n_levels, n_dm, n_seg;
    int32_t seg;              // level-0 samples per segment
    float threshold;
    int32_t level_shift[kMaxLevels];
    int32_t level_slots[kMaxLevels];
    int64_t level_pitch[kMaxLevels];
    int64_t level_off[kMaxLevels];
};

// Launchers (spd_kernels.hip).  Return hipError_t as int.
int launch_scales(const ScaleArgs &a, void *stream);
int launch_evalmask(const MaskArgs &a, void *stream);
int launch_lossy(const LossyArgs &a, bool carry, int lds_bytes, void *stream);
int launch_exhaustive(const ExhArgs &a, bool dense, void *stream);
int launch_peaks(const PeakArgs &a, void *stream);
const char *hip_error_text(int err);

}  // namespace spd
