/*
 * spd.h -- boxcar single-pulse search on AMD Instinct MI355X (gfx950), C ABI.
 *
 * Implements the single pulse detection (SPD) step of Adamek & Armour, "Single Pulse Detection
 * Algorithms for Real-time Fast Radio Burst Searches using GPUs" (arXiv:1910.08324):
 * boxcar matched filtering of dedispersed time series, one row per DM trial, with
 *   - the ideal (exhaustive) search: every width 1..L_end at every sample (Section 3.1);
 *   - BoxDIT: boxcars up to L^i_max on data decimated i times, widths
 *       sum_{k<i} 2^k L^k_max + 2^i m,  m = 1..L^i_max, every 2^i samples (Algorithm 1, Section 3.1);
 *   - IGRID IG(d): base widths 2^j with P layers (boxcars every 2^j / P samples) and the extra
 *     widths 2^j + q 2^j / 2^d, q < 2^d, from traversing the tree to depth d (Section 3.2, Table 1);
 * each producing, per separation level k (boxcars every 2^k samples), the highest SNR Y_k and the
 * width W_k that produced it (the per-iteration output equation of Section 3), followed by
 * thresholded peak finding that selects candidates (Section 4.6).
 *
 * SNR of a boxcar of width L starting at s (Section 2, eqs. SNR and SNRlong with the white-noise
 * scaling mu(X_L) = L mu, sigma(X_L) = sqrt(L) sigma):
 *     SNR(s, L) = (sum_{j<L} x[s+j] - L mu) / (sqrt(L) sigma)
 * Y_k[m] is the maximum over the level's widths L with s + L <= n_in, s = m 2^k; W_k[m] is the
 * smallest width reaching it; if no width fits, Y_k[m] = -inf and W_k[m] = 0.
 *
 * Candidate rule (the paper names its peak finder without defining it; this is the definition
 * implemented): on each level plane, slot (d, m) is a candidate iff Y > threshold and, for each
 * in-bounds neighbour (d+a, m+b), a, b in {-1,0,1}, Y > Y_nb if the neighbour precedes (d, m) in
 * row-major order and Y >= Y_nb if it follows.  Candidates are ordered by (level, dm, start).
 *
 * Conventions
 *   - Every function returns SPD_OK (0) or a negative status; nothing throws across the ABI.
 *   - spd_search is asynchronous on the given HIP stream; it never allocates, never frees and
 *     never synchronises.  The caller owns every buffer and keeps it alive until the stream has
 *     finished the call.  One call in flight per workspace.
 *   - Device pointers are HIP device memory on the current device.  Host pointers are marked.
 */
#ifndef SPD_H
#define SPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPD_ABI_VERSION 5

/* Status codes. */
#define SPD_OK          0
#define SPD_EINVAL     -1  /* an argument is out of range or inconsistent (see each field)  */
#define SPD_EALIGN     -2  /* t0 is not a multiple of 2^K (K = top level), or a bad pointer   */
#define SPD_EWORKSPACE -3  /* workspace is NULL or smaller than spd_plan_info.workspace_bytes */
#define SPD_EHIP       -4  /* a HIP launch failed; spd_error_string has the text               */

/* Search methods. */
#define SPD_EXHAUSTIVE 0
#define SPD_BOXDIT     1
#define SPD_IGRID      2

/* Output flags (at least one must be set). */
#define SPD_WRITE_PLANES     1u  /* write the per-level Y (float) and W (uint16) planes        */
#define SPD_WRITE_CANDIDATES 2u  /* run the peak finder and write the candidate list           */

#define SPD_MAX_LEVELS 24
#define SPD_MAX_LEVEL_WIDTHS 64   /* widths per level for BoxDIT and IGRID                     */
#define SPD_MAX_LEND 65535        /* widths are stored as uint16                               */
#define SPD_MAX_LIST_LEND 16384   /* largest width when an explicit exhaustive list is given   */
#define SPD_MAX_LAUNCHES 26       /* kernel launches of one spd_filter call                    */

/*
 * Search parameters.  All pointers in this struct are HOST pointers, read during the call only.
 *   method          SPD_EXHAUSTIVE, SPD_BOXDIT or SPD_IGRID.
 *   l_end           largest boxcar width L_end, 1..65535.  Lossy width sets are cut at l_end.
 *   widths/n_widths EXHAUSTIVE only: strictly increasing widths in [1, l_end] with l_end <= 16384,
 *                   or NULL / 0 for every width 1..l_end.
 *   boxdit_lmax     BOXDIT only: L^i_max per iteration (n_boxdit_lmax >= 1 entries; the last one
 *                   repeats).  Each even (the shifted decimation of Section 3.1 needs L^i_max
 *                   divisible by D = 2) and 2..64.
 *   igrid_depth     IGRID only: d in 0..4.
 *   igrid_layers    IGRID only: P, a power of two with 2^d <= P <= 64, or 0 for P = 2^(d+1) (the
 *                   paper's 4/8/16 layers for IG(1)/(2)/(3)).  d = 0, P = 1 is the plain DIT search.
 *   threshold       candidates need SNR strictly above it.
 *   flags           SPD_WRITE_PLANES | SPD_WRITE_CANDIDATES.
 *   segment         samples per work item along time (0 = chosen by the library).  Results do not
 *                   depend on it.  BoxDIT / IGRID: a multiple of 256 in 256..32768 that leaves
 *                   every launch of the level cascade room for its halo and its on-chip buffers
 *                   (spd_plan returns SPD_EINVAL otherwise); exhaustive: 256, or 512 / 1024 (a wave
 *                   takes 2 / 4 consecutive 256-sample items) when L_end <= 512.
 *   step_levels     BoxDIT / IGRID: separation levels computed on chip per kernel launch, 1..6,
 *                   or 0 for the library's choice (4, fewer if a tile's buffers would not fit).
 *                   Results do not depend on it.  Exhaustive: must be 0.
 *   rho, n_rho      NULL / 0 for the white-noise scaling sigma(L) = sqrt(L) sigma (Section 2.1).
 *                   Otherwise a DEVICE array [n_dm][n_rho] (the one exception to "host
 *                   pointers" here; read by the kernels): rho[d][k] = sd of row d decimated to
 *                   width 2^k over sqrt(2^k) sd_0, as spd_msd writes it, and the search uses
 *                   sigma(L) = sqrt(L) sigma[d] rho_d(L), rho_d linear in log2 L between adjacent
 *                   powers of two and held at rho[d][n_rho-1] above (Section 4.6).  1..24 levels.
 *                   Not supported by the batched search.
 */
typedef struct {
    int32_t method;
    int32_t l_end;
    const int32_t *widths;
    int32_t n_widths;
    const int32_t *boxdit_lmax;
    int32_t n_boxdit_lmax;
    int32_t igrid_depth;
    int32_t igrid_layers;
    float threshold;
    uint32_t flags;
    int32_t segment;
    int32_t step_levels;
    const float *rho;
    int32_t n_rho;
} spd_params;

/* One candidate (24 bytes).  start = t0 + m 2^k is the first sample of the boxcar; the pulse
 * centre is start + width / 2 (Section 4.4 reports detections at the centre). */
typedef struct {
    int64_t start;
    int32_t dm;
    int32_t width;
    int32_t level;
    float snr;
} spd_candidate;

/* Output geometry and workspace size of a search. */
typedef struct {
    int32_t n_levels;                         /* K + 1                                        */
    int32_t top_level;                        /* K: the last level's boxcars are 2^K apart    */
    int32_t max_width;                        /* widest boxcar evaluated                      */
    int32_t required_halo;                    /* max_width - 1                                 */
    int32_t level_shift[SPD_MAX_LEVELS];      /* level i places boxcars every 2^level_shift[i] */
    int32_t level_nwidths[SPD_MAX_LEVELS];    /* number of widths of level i                   */
    int64_t plane_offset[SPD_MAX_LEVELS];     /* element offset of level i in snr / width      */
    int64_t plane_slots[SPD_MAX_LEVELS];      /* slots per DM row = ceil(n_out / 2^k)           */
    int64_t plane_pitch[SPD_MAX_LEVELS];      /* elements between DM rows (multiple of 64)      */
    int64_t plane_elems;                      /* elements of the snr buffer (and width buffer)  */
    int64_t workspace_bytes;                  /* device workspace spd_search needs              */
    int32_t segment;                          /* samples per work item along time              */
    int32_t n_segments;                       /* work items per DM row                          */
    /* the kernel launches of spd_filter, in stream order (for measurement and accounting) */
    int32_t n_launches;
    int32_t launch_first_level[SPD_MAX_LAUNCHES]; /* first level computed; -1 for a set-up launch */
    int32_t launch_levels[SPD_MAX_LAUNCHES];      /* levels computed (planes written)           */
    int64_t launch_in_units[SPD_MAX_LAUNCHES];    /* floats read per DM row (samples, or decimated
                                                     series and carried prefixes handed on)   */
    int64_t launch_out_units[SPD_MAX_LAUNCHES];   /* floats per DM row handed to the next launch */
    int32_t launch_threads[SPD_MAX_LAUNCHES];     /* threads per work-group of each launch       */
    int32_t launch_tile[SPD_MAX_LAUNCHES];        /* units of the launch's input per work-group
                                                     (cascade launches; 0 for the others)     */
} spd_plan_info;

/*
 * spd_plan: validate parameters and describe the outputs of a search over n_dm rows.
 *   n_in  samples available per row (the boxcar at s may use x[s .. s+L-1] only if s+L <= n_in)
 *   n_out output slots at level 0 (starts 0..n_out-1); 1 <= n_out <= n_in <= 2^31 - 2^20.
 * Returns SPD_OK and fills *out, or SPD_EINVAL.  No device work.
 */
int spd_plan(const spd_params *params, int32_t n_dm, int32_t n_in, int32_t n_out,
             spd_plan_info *out);

/*
 * spd_level_widths: the widths (in samples, ascending) of level `level` of the search.
 * Writes at most `cap` entries to the HOST array `out` and the full count to *n.
 * Returns SPD_OK, or SPD_EINVAL for a bad level or parameters.  No device work.
 */
int spd_level_widths(const spd_params *params, int32_t level, int32_t *out, int32_t cap,
                     int32_t *n);

/*
 * spd_search: run the search on `hip_stream` (a hipStream_t; NULL = default stream).
 *   x          device float [n_dm][ld], ld >= n_in; row d is DM trial d.  Read only.
 *   t0         absolute sample index of x[:, 0]; must be a multiple of 2^K so that consecutive
 *              blocks of a stream see the same boxcar grid.  Only shifts candidate starts.
 *   mean,sigma device float [n_dm]: noise mean and standard deviation per row, sigma > 0
 *              (a precondition: the library does not read them on the host).
 *   snr,width  device planes laid out as in spd_plan_info (plane_elems elements each, level i at
 *              plane_offset[i], row d at + d * plane_pitch[i]; slots beyond plane_slots[i] in a
 *              row are left untouched).  Required with SPD_WRITE_PLANES, ignored otherwise.
 *   cand       device spd_candidate[cand_cap]; the first min(total, cand_cap) candidates in
 *              (level, dm, start) order are written.  Required (cand_cap may be 0) with
 *              SPD_WRITE_CANDIDATES.
 *   cand_count device int64: receives the TOTAL number of candidates, which may exceed cand_cap.
 *   workspace  device memory of at least spd_plan_info.workspace_bytes bytes, 256-byte aligned.
 * Returns SPD_OK once all kernels are enqueued, SPD_EINVAL / SPD_EALIGN / SPD_EWORKSPACE for bad
 * arguments (nothing enqueued), or SPD_EHIP if a launch failed.
 */
int spd_search(const spd_params *params, const float *x, int64_t ld, int32_t n_dm, int32_t n_in,
               int32_t n_out, int64_t t0, const float *mean, const float *sigma, float *snr,
               uint16_t *width, spd_candidate *cand, int64_t cand_cap, int64_t *cand_count,
               void *workspace, int64_t workspace_bytes, void *hip_stream);

/*
 * The two stages of spd_search as separate calls, for callers that time or overlap them.
 * spd_search == spd_filter followed by spd_peaks on the same stream, parameters, sizes,
 * planes and workspace.
 *
 * spd_filter: the boxcar search only (Sections 3.1 and 3.2): writes the planes (to snr/width,
 *   or into the workspace when SPD_WRITE_PLANES is not set) and, when SPD_WRITE_CANDIDATES is
 *   set, records in the workspace the slots above the threshold for spd_peaks.  BoxDIT and
 *   IGRID run as a chain of cascade launches, each computing up to step_levels levels on chip and
 *   handing its last decimated series (and, for BoxDIT, the carried prefixes) to the next
 *   through the workspace; spd_plan_info lists them.  Arguments as for spd_search.
 * spd_peaks: candidate selection from the planes and records left by spd_filter (params->flags
 *   must include SPD_WRITE_CANDIDATES; snr/width as given to spd_filter).  Arguments as for
 *   spd_search.
 */
int spd_filter(const spd_params *params, const float *x, int64_t ld, int32_t n_dm, int32_t n_in,
               int32_t n_out, const float *mean, const float *sigma, float *snr, uint16_t *width,
               void *workspace, int64_t workspace_bytes, void *hip_stream);

int spd_peaks(const spd_params *params, int32_t n_dm, int32_t n_in, int32_t n_out, int64_t t0,
              const float *snr, const uint16_t *width, spd_candidate *cand, int64_t cand_cap,
              int64_t *cand_count, void *workspace, int64_t workspace_bytes, void *hip_stream);

/*
 * spd_filter_timed: spd_filter with a HIP event recorded on `hip_stream` before the first kernel
 *   launch and after each one.  It then waits for the last event and writes each launch's
 *   duration in milliseconds to the HOST array launch_ms (at most `cap` entries, in the order of
 *   spd_plan_info's launch list) and the number of launches to the HOST int *n_launches.  Meant
 *   for measurement: unlike the other calls it creates and destroys HIP events and blocks the
 *   calling thread until the filter has finished.  Returns as spd_filter, or SPD_EHIP if an
 *   event call failed.
 */
int spd_filter_timed(const spd_params *params, const float *x, int64_t ld, int32_t n_dm,
                     int32_t n_in, int32_t n_out, const float *mean, const float *sigma,
                     float *snr, uint16_t *width, void *workspace, int64_t workspace_bytes,
                     void *hip_stream, float *launch_ms, int32_t cap, int32_t *n_launches);

/*
 * Tile-gated search: the lossy search everywhere and the exhaustive set (Section 3.1, the ideal
 * search the paper measures its losses against) only on flagged tiles of the DM x time block,
 * as a tile proposal selects them (spd_proposal.h).
 *
 * spd_gated_plan: HOST *workspace_bytes for spd_search_gated with these sizes.
 * spd_search_gated: on `hip_stream`,
 *   1. the lossy search `lossy` (BoxDIT or IGRID, SPD_WRITE_CANDIDATES required; its planes to
 *      snr/width with SPD_WRITE_PLANES, as for spd_search);
 *   2. the exhaustive search `exh` (SPD_EXHAUSTIVE, SPD_WRITE_CANDIDATES required) at the slots
 *      of flagged tiles only.  With SPD_WRITE_PLANES its level-0 plane goes to exh_snr/exh_width
 *      (layout of spd_plan for `exh`); slots outside flagged tiles are left untouched.
 *   Tiles: tile (r, c) holds DM rows [r tile_rows, (r+1) tile_rows) and output slots (samples)
 *   [c tile_len, (c+1) tile_len); tile_flag is a DEVICE uint8 array
 *   [ceil(n_dm / tile_rows)][ceil(n_out / tile_len)], nonzero = flagged.  tile_rows >= 1;
 *   tile_len a multiple of 1024.
 *   Candidates (cand, cand_cap, cand_count as for spd_search): first the lossy search's
 *   candidates whose (dm, start - t0) lies in an unflagged tile, in (level, dm, start) order,
 *   then the exhaustive search's candidates in flagged tiles in (dm, start) order (level 0).
 *   The exhaustive candidates' 3x3 test sees only neighbours inside flagged tiles (the plane
 *   exists only there); the lossy candidates' test sees the complete lossy planes.  Values and
 *   widths are bitwise those of spd_search with the same parameters at the same slots.
 *   Returns as spd_search (SPD_EINVAL also for the wrong method in either params or a bad tile
 *   shape).
 */
int spd_gated_plan(const spd_params *lossy, const spd_params *exh, int32_t n_dm, int32_t n_in,
                   int32_t n_out, int32_t tile_rows, int32_t tile_len, int64_t *workspace_bytes);

int spd_search_gated(const spd_params *lossy, const spd_params *exh, const float *x, int64_t ld,
                     int32_t n_dm, int32_t n_in, int32_t n_out, int64_t t0, const float *mean,
                     const float *sigma, const uint8_t *tile_flag, int32_t tile_rows,
                     int32_t tile_len, float *snr, uint16_t *width, float *exh_snr,
                     uint16_t *exh_width, spd_candidate *cand, int64_t cand_cap,
                     int64_t *cand_count, void *workspace, int64_t workspace_bytes,
                     void *hip_stream);

/*
 * spd_search_noalloc: spd_search without a workspace argument, for callers that cannot allocate
 *   device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 *   allocation).  The workspace is a fixed array inside the library, SPD_NOALLOC_SCRATCH_BYTES
 *   per GPU, allocated with the library's code on each GPU it runs on and held until the
 *   process ends.  Arguments, outputs and results are those of spd_search (bitwise: the same
 *   kernels run); the call allocates and frees nothing.
 *   Limit: searches whose spd_plan_info.workspace_bytes exceeds SPD_NOALLOC_SCRATCH_BYTES return
 *   SPD_EWORKSPACE with nothing enqueued (use spd_search with a workspace of your own).
 *   Sharing: every call on one GPU uses that GPU's one array, so calls that overlap in time on
 *   one GPU (other streams, other threads) race on it; serialise them.  A call may follow the
 *   previous one on the same stream at once: nothing in the array needs clearing.
 *   The first call on a device resolves the array's device address (SPD_EHIP if that fails).
 */
#define SPD_NOALLOC_SCRATCH_BYTES (64 << 20)

int spd_search_noalloc(const spd_params *params, const float *x, int64_t ld, int32_t n_dm,
                       int32_t n_in, int32_t n_out, int64_t t0, const float *mean,
                       const float *sigma, float *snr, uint16_t *width, spd_candidate *cand,
                       int64_t cand_cap, int64_t *cand_count, void *hip_stream);

/* Human-readable text for a status code (static storage; includes the last HIP error text for
 * SPD_EHIP on this thread). */
const char *spd_error_string(int status);

/* SPD_ABI_VERSION of the loaded library. */
int spd_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPD_H */
