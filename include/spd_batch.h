/*
 * spd_batch.h -- many beams in one fused launch per cascade step (C ABI, gfx950).
 *
 * A batch is a set of beams (blocks of dedispersed DM rows, each with its own number of rows and
 * samples) searched with the same BoxDIT or IGRID parameters (Sections 3.1, 3.2 of Adamek &
 * Armour, arXiv:1910.08324).  Every cascade step of the search runs as ONE kernel launch over all
 * beams: a persistent grid walks the (beam, DM row, tile) work items of the whole batch; each
 * pass of the peak finder is likewise one launch over the waves of every beam.  Every beam's
 * planes and candidates are bitwise identical to those of spd_search on that beam alone with the
 * same parameters.
 *
 * Use:
 *   1. spd_batch_plan: workspace and descriptor-table sizes.
 *   2. spd_batch_table: the library writes the batch's descriptor table into a HOST buffer;
 *      the caller copies those bytes to device memory (the library never copies or allocates).
 *      The table depends on the beams' pointers (inputs, planes, candidate buffers) and on the
 *      workspace address, so it is made again when any of them changes.
 *   3. spd_batch_search (asynchronous on the stream), as often as wanted.
 * The exhaustive method is not batched (SPD_EINVAL): it is bound by arithmetic, not by launches.
 */
#ifndef SPD_BATCH_H
#define SPD_BATCH_H

#include <stdint.h>

#include "spd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One beam of a batch: the arguments of spd_search for it (device pointers). */
typedef struct {
    const float *x;          /* [n_dm][ld], ld >= n_in                                    */
    int64_t ld;
    int32_t n_dm, n_in, n_out;
    int32_t reserved;
    int64_t t0;              /* multiple of 2^K, as for spd_search                           */
    const float *mean;       /* [n_dm]                                                      */
    const float *sigma;      /* [n_dm], > 0                                                 */
    float *snr;              /* planes (SPD_WRITE_PLANES), else ignored (planes go to the    */
    uint16_t *width;         /*   workspace)                                               */
    spd_candidate *cand;     /* SPD_WRITE_CANDIDATES: as for spd_search                      */
    int64_t cand_cap;
    int64_t *cand_count;
} spd_beam;

/*
 * spd_batch_plan: HOST outputs *workspace_bytes (device workspace, 256-byte aligned) and
 * *table_bytes (descriptor table) for n_beams beams (HOST array).  Returns SPD_EINVAL for the
 * exhaustive method, n_beams < 1, or a beam spd_plan would reject.
 */
int spd_batch_plan(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                   int64_t *workspace_bytes, int64_t *table_bytes);

/*
 * spd_batch_table: write the descriptor table for this batch and this workspace (a device
 * address, not dereferenced here) into the HOST buffer `table` (table_bytes from
 * spd_batch_plan).  Copy it to device memory (16-byte aligned) for spd_batch_search.
 */
int spd_batch_table(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                    void *workspace, void *table, int64_t table_bytes);

/*
 * spd_batch_search: search every beam.  table_dev is the device copy of spd_batch_table's
 * output for the same params, beams and workspace.  grid: work-groups of the persistent
 * cascade launches (each loops over work items), or 0 for one work-group per item.
 * Returns SPD_OK once everything is enqueued, SPD_EINVAL / SPD_EALIGN / SPD_EWORKSPACE for bad
 * arguments (nothing enqueued), SPD_EHIP for a failed launch.
 */
int spd_batch_search(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                     const void *table_dev, void *workspace, int64_t workspace_bytes,
                     int32_t grid, void *hip_stream);

/*
 * spd_copy_rows: dst[r][c] = src[r][c] for r < n_rows, c < n_cols.  dst and src are DEVICE float
 * arrays with row strides ld_dst, ld_src >= n_cols (in floats); the two must not overlap.  A
 * streaming search appends each arriving block of a beam after the samples it keeps on the
 * device with this copy (16-byte vector accesses when both sides allow them).  n_cols == 0 or
 * n_rows == 0 enqueues nothing.  Asynchronous on the stream; SPD_EINVAL for negative sizes, a
 * stride below n_cols or a NULL pointer with work to do, SPD_EHIP for a failed launch.
 */
int spd_copy_rows(float *dst, int64_t ld_dst, const float *src, int64_t ld_src, int32_t n_rows,
                  int32_t n_cols, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SPD_BATCH_H */
