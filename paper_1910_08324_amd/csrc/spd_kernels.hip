// Boxcar single-pulse search kernels for gfx950 (CDNA4, wave64).
//
// step_kernel        BoxDIT and IGRID: one launch per step of up to six separation levels.
//                    A work-group takes one tile of a DM row into LDS, forms the decimated
//                    levels on chip and evaluates every level's width set; only the planes and
//                    the last level (1/64 of the input) go back to HBM.
// exh_kernel         exhaustive search (every width 1..L_end): one wave per 256 output slots,
//                    4 consecutive starts per lane, the input window streamed through an LDS ring.
// peak_* kernels     thresholded 3x3 peak finding over the per-level planes, with output in
//                    (level, dm, start) order: count -> scan -> scatter.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "spd_internal.h"

namespace spd {

#define SPD_NEG_INF (-__builtin_huge_valf())

// Work-group barrier that orders LDS only: global loads and stores stay in flight across it
// (a full __syncthreads() also waits for every outstanding global access of the wave).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ----------------------------------------------------------------------------------------
// 1/sqrt(L) table of the exhaustive search.  Computed in FP64 and rounded once to FP32, so
// every kernel scales a boxcar sum by the correctly rounded 1/sqrt(L) (white-noise scaling,
// Section 2.1).  The cascade kernel builds its own small table in LDS the same way.
// ----------------------------------------------------------------------------------------
// rho_d(L) of a measured standard-deviation table (Section 4.6): linear in log2 L between the
// values at adjacent powers of two, held at the last level above it.
__device__ __forceinline__ double rho_of_width(const float *rho_row, int n_rho, double L) {
    const double a = log2(L);
    int k = (int)floor(a + 1e-12);
    if (k >= n_rho - 1) return (double)rho_row[n_rho - 1];
    if (k < 0) k = 0;
    const double f = a - k;
    return (1.0 - f) * (double)rho_row[k] + f * (double)rho_row[k + 1];
}

__global__ void scales_kernel(const ScaleArgs A) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int d = blockIdx.y;
    if (t >= A.n) return;
    if (!A.rho) {
        A.scale[t] = (float)(1.0 / sqrt((double)(t + 1)));
        return;
    }
    const double L = (double)(t + 1);
    const double r = rho_of_width(A.rho + (int64_t)d * A.ld_rho, A.n_rho, L);
    A.scale[(int64_t)d * A.row_ld + t] = (float)(1.0 / (sqrt(L) * r));
}

__global__ void evalmask_kernel(const MaskArgs A) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.n_words) A.evalmask[t] = A.bits[t];
}

// ----------------------------------------------------------------------------------------
// BoxDIT / IGRID cascade: one launch per step of up to kStepMaxLevels levels.
//
// Work-group = (DM row d, tile t) of NTH threads (256; 128 for short IG(1) tiles).  The tile
// covers T units of the step's input series (the normalised samples in the first step, the
// decimated series y_{k0} afterwards) plus the halo its widest boxcars reach.  The whole tile
// lives in LDS:
//   1. load the window (coalesced float4), normalising z = (x - mu) / sigma in the first step;
//   2. form the decimated levels in place, one pass and one barrier per level;
//   3. evaluate every level's width set at every slot of the tile, 4 consecutive slots per
//      thread from a register window, writing the SNR/width planes (BoxDIT adds the carried
//      prefix and hands each level's longest boxcar on as the next level's prefix);
//   4. hand the last formed level (and its prefixes) to the next step through HBM.
// Slots whose SNR is above the threshold and not below its time neighbours are recorded as
// pre-candidates for the peak finder (a superset of the final candidates).
//
// The width sets of the paper's configurations are compiled in (FAM selects one): the unit
// counts of a level are then constants, so the bank is straight-line code with 4 VALU
// operations per (slot, width) plus one add per (slot, unit).  Other width sets, and groups
// near the end of the data where some widths do not fit, take the generic path.
// ----------------------------------------------------------------------------------------

// unit-count bitmask (bit U-1) of IGRID IG(d) with P layers: level 0 and level >= 1
__host__ __device__ constexpr uint64_t ig_mask_l0(int P, int d) {
    uint64_t m = 0;
    for (int W = 1; W <= P; W <<= 1) {
        const int inc = (W >> d) > 1 ? (W >> d) : 1;
        for (int q = 0; q < (1 << d); ++q)
            if (W + q * inc < 2 * W) m |= 1ull << (W + q * inc - 1);
    }
    return m;
}
__host__ __device__ constexpr uint64_t ig_mask_lk(int P, int d) {
    uint64_t m = 0;
    for (int q = 0; q < (1 << d); ++q) m |= 1ull << (P + q * (P >> d) - 1);
    return m;
}
__host__ __device__ constexpr uint64_t run_mask(int L) { return L >= 64 ? ~0ull : ((1ull << L) - 1); }

// Compiled-in width patterns of each family: (UMAX, MASK) for pattern 1 and pattern 2, and the
// waves per SIMD the kernel is compiled for (register budget: 8 waves leave 64 VGPRs and 96
// SGPRs per lane; IG(3)'s 30-unit window needs a few more VGPRs than that).
template <int FAM> struct Fam;
template <> struct Fam<0> { static constexpr int U1 = 1, U2 = 1, WAVES = 7;
                            static constexpr uint64_t M1 = 1, M2 = 1; };
template <> struct Fam<1> { static constexpr int U1 = 6, U2 = 6, WAVES = 8;
                            static constexpr uint64_t M1 = ig_mask_l0(4, 1), M2 = ig_mask_lk(4, 1); };
template <> struct Fam<2> { static constexpr int U1 = 14, U2 = 14, WAVES = 8;
                            static constexpr uint64_t M1 = ig_mask_l0(8, 2), M2 = ig_mask_lk(8, 2); };
template <> struct Fam<3> { static constexpr int U1 = 30, U2 = 30, WAVES = 7;
                            static constexpr uint64_t M1 = ig_mask_l0(16, 3), M2 = ig_mask_lk(16, 3); };
template <> struct Fam<4> { static constexpr int U1 = 8, U2 = 8, WAVES = 8;
                            static constexpr uint64_t M1 = run_mask(8), M2 = run_mask(8); };
template <> struct Fam<5> { static constexpr int U1 = 16, U2 = 16, WAVES = 8;
                            static constexpr uint64_t M1 = run_mask(16), M2 = run_mask(16); };
template <> struct Fam<6> { static constexpr int U1 = 32, U2 = 32, WAVES = 8;
                            static constexpr uint64_t M1 = run_mask(32), M2 = run_mask(32); };
template <> struct Fam<7> { static constexpr int U1 = 1, U2 = 1, WAVES = 8;
                            static constexpr uint64_t M1 = 1, M2 = 1; };

// How much of a group's LDS window is read ahead, before the previous batch's barrier (PRE4
// float4 of the NW the banks use; the rest is read when the bank starts), and the waves per
// SIMD the launch is compiled for.  Reading a little ahead lets each bank start on data already
// in registers without costing occupancy; reading the whole window ahead costs registers, hence
// waves, and was slower for most sets.  Measured on the 4096 x 262144 beam (dominant launch,
// planes / candidates only, against no read-ahead): IG(1) 3.44 -> 3.19 / 3.29 -> 3.22 ms,
// IG(2) 5.24 -> 4.48 / 5.13 -> 4.27, IG(3) 8.59 -> 7.70 / 8.45 -> 7.60, BD-8 4.73 -> 4.33 /
// 4.48 -> 3.62, BD-16 6.56 -> 5.96 / 6.24 -> 5.32, BD-32 9.70 -> 9.44 / 9.29 -> 8.45.
template <int FAM, bool W> struct StepShape {
    static constexpr int NW = (FAM >= 1 && FAM <= 7) ? (kGroup + Fam<FAM>::U1 - 1 + 3) / 4 : 1;
    static constexpr int PRE4 = FAM == 1 ? (W ? 1 : 3) : FAM == 2 ? 2 : FAM == 3 ? 3 : FAM == 4 ? 2
                              : FAM == 5 ? 2 : FAM == 6 ? 4 : 0;
    static constexpr int WAVES = FAM == 6 ? 7 : Fam<FAM>::WAVES;
};


// All widths of the group fit: straight-line evaluation of a compiled-in width pattern.
// X enters holding the carried prefixes and leaves holding the sum over UMAX units.
// W: bu receives the unit count of the best width (0 if none); without W only the maximum is
// kept (the same value: the largest of the same products).
template <int NW>
__device__ __forceinline__ void window_load(const float *y, float w[4 * NW]) {
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const float4 v = *reinterpret_cast<const float4 *>(y + 4 * q);
        w[4 * q + 0] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
    }
}

// the same on a window already in registers, split in two arrays: wa holds its first 4 P4 units
// (m0 .. m0 + 4 P4 - 1 of the level), wb the rest
template <int UMAX, uint64_t MASK, bool W, int P4>
__device__ __forceinline__ void bank_fixed_split(const float *wa, const float *wb, const float *rt,
                                                 float X[kGroup], float best[kGroup], int bu[kGroup]) {
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
#pragma unroll
        for (int q = 0; q < kGroup; ++q) X[q] += (q + u < 4 * P4) ? wa[q + u] : wb[q + u - 4 * P4];
        if (((MASK >> u) & 1ull) != 0) {        // folded after unrolling
            const float r = rt[u];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const float v = X[q] * r;
                if (W) {
                    const bool gt = v > best[q];
                    best[q] = gt ? v : best[q];
                    bu[q] = gt ? (u + 1) : bu[q];
                } else {
                    best[q] = fmaxf(best[q], v);
                }
            }
        }
    }
}

template <int UMAX, uint64_t MASK, bool W>
__device__ __forceinline__ void bank_fixed(const float *y, const float *rt, float X[kGroup],
                                           float best[kGroup], int bu[kGroup]) {
    constexpr int NW = (kGroup + UMAX - 1 + 3) / 4;
    float w[4 * NW];
    window_load<NW>(y, w);
    bank_fixed_split<UMAX, MASK, W, NW>(w, w, rt, X, best, bu);
}

// Any width set, with the valid-only check per slot.  Xc receives the sum over `ufull` units
// (the carry handed to the next BoxDIT level).  W as for bank_fixed.
template <bool W>
__device__ __forceinline__ void bank_generic(const float *y, const float *rt, int umax,
                                             uint64_t emask, int ufull, int k, int base,
                                             const int64_t room[kGroup], float X[kGroup],
                                             float Xc[kGroup], float best[kGroup],
                                             int bu[kGroup]) {
    float4 wa = *reinterpret_cast<const float4 *>(y);
    for (int u4 = 0; u4 < umax; u4 += 4) {
        const float4 wb = *reinterpret_cast<const float4 *>(y + u4 + 4);
        const float w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int u = u4 + t;
            if (u >= umax) break;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) X[q] += w[q + t];
            if ((emask >> u) & 1ull) {
                const float r = rt[u];
                const int64_t Lw = (int64_t)base + ((int64_t)(u + 1) << k);
#pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    float v = X[q] * r;
                    if (Lw > room[q]) v = SPD_NEG_INF;
                    if (W) {
                        const bool gt = v > best[q];
                        best[q] = gt ? v : best[q];
                        bu[q] = gt ? (u + 1) : bu[q];
                    } else {
                        best[q] = fmaxf(best[q], v);
                    }
                }
            }
            if (u + 1 == ufull) {
#pragma unroll
                for (int q = 0; q < kGroup; ++q) Xc[q] = X[q];
            }
        }
        wa = wb;
    }
}

// Where a tile finds its beam's buffers and sizes: in the launch arguments (one beam per
// launch) or in a table in device memory (many beams per launch).
struct ArgGeom {
    const StepArgs &A;
    __device__ const float *in() const { return A.in; }
    __device__ const float *cin() const { return A.cin; }
    __device__ float *out() const { return A.out; }
    __device__ float *cout() const { return A.cout; }
    __device__ const float *mean() const { return A.mean; }
    __device__ const float *sigma() const { return A.sigma; }
    __device__ float *Y() const { return A.Y; }
    __device__ uint16_t *W() const { return A.W; }
    __device__ uint32_t *slab_cnt() const { return A.slab_cnt; }
    __device__ uint32_t *slab_ent() const { return A.slab_ent; }
    __device__ int64_t ld_in() const { return A.ld_in; }
    __device__ int64_t ld_cin() const { return A.ld_cin; }
    __device__ int64_t ld_out() const { return A.ld_out; }
    __device__ int n_in() const { return A.n_in; }
    __device__ int in_len() const { return A.in_len; }
    __device__ int n_tiles() const { return A.n_tiles; }
    __device__ int vec_ok() const { return A.vec_ok; }
    __device__ int64_t plane_off(int j) const { return A.lv[j].plane_off; }
    __device__ int64_t pitch(int j) const { return A.lv[j].pitch; }
    __device__ int64_t slab_base(int j) const { return A.lv[j].slab_base; }
    __device__ int slots(int j) const { return A.lv[j].slots; }
    __device__ RecStep *rec() const { return A.rec; }
    __device__ uint32_t *amask() const { return A.amask; }
    __device__ int64_t mask_off(int j) const { return A.lv[j].mask_off; }
    __device__ int64_t cnt_off(int j) const { return A.lv[j].cnt_off; }
};

// The table is read-only during a launch and every lane of a work-group reads the same entry,
// so it is addressed in the constant address space: its fields load as scalar (SMEM) reads.
typedef __attribute__((address_space(4))) const BeamView *ConstBeamPtr;
typedef __attribute__((address_space(4))) const int64_t *ConstI64Ptr;

struct TabGeom {
    ConstBeamPtr V;
    __device__ const float *in() const { return V->in; }
    __device__ const float *cin() const { return V->cin; }
    __device__ float *out() const { return V->out; }
    __device__ float *cout() const { return V->cout; }
    __device__ const float *mean() const { return V->mean; }
    __device__ const float *sigma() const { return V->sigma; }
    __device__ float *Y() const { return V->Y; }
    __device__ uint16_t *W() const { return V->W; }
    __device__ uint32_t *slab_cnt() const { return V->slab_cnt; }
    __device__ uint32_t *slab_ent() const { return V->slab_ent; }
    __device__ int64_t ld_in() const { return V->ld_in; }
    __device__ int64_t ld_cin() const { return V->ld_cin; }
    __device__ int64_t ld_out() const { return V->ld_out; }
    __device__ int n_in() const { return V->n_in; }
    __device__ int in_len() const { return V->in_len; }
    __device__ int n_tiles() const { return V->n_tiles; }
    __device__ int vec_ok() const { return V->vec_ok; }
    __device__ int64_t plane_off(int j) const { return V->plane_off[j]; }
    __device__ int64_t pitch(int j) const { return V->pitch[j]; }
    __device__ int64_t slab_base(int j) const { return V->slab_base[j]; }
    __device__ int slots(int j) const { return V->slots[j]; }
    __device__ RecStep *rec() const { return V->rec; }
    __device__ uint32_t *amask() const { return V->amask; }
    __device__ int64_t mask_off(int j) const { return V->mask_off[j]; }
    __device__ int64_t cnt_off(int j) const { return V->cnt_off[j]; }
};

// The step's record for the peak finder (candidates only): pointers, sizes and level constants,
// exactly those the tiles of this launch use.  Written by one work-group.
template <int NTH, class G>
__device__ __forceinline__ void write_rec(const StepArgs &A, const G &V, RecStep *R) {
    const int tid = threadIdx.x;
    for (int i = tid; i < A.J * kMaxLevelWidths; i += NTH) {
        const int j = i / kMaxLevelWidths, u = i - j * kMaxLevelWidths;
        R->lv[j].rt[u] = A.rtab[j][u];
    }
    if (tid < A.J) {
        const StepLevel &L = A.lv[tid];
        RecLevel &r = R->lv[tid];
        r.k = L.k;
        r.cshift = L.cshift;
        r.umax = L.umax;
        r.ufull = L.ufull;
        r.base = L.base;
        r.slots = V.slots(tid);
        r.evalmask = L.evalmask;
    }
    if (tid == 0) {
        R->in = V.in();
        R->cin = V.cin();
        R->mean = V.mean();
        R->sigma = V.sigma();
        R->rho = A.rho;
        R->ld_in = V.ld_in();
        R->ld_cin = V.ld_cin();
        R->ld_rho = A.ld_rho;
        R->n_rho = A.n_rho;
        R->in_len = V.in_len();
        R->n_in = V.n_in();
        R->normalise = A.normalise;
        R->carry = A.carry;
        R->J = A.J;
    }
}

// One tile (DM row d, tile `tile`) of a cascade launch.  A holds what every beam of the launch
// shares (levels, width patterns, tile length); G the beam's buffers and sizes.  W: the planes
// are stored (A.write_planes), so the banks also track the best width; candidates-only
// launches keep the maxima only.
template <bool FIRST, int FAM, bool RHO, int NTH, bool W, class G>
__device__ __forceinline__ void step_tile(const StepArgs &A, const G &V, const int d,
                                          const int tile, float *lds, uint32_t *st_cnt) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int T = A.T;
    if (RHO) {
        // this row's 1/sigma(L) relative to 1/(sqrt(L) sigma): scale[j][u-1] = rtab[j][u-1] / rho(L)
        const float *rr = A.rho + (int64_t)d * A.ld_rho;
        float *sc = lds + A.lds_sc;
        for (int i = tid; i < A.J * kMaxLevelWidths; i += NTH) {
            const int j = i / kMaxLevelWidths, u = i - j * kMaxLevelWidths + 1;
            if (u <= A.lv[j].umax) {
                const double L = (double)A.lv[j].base + ldexp((double)u, A.lv[j].k);
                sc[i] = (float)((double)A.rtab[j][u - 1] / rho_of_width(rr, A.n_rho, L));
            }
        }
    }
    // carried prefixes: BoxDIT families always, IGRID families never (known at compile time, so
    // their code and branches vanish), the generic kernel as the launch says
    constexpr int kCarry = (FAM >= 4 && FAM <= 6) ? 1 : (FAM == 0 ? -1 : 0);
    const bool carry = kCarry < 0 ? (A.carry != 0) : (kCarry == 1);
    const int64_t u0 = (int64_t)tile * T;
    if (tid < kStepMaxLevels) st_cnt[tid] = 0;
    if (d == 0 && tile == 0 && V.rec()) write_rec<NTH>(A, V, V.rec());

    // ---- 1. window of the input series (normalised in the first step) and carried prefixes
    {
        const float *inr = V.in() + (int64_t)d * V.ld_in();
        float mu = 0.0f, inv = 1.0f;
        if (FIRST) {
            mu = V.mean()[d];
            inv = 1.0f / V.sigma()[d];
        }
        const int N0 = A.lv[0].n_units;
        float *y0 = lds + A.lv[0].lds_y;
        const int64_t len = V.in_len();
        // kLoadBatch float4 loads per thread are issued before any of them is used, so a tile's
        // window costs about one memory round trip rather than one per float4
        // (unconditional loads: lanes past the data read the row's last whole float4 instead,
        // and use the element-wise path below)
        constexpr int kLoadBatch = 8;
        const bool vec = V.vec_ok() && len >= 4;
        // the last float4 a lane may read: inside the data and inside this tile's window (lanes
        // past the window re-read it, served by the cache, instead of fetching the next tile's)
        const int64_t rmax = vec ? min((len - 4) & ~(int64_t)3, u0 + ((N0 - 4) & ~3)) : 0;
        for (int i0 = tid * 4; i0 < N0; i0 += NTH * 4 * kLoadBatch) {
            float4 v[kLoadBatch];
            if (vec) {
#pragma unroll
                for (int b = 0; b < kLoadBatch; ++b) {
                    const int64_t r = u0 + i0 + b * NTH * 4;
                    v[b] = *reinterpret_cast<const float4 *>(inr + (r < rmax ? r : rmax));
                }
            }
#pragma unroll
            for (int b = 0; b < kLoadBatch; ++b) {
                const int i = i0 + b * NTH * 4;
                if (i >= N0) continue;
                const int64_t r = u0 + i;
                float4 w;
                if (vec && r + 3 < len) {
                    w = v[b];
                    if (FIRST) {
                        w.x = (w.x - mu) * inv;
                        w.y = (w.y - mu) * inv;
                        w.z = (w.z - mu) * inv;
                        w.w = (w.w - mu) * inv;
                    }
                } else {
                    float e[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        e[q] = 0.0f;
                        if (r + q < len) e[q] = FIRST ? (inr[r + q] - mu) * inv : inr[r + q];
                    }
                    w = make_float4(e[0], e[1], e[2], e[3]);
                }
                *reinterpret_cast<float4 *>(y0 + i) = w;
            }
        }
        if (!FIRST && carry && V.cin()) {
            const float *cr = V.cin() + (int64_t)d * V.ld_cin();
            float *c0 = lds + A.lv[0].lds_c;
            for (int i = tid; i < T; i += NTH) {
                const int64_t m = u0 + i;
                c0[i] = (m < V.slots(0)) ? cr[m] : 0.0f;
            }
        }
    }
    lds_barrier();

    // ---- 2+3. cascade fused with the width sets.  Level j is evaluated in batches of
    // NTH groups (the work-group size); each group also forms its two units of level j+1 (and, for BoxDIT,
    // its two carried prefixes) in registers.  After a barrier that ends the batch's reads they
    // are written in place: unit n of level j+1 goes to index n of the same buffer, below every
    // unit of level j a later batch still reads (and likewise for the carries).  The units of
    // level j+1 past the tile's slots (its halo) are formed after the last batch.
    const int jtop = A.has_out ? A.J : A.J - 1;
    float *ybuf = lds + A.lv[0].lds_y;
    float *cbuf = lds + A.lv[0].lds_c;
    for (int j = 0; j < A.J; ++j) {
        const bool form_next = j + 1 <= jtop;
        const int cs1 = form_next ? A.lv[j + 1].cshift : 0;
        const int n_next = form_next ? A.lv[j + 1].n_units : 0;
        const StepLevel &L = A.lv[j];
        const int Sj = T >> j;
        const int ms0 = tile * Sj;                         // absolute slot of tile slot 0
        const int ngroups = Sj / kGroup;
        const float *yj = ybuf;
        const float *cj = cbuf;
        const bool has_carry = carry && (j > 0 || V.cin() != nullptr);
        const bool to_lds = carry && (j + 1 < A.J);
        const bool to_glb = carry && (j + 1 == A.J) && A.has_out;
        float *cg = to_glb ? V.cout() + (int64_t)d * V.ld_out() + (int64_t)tile * (T >> A.J) : nullptr;
        const bool sync_batches = form_next || to_lds;   // a batch writes into the live buffers
        const int k = L.k;
        const int umax = L.umax;
        const int base = L.base;
        const int pat = L.pattern;
        const float *rt = RHO ? lds + A.lds_sc + j * kMaxLevelWidths : A.rtab[j];
        float *rowY = V.Y() + V.plane_off(j) + (int64_t)d * V.pitch(j);
        uint16_t *rowW = V.W() + V.plane_off(j) + (int64_t)d * V.pitch(j);
        // a group is "fast" when the widest boxcar of its last slot ends inside the data
        const int64_t fast_lim = (int64_t)V.n_in() - base - ((int64_t)umax << k);
        // the first kP4 float4 of a group's window are read from LDS before the previous batch's
        // barrier (they lie above every unit that batch writes), so their latency overlaps the
        // previous batch's stores and barrier
        constexpr int kNW = StepShape<FAM, W>::NW;
        constexpr int kP4 = StepShape<FAM, W>::PRE4;
        constexpr bool kPre = kP4 > 0;
        float win[4 * (kPre ? kP4 : 1)];
        float win2[4 * (kNW > kP4 ? kNW - kP4 : 1)];
        if (kPre && tid < ngroups) window_load<(kPre ? kP4 : 1)>(yj + tid * kGroup, win);
        for (int gb = 0; gb < ngroups; gb += NTH) {
            const int g = gb + tid;
            const int m0 = g * kGroup;
            const int ma = ms0 + m0;
            const bool act = (g < ngroups) && (ma < V.slots(j));
            float best[kGroup];
            int bu[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                best[q] = SPD_NEG_INF;
                bu[q] = 0;
            }
            // y_{j+1}[n] = y_j[2n + cshift] + y_j[2n + cshift + 1] for 2n + cshift = m0, m0 + 2
            const int n0 = (m0 - cs1) >> 1;
            float nu0 = 0.0f, nu1 = 0.0f;
            if (form_next && g < ngroups) {
                if (kPre) {
                    nu0 = win[0] + win[1];
                    nu1 = win[2] + win[3];
                } else {
                    const float4 w0 = *reinterpret_cast<const float4 *>(yj + m0);
                    nu0 = w0.x + w0.y;
                    nu1 = w0.z + w0.w;
                }
            }
            float Xc[kGroup];
            if (act) {
                float X[kGroup];
#pragma unroll
                for (int q = 0; q < kGroup; ++q) X[q] = has_carry ? cj[m0 + q] : 0.0f;
                const bool fast = ((int64_t)(ma + kGroup - 1) << k) <= fast_lim;
                if (FAM != 0 && fast && pat == 1) {
                    if constexpr (kPre) {
                        if constexpr (kNW > kP4) window_load<kNW - kP4>(yj + m0 + 4 * kP4, win2);
                        bank_fixed_split<Fam<FAM>::U1, Fam<FAM>::M1, W, kP4>(win, win2, rt, X, best, bu);
                    } else {
                        bank_fixed<Fam<FAM>::U1, Fam<FAM>::M1, W>(yj + m0, rt, X, best, bu);
                    }
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) Xc[q] = X[q];
                } else if (FAM != 0 && fast && pat == 2) {
                    if constexpr (kPre) {
                        if constexpr (kNW > kP4) window_load<kNW - kP4>(yj + m0 + 4 * kP4, win2);
                        bank_fixed_split<Fam<FAM>::U2, Fam<FAM>::M2, W, kP4>(win, win2, rt, X, best, bu);
                    } else {
                        bank_fixed<Fam<FAM>::U2, Fam<FAM>::M2, W>(yj + m0, rt, X, best, bu);
                    }
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) Xc[q] = X[q];
                } else {
                    int64_t room[kGroup];
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) room[q] = (int64_t)V.n_in() - ((int64_t)(ma + q) << k);
                    bank_generic<W>(yj + m0, rt, umax, L.evalmask, L.ufull, k, base, room, X, Xc, best, bu);
                }
                if (cg) {
                    // the last level's longest boxcar is the next step's carried prefix
                    cg[(m0 >> 1) + 0] = Xc[0];
                    cg[(m0 >> 1) + 1] = Xc[2];
                }
                int bw[kGroup];
#pragma unroll
                for (int q = 0; q < kGroup; ++q) bw[q] = bu[q] ? base + (bu[q] << k) : 0;
                if (!W) {
                    // candidates only: nothing stored; the peak finder forms what it reads again
                } else if (ma + kGroup <= V.slots(j)) {
                    *reinterpret_cast<float4 *>(rowY + ma) = make_float4(best[0], best[1], best[2], best[3]);
                    *reinterpret_cast<uint2 *>(rowW + ma) =
                        make_uint2((uint32_t)bw[0] | ((uint32_t)bw[1] << 16),
                                   (uint32_t)bw[2] | ((uint32_t)bw[3] << 16));
                } else {
#pragma unroll
                    for (int q = 0; q < kGroup; ++q)
                        if (ma + q < V.slots(j)) {
                            rowY[ma + q] = best[q];
                            rowW[ma + q] = (uint16_t)bw[q];
                        }
                }
            }
            // the window of this thread's group in the next batch
            if (kPre && g + NTH < ngroups) window_load<(kPre ? kP4 : 1)>(yj + (g + NTH) * kGroup, win);
            if (A.want_cand) {
                const float gmax = fmaxf(fmaxf(best[0], best[1]), fmaxf(best[2], best[3]));
                if (__ballot(gmax > A.threshold)) {
                    if (V.amask()) {
                        // candidates only: one bit per group of kGroup slots, set where any of
                        // them is above the threshold (the bits start cleared): the wave's
                        // ballot is its 64 groups, two words of the slab
                        const uint64_t gbits = __ballot(act && gmax > A.threshold);
                        const int word = (gb + 64 * (tid >> 6)) >> 5;
                        if (lane == 0) {
                            uint32_t *mw = V.amask() + V.mask_off(j) +
                                           ((int64_t)d * V.n_tiles() + tile) * L.mask_wps + word;
                            if ((uint32_t)gbits && word < L.mask_wps) mw[0] = (uint32_t)gbits;
                            if ((uint32_t)(gbits >> 32) && word + 1 < L.mask_wps)
                                mw[1] = (uint32_t)(gbits >> 32);
                        }
                    }
                    // time neighbours: inside the group, or the adjacent groups of the
                    // neighbouring lanes; unknown neighbours (wave edges) count as -inf
                    float left = __shfl_up(best[kGroup - 1], 1);
                    float right = __shfl_down(best[0], 1);
                    if (lane == 0) left = SPD_NEG_INF;
                    if (lane == 63) right = SPD_NEG_INF;
                    int nh = 0;
                    bool hit[kGroup];
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) {
                        const float l = q > 0 ? best[q - 1] : left;
                        const float rr = q + 1 < kGroup ? best[q + 1] : right;
                        hit[q] = act && (ma + q < V.slots(j)) && best[q] > A.threshold &&
                                 best[q] > l && best[q] >= rr;
                        nh += hit[q];
                    }
                    if (nh) {
                        const int64_t slab = V.slab_base(j) + (int64_t)d * V.n_tiles() + tile;
                        uint32_t pos = atomicAdd(&st_cnt[j], (uint32_t)nh);
#pragma unroll
                        for (int q = 0; q < kGroup; ++q) {
                            if (hit[q]) {
                                if (pos < (uint32_t)kSlabCap)
                                    V.slab_ent()[slab * kSlabCap + pos] = (uint32_t)(ma + q);
                                ++pos;
                            }
                        }
                    }
                }
            }
            if (sync_batches) {
                lds_barrier();                   // the batch's reads of level j are done
                if (form_next && g < ngroups) {
                    float *yn = ybuf;
                    if (n0 >= 0 && n0 < n_next) yn[n0] = nu0;
                    if (n0 + 1 >= 0 && n0 + 1 < n_next) yn[n0 + 1] = nu1;
                }
                if (to_lds && act) {
                    // this level's longest boxcar is the next level's carried prefix
                    cbuf[(m0 >> 1) + 0] = Xc[0];
                    cbuf[(m0 >> 1) + 1] = Xc[2];
                }
            }
        }
        if (form_next) {
            // halo units of level j+1: read at index >= S_j, written below it
            for (int n = max(0, (Sj - cs1) >> 1) + tid; n < n_next; n += NTH) {
                const float2 p = *reinterpret_cast<const float2 *>(yj + 2 * n + cs1);
                ybuf[n] = p.x + p.y;
            }
        }
        lds_barrier();                       // level j+1 is complete
    }

    // ---- 4. hand on the last formed level
    if (A.has_out) {
        const float *yJ = lds + A.lv[0].lds_y;
        float *o = V.out() + (int64_t)d * V.ld_out() + (int64_t)tile * (T >> A.J);
        for (int n = tid; n < (T >> A.J); n += NTH) o[n] = yJ[n];
    }
    if (A.want_cand) {
        lds_barrier();
        // the tile's counts of all its levels side by side (one short write per work-group)
        if (tid < A.J)
            V.slab_cnt()[V.cnt_off(tid) + ((int64_t)d * V.n_tiles() + tile) * A.J] = st_cnt[tid];
    }
}


// One launch for one beam: work-group = (DM row, tile) of NTH threads.
template <bool FIRST, int FAM, bool RHO, int NTH, bool W>
__global__ __launch_bounds__(NTH, (StepShape<FAM, W>::WAVES)) void step_kernel(const StepArgs A) {
    extern __shared__ float lds[];
    __shared__ uint32_t st_cnt[kStepMaxLevels];
    const int d = blockIdx.x / A.n_tiles;
    const int tile = blockIdx.x - d * A.n_tiles;
    if (d >= A.n_dm) return;
    step_tile<FIRST, FAM, RHO, NTH, W>(A, ArgGeom{A}, d, tile, lds, st_cnt);
}

// One launch for many beams (same levels and tile length, any sizes): a persistent grid walks
// the work items (beam, DM row, tile) in order; item i belongs to the beam b with
// item_base[b] <= i < item_base[b + 1].
template <bool FIRST, int FAM, bool W>
__global__ __launch_bounds__(kStepThreads, (StepShape<FAM, W>::WAVES)) void step_kernel_batch(const StepBatchArgs B) {
    extern __shared__ float lds[];
    __shared__ uint32_t st_cnt[kStepMaxLevels];
    const ConstBeamPtr beams = (ConstBeamPtr)B.beams;
    const ConstI64Ptr base = (ConstI64Ptr)B.item_base;
    int b = 0;
    for (int64_t item = blockIdx.x; item < B.n_items; item += gridDim.x) {
        while (b + 1 < B.n_beams && base[b + 1] <= item) ++b;
        const TabGeom V{beams + b};
        const int64_t local = item - base[b];
        const int d = (int)(local / V.n_tiles());
        const int tile = (int)(local - (int64_t)d * V.n_tiles());
        if (item != (int64_t)blockIdx.x) lds_barrier();   // the previous item is done with LDS
        step_tile<FIRST, FAM, false, kStepThreads, W>(B.s, V, d, tile, lds, st_cnt);
    }
}

// ----------------------------------------------------------------------------------------
// Exhaustive search kernel.
//
// Work item = (row d, 256 output slots starting at s0).  Lane l owns the 4 consecutive starts
// s0 + 4l + v.  Widths are visited in increasing order with one running sum per start, in
// groups of 16 or 64 widths: inside a group only the maximum is tracked (add, multiply, max per
// start and width); after the group the best group, and the running sum entering it, are
// kept.  The winning width inside the winning group is recovered at the end by replaying that
// group's steps with the same FP32 operations, so it is the smallest width attaining the
// maximum, exactly as a per-width argmax would give.
// The input window z[s0 .. s0 + 256 + L_end) streams through a 1024-float LDS ring, 512 new
// samples per block of 512 widths.  The ring's first 16 float4 are mirrored after its end, so a
// group reads its 17 consecutive float4 at immediate offsets from one base address.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ float load_z(const float *xr, int r, int n_in, float mu, float inv) {
    return r < n_in ? (xr[r] - mu) * inv : 0.0f;
}

// The width scales of a row are read-only during the launch and indexed by the group's widths,
// which every lane shares: addressed in the constant address space they load as scalar reads.
typedef __attribute__((address_space(4))) const float *ConstFloatPtr;

constexpr int kRing4 = 256;        // float4 slots of the ring (1024 samples)
constexpr int kGuard4 = 16;        // mirrored slots after the ring's end

__device__ __forceinline__ void ring_put(float4 *ring4, int i, float4 v) {   // 0 <= i < kRing4
    ring4[i] = v;
    if (i < kGuard4) ring4[kRing4 + i] = v;
}

// G widths L0 .. L0+G-1 at the lane's 4 starts: running sums X, group maxima gm.  The window
// z[s0 + 4 lane + L0 - 1 ..] is read from the LDS ring one float4 per 4 widths.
template <bool CHECK, bool DENSE, int G>
__device__ __forceinline__ void exh_group(const float4 *ring4, int jb4, int L0, ConstFloatPtr scale,
                                          const uint32_t *evalmask, int Lw, const int room[4],
                                          float X[4], float gm[4]) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f *win = reinterpret_cast<const v4f *>(ring4 + (jb4 & (kRing4 - 1)));
    v4f wa = win[0];
#pragma unroll 4
    for (int t = 0; t < G / 4; ++t) {
        const v4f wb = win[t + 1];
        const float w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
        const int L = L0 + 4 * t;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            const float r = scale[L - 1 + tt];
            bool on = true;
            if (!DENSE) on = (evalmask[(L - 1 + tt) >> 5] >> ((L - 1 + tt) & 31)) & 1u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                X[v] += w[v + tt];
                float snr = X[v] * r;
                if (CHECK) {
                    const bool ok = (L + tt <= Lw) && (L + tt <= room[v]);
                    snr = ok ? snr : SPD_NEG_INF;
                }
                if (!DENSE) snr = on ? snr : SPD_NEG_INF;
                gm[v] = fmaxf(gm[v], snr);
            }
        }
        wa = wb;
    }
}

// G: widths per max-only group.  L_end up to 4096 takes groups of 16 (a shorter argmax replay
// per start, which there costs as much as the width loop: 2x faster at L_end 256, 1.8x at 1024);
// larger L_end groups of 64 (less bookkeeping per width).
template <bool DENSE, bool MULTI, int G>
__global__ __launch_bounds__(64) void exh_kernel(const ExhArgs A) {
    __shared__ float4 ring4[kRing4 + kGuard4];

    // A wave takes `per` consecutive work items of a row (MULTI: several, when every width fits
    // one block of the ring, so each further item needs only 256 new samples, loaded while the
    // previous item computes).  Ring position 0 holds sample `base`.
    const int lane = threadIdx.x;
    const int per = MULTI ? A.segs_per_wave : 1;
    const int waves_per_row = (A.n_seg + per - 1) / per;
    const int d = blockIdx.x / waves_per_row;
    const int g0 = (blockIdx.x - d * waves_per_row) * per;
    if (d >= A.n_dm) return;
    const int g_end = min(g0 + per, A.n_seg);
    if (A.tile_flag) {
        // tile-gated: a wave's items lie in one tile (tile_len is a multiple of 1024 samples)
        const int64_t t = (int64_t)(d / A.tile_rows) * A.n_col_tiles + (g0 * kExhSlots) / A.tile_len;
        if (!A.tile_flag[t]) {
            if (A.want_cand && lane == 0)
                for (int g = g0; g < g_end; ++g) A.slab_cnt[(int64_t)d * A.n_seg + g] = 0;
            return;
        }
    }
    const int base = g0 * kExhSlots;
    const float *xr = A.x + (int64_t)d * A.ld;
    const float *srow = A.scale + (int64_t)d * A.scale_ld;     // this row's 1/sigma(L) factors
    const float mu = A.mean[d];
    const float inv = 1.0f / A.sigma[d];
    const int Lw = A.l_end;
    const int n_in = A.n_in;

    auto load4 = [&](int r) -> float4 {          // z[r .. r + 3], r a multiple of 4
        float4 v;
        if (A.vec_ok && r + 3 < n_in) {
            v = *reinterpret_cast<const float4 *>(xr + r);
            v.x = (v.x - mu) * inv;
            v.y = (v.y - mu) * inv;
            v.z = (v.z - mu) * inv;
            v.w = (v.w - mu) * inv;
        } else {
            v.x = load_z(xr, r + 0, n_in, mu, inv);
            v.y = load_z(xr, r + 1, n_in, mu, inv);
            v.z = load_z(xr, r + 2, n_in, mu, inv);
            v.w = load_z(xr, r + 3, n_in, mu, inv);
        }
        return v;
    };

#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = q * 256 + lane * 4;
        ring_put(ring4, j >> 2, load4(base + j));
    }
    int loaded_to = base + 1024;
    __syncthreads();

    const int nblk = (Lw + kExhBlock - 1) / kExhBlock;
    for (int g = g0; g < g_end; ++g) {
    const int s0 = g * kExhSlots;
    const int ro4 = (s0 - base) >> 2;              // ring offset (float4) of this item's window
    // the next item's window reaches 256 samples further: fetch them now, store after this item
    const bool fetch = MULTI && (g + 1 < g_end) && (s0 + kExhSlots + 768 > loaded_to);
    float4 nx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (fetch) nx = load4(loaded_to + lane * 4);

    float X[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float best[4] = {SPD_NEG_INF, SPD_NEG_INF, SPD_NEG_INF, SPD_NEG_INF};
    float bx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int bg[4] = {0, 0, 0, 0};
    int room[4];                                    // widest valid width per start
#pragma unroll
    for (int v = 0; v < 4; ++v) room[v] = n_in - (s0 + 4 * lane + v);

    for (int b = 0; b < nblk; ++b) {
        const bool refill = (b + 1 < nblk);
        float4 pf0, pf1;
        const int jn = b * kExhBlock + 1024;
        if (refill) {
            pf0 = load4(s0 + jn + lane * 4);
            pf1 = load4(s0 + jn + 256 + lane * 4);
        }
        for (int gi = 0; gi < kExhBlock / G; ++gi) {
            const int L0 = b * kExhBlock + gi * G + 1;
            if (L0 > Lw) break;
            // wave-uniform: every width of the group fits at every start of the work item
            const bool fast = (L0 + G - 1 <= Lw) &&
                              ((int64_t)s0 + kExhSlots - 1 + L0 + G - 1 <= n_in);
            float Xs[4], gm[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Xs[v] = X[v];
                gm[v] = SPD_NEG_INF;
            }
            const int jb4 = ro4 + lane + ((L0 - 1) >> 2);
            if (fast)
                exh_group<false, DENSE, G>(ring4, jb4, L0, (ConstFloatPtr)srow, A.evalmask, Lw, room, X, gm);
            else
                exh_group<true, DENSE, G>(ring4, jb4, L0, (ConstFloatPtr)srow, A.evalmask, Lw, room, X, gm);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (gm[v] > best[v]) {
                    best[v] = gm[v];
                    bg[v] = (L0 - 1) / G;
                    bx[v] = Xs[v];
                }
            }
        }
        if (refill) {
            __syncthreads();
            ring_put(ring4, ((jn >> 2) + lane) & (kRing4 - 1), pf0);
            ring_put(ring4, ((jn >> 2) + 64 + lane) & (kRing4 - 1), pf1);
            __syncthreads();
        }
    }

    // ---- recover the smallest width attaining the maximum inside the winning group.  With a
    // single block of widths the ring still holds the whole window (it was never refilled), so
    // the replay reads the same values from LDS; otherwise it reloads them.
    int bw[4] = {0, 0, 0, 0};
    const float *ring = reinterpret_cast<const float *>(ring4);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (best[v] == SPD_NEG_INF) continue;
        const int sv = s0 + 4 * lane + v;
        const int Lb = bg[v] * G + 1;
        float Xr = bx[v], bm = SPD_NEG_INF;
        for (int t = 0; t < G; ++t) {
            const int L = Lb + t;
            if (L > Lw) break;
            Xr += (nblk == 1) ? ring[(4 * ro4 + 4 * lane + v + L - 1) & (4 * kRing4 - 1)]
                              : load_z(xr, sv + L - 1, n_in, mu, inv);
            float snr = Xr * srow[L - 1];
            bool ok = L <= room[v];
            if (!DENSE) ok = ok && ((A.evalmask[(L - 1) >> 5] >> ((L - 1) & 31)) & 1u);
            if (ok && snr > bm) {
                bm = snr;
                bw[v] = L;
            }
        }
    }

    // ---- outputs
    const int m0 = s0 + 4 * lane;
    float *Yr = A.Y + (int64_t)d * A.pitch;
    uint16_t *Wr = A.W + (int64_t)d * A.pitch;
    if (m0 + 3 < A.n_out) {
        *reinterpret_cast<float4 *>(Yr + m0) = make_float4(best[0], best[1], best[2], best[3]);
        const uint32_t lo = (uint32_t)bw[0] | ((uint32_t)bw[1] << 16);
        const uint32_t hi = (uint32_t)bw[2] | ((uint32_t)bw[3] << 16);
        *reinterpret_cast<uint2 *>(Wr + m0) = make_uint2(lo, hi);
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (m0 + v < A.n_out) {
                Yr[m0 + v] = best[v];
                Wr[m0 + v] = (uint16_t)bw[v];
            }
        }
    }
    if (A.want_cand) {
        // pre-candidates: above the threshold and not below either time neighbour (neighbours
        // held by other work items are unknown and treated as -inf)
        float left = __shfl_up(best[3], 1);
        float right = __shfl_down(best[0], 1);
        if (lane == 0) left = SPD_NEG_INF;
        if (lane == 63) right = SPD_NEG_INF;
        bool hit[4];
        int mine = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float l = v > 0 ? best[v - 1] : left;
            const float r = v < 3 ? best[v + 1] : right;
            hit[v] = (m0 + v < A.n_out) && best[v] > A.threshold && best[v] > l && best[v] >= r;
            mine += hit[v];
        }
        const uint64_t any = __ballot(mine > 0);
        uint32_t total = 0;
        if (any) {
            int pre = mine;                              // inclusive prefix over lanes
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(pre, off);
                if (lane >= off) pre += t;
            }
            total = (uint32_t)__shfl(pre, 63);
            int pos = pre - mine;
            const int64_t slab = (int64_t)d * A.n_seg + g;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (hit[v]) {
                    if (pos < kExhSlabCap) A.slab_ent[slab * kExhSlabCap + pos] = (uint32_t)(m0 + v);
                    ++pos;
                }
            }
        }
        if (lane == 0) A.slab_cnt[(int64_t)d * A.n_seg + g] = total;
    }
    if (fetch) {
        ring_put(ring4, (((loaded_to - base) >> 2) + lane) & (kRing4 - 1), nx);
        loaded_to += 256;
    }
    __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------
// Peak finding (candidate selection).  A slot is a candidate iff its SNR is above the
// threshold and it passes the 3x3 neighbour test (strict against neighbours earlier in
// row-major order, non-strict against later ones).  The search kernels recorded, per
// (level, row, tile) slab, the slots above the threshold that are not below their time
// neighbours; a slab that overflowed is rescanned densely over its tile.  Three passes keep the
// output in (level, dm, start) order without a global sort: per-wave survivor counts (each
// slab's entries sorted in the wave), one scan, scatter.
// ----------------------------------------------------------------------------------------
// When only candidates are requested the lossy searches store no planes, and the peak finder
// forms each slot value it reads again from the step's record: the units of the level as
// pairwise sums of the step's input series (level by level, as the cascade forms them), the
// BoxDIT carried prefix through the levels below, and the level's widths in increasing order
// with the same FP32 operations as step_tile.  Value and width are therefore bitwise those the
// planes would hold; the work is small because only slots near pre-candidates are formed.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ float rec_in(const RecStep &R, const float *inr, float mu, float inv,
                                        int64_t r) {
    if (r >= R.in_len) return 0.0f;                   // the tile pads past the data with zeros
    return R.normalise ? (inr[r] - mu) * inv : inr[r];
}

// pairwise sum of the 2^J input units from a, in the cascade's order
template <int J>
__device__ __forceinline__ float rec_tree(const RecStep &R, const float *inr, float mu, float inv,
                                          int64_t a) {
    float v[1 << J];
#pragma unroll
    for (int i = 0; i < (1 << J); ++i) v[i] = rec_in(R, inr, mu, inv, a + i);
#pragma unroll
    for (int h = (1 << J); h > 1; h >>= 1) {
#pragma unroll
        for (int i = 0; i < h / 2; ++i) v[i] = v[2 * i] + v[2 * i + 1];
    }
    return v[0];
}

// unit n of level j of the step: y_j[n] = y_{j-1}[2n + cshift_j] + y_{j-1}[2n + cshift_j + 1]
__device__ __noinline__ float rec_unit(const RecStep &R, const float *inr, float mu, float inv,
                                       int j, int64_t n) {
    int64_t a = n;
    for (int i = j; i >= 1; --i) a = 2 * a + R.lv[i].cshift;
    switch (j) {
        case 0: return rec_in(R, inr, mu, inv, a);
        case 1: return rec_tree<1>(R, inr, mu, inv, a);
        case 2: return rec_tree<2>(R, inr, mu, inv, a);
        case 3: return rec_tree<3>(R, inr, mu, inv, a);
        case 4: return rec_tree<4>(R, inr, mu, inv, a);
        default: return rec_tree<5>(R, inr, mu, inv, a);
    }
}

// Y and W of slot m (absolute) of level j of the step, row d
__device__ __noinline__ float rec_slot(const RecStep &R, int d, int j, int64_t m, int *w_out) {
    const float *inr = R.in + (int64_t)d * R.ld_in;
    float mu = 0.0f, inv = 1.0f;
    if (R.normalise) {
        mu = R.mean[d];
        inv = 1.0f / R.sigma[d];
    }
    const RecLevel &L = R.lv[j];
    // carried prefix (BoxDIT): from the previous step's hand-off, then through levels 0..j-1,
    // each adding its ufull units at the slot that leads to m
    float X = 0.0f;
    if (R.carry && (j > 0 || R.cin != nullptr)) {
        const int64_t p0 = m << j;
        if (R.cin && p0 < R.lv[0].slots) X = R.cin[(int64_t)d * R.ld_cin + p0];
        for (int i = 0; i < j; ++i) {
            const int64_t p = m << (j - i);
            const int uf = R.lv[i].ufull;
            for (int u = 0; u < uf; ++u) X += rec_unit(R, inr, mu, inv, i, p + u);
        }
    }
    const float *rr = R.rho ? R.rho + (int64_t)d * R.ld_rho : nullptr;
    const int64_t room = (int64_t)R.n_in - (m << L.k);
    float best = SPD_NEG_INF;
    int bu = 0;
    for (int u = 0; u < L.umax; ++u) {
        X += rec_unit(R, inr, mu, inv, j, m + u);
        if ((L.evalmask >> u) & 1ull) {
            float r = L.rt[u];
            if (rr) {
                const double Lw = (double)L.base + ldexp((double)(u + 1), L.k);
                r = (float)((double)L.rt[u] / rho_of_width(rr, R.n_rho, Lw));
            }
            float v = X * r;
            if ((int64_t)L.base + ((int64_t)(u + 1) << L.k) > room) v = SPD_NEG_INF;
            if (v > best) {
                best = v;
                bu = u + 1;
            }
        }
    }
    *w_out = bu ? L.base + (bu << L.k) : 0;
    return best;
}

// Y of the slots m0, m0+1, m0+2 of level j in row d whose bit in `need` (bit i: slot m0+i) is
// set, into y[i]: each unit of the level is formed once and added, in order, to the running sum
// of every slot that covers it, so every slot's sum and SNR are those rec_slot forms.
__device__ __noinline__ void rec_slots3(const RecStep &R, int d, int j, int64_t m0, int need,
                                       float y[3]) {
    const float *inr = R.in + (int64_t)d * R.ld_in;
    float mu = 0.0f, inv = 1.0f;
    if (R.normalise) {
        mu = R.mean[d];
        inv = 1.0f / R.sigma[d];
    }
    const RecLevel &L = R.lv[j];
    float X[3] = {0.0f, 0.0f, 0.0f}, best[3];
    int64_t room[3];
    for (int i = 0; i < 3; ++i) {
        best[i] = SPD_NEG_INF;
        room[i] = 0;
        if (!((need >> i) & 1)) continue;                   // (m0 + i may be -1 then)
        room[i] = (int64_t)R.n_in - ((m0 + i) << L.k);
        if (R.carry && (j > 0 || R.cin != nullptr)) {
            const int64_t m = m0 + i, p0 = m << j;
            if (R.cin && p0 < R.lv[0].slots) X[i] = R.cin[(int64_t)d * R.ld_cin + p0];
            for (int l = 0; l < j; ++l) {
                const int64_t p = m << (j - l);
                const int uf = R.lv[l].ufull;
                for (int u = 0; u < uf; ++u) X[i] += rec_unit(R, inr, mu, inv, l, p + u);
            }
        }
    }
    const float *rr = R.rho ? R.rho + (int64_t)d * R.ld_rho : nullptr;
    const int first = (need & 1) ? 0 : (need & 2) ? 1 : 2;
    const int last = (need & 4) ? 2 : (need & 2) ? 1 : 0;
    for (int v = first; v < L.umax + last; ++v) {           // unit m0 + v
        const float yu = rec_unit(R, inr, mu, inv, j, m0 + v);
        for (int i = first; i <= last; ++i) {
            const int u = v - i;                            // width index of slot m0 + i
            if (!((need >> i) & 1) || u < 0 || u >= L.umax) continue;
            X[i] += yu;
            if ((L.evalmask >> u) & 1ull) {
                float r = L.rt[u];
                if (rr) {
                    const double Lw = (double)L.base + ldexp((double)(u + 1), L.k);
                    r = (float)((double)L.rt[u] / rho_of_width(rr, R.n_rho, Lw));
                }
                float val = X[i] * r;
                if ((int64_t)L.base + ((int64_t)(u + 1) << L.k) > room[i]) val = SPD_NEG_INF;
                if (val > best[i]) best[i] = val;
            }
        }
    }
    for (int i = 0; i < 3; ++i) y[i] = best[i];
}

// The helpers take the arguments either from the launch (one beam) or from a per-beam table in
// the constant address space (a batch); PA is the (qualified) PeakArgs type.
// SNR (and width, if w) of slot m of level k in row d: from the planes, or formed again.
template <class PA>
__device__ __forceinline__ float slot_value(PA &A, int k, int d, int m, int *w) {
    if (A.rec) {
        int wl;
        const float y = rec_slot(A.rec[A.level_step[k]], d, A.level_j[k], m, &wl);
        if (w) *w = wl;
        return y;
    }
    const int64_t i = A.level_off[k] + (int64_t)d * A.level_pitch[k] + m;
    if (w) *w = A.W[i];
    return A.Y[i];
}

// tile gating of the candidates (flag_mode): may slot m of level k in row d be a candidate, and
// does its value exist (mode 2: only inside flagged tiles)?
template <class PA>
__device__ __forceinline__ bool slot_kept(PA &A, int k, int d, int m) {
    if (A.flag_mode == 0) return true;
    const int64_t s = (int64_t)m << A.level_shift[k];
    const bool f = A.tile_flag[(int64_t)(d / A.tile_rows) * A.n_col_tiles + s / A.tile_len] != 0;
    return A.flag_mode == 2 ? f : !f;
}

// candidates only: may slot m of level k in row d be above the threshold?  (The bit of its
// group of kGroup slots: clear means every slot of the group is at or below the threshold.)
template <class PA>
__device__ __forceinline__ bool slot_above(PA &A, int k, int d, int m) {
    const int ts = A.tile_slots[k];
    const int t = m / ts, g = (m - t * ts) / kGroup;
    const uint32_t w = A.amask[A.mask_off[k] + ((int64_t)d * A.tiles_per_row[k] + t) * A.mask_wps[k] +
                               (g >> 5)];
    return (w >> (g & 31)) & 1u;
}

// The 3x3 test when the planes are not stored: a neighbour at or below the threshold cannot
// block a slot above it, so only neighbours whose group bit is set are formed again, with the
// slot itself if any is (y_known: its value is already y_in); the slots of one row are formed
// together.
// time_tested: m is a pre-candidate, so the cascade already compared it exactly with its time
// neighbours that lie in the same wave's 256 slots of the tile (only those across a wave or
// tile edge are unknown to it).
template <class PA>
__device__ __forceinline__ bool peak_test_rec(PA &A, int k, int d, int m, bool y_known = false,
                                              float y_in = 0.0f, bool time_tested = false) {
    const int slots = A.level_slots[k];
    const int ts = A.tile_slots[k];
    const int lm = m - (m / ts) * ts;                     // slot within its tile
    const bool left_known = time_tested && (lm & 255) != 0;
    const bool right_known = time_tested && ((lm + 1) & 255) != 0 && lm + 1 < ts;
    int need[3] = {0, 0, 0};
    bool any = false;
#pragma unroll
    for (int a = -1; a <= 1; ++a) {
        const int dn = d + a;
        if (dn < 0 || dn >= A.n_dm) continue;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            if (a == 0 && b == 0) continue;
            if (a == 0 && ((b < 0 && left_known) || (b > 0 && right_known))) continue;
            const int mn = m + b;
            if (mn < 0 || mn >= slots) continue;
            if (slot_above(A, k, dn, mn)) {
                need[a + 1] |= 1 << (b + 1);
                any = true;
            }
        }
    }
    if (!any) return true;
    const RecStep &R = A.rec[A.level_step[k]];
    const int j = A.level_j[k];
    float y = y_in;
    if (!y_known) need[1] |= 2;                 // the slot itself, formed with its row
    float v[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (need[a]) rec_slots3(R, d + a - 1, j, (int64_t)m - 1, need[a], v[a]);
    if (!y_known) y = v[1][1];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (!((need[a] >> b) & 1) || (a == 1 && b == 1)) continue;
            const bool earlier = (a < 1) || (a == 1 && b < 1);
            if (earlier ? !(y > v[a][b]) : !(y >= v[a][b])) return false;
        }
    return true;
}

template <class PA>
__device__ __forceinline__ bool peak_test(PA &A, int k, int d, int m, float y) {
    const int slots = A.level_slots[k];
#pragma unroll
    for (int a = -1; a <= 1; ++a) {
        const int dn = d + a;
        if (dn < 0 || dn >= A.n_dm) continue;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            if (a == 0 && b == 0) continue;
            const int mn = m + b;
            if (mn < 0 || mn >= slots) continue;
            if (A.flag_mode == 2 && !slot_kept(A, k, dn, mn)) continue;   // no value there
            const float yn = slot_value(A, k, dn, mn, nullptr);
            const bool earlier = (a < 0) || (a == 0 && b < 0);
            if (earlier ? !(y > yn) : !(y >= yn)) return false;
        }
    }
    return true;
}

struct SlabPos {
    int k, d, t, mlo, mhi;
};

template <class PA>
__device__ __forceinline__ SlabPos slab_decode(PA &A, int64_t s) {
    SlabPos p;
    int k = 0;
    while (k + 1 < A.n_levels && s >= A.slab_base[k + 1]) ++k;
    const int64_t r = s - A.slab_base[k];
    p.k = k;
    p.d = (int)(r / A.tiles_per_row[k]);
    p.t = (int)(r - (int64_t)p.d * A.tiles_per_row[k]);
    p.mlo = p.t * A.tile_slots[k];
    p.mhi = min(p.mlo + A.tile_slots[k], A.level_slots[k]);
    return p;
}

template <class PA>
__device__ __forceinline__ int64_t slab_cnt_index(PA &A, int64_t s) {
    int k = 0;
    while (k + 1 < A.n_levels && s >= A.slab_base[k + 1]) ++k;
    return A.cnt_off[k] + (s - A.slab_base[k]) * A.cnt_stride[k];
}

template <class PA>
__device__ __forceinline__ float plane_at(PA &A, int k, int d, int m) {
    return slot_value(A, k, d, m, nullptr);
}

__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t key, int lane) {
    // bitonic sort of one key per lane, ascending across the 64 lanes
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t other = (uint32_t)__shfl_xor((int)key, j);
            const bool asc = (lane & k) == 0;
            const bool low = (lane & j) == 0;
            key = (asc == low) ? min(key, other) : max(key, other);
        }
    }
    return key;
}

// count pass of wave w of a beam
template <class PA>
__device__ __forceinline__ void peak_count_wave(PA &A, int w, int lane) {
    const int64_t sbeg = (int64_t)w * A.slabs_per_wave;
    const int64_t send = min(sbeg + A.slabs_per_wave, A.n_slabs);
    int64_t total = 0;
    for (int64_t sb = sbeg; sb < send; sb += 64) {
        const int64_t s = sb + lane;
        const uint32_t c = (s < send) ? A.slab_cnt[slab_cnt_index(A, s)] : 0u;
        if (s < send && c == 0) A.surv[s] = 0;
        uint64_t nz = __ballot(c != 0);
        while (nz) {
            const int l = __ffsll((unsigned long long)nz) - 1;
            nz &= nz - 1;
            const int64_t ss = sb + l;
            const uint32_t cc = (uint32_t)__shfl((int)c, l);
            const SlabPos p = slab_decode(A, ss);
            uint32_t nsurv = 0;
            uint64_t msk = 0;
            if (cc <= (uint32_t)A.slab_cap) {
                uint32_t key = (lane < (int)cc) ? A.slab_ent[ss * A.slab_cap + lane] : 0xffffffffu;
                key = wave_sort_u32(key, lane);
                bool ok = false;
                if (lane < (int)cc) {
                    A.slab_ent[ss * A.slab_cap + lane] = key;
                    const int m = (int)key;
                    if (A.amask)
                        ok = slot_kept(A, p.k, p.d, m) &&
                             peak_test_rec(A, p.k, p.d, m, false, 0.0f, true);
                    else
                        ok = slot_kept(A, p.k, p.d, m) &&
                             peak_test(A, p.k, p.d, m, plane_at(A, p.k, p.d, m));
                }
                msk = __ballot(ok);
                nsurv = __popcll(msk);
            } else {
                for (int mb = p.mlo; mb < p.mhi; mb += 64) {
                    const int m = mb + lane;
                    bool ok = false;
                    if (m < p.mhi && slot_kept(A, p.k, p.d, m)) {
                        if (A.amask) {
                            if (slot_above(A, p.k, p.d, m)) {
                                const float y = plane_at(A, p.k, p.d, m);
                                ok = (y > A.threshold) && peak_test_rec(A, p.k, p.d, m, true, y);
                            }
                        } else {
                            const float y = plane_at(A, p.k, p.d, m);
                            ok = (y > A.threshold) && peak_test(A, p.k, p.d, m, y);
                        }
                    }
                    nsurv += __popcll(__ballot(ok));
                }
            }
            if (lane == 0) {
                A.surv[ss] = nsurv;
                A.mask[ss] = msk;
            }
            total += nsurv;
        }
    }
    if (lane == 0) A.wave_tot[w] = total;
}

__global__ __launch_bounds__(256) void peak_count_kernel(const PeakArgs A) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= A.n_waves) return;
    peak_count_wave(A, w, threadIdx.x & 63);
}

// exclusive scan of a beam's per-wave totals by one 1024-thread work-group
template <class PA>
__device__ __forceinline__ void peak_scan_block(PA &A, int64_t *part) {
    const int t = threadIdx.x;
    const int per = (A.n_waves + 1023) / 1024;
    // candidates already written before this list (read before the first barrier: the last
    // thread may overwrite the same count at the end)
    const int64_t base = A.base_count ? *A.base_count : 0;
    int64_t loc = 0;
    for (int i = 0; i < per; ++i) {
        const int w = t * per + i;
        if (w < A.n_waves) loc += A.wave_tot[w];
    }
    part[t] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = base + part[t] - loc;               // exclusive prefix
    for (int i = 0; i < per; ++i) {
        const int w = t * per + i;
        if (w < A.n_waves) {
            A.wave_off[w] = run;
            run += A.wave_tot[w];
        }
    }
    if (t == 1023) *A.cand_count = base + part[1023];
}

__global__ __launch_bounds__(1024) void peak_scan_kernel(const PeakArgs A) {
    __shared__ int64_t part[1024];
    peak_scan_block(A, part);
}

template <class PA>
__device__ __forceinline__ void put_cand(PA &A, int64_t idx, int k, int d, int m, float y, int w) {
    if (idx >= A.cand_cap) return;
    spd_candidate c;
    c.start = A.t0 + ((int64_t)m << A.level_shift[k]);
    c.dm = d;
    c.width = w;
    c.level = k;
    c.snr = y;
    A.cand[idx] = c;
}

// scatter pass of wave w of a beam
template <class PA>
__device__ __forceinline__ void peak_scatter_wave(PA &A, int w, int lane) {
    const int64_t sbeg = (int64_t)w * A.slabs_per_wave;
    const int64_t send = min(sbeg + A.slabs_per_wave, A.n_slabs);
    int64_t off = A.wave_off[w];
    for (int64_t sb = sbeg; sb < send; sb += 64) {
        const int64_t s = sb + lane;
        const uint32_t sv = (s < send) ? A.surv[s] : 0u;
        uint64_t nz = __ballot(sv != 0);
        while (nz) {
            const int l = __ffsll((unsigned long long)nz) - 1;
            nz &= nz - 1;
            const int64_t ss = sb + l;
            const uint32_t nsurv = (uint32_t)__shfl((int)sv, l);
            const uint32_t cc = A.slab_cnt[slab_cnt_index(A, ss)];
            const SlabPos p = slab_decode(A, ss);
            if (cc <= (uint32_t)A.slab_cap) {
                const uint64_t msk = A.mask[ss];
                if (lane < (int)cc && ((msk >> lane) & 1ull)) {
                    const int m = (int)A.slab_ent[ss * A.slab_cap + lane];
                    int w;
                    const float y = slot_value(A, p.k, p.d, m, &w);
                    put_cand(A, off + __popcll(msk & lanes_below(lane)), p.k, p.d, m, y, w);
                }
            } else {
                int64_t run = 0;
                for (int mb = p.mlo; mb < p.mhi; mb += 64) {
                    const int m = mb + lane;
                    bool ok = false;
                    float y = 0.0f;
                    int w = 0;
                    if (m < p.mhi && slot_kept(A, p.k, p.d, m)) {
                        if (A.amask) {
                            if (slot_above(A, p.k, p.d, m)) {
                                y = slot_value(A, p.k, p.d, m, &w);
                                ok = (y > A.threshold) && peak_test_rec(A, p.k, p.d, m, true, y);
                            }
                        } else {
                            y = slot_value(A, p.k, p.d, m, &w);
                            ok = (y > A.threshold) && peak_test(A, p.k, p.d, m, y);
                        }
                    }
                    const uint64_t b = __ballot(ok);
                    if (ok) put_cand(A, off + run + __popcll(b & lanes_below(lane)), p.k, p.d, m, y, w);
                    run += __popcll(b);
                }
            }
            off += nsurv;
        }
    }
}

__global__ __launch_bounds__(256) void peak_scatter_kernel(const PeakArgs A) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= A.n_waves) return;
    peak_scatter_wave(A, w, threadIdx.x & 63);
}

// Batched: the peak-finder arguments of every beam in a table in the constant address space
// (read with scalar loads), the waves of all beams in one index space: wave i belongs to beam b
// with wave_base[b] <= i < wave_base[b + 1].  One launch per pass for the whole batch; the scan
// takes one work-group per beam.
typedef __attribute__((address_space(4))) const PeakArgs CPeakArgs;

__device__ __forceinline__ int peak_beam_of(const PeakBatchArgs &B, int64_t wg) {
    const ConstI64Ptr base = (ConstI64Ptr)B.wave_base;
    int lo = 0, hi = B.n_beams - 1;                     // last b with base[b] <= wg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void peak_count_batch_kernel(const PeakBatchArgs B) {
    const int64_t wg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wg >= B.n_waves) return;
    const int b = peak_beam_of(B, wg);
    CPeakArgs &A = ((CPeakArgs *)B.tab)[b];
    peak_count_wave(A, (int)(wg - ((ConstI64Ptr)B.wave_base)[b]), threadIdx.x & 63);
}

__global__ __launch_bounds__(1024) void peak_scan_batch_kernel(const PeakBatchArgs B) {
    __shared__ int64_t part[1024];
    CPeakArgs &A = ((CPeakArgs *)B.tab)[blockIdx.x];
    peak_scan_block(A, part);
}

__global__ __launch_bounds__(256) void peak_scatter_batch_kernel(const PeakBatchArgs B) {
    const int64_t wg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wg >= B.n_waves) return;
    const int b = peak_beam_of(B, wg);
    CPeakArgs &A = ((CPeakArgs *)B.tab)[b];
    peak_scatter_wave(A, (int)(wg - ((ConstI64Ptr)B.wave_base)[b]), threadIdx.x & 63);
}

// ----------------------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------------------
int launch_scales(const ScaleArgs &a, void *stream) {
    if (a.n <= 0) return 0;
    const unsigned rows = a.rho ? (unsigned)a.n_rows : 1u;
    hipLaunchKernelGGL(scales_kernel, dim3((a.n + 255) / 256, rows), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_evalmask(const MaskArgs &a, void *stream) {
    hipLaunchKernelGGL(evalmask_kernel, dim3((a.n_words + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// IG(1) tiles of at most kSmallTileMax units run on work-groups of kSmallStepThreads (the
// planner sets StepArgs::nth): its light width sets leave the launch bound by the plane writes,
// which go faster from more, smaller work-groups (3.77 ms against 3.91 ms at the best tile of
// either size on the 4096 x 262144 beam; the denser sets are faster on 256 threads).  Results do
// not depend on the work-group size.
template <bool FIRST, int FAM, int NTH>
static void launch_nth(const StepArgs &a, int lds_bytes, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.n_dm * a.n_tiles));
    if (a.rho && a.write_planes)
        hipLaunchKernelGGL((step_kernel<FIRST, FAM, true, NTH, true>), grid, dim3(NTH), lds_bytes, st, a);
    else if (a.rho)
        hipLaunchKernelGGL((step_kernel<FIRST, FAM, true, NTH, false>), grid, dim3(NTH), lds_bytes, st, a);
    else if (a.write_planes)
        hipLaunchKernelGGL((step_kernel<FIRST, FAM, false, NTH, true>), grid, dim3(NTH), lds_bytes, st, a);
    else
        hipLaunchKernelGGL((step_kernel<FIRST, FAM, false, NTH, false>), grid, dim3(NTH), lds_bytes, st, a);
}

// The work-group size is the planner's (StepArgs::nth): 128 threads only for IG(1).
template <bool FIRST, int FAM>
static int launch_one(const StepArgs &a, int lds_bytes, hipStream_t st) {
    if (a.nth == kSmallStepThreads) {
        if (FAM != 1) return (int)hipErrorInvalidValue;
        launch_nth<FIRST, 1, kSmallStepThreads>(a, lds_bytes, st);
    } else if (a.nth == kStepThreads) {
        launch_nth<FIRST, FAM, kStepThreads>(a, lds_bytes, st);
    } else {
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <bool FIRST>
static int launch_step_fam(const StepArgs &a, int fam, int lds_bytes, hipStream_t st) {
    switch (fam) {
        case 1: return launch_one<FIRST, 1>(a, lds_bytes, st);
        case 2: return launch_one<FIRST, 2>(a, lds_bytes, st);
        case 3: return launch_one<FIRST, 3>(a, lds_bytes, st);
        case 4: return launch_one<FIRST, 4>(a, lds_bytes, st);
        case 5: return launch_one<FIRST, 5>(a, lds_bytes, st);
        case 6: return launch_one<FIRST, 6>(a, lds_bytes, st);
        case 7: return launch_one<FIRST, 7>(a, lds_bytes, st);
        default: return launch_one<FIRST, 0>(a, lds_bytes, st);
    }
}

template <bool FIRST, int FAM>
static int launch_batch(const StepBatchArgs &a, int lds_bytes, int grid, hipStream_t st) {
    if (a.s.write_planes)
        hipLaunchKernelGGL((step_kernel_batch<FIRST, FAM, true>), dim3((unsigned)grid),
                           dim3(kStepThreads), lds_bytes, st, a);
    else
        hipLaunchKernelGGL((step_kernel_batch<FIRST, FAM, false>), dim3((unsigned)grid),
                           dim3(kStepThreads), lds_bytes, st, a);
    return (int)hipGetLastError();
}

template <bool FIRST>
static int launch_batch_fam(const StepBatchArgs &a, int fam, int lds_bytes, int grid, hipStream_t st) {
    switch (fam) {
        case 1: return launch_batch<FIRST, 1>(a, lds_bytes, grid, st);
        case 2: return launch_batch<FIRST, 2>(a, lds_bytes, grid, st);
        case 3: return launch_batch<FIRST, 3>(a, lds_bytes, grid, st);
        case 4: return launch_batch<FIRST, 4>(a, lds_bytes, grid, st);
        case 5: return launch_batch<FIRST, 5>(a, lds_bytes, grid, st);
        case 6: return launch_batch<FIRST, 6>(a, lds_bytes, grid, st);
        case 7: return launch_batch<FIRST, 7>(a, lds_bytes, grid, st);
        default: return launch_batch<FIRST, 0>(a, lds_bytes, grid, st);
    }
}

int launch_step_batch(const StepBatchArgs &a, int fam, int lds_bytes, int grid, void *stream) {
    if (a.s.normalise) return launch_batch_fam<true>(a, fam, lds_bytes, grid, (hipStream_t)stream);
    return launch_batch_fam<false>(a, fam, lds_bytes, grid, (hipStream_t)stream);
}

int launch_step(const StepArgs &a, int fam, int lds_bytes, void *stream) {
    // the first step (raw samples, normalised on load) and the later steps (decimated series)
    // are separate instantiations, so profiles tell them apart
    if (a.normalise) return launch_step_fam<true>(a, fam, lds_bytes, (hipStream_t)stream);
    return launch_step_fam<false>(a, fam, lds_bytes, (hipStream_t)stream);
}

uint64_t family_mask(int fam, int pattern) {
    switch (fam) {
        case 1: return pattern == 1 ? Fam<1>::M1 : Fam<1>::M2;
        case 2: return pattern == 1 ? Fam<2>::M1 : Fam<2>::M2;
        case 3: return pattern == 1 ? Fam<3>::M1 : Fam<3>::M2;
        case 4: return Fam<4>::M1;
        case 5: return Fam<5>::M1;
        case 6: return Fam<6>::M1;
        case 7: return Fam<7>::M1;
        default: return 0;
    }
}

int launch_exhaustive(const ExhArgs &a, bool dense, void *stream) {
    const int64_t per_row = (a.n_seg + a.segs_per_wave - 1) / a.segs_per_wave;
    const dim3 grid((unsigned)((int64_t)a.n_dm * per_row));
    const bool multi = a.segs_per_wave > 1;
    // groups of 16 widths up to L_end 4096, of 64 above (measured crossover on gfx950)
    const bool small = a.l_end <= kExhSmallGroupMax;
    hipStream_t st = (hipStream_t)stream;
    if (multi) {
        if (dense)
            hipLaunchKernelGGL((exh_kernel<true, true, 16>), grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL((exh_kernel<false, true, 16>), grid, dim3(64), 0, st, a);
    } else if (small) {
        if (dense)
            hipLaunchKernelGGL((exh_kernel<true, false, 16>), grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL((exh_kernel<false, false, 16>), grid, dim3(64), 0, st, a);
    } else {
        if (dense)
            hipLaunchKernelGGL((exh_kernel<true, false, 64>), grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL((exh_kernel<false, false, 64>), grid, dim3(64), 0, st, a);
    }
    return (int)hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, void *stream) {
    if (n <= 0) return 0;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       p, n, v);
    return (int)hipGetLastError();
}

int launch_peaks(const PeakArgs &a, void *stream) {
    const dim3 grid((unsigned)((a.n_waves + 3) / 4));
    hipLaunchKernelGGL(peak_count_kernel, grid, dim3(256), 0, (hipStream_t)stream, a);
    int err = (int)hipGetLastError();
    if (err) return err;
    hipLaunchKernelGGL(peak_scan_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, a);
    err = (int)hipGetLastError();
    if (err) return err;
    hipLaunchKernelGGL(peak_scatter_kernel, grid, dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_peaks_batch(const PeakBatchArgs &a, void *stream) {
    if (a.n_waves <= 0) return 0;
    const dim3 grid((unsigned)((a.n_waves + 3) / 4));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(peak_count_batch_kernel, grid, dim3(256), 0, st, a);
    int err = (int)hipGetLastError();
    if (err) return err;
    hipLaunchKernelGGL(peak_scan_batch_kernel, dim3((unsigned)a.n_beams), dim3(1024), 0, st, a);
    err = (int)hipGetLastError();
    if (err) return err;
    hipLaunchKernelGGL(peak_scatter_batch_kernel, grid, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

const char *hip_error_text(int err) { return hipGetErrorString((hipError_t)err); }

}  // namespace spd
