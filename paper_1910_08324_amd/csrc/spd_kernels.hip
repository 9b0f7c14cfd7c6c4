// Boxcar single-pulse search kernels for gfx950 (CDNA4, wave64).
//
// lossy_kernel       BoxDIT and IGRID: one wave streams one (DM row, time segment) work item
//                    through an on-chip decimation cascade.  Every input sample is read from HBM
//                    once (plus the look-ahead halo of the segment), every plane value is written
//                    once, and no intermediate level ever leaves LDS.
// exh_kernel         exhaustive search (every width 1..L_end): one wave per 256 output slots,
//                    4 consecutive starts per lane, the input window streamed through an LDS ring.
// peak_* kernels     thresholded 3x3 peak finding over the per-level planes, with output in
//                    (level, dm, start) order: count -> scan -> scatter.
#include <hip/hip_runtime.h>

#include <math.h>

#include "spd_internal.h"

namespace spd {

#define SPD_NEG_INF (-__builtin_huge_valf())

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ----------------------------------------------------------------------------------------
// 1/sqrt(L) table of the exhaustive search.  Computed in FP64 and rounded once to FP32, so
// every kernel scales a boxcar sum by the correctly rounded 1/sqrt(L) (white-noise scaling,
// Section 2.1).  The cascade kernel builds its own small table in LDS the same way.
// ----------------------------------------------------------------------------------------
__global__ void scales_kernel(const ScaleArgs A) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.n) A.scale[t] = (float)(1.0 / sqrt((double)(t + 1)));
}

__global__ void evalmask_kernel(const MaskArgs A) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.n_words) A.evalmask[t] = A.bits[t];
}

// ----------------------------------------------------------------------------------------
// BoxDIT / IGRID cascade kernel.
//
// Work item = (row d, segment g): output slots [g seg / 2^k, min((g+1) seg / 2^k, slots_k)) of
// every level k.  The wave streams the row forward from s0 = g seg in chunks of kLossyChunk
// samples.  For each level it keeps, in LDS, a window of its decimated series y_k (and for
// BoxDIT the carried prefix sums), and it emits a slot as soon as every unit that slot's
// widest boxcar needs has been formed.  State per level (all wave-uniform):
//   a[k]   units of y_k formed so far          e[k]  next slot to emit
//   yb[k]  unit held at window index 0          cb[k] slot held at carry-window index 0
//   cw[k]  carries written so far (BoxDIT)      cnt[k] pre-candidates found (slab fill)
// After each chunk every window is compacted to its live tail so the LDS footprint stays at
// about 2 * chunk + levels * (widest unit count) floats.
// ----------------------------------------------------------------------------------------
template <bool CARRY>
__global__ __launch_bounds__(64) void lossy_kernel(const LossyArgs A) {
    extern __shared__ float lds[];
    __shared__ int st_a[kMaxLevels], st_e[kMaxLevels], st_yb[kMaxLevels], st_cb[kMaxLevels];
    __shared__ int st_cw[kMaxLevels];
    __shared__ uint32_t st_cnt[kMaxLevels];

    const int lane = threadIdx.x;
    const int d = blockIdx.x / A.n_seg;
    const int g = blockIdx.x - d * A.n_seg;
    if (d >= A.n_dm) return;
    const int nlev = A.n_levels;
    const int s0 = g * A.seg;                       // first sample of the segment (row coords)
    const float *xr = A.x + (int64_t)d * A.ld;
    const float mu = A.mean[d];
    const float inv = 1.0f / A.sigma[d];
    const float thr = A.threshold;

    if (lane < nlev) {
        st_a[lane] = 0;
        st_e[lane] = 0;
        st_yb[lane] = 0;
        st_cb[lane] = 0;
        st_cw[lane] = 0;
        st_cnt[lane] = 0;
    }
    // 1/sqrt(L) of every (level, width), rounded once from FP64 (white-noise scaling)
    for (int t = lane; t < A.n_scale; t += 64) {
        int lev = 0;
        while (lev + 1 < nlev && t >= A.lv[lev + 1].scale_off) ++lev;
        const LevelDesc &D = A.lv[lev];
        const double L = (double)D.base + (double)((int64_t)D.units[t - D.scale_off] << lev);   // level index = log2 separation
        lds[A.lds_scale + t] = (float)(1.0 / sqrt(L));
    }
    __syncthreads();

    constexpr int C = kLossyChunk;
    for (int ch = 0; ch < A.max_chunks; ++ch) {
        // ---- 1. load + normalise chunk ch into the level-0 window: z = (x - mu) / sigma
        {
            const int a0 = st_a[0];
            float *y0 = lds + A.lv[0].lds_y - st_yb[0] + a0;
            const int r0 = s0 + ch * C;
#pragma unroll
            for (int q = 0; q < C / 256; ++q) {
                const int j = q * 256 + lane * 4;
                const int r = r0 + j;
                float4 v;
                if (A.vec_ok && r + 3 < A.n_in) {
                    v = *reinterpret_cast<const float4 *>(xr + r);
                    v.x = (v.x - mu) * inv;
                    v.y = (v.y - mu) * inv;
                    v.z = (v.z - mu) * inv;
                    v.w = (v.w - mu) * inv;
                } else {
                    v.x = (r + 0 < A.n_in) ? (xr[r + 0] - mu) * inv : 0.0f;
                    v.y = (r + 1 < A.n_in) ? (xr[r + 1] - mu) * inv : 0.0f;
                    v.z = (r + 2 < A.n_in) ? (xr[r + 2] - mu) * inv : 0.0f;
                    v.w = (r + 3 < A.n_in) ? (xr[r + 3] - mu) * inv : 0.0f;
                }
                *reinterpret_cast<float4 *>(y0 + j) = v;
            }
            __syncthreads();
            if (lane == 0) st_a[0] = a0 + C;
            __syncthreads();
        }

        // ---- 2. decimation cascade: y_k[n] = y_{k-1}[2n + cshift] + y_{k-1}[2n + cshift + 1]
        for (int k = 1; k < nlev; ++k) {
            const int cs = A.lv[k].cshift;
            const int ap = st_a[k - 1];
            const int aold = st_a[k];
            const int anew = ap >= cs + 2 ? (ap - cs) >> 1 : 0;
            const float *yp = lds + A.lv[k - 1].lds_y - st_yb[k - 1];
            float *yk = lds + A.lv[k].lds_y - st_yb[k];
            for (int n = aold + lane; n < anew; n += 64) {
                const int src = 2 * n + cs;
                yk[n] = yp[src] + yp[src + 1];
            }
            __syncthreads();
            if (lane == 0) st_a[k] = anew > aold ? anew : aold;
            __syncthreads();
        }

        // ---- 3. emit every slot whose widest boxcar is complete, level by level
        bool all_done = true;
        for (int k = 0; k < nlev; ++k) {
            const LevelDesc &D = A.lv[k];
            const int endk = min(A.seg >> k, D.slots - (s0 >> k));
            const int e = st_e[k];
            const int hi = min(st_a[k] - D.umax + 1, endk);
            if (hi > e) {
                const float *yk = lds + D.lds_y - st_yb[k];
                const float *ck = lds + D.lds_c - st_cb[k];
                const bool pass_carry = CARRY && (k + 1 < nlev);
                float *cn = pass_carry ? (lds + A.lv[k + 1].lds_c - st_cb[k + 1]) : nullptr;
                const int ufull = D.ufull;
                const float *sc = lds + A.lds_scale + D.scale_off;
                const int64_t rowoff = D.plane_off + (int64_t)d * D.pitch + (s0 >> k);
                const int64_t slab = ((int64_t)k * A.n_dm + d) * A.n_seg + g;
                uint32_t cnt = st_cnt[k];
                for (int mb = e; mb < hi; mb += 64) {
                    const int m = mb + lane;
                    const bool act = m < hi;
                    float best = SPD_NEG_INF;
                    int bw = 0;
                    if (act) {
                        float X = (CARRY && k > 0) ? ck[m] : 0.0f;   // level 0 has no carried prefix
                        const int64_t s = (int64_t)s0 + ((int64_t)m << k);
                        const int64_t room = (int64_t)A.n_in - s;   // widths <= room are valid
                        int u = 0;
                        for (int j = 0; j < D.nw; ++j) {
                            const int uj = D.units[j];
                            for (; u < uj; ++u) X += yk[m + u];
                            const int Lw = D.base + (uj << k);
                            if (Lw <= room) {
                                const float v = X * sc[j];
                                if (v > best) {
                                    best = v;
                                    bw = Lw;
                                }
                            }
                        }
                        if (pass_carry && !(m & 1)) {
                            for (; u < ufull; ++u) X += yk[m + u];
                            cn[m >> 1] = X;
                        }
                        A.Y[rowoff + m] = best;
                        A.W[rowoff + m] = (uint16_t)bw;
                    }
                    if (A.want_cand) {
                        const bool hit = act && best > thr;
                        const uint64_t b = __ballot(hit);
                        if (b) {
                            if (hit) {
                                const uint32_t pos = cnt + __popcll(b & lanes_below(lane));
                                if (pos < kSlabCap)
                                    A.slab_ent[slab * kSlabCap + pos] = (uint32_t)((s0 >> k) + m);
                            }
                            cnt += __popcll(b);
                        }
                    }
                }
                __syncthreads();
                if (lane == 0) {
                    st_e[k] = hi;
                    st_cnt[k] = cnt;
                    if (pass_carry) st_cw[k + 1] = (hi + 1) >> 1;
                }
                __syncthreads();
            }
            if (max(e, hi) < endk) all_done = false;
        }
        if (all_done) break;

        // ---- 4. compact every window to its live tail
        for (int k = 0; k < nlev; ++k) {
            const LevelDesc &D = A.lv[k];
            const int endk = min(A.seg >> k, D.slots - (s0 >> k));
            const int a = st_a[k];
            const int e = st_e[k];
            int lo = a;
            if (e < endk) lo = min(lo, e);
            if (k + 1 < nlev) lo = min(lo, 2 * st_a[k + 1] + A.lv[k + 1].cshift);
            if (k == 0) lo &= ~3;                        // keep float4 alignment of loads
            const int yb = st_yb[k];
            float *yw = lds + D.lds_y;
            const int len = a - lo;
            float v0 = 0.0f, v1 = 0.0f;
            if (lane < len) v0 = yw[lo - yb + lane];
            if (lane + 64 < len) v1 = yw[lo - yb + lane + 64];
            int clen = 0, clo = 0;
            float c0 = 0.0f, c1 = 0.0f;
            if (CARRY && k > 0) {
                clo = e;
                clen = max(0, st_cw[k] - clo);
                float *cwin = lds + D.lds_c;
                const int cb = st_cb[k];
                if (lane < clen) c0 = cwin[clo - cb + lane];
                if (lane + 64 < clen) c1 = cwin[clo - cb + lane + 64];
            }
            __syncthreads();
            if (lane < len) yw[lane] = v0;
            if (lane + 64 < len) yw[lane + 64] = v1;
            if (CARRY && k > 0) {
                float *cwin = lds + D.lds_c;
                if (lane < clen) cwin[lane] = c0;
                if (lane + 64 < clen) cwin[lane + 64] = c1;
            }
            __syncthreads();
            if (lane == 0) {
                st_yb[k] = lo;
                if (CARRY && k > 0) st_cb[k] = clo;
            }
            __syncthreads();
        }
    }

    if (A.want_cand && lane < nlev)
        A.slab_cnt[((int64_t)lane * A.n_dm + d) * A.n_seg + g] = st_cnt[lane];
}

// ----------------------------------------------------------------------------------------
// Exhaustive search kernel.
//
// Work item = (row d, 256 output slots starting at s0).  Lane l owns the 4 consecutive starts
// s0 + 4l + v.  Widths are visited in increasing order with one running sum per start, in
// groups of 64 widths: inside a group only the maximum is tracked (add, multiply, max per
// start and width); after the group the best group, and the running sum entering it, are
// kept.  The winning width inside the winning group is recovered at the end by replaying that
// group's 64 steps with the same FP32 operations, so it is the smallest width attaining the
// maximum, exactly as a per-width argmax would give.
// The input window z[s0 .. s0 + 256 + L_end) streams through a 2048-float LDS ring, 512 new
// samples per block of 512 widths.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ float load_z(const float *xr, int r, int n_in, float mu, float inv) {
    return r < n_in ? (xr[r] - mu) * inv : 0.0f;
}

template <bool DENSE>
__global__ __launch_bounds__(64) void exh_kernel(const ExhArgs A) {
    __shared__ float4 ring4[512];                  // 2048 floats

    const int lane = threadIdx.x;
    const int d = blockIdx.x / A.n_seg;
    const int g = blockIdx.x - d * A.n_seg;
    if (d >= A.n_dm) return;
    const int s0 = g * kExhSlots;
    const float *xr = A.x + (int64_t)d * A.ld;
    const float mu = A.mean[d];
    const float inv = 1.0f / A.sigma[d];
    const int Lw = A.l_end;
    const int n_in = A.n_in;

    auto load4 = [&](int j) -> float4 {          // z[s0 + j .. s0 + j + 3], j multiple of 4
        const int r = s0 + j;
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
        ring4[j >> 2] = load4(j);
    }
    __syncthreads();

    float X[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float best[4] = {SPD_NEG_INF, SPD_NEG_INF, SPD_NEG_INF, SPD_NEG_INF};
    float bx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int bg[4] = {0, 0, 0, 0};
    int room[4];                                    // widest valid width per start
#pragma unroll
    for (int v = 0; v < 4; ++v) room[v] = n_in - (s0 + 4 * lane + v);

    const int nblk = (Lw + kExhBlock - 1) / kExhBlock;
    for (int b = 0; b < nblk; ++b) {
        const bool refill = (b + 1 < nblk);
        float4 pf0, pf1;
        const int jn = b * kExhBlock + 1024;
        if (refill) {
            pf0 = load4(jn + lane * 4);
            pf1 = load4(jn + 256 + lane * 4);
        }
        for (int gi = 0; gi < kExhBlock / kExhGroup; ++gi) {
            const int L0 = b * kExhBlock + gi * kExhGroup + 1;
            if (L0 > Lw) break;
            const bool fast = (L0 + kExhGroup - 1 <= Lw) &&
                              ((int64_t)s0 + kExhSlots - 1 + L0 + kExhGroup - 1 <= n_in);
            float Xs[4], gm[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Xs[v] = X[v];
                gm[v] = SPD_NEG_INF;
            }
            const int jb4 = lane + ((L0 - 1) >> 2);
            float4 wa = ring4[jb4 & 511];
#pragma unroll 4
            for (int t = 0; t < kExhGroup / 4; ++t) {
                const float4 wb = ring4[(jb4 + t + 1) & 511];
                const float w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
                const int L = L0 + 4 * t;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    const float r = A.scale[L - 1 + tt];
                    bool on = true;
                    if (!DENSE) on = (A.evalmask[(L - 1 + tt) >> 5] >> ((L - 1 + tt) & 31)) & 1u;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        X[v] += w[v + tt];
                        float snr = X[v] * r;
                        if (!fast) {
                            const bool ok = (L + tt <= Lw) && (L + tt <= room[v]);
                            snr = ok ? snr : SPD_NEG_INF;
                        }
                        if (!DENSE) snr = on ? snr : SPD_NEG_INF;
                        gm[v] = fmaxf(gm[v], snr);
                    }
                }
                wa = wb;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (gm[v] > best[v]) {
                    best[v] = gm[v];
                    bg[v] = (L0 - 1) / kExhGroup;
                    bx[v] = Xs[v];
                }
            }
        }
        if (refill) {
            __syncthreads();
            ring4[((jn >> 2) + lane) & 511] = pf0;
            ring4[((jn >> 2) + 64 + lane) & 511] = pf1;
            __syncthreads();
        }
    }

    // ---- recover the smallest width attaining the maximum inside the winning group
    int bw[4] = {0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (best[v] == SPD_NEG_INF) continue;
        const int sv = s0 + 4 * lane + v;
        const int Lb = bg[v] * kExhGroup + 1;
        float Xr = bx[v], bm = SPD_NEG_INF;
        for (int t = 0; t < kExhGroup; ++t) {
            const int L = Lb + t;
            if (L > Lw) break;
            Xr += load_z(xr, sv + L - 1, n_in, mu, inv);
            float snr = Xr * A.scale[L - 1];
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
        bool hit[4];
        int mine = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            hit[v] = (m0 + v < A.n_out) && best[v] > A.threshold;
            mine += hit[v];
        }
        const uint64_t any = __ballot(mine > 0);
        uint32_t base = 0;
        if (any) {
            // exclusive prefix of `mine` over lanes (lane-major, then v)
            int pre = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(pre, off);
                if (lane >= off) pre += t;
            }
            const int total = __shfl(pre, 63);
            pre -= mine;
            const int64_t slab = (int64_t)d * A.n_seg + g;
            int pos = pre;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (hit[v]) {
                    if (pos < kExhSlabCap) A.slab_ent[slab * kExhSlabCap + pos] = (uint32_t)(m0 + v);
                    ++pos;
                }
            }
            base = (uint32_t)total;
        }
        if (lane == 0) A.slab_cnt[(int64_t)d * A.n_seg + g] = base;
    }
}

// ----------------------------------------------------------------------------------------
// Peak finding (candidate selection).  A slot is a candidate iff its SNR is above the
// threshold and it passes the 3x3 neighbour test (strict against neighbours earlier in
// row-major order, non-strict against later ones).  Pre-candidates (SNR above threshold) were
// collected per (level, row, segment) slab by the search kernel in slot order; a slab that
// overflowed is rescanned densely over its slot range.  Three passes keep the output in
// (level, dm, start) order without sorting: per-wave survivor counts, one scan, scatter.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ bool peak_test(const PeakArgs &A, int k, int d, int m, float y) {
    const float *P = A.Y + A.level_off[k];
    const int64_t pitch = A.level_pitch[k];
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
            const float yn = P[(int64_t)dn * pitch + mn];
            const bool earlier = (a < 0) || (a == 0 && b < 0);
            if (earlier ? !(y > yn) : !(y >= yn)) return false;
        }
    }
    return true;
}

struct SlabPos {
    int k, d, g;
};

__device__ __forceinline__ SlabPos slab_decode(const PeakArgs &A, int64_t s) {
    SlabPos p;
    p.g = (int)(s % A.n_seg);
    const int64_t r = s / A.n_seg;
    p.d = (int)(r % A.n_dm);
    p.k = (int)(r / A.n_dm);
    return p;
}

__device__ __forceinline__ float plane_at(const PeakArgs &A, int k, int d, int m) {
    return A.Y[A.level_off[k] + (int64_t)d * A.level_pitch[k] + m];
}

__global__ __launch_bounds__(256) void peak_count_kernel(const PeakArgs A) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= A.n_waves) return;
    const int64_t sbeg = (int64_t)w * A.slabs_per_wave;
    const int64_t send = min(sbeg + A.slabs_per_wave, A.n_slabs);
    int64_t total = 0;
    for (int64_t sb = sbeg; sb < send; sb += 64) {
        const int64_t s = sb + lane;
        const uint32_t c = (s < send) ? A.slab_cnt[s] : 0u;
        if (s < send && c == 0) A.surv[s] = 0;
        uint64_t nz = __ballot(c != 0);
        while (nz) {
            const int l = __ffsll((unsigned long long)nz) - 1;
            nz &= nz - 1;
            const int64_t ss = sb + l;
            const uint32_t cc = __shfl(c, l);
            const SlabPos p = slab_decode(A, ss);
            uint32_t nsurv = 0;
            uint64_t msk = 0;
            if (cc <= (uint32_t)A.slab_cap) {
                bool ok = false;
                if (lane < (int)cc) {
                    const int m = (int)A.slab_ent[ss * A.slab_cap + lane];
                    ok = peak_test(A, p.k, p.d, m, plane_at(A, p.k, p.d, m));
                }
                msk = __ballot(ok);
                nsurv = __popcll(msk);
            } else {
                const int segk = A.seg >> A.level_shift[p.k];
                const int mlo = p.g * segk;
                const int mhi = min(mlo + segk, A.level_slots[p.k]);
                for (int mb = mlo; mb < mhi; mb += 64) {
                    const int m = mb + lane;
                    bool ok = false;
                    if (m < mhi) {
                        const float y = plane_at(A, p.k, p.d, m);
                        ok = (y > A.threshold) && peak_test(A, p.k, p.d, m, y);
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

__global__ __launch_bounds__(1024) void peak_scan_kernel(const PeakArgs A) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (A.n_waves + 1023) / 1024;
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
    int64_t run = part[t] - loc;                      // exclusive prefix
    for (int i = 0; i < per; ++i) {
        const int w = t * per + i;
        if (w < A.n_waves) {
            A.wave_off[w] = run;
            run += A.wave_tot[w];
        }
    }
    if (t == 1023) *A.cand_count = part[1023];
}

__device__ __forceinline__ void put_cand(const PeakArgs &A, int64_t idx, int k, int d, int m,
                                         float y) {
    if (idx >= A.cand_cap) return;
    spd_candidate c;
    c.start = A.t0 + ((int64_t)m << A.level_shift[k]);
    c.dm = d;
    c.width = A.W[A.level_off[k] + (int64_t)d * A.level_pitch[k] + m];
    c.level = k;
    c.snr = y;
    A.cand[idx] = c;
}

__global__ __launch_bounds__(256) void peak_scatter_kernel(const PeakArgs A) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= A.n_waves) return;
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
            const uint32_t nsurv = __shfl(sv, l);
            const uint32_t cc = A.slab_cnt[ss];
            const SlabPos p = slab_decode(A, ss);
            if (cc <= (uint32_t)A.slab_cap) {
                const uint64_t msk = A.mask[ss];
                if (lane < (int)cc && ((msk >> lane) & 1ull)) {
                    const int m = (int)A.slab_ent[ss * A.slab_cap + lane];
                    put_cand(A, off + __popcll(msk & lanes_below(lane)), p.k, p.d, m,
                             plane_at(A, p.k, p.d, m));
                }
            } else {
                const int segk = A.seg >> A.level_shift[p.k];
                const int mlo = p.g * segk;
                const int mhi = min(mlo + segk, A.level_slots[p.k]);
                int64_t run = 0;
                for (int mb = mlo; mb < mhi; mb += 64) {
                    const int m = mb + lane;
                    bool ok = false;
                    float y = 0.0f;
                    if (m < mhi) {
                        y = plane_at(A, p.k, p.d, m);
                        ok = (y > A.threshold) && peak_test(A, p.k, p.d, m, y);
                    }
                    const uint64_t b = __ballot(ok);
                    if (ok) put_cand(A, off + run + __popcll(b & lanes_below(lane)), p.k, p.d, m, y);
                    run += __popcll(b);
                }
            }
            off += nsurv;
        }
    }
}

// ----------------------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------------------
int launch_scales(const ScaleArgs &a, void *stream) {
    if (a.n <= 0) return 0;
    hipLaunchKernelGGL(scales_kernel, dim3((a.n + 255) / 256), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_evalmask(const MaskArgs &a, void *stream) {
    hipLaunchKernelGGL(evalmask_kernel, dim3((a.n_words + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_lossy(const LossyArgs &a, bool carry, int lds_bytes, void *stream) {
    const dim3 grid((unsigned)((int64_t)a.n_dm * a.n_seg));
    if (carry)
        hipLaunchKernelGGL(lossy_kernel<true>, grid, dim3(64), lds_bytes, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(lossy_kernel<false>, grid, dim3(64), lds_bytes, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_exhaustive(const ExhArgs &a, bool dense, void *stream) {
    const dim3 grid((unsigned)((int64_t)a.n_dm * a.n_seg));
    if (dense)
        hipLaunchKernelGGL(exh_kernel<true>, grid, dim3(64), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(exh_kernel<false>, grid, dim3(64), 0, (hipStream_t)stream, a);
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

const char *hip_error_text(int err) { return hipGetErrorString((hipError_t)err); }

}  // namespace spd
