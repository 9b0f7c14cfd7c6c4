// Noise statistics per DM trial (declared in include/spd_msd.h): robust mean and standard
// deviation with iterative outlier rejection, for the samples and for every power-of-two
// decimation of them.  One work-group per row, FP64 throughout.
//
// A pass reads the row once and serves every level at the same time.  The row streams through
// in tiles of 1024 samples, one float4 per thread; inside a tile the decimated values of levels
// 1..8 are formed in registers (levels 1, 2 within a thread, 3..8 by pairwise sums across lanes,
// moved by DPP row shifts and readlane rather than through LDS)
// and each lane accumulates the values it holds.  Values of levels 9 and up (at most 1/256 of the
// samples) are formed once, in the first pass, into the workspace, and later passes read them
// from there.  Per level, each thread keeps a count and the sums of (value - shift) and of its
// square, with the shift the level's current mean estimate; after the pass the threads' partial
// statistics (count, mean, sum of squared deviations) are merged pairwise with Chan, Golub &
// LeVeque's formula in a fixed order.  Levels 0..2, which every lane serves, count their kept
// values per wave instead, and their lanes' sums around the common shift are totalled directly.  Levels converge independently; the row's passes stop
// when every level has.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "spd.h"
#include "spd_msd.h"

namespace spdm {

constexpr int kThreads = 256;
constexpr int kTile = 4 * kThreads;   // samples per tile
constexpr int kRegLevels = 9;          // levels 0..8 formed in registers
constexpr int kWsFirst = 9;            // levels 9.. live in the workspace

struct Part {
    double n, mean, m2;
};

__device__ __forceinline__ Part merge(Part a, Part b) {
    if (a.n == 0.0) return b;
    if (b.n == 0.0) return a;
    const double n = a.n + b.n;
    const double d = b.mean - a.mean;
    Part r;
    r.n = n;
    r.mean = a.mean + d * (b.n / n);
    r.m2 = a.m2 + b.m2 + d * d * (a.n * b.n / n);
    return r;
}

// merge the 256 threads' partials: butterflies inside each wave, then the four waves in order
__device__ Part block_merge(Part p, Part *sh) {
    for (int o = 1; o < 64; o <<= 1) {
        Part q;
        q.n = __shfl_xor(p.n, o);
        q.mean = __shfl_xor(p.mean, o);
        q.m2 = __shfl_xor(p.m2, o);
        // both lanes of a pair combine (lower, upper) in the same order, so they agree
        const bool upper = (threadIdx.x & o) != 0;
        p = upper ? merge(q, p) : merge(p, q);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
    __syncthreads();
    return merge(merge(sh[0], sh[1]), merge(sh[2], sh[3]));
}

// totals over the work-group of per-thread (count, sum, sum of squares) in a fixed order:
// butterflies inside each wave (a + b == b + a, so the lanes agree), then the four waves in order
__device__ Part block_sums(Part p, Part *sh) {
    for (int o = 1; o < 64; o <<= 1) {
        p.n += __shfl_xor(p.n, o);
        p.mean += __shfl_xor(p.mean, o);
        p.m2 += __shfl_xor(p.m2, o);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = p;
    __syncthreads();
    Part t;
    t.n = (sh[0].n + sh[1].n) + (sh[2].n + sh[3].n);
    t.mean = (sh[0].mean + sh[1].mean) + (sh[2].mean + sh[3].mean);
    t.m2 = (sh[0].m2 + sh[1].m2) + (sh[2].m2 + sh[3].m2);
    return t;
}

// a thread's running sums of one level: count, sum and sum of squares of (value - shift)
struct Acc {
    int n;
    double s1, s2;
};

__device__ __forceinline__ void acc_reset(Acc &a) {
    a.n = 0;
    a.s1 = a.s2 = 0.0;
}

__device__ __forceinline__ Part acc_part(const Acc &a, double shift) {
    Part p = {0.0, 0.0, 0.0};
    if (a.n > 0) {
        p.n = (double)a.n;
        p.mean = shift + a.s1 / p.n;
        p.m2 = fmax(0.0, a.s2 - a.s1 * (a.s1 / p.n));
    }
    return p;
}

// the estimate of one level, shared by the work-group
struct Level {
    double shift;       // subtracted before summing
    double m, lim;      // a value is kept in a rejection pass if |value - m| <= lim
    double sd, kept;
    int active;         // still being refined
    int iters;          // rejection passes that changed the estimate
};

struct MsdArgs {
    const float *x;
    int64_t ld;
    double *ws;          // per row: the values of levels 9.. (n >> 9 of level 9, then level 10, ...)
    int64_t ws_row;      // doubles per row
    float *mean, *sigma, *rho, *level_sd;
    int32_t *passes;
    int32_t n_dm, n_in, levels, max_iter;
    double tau;
};

// take value v of a level (valid or not) into the thread's sums.  After the first pass the
// shift is the level's mean, so one difference serves the test and the sums.
__device__ __forceinline__ void take(Acc &a, const Level &L, bool first, bool valid, double v) {
    const double d = v - L.shift;
    const bool ok = valid && (first || fabs(d) <= L.lim);
    const double e = ok ? d : 0.0;           // (d may be NaN for a value past the data)
    a.n += ok ? 1 : 0;
    a.s1 += e;
    a.s2 = fma(e, e, a.s2);
}

// v of lane l + 2^(K-3), for the lanes that are multiples of 2^(K-2) (other lanes get values
// that are never used).  Within a row of 16 lanes a DPP row shift moves the value in registers;
// across rows the two (or one) values needed are read out with readlane.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int K>
__device__ __forceinline__ double from_lane_above(double v, int lane) {
    constexpr int span = 1 << (K - 3);
    if constexpr (span <= 8) {
        return dpp_f64<0x100 + span>(v);                // row_shl:span (lane l reads l + span)
    } else if constexpr (span == 16) {
        const double a = readlane_f64(v, 16), b = readlane_f64(v, 48);
        return lane < 32 ? a : b;
    } else {
        return readlane_f64(v, 32);
    }
}

// one step of the cross-lane cascade: level K from pairs of level K-1 values; each holder lane
// (a multiple of 2^(K-2)) parks its value in the wave's slot of level K (NaN past the data;
// in a FULL tile every value of levels 3..8 lies inside it)
template <int K, bool FULL>
__device__ __forceinline__ void level_step(double &v, double *slots, int lane, int s, int n) {
    constexpr int kSlotK = K == 3 ? 0 : K == 4 ? 32 : K == 5 ? 48 : K == 6 ? 56 : K == 7 ? 60 : 62;
    v = v + from_lane_above<K>(v, lane);
    if ((lane & ((2 << (K - 3)) - 1)) == 0)
        slots[kSlotK + (lane >> (K - 2))] = (FULL || s + (1 << K) <= n) ? v : __builtin_nan("");
}

// take for a level every lane of the wave serves: the count of kept values is kept per wave
// (a ballot's population count, on the scalar unit) instead of per lane
__device__ __forceinline__ void take_w(Acc &a, uint32_t &nw, const Level &L, bool first,
                                       bool valid, double v) {
    const double d = v - L.shift;
    const bool ok = valid && (first || fabs(d) <= L.lim);
    const double e = ok ? d : 0.0;           // (d may be NaN for a value past the data)
    nw += (uint32_t)__popcll(__ballot(ok));
    a.s1 += e;
    a.s2 = fma(e, e, a.s2);
}

// statistics of a level all of whose values share one shift: the work-group's totals of the
// lanes' sums and the waves' counts give the mean and the sum of squared deviations
__device__ __forceinline__ Part wave_counted_part(const Acc &a, uint32_t nw, double shift, Part *sh) {
    Part p = {(threadIdx.x & 63) == 0 ? (double)nw : 0.0, a.s1, a.s2};
    const Part t = block_sums(p, sh);
    Part u = {0.0, 0.0, 0.0};
    if (t.n > 0.0) {
        u.n = t.n;
        u.mean = shift + t.mean / t.n;
        u.m2 = fmax(0.0, t.m2 - t.mean * (t.mean / t.n));
    }
    return u;
}

__global__ __launch_bounds__(kThreads) void msd_kernel(const MsdArgs A) {
    __shared__ Part sh[4];
    __shared__ Level lv[SPD_MAX_LEVELS];
    __shared__ double t8[4];                   // level-8 value of each wave in the current tile
    __shared__ double slot_buf[4][64];         // per wave: this tile's level 3..8 values
    __shared__ int any_active;
    const int d = blockIdx.x;
    if (d >= A.n_dm) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n = A.n_in;
    const int K = A.levels;
    const int kreg = min(K, kRegLevels);
    const float *xr = A.x + (int64_t)d * A.ld;
    double *wr = A.ws + (int64_t)d * A.ws_row;
    const int n_tiles = (n + kTile - 1) / kTile;
    const bool vec = (((uintptr_t)xr) & 15) == 0;
    // a tile gives each wave 32 + 16 + 8 + 4 + 2 + 1 values of levels 3..8: lanes 0..31 take
    // level 3, 32..47 level 4, 48..55 level 5, 56..59 level 6, 60..61 level 7, 62 level 8
    const int my_k = lane < 32 ? 3 : lane < 48 ? 4 : lane < 56 ? 5 : lane < 60 ? 6 : lane < 62 ? 7
                                                                                   : lane < 63 ? 8 : kRegLevels;
    double *slots = slot_buf[wave];
    slots[63] = __builtin_nan("");               // lane 63 has no value

    if (tid < K) {
        Level &L = lv[tid];
        L.shift = (double)xr[0] * (double)(1 << tid);   // first pass: a value of the right size
        L.m = 0.0;
        L.lim = 0.0;
        L.sd = 0.0;
        L.kept = 0.0;
        L.active = 1;
        L.iters = 0;
    }
    __syncthreads();

    int pass = 0;
    for (; pass <= A.max_iter; ++pass) {
        const bool first = pass == 0;
        if (!first) {
            if (tid == 0) {
                int a = 0;
                for (int k = 0; k < K; ++k) a |= lv[k].active;
                any_active = a;
            }
            __syncthreads();
            if (!any_active) break;
        }
        // the samples are read again only while a level formed from them in registers is open
        // (levels 9.. come from the workspace after the first pass)
        bool read_row = first;
        for (int k = 0; k < kreg; ++k) read_row = read_row || lv[k].active;
        Acc a0, a1, a2, am;                      // levels 0, 1, 2 and this lane's level of 3..8
        uint32_t n0w = 0, n1w = 0, n2w = 0;      // the wave's kept counts of levels 0, 1, 2
        acc_reset(a0);
        acc_reset(a1);
        acc_reset(a2);
        acc_reset(am);
        const Level L0 = lv[0];
        const Level L1 = lv[min(1, K - 1)];
        const Level L2 = lv[min(2, K - 1)];
        const Level Lm = lv[min(my_k, K - 1)];
        const bool on0 = first || L0.active;
        const bool on1 = K > 1 && (first || L1.active);
        const bool on2 = K > 2 && (first || L2.active);
        const bool onm = my_k < kreg && (first || Lm.active);

        auto fetch = [&](int tile, float4 &f) {
            const int s = tile * kTile + 4 * tid;
            if (vec && s + 3 < n) {
                f = *reinterpret_cast<const float4 *>(xr + s);
            } else {
                f.x = s + 0 < n ? xr[s + 0] : 0.0f;
                f.y = s + 1 < n ? xr[s + 1] : 0.0f;
                f.z = s + 2 < n ? xr[s + 2] : 0.0f;
                f.w = s + 3 < n ? xr[s + 3] : 0.0f;
            }
        };
        float4 nxt = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (read_row) fetch(0, nxt);
        // one tile; FULL: every sample of the tile is inside the data (all tiles but the last),
        // so the per-value validity tests fold away
        auto tile_body = [&](auto full_tag, int tile, float4 cur) {
            constexpr bool FULL = decltype(full_tag)::value;
            const int s = tile * kTile + 4 * tid;                // first sample of this thread
            const double v0[4] = {(double)cur.x, (double)cur.y, (double)cur.z, (double)cur.w};
            if (on0)
#pragma unroll
                for (int q = 0; q < 4; ++q) take_w(a0, n0w, L0, first, FULL || s + q < n, v0[q]);
            // levels 1, 2 within the thread
            const double v1a = v0[0] + v0[1], v1b = v0[2] + v0[3];
            if (on1) {
                take_w(a1, n1w, L1, first, FULL || s + 2 <= n, v1a);
                take_w(a1, n1w, L1, first, FULL || s + 4 <= n, v1b);
            }
            double v = v1a + v1b;
            if (on2) take_w(a2, n2w, L2, first, FULL || s + 4 <= n, v);
            // levels 3..8 across lanes: after step k, lane l holds the value of level k that starts
            // at its own samples when l is a multiple of 2^(k-2); holders park their values in the
            // wave's 64 slots (level k from slot 64 - 2^(9-k), one per holder, NaN past the data), and
            // every lane then takes the one value of its own level in its slot
            level_step<3, FULL>(v, slots, lane, s, n);
            level_step<4, FULL>(v, slots, lane, s, n);
            level_step<5, FULL>(v, slots, lane, s, n);
            level_step<6, FULL>(v, slots, lane, s, n);
            level_step<7, FULL>(v, slots, lane, s, n);
            level_step<8, FULL>(v, slots, lane, s, n);
            if (onm) {
                const double mv = slots[lane];                   // written by this wave above
                take(am, Lm, first, FULL || !__builtin_isnan(mv), mv);
            }
            // levels 9 and 10 (and the level-10 values the higher levels are built from): the
            // first pass writes them to the workspace
            if (first && K > kWsFirst) {
                if (lane == 0) t8[wave] = v;
                __syncthreads();
                if (tid == 0) {
                    const int64_t i9 = (int64_t)tile * 2;
                    const double a9 = t8[0] + t8[1], b9 = t8[2] + t8[3];
                    const int64_t n9 = n >> 9;
                    if (i9 < n9) wr[i9] = a9;
                    if (i9 + 1 < n9) wr[i9 + 1] = b9;
                    if (K > 10 && tile < (n >> 10)) wr[n9 + tile] = a9 + b9;
                }
                __syncthreads();
            }
        };
        for (int tile = 0; read_row && tile < n_tiles; ++tile) {
            const float4 cur = nxt;
            if (tile + 1 < n_tiles) fetch(tile + 1, nxt);        // in flight while this tile computes
            if ((tile + 1) * kTile <= n)                         // uniform over the work-group
                tile_body(std::true_type{}, tile, cur);
            else
                tile_body(std::false_type{}, tile, cur);
        }
        if (first && K > 11) {
            // levels 11.. from pairs of the level below, all in the workspace
            int64_t off_prev = (int64_t)(n >> 9), off = off_prev + (n >> 10);
            for (int k = 11; k < K; ++k) {
                const int64_t cnt = (int64_t)(n >> k);
                for (int64_t i = tid; i < cnt; i += kThreads) wr[off + i] = wr[off_prev + 2 * i] + wr[off_prev + 2 * i + 1];
                off_prev = off;
                off += cnt;
                __syncthreads();
            }
        }

        // merge the pass's statistics and update every level still being refined (the decision
        // to skip a level is uniform across the work-group)
        auto update_merged = [&](int k, const Part u) {
            if (tid == 0) {
                Level &S = lv[k];
                if (first) {
                    S.m = u.mean;
                    S.sd = u.n > 1.0 ? sqrt(u.m2 / (u.n - 1.0)) : 0.0;
                    S.kept = u.n;
                    S.active = A.max_iter > 0;
                } else if (u.n == S.kept || u.n < 2.0) {
                    S.active = 0;
                } else {
                    S.kept = u.n;
                    S.m = u.mean;
                    S.sd = sqrt(u.m2 / (u.n - 1.0));
                    S.iters += 1;
                    if (S.iters >= A.max_iter) S.active = 0;
                }
                S.lim = A.tau * S.sd;
                S.shift = S.m;
            }
            __syncthreads();
        };
        auto update = [&](int k, Part p) { update_merged(k, block_merge(p, sh)); };
        if (K > 0 && (first || lv[0].active)) update_merged(0, wave_counted_part(a0, n0w, lv[0].shift, sh));
        if (K > 1 && (first || lv[1].active)) update_merged(1, wave_counted_part(a1, n1w, lv[1].shift, sh));
        if (K > 2 && (first || lv[2].active)) update_merged(2, wave_counted_part(a2, n2w, lv[2].shift, sh));
        for (int k = 3; k < kreg; ++k) {
            if (first || lv[k].active) {
                Part p = {0.0, 0.0, 0.0};
                if (my_k == k) p = acc_part(am, lv[k].shift);
                update(k, p);
            }
        }
        int64_t off = 0;
        for (int k = kWsFirst; k < K; ++k) {
            const int64_t cnt = (int64_t)(n >> k);
            const Level Lk = lv[k];
            if (first || Lk.active) {
                Acc a;
                acc_reset(a);
                for (int64_t i = tid; i < cnt; i += kThreads) take(a, Lk, first, true, wr[off + i]);
                update(k, acc_part(a, Lk.shift));
            }
            off += cnt;
        }
    }

    if (tid < K) {
        const double sd0 = lv[0].sd;
        const double sd = lv[tid].sd;
        if (tid == 0) {
            A.mean[d] = (float)lv[0].m;
            A.sigma[d] = (float)sd0;
            if (A.passes) A.passes[d] = pass;
        }
        if (A.rho) A.rho[(int64_t)d * K + tid] = (float)(sd / (sqrt((double)(1 << tid)) * sd0));
        if (A.level_sd) A.level_sd[(int64_t)d * K + tid] = (float)sd;
    }
}

}  // namespace spdm

extern "C" {

int spd_msd_workspace(int32_t n_dm, int32_t n_in, int32_t levels, int64_t *bytes) {
    if (!bytes || n_dm < 1 || n_in < 2 || n_in > INT32_MAX - 4096 || levels < 1 ||
        levels > SPD_MAX_LEVELS || ((int64_t)n_in >> (levels - 1)) < 2)
        return SPD_EINVAL;
    // levels 9.. of every row: fewer than n_in / 256 values
    *bytes = (int64_t)n_dm * ((n_in >> 8) + 8) * 8 + 256;
    return SPD_OK;
}

int spd_msd(const float *x, int64_t ld, int32_t n_dm, int32_t n_in, int32_t levels, float tau,
            int32_t max_iter, float *mean, float *sigma, float *rho, float *level_sd,
            int32_t *passes, void *workspace, int64_t workspace_bytes, void *hip_stream) {
    int64_t need = 0;
    const int st = spd_msd_workspace(n_dm, n_in, levels, &need);
    if (st != SPD_OK) return st;
    if (!x || ld < n_in || !mean || !sigma || !(tau > 0.0f) || max_iter < 0) return SPD_EINVAL;
    if (!workspace || workspace_bytes < need) return SPD_EWORKSPACE;
    if ((uintptr_t)workspace & 255) return SPD_EALIGN;
    spdm::MsdArgs a;
    a.x = x;
    a.ld = ld;
    a.ws = static_cast<double *>(workspace);
    a.ws_row = (n_in >> 8) + 8;
    a.mean = mean;
    a.sigma = sigma;
    a.rho = rho;
    a.level_sd = level_sd;
    a.passes = passes;
    a.n_dm = n_dm;
    a.n_in = n_in;
    a.levels = levels;
    a.max_iter = max_iter;
    a.tau = (double)tau;
    hipLaunchKernelGGL(spdm::msd_kernel, dim3(n_dm), dim3(spdm::kThreads), 0,
                       static_cast<hipStream_t>(hip_stream), a);
    return hipGetLastError() == hipSuccess ? SPD_OK : SPD_EHIP;
}

}  // extern "C"
