// Noise statistics per DM trial (declared in include/spd_msd.h): robust mean and standard
// deviation with iterative outlier rejection, for the samples and for every power-of-two
// decimation of them.  One work-group per row, FP64 throughout.
//
// A read of the row serves every level at once.  The row streams through in tiles of 1024
// samples, one float4 per thread; inside a tile the decimated values of levels 1..8 are formed
// in registers (levels 1, 2 within a thread, 3..8 by pairwise sums across lanes, moved by DPP
// row shifts and readlane rather than through LDS).  Levels 0..5 are accumulated as they stream
// by: per level, each thread keeps a count and the sums of (value - shift) and of its square,
// the shift being the level's current mean estimate; levels 0..2, which every lane serves, count
// their kept values per wave and total their lanes' sums directly, levels 3..5 merge per-lane
// partials (count, mean, sum of squared deviations) with Chan, Golub & LeVeque's formula in a
// fixed order.  Levels 6 and up (at most 1/32 of the values) are stored whole in the workspace by
// the first read and taken from there in every pass.  Levels converge independently; the row's
// passes stop when every level has.
//
// Most passes need not read the row.  Before the first read a pre-estimate (mean and sd of 8
// tiles spread over the row) centres a band for each level 0..5; the first read (the estimate
// that keeps every value) lists, per level and wave, every value outside the band and keeps the
// count and sums of the values it did not list.  While the limit of a later pass still covers
// the whole band (|value - list centre| <= band half-width implies |value - mean| <= limit,
// checked with a margin for rounding), every unlisted value is kept, so the pass needs only the
// listed values: it tests them exactly as a full read would and adds the unlisted statistics;
// such a pass runs its levels side by side, one wave per level.  The kept sets, hence the counts,
// pass counts and stopping decisions, are those of full reads; only the order of the FP64 sums
// differs (and is fixed).  When the band is no longer covered, or a list overflowed its room, the
// pass reads the row again and lists anew around its own estimate (0.8 of its limit).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "spd.h"
#include "spd_msd.h"

namespace spdm {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTile = 4 * kThreads;   // samples per tile
constexpr int kRegLevels = 9;          // levels 0..8 formed in registers
constexpr int kListLevels = 6;         // levels 0..5 are summed as the row streams by
constexpr int kArrFirst = 6;           // levels 6.. are stored whole by the first pass
constexpr double kListFrac = 0.8;      // a rebuild lists values beyond 0.8 of the limit
constexpr int kProbeTiles = 8;         // tiles of the pre-estimate, spread over the row

// Per row, the workspace holds the values of levels 6.. (level 6 first, then 7, ...; fewer than
// n / 32 in all), then for each level k < 6 one list per wave with room for 1/16 of the wave's
// values of the level, plus 16.
__host__ __device__ inline int64_t arr_offset(int n, int k) {   // of level k >= 6
    int64_t o = 0;
    for (int i = kArrFirst; i < k; ++i) o += (int64_t)(n >> i);
    return o;
}
__host__ __device__ constexpr int list_room(int n, int k) { return ((n >> k) >> 6) + 16; }
__host__ __device__ inline int64_t list_offset(int n, int k) {   // of level k's first list
    int64_t o = (int64_t)(n >> 5) + 8;
    for (int i = 0; i < k; ++i) o += (int64_t)kWaves * list_room(n, i);
    return o;
}
__host__ __device__ inline int64_t ws_row_doubles(int n) { return list_offset(n, kListLevels); }

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

// the same two reductions over one wave only (every lane receives the result)
__device__ __forceinline__ Part wave_merge(Part p) {
    for (int o = 1; o < 64; o <<= 1) {
        Part q;
        q.n = __shfl_xor(p.n, o);
        q.mean = __shfl_xor(p.mean, o);
        q.m2 = __shfl_xor(p.m2, o);
        const bool upper = (threadIdx.x & o) != 0;
        p = upper ? merge(q, p) : merge(p, q);
    }
    return p;
}

__device__ __forceinline__ Part wave_sums(Part p) {
    for (int o = 1; o < 64; o <<= 1) {
        p.n += __shfl_xor(p.n, o);
        p.mean += __shfl_xor(p.mean, o);
        p.m2 += __shfl_xor(p.m2, o);
    }
    return p;
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
    double lc, lt;      // last full read: values with |value - lc| > lt are listed
    double nn, ns1, ns2;  // the unlisted values: count and sums of (value - lc) and its square
    int active;         // still being refined
    int iters;          // rejection passes that changed the estimate
    int listed;         // the lists hold every value beyond lt (none overflowed)
};

// every unlisted value is kept by a pass with this level's current mean and limit: the band
// |v - lc| <= lt lies inside |v - m| <= lim with room for the rounding of both differences
__device__ __forceinline__ bool band_covered(const Level &L) {
    const double slack = 1e-12 * (L.lim + L.lt + fabs(L.lc) + fabs(L.m));
    return L.listed && L.lt + fabs(L.lc - L.m) + slack <= L.lim;
}

struct MsdArgs {
    const float *x;
    int64_t ld;
    double *ws;          // per row: the values of levels 6.., then the lists of levels 0..5
    int64_t ws_row;      // doubles per row
    float *mean, *sigma, *rho, *level_sd;
    int32_t *passes;
    int32_t n_dm, n_in, levels, max_iter;
    double tau;
};

// a level's estimate after a pass with statistics u (one thread)
__device__ __forceinline__ void update_level(Level &S, const Part &u, bool probe, bool first,
                                             const MsdArgs &A) {
    if (probe) {
        // centre and band of the first pass's lists: 0.9 of the limit the pre-estimate gives,
        // less by three standard errors of its sd
        const double sd = u.n > 1.0 ? sqrt(u.m2 / (u.n - 1.0)) : 0.0;
        const double frac = 0.9 / (1.0 + 3.0 / sqrt(fmax(2.0 * u.n, 1.0)));
        S.shift = u.n > 0.0 ? u.mean : S.shift;
        S.lc = S.shift;
        S.lt = frac * A.tau * sd;
        return;
    }
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

// how many of the lanes below this one have their bit set in b (mbcnt)
__device__ __forceinline__ int count_below(uint64_t b) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

// append the values of the lanes whose `far` is set to the wave's list, in lane order after the
// values appended before (a full list still counts them, which marks the overflow)
__device__ __forceinline__ void list_append(bool far, double v, double *list, int &cnt, int room) {
    const uint64_t b = __ballot(far);
    if (b) {
        const int i = cnt + count_below(b);
        if (far && i < room) list[i] = v;
        cnt += __popcll(b);
    }
}

// take for a level every lane of the wave serves: the count of kept values is kept per wave
// (a ballot's population count, on the scalar unit) instead of per lane.  LIST: values beyond
// the list threshold also go to the wave's list of the level.
template <bool LIST>
__device__ __forceinline__ void take_w(Acc &a, uint32_t &nw, const Level &L, bool first,
                                       bool valid, double v, double *list, int &cnt, int room) {
    const double d = v - L.shift;
    const bool ok = valid && (first || fabs(d) <= L.lim);
    const double e = ok ? d : 0.0;           // (d may be NaN for a value past the data)
    nw += (uint32_t)__popcll(__ballot(ok));
    a.s1 += e;
    a.s2 = fma(e, e, a.s2);
    if (LIST) list_append(valid && !(fabs(d) <= L.lt), v, list, cnt, room);   // lc == shift
}

// statistics of a level all of whose values share one shift: the work-group's totals of the
// lanes' sums and the waves' counts give the mean and the sum of squared deviations (`tot`
// receives the totals: count and the sums of (value - shift) and its square)
__device__ __forceinline__ Part wave_counted_part(const Acc &a, uint32_t nw, double shift, Part *sh,
                                                  Part *tot = nullptr) {
    Part p = {(threadIdx.x & 63) == 0 ? (double)nw : 0.0, a.s1, a.s2};
    const Part t = block_sums(p, sh);
    if (tot) *tot = t;
    Part u = {0.0, 0.0, 0.0};
    if (t.n > 0.0) {
        u.n = t.n;
        u.mean = shift + t.mean / t.n;
        u.m2 = fmax(0.0, t.m2 - t.mean * (t.mean / t.n));
    }
    return u;
}

__global__ __launch_bounds__(kThreads, 4) void msd_kernel(const MsdArgs A) {
    __shared__ Part sh[4];
    __shared__ Level lv[SPD_MAX_LEVELS];
    __shared__ double t8[4];                   // level-8 value of each wave in the current tile
    __shared__ double slot_buf[4][64];         // per wave: this tile's level 3..8 values
    __shared__ int list_cnt[kWaves][kListLevels];  // values each wave listed in the last full read
    __shared__ int any_active, pass_mode;
    const int d = blockIdx.x;
    if (d >= A.n_dm) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform over the wave
    const int n = A.n_in;
    const int K = A.levels;
    const int klist = min(K, kListLevels);
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
    // this wave's list of level k
    auto list_of = [&](int k) { return wr + list_offset(n, k) + (int64_t)wave * list_room(n, k); };

    if (tid < K) {
        Level &L = lv[tid];
        L.shift = (double)xr[0] * (double)(1 << tid);   // pre-estimate: a value of the right size
        L.m = 0.0;
        L.lim = 0.0;
        L.sd = 0.0;
        L.kept = 0.0;
        L.lc = L.shift;
        L.lt = 0.0;
        L.nn = L.ns1 = L.ns2 = 0.0;
        L.active = 1;
        L.iters = 0;
        L.listed = 0;
    }
    __syncthreads();

    // Kinds of pass: the pre-estimate (mean and sd of a few tiles spread over the row, which
    // centre the first pass's lists and set their band), a full read (the first estimate, or a
    // rejection pass, both listing the values beyond the band), a list pass (the listed values
    // only).  The pre-estimate counts as no pass.
    enum { kProbe = 0, kRead = 1, kList = 2 };
    const int n_probe = min(n_tiles, kProbeTiles);
    int pass = -1;
    for (; pass <= A.max_iter; ++pass) {
        const bool probe = pass < 0;
        const bool first = pass <= 0;            // every valid value is kept
        if (tid == 0) {
            int a = 0;
            bool lists = pass > 0;
            for (int k = 0; k < K; ++k) a |= lv[k].active;
            for (int k = 0; k < klist; ++k)
                if (lv[k].active) lists = lists && band_covered(lv[k]);
            const int mode = probe ? kProbe : lists ? kList : kRead;
            if (mode == kRead && pass > 0) {
                for (int k = 0; k < klist; ++k) {
                    Level &L = lv[k];
                    L.lc = L.shift;                 // the current mean
                    L.lt = kListFrac * L.lim;
                }
            }
            any_active = pass <= 0 ? 1 : a;
            pass_mode = mode;
        }
        __syncthreads();
        if (!any_active) break;
        const int mode = pass_mode;
        const bool build = mode == kRead;
        // the samples are read again only while a level of 0..5 is open and its listed values do
        // not suffice (levels 6.. come from the workspace after the first pass)
        bool read_row = first;
        for (int k = 0; k < klist; ++k) read_row = read_row || lv[k].active;
        read_row = read_row && mode != kList;
        Acc a0, a1, a2, am;                      // levels 0, 1, 2 and this lane's level of 3..8
        uint32_t n0w = 0, n1w = 0, n2w = 0;      // the wave's kept counts of levels 0, 1, 2
        int lc_[kListLevels];                    // the wave's listed counts (full read)
#pragma unroll
        for (int k = 0; k < kListLevels; ++k) lc_[k] = 0;
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
        const bool onm = my_k < klist && (first || Lm.active);   // lanes of levels 3..5
        const bool arr = pass == 0 && my_k >= kArrFirst && my_k < K;   // lanes of 6..8

        auto fetch = [&](int tile, float4 &f) {
            const int s = tile * kTile + 4 * tid;
            if (vec && s + 3 < n) {
                // streamed once per full read: keep the cache for the lists being written
                typedef float v4f __attribute__((ext_vector_type(4)));
                const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(xr + s));
                f = make_float4(t.x, t.y, t.z, t.w);
            } else {
                f.x = s + 0 < n ? xr[s + 0] : 0.0f;
                f.y = s + 1 < n ? xr[s + 1] : 0.0f;
                f.z = s + 2 < n ? xr[s + 2] : 0.0f;
                f.w = s + 3 < n ? xr[s + 3] : 0.0f;
            }
        };
        // the pre-estimate reads tiles (i n_tiles) / n_probe, a full read every tile
        auto tile_at = [&](int i) { return probe ? (int)(((int64_t)i * n_tiles) / n_probe) : i; };
        const int n_read = probe ? n_probe : n_tiles;
        float4 nxt = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (read_row) fetch(tile_at(0), nxt);
        // one tile; FULL: every sample of the tile is inside the data (all tiles but the last),
        // so the per-value validity tests fold away; LIST: the values beyond the band are listed
        auto tile_body = [&](auto full_tag, auto list_tag, int tile, float4 cur) {
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr bool LIST = decltype(list_tag)::value;
            const int s = tile * kTile + 4 * tid;                // first sample of this thread
            const double v0[4] = {(double)cur.x, (double)cur.y, (double)cur.z, (double)cur.w};
            if (on0)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    take_w<LIST>(a0, n0w, L0, first, FULL || s + q < n, v0[q], list_of(0), lc_[0],
                                 list_room(n, 0));
            // levels 1, 2 within the thread
            const double v1a = v0[0] + v0[1], v1b = v0[2] + v0[3];
            if (on1) {
                take_w<LIST>(a1, n1w, L1, first, FULL || s + 2 <= n, v1a, list_of(1), lc_[1],
                             list_room(n, 1));
                take_w<LIST>(a1, n1w, L1, first, FULL || s + 4 <= n, v1b, list_of(1), lc_[1],
                             list_room(n, 1));
            }
            double v = v1a + v1b;
            if (on2)
                take_w<LIST>(a2, n2w, L2, first, FULL || s + 4 <= n, v, list_of(2), lc_[2],
                             list_room(n, 2));
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
            bool far = false;
            double mv = 0.0;
            if (onm) {
                mv = slots[lane];                                // written by this wave above
                const bool valid = FULL || !__builtin_isnan(mv);
                take(am, Lm, first, valid, mv);
                if (LIST) far = valid && !(fabs(mv - Lm.shift) <= Lm.lt);   // lc == shift
            }
            if (arr) {
                // the first pass stores levels 6..8 whole: level k's values of a tile in wave,
                // then lane order (lanes 56.., 60.., 62 hold levels 6, 7, 8)
                const int k = my_k;
                const int lane0 = k == 6 ? 56 : k == 7 ? 60 : 62;
                const int64_t i = (int64_t)tile * (kTile >> k) + wave * (256 >> k) + (lane - lane0);
                if (i < (n >> k)) wr[arr_offset(n, k) + i] = slots[lane];
            }
            if (LIST) {
                // each level's lanes form one run of the wave: append level by level (the
                // ballot and the counts stay in uniform control flow)
                const uint64_t b = __ballot(far);
                if (b) {
#pragma unroll
                    for (int k = 3; k < kListLevels; ++k) {
                        const uint64_t run = k == 3 ? 0xffffffffull : k == 4 ? 0xffffull << 32
                                                                    : 0xffull << 48;
                        const uint64_t bk = b & run;
                        if (bk) {
                            const int i = lc_[k] + count_below(bk);
                            if (far && my_k == k && i < list_room(n, k)) list_of(k)[i] = mv;
                            lc_[k] += __popcll(bk);
                        }
                    }
                }
            }
            // levels 9 and 10 (and the level-10 values the higher levels are built from): the
            // first pass writes them to the workspace
            if (pass == 0 && K > 9) {
                if (lane == 0) t8[wave] = v;
                __syncthreads();
                if (tid == 0) {
                    const int64_t i9 = (int64_t)tile * 2;
                    const double a9 = t8[0] + t8[1], b9 = t8[2] + t8[3];
                    double *w9 = wr + arr_offset(n, 9);
                    const int64_t n9 = n >> 9;
                    if (i9 < n9) w9[i9] = a9;
                    if (i9 + 1 < n9) w9[i9 + 1] = b9;
                    if (K > 10 && tile < (n >> 10)) w9[n9 + tile] = a9 + b9;
                }
                __syncthreads();
            }
        };
        for (int i = 0; read_row && i < n_read; ++i) {
            const int tile = tile_at(i);
            const float4 cur = nxt;
            if (i + 1 < n_read) fetch(tile_at(i + 1), nxt);      // in flight while this tile computes
            const bool full = (tile + 1) * kTile <= n;            // uniform over the work-group
            if (build) {
                if (full)
                    tile_body(std::true_type{}, std::true_type{}, tile, cur);
                else
                    tile_body(std::false_type{}, std::true_type{}, tile, cur);
            } else {
                if (full)
                    tile_body(std::true_type{}, std::false_type{}, tile, cur);
                else
                    tile_body(std::false_type{}, std::false_type{}, tile, cur);
            }
        }
        if (build && lane == 0)
            for (int k = 0; k < klist; ++k) list_cnt[wave][k] = lc_[k];
        if (pass == 0 && K > 11) {
            // levels 11.. from pairs of the level below, all in the workspace
            int64_t off_prev = arr_offset(n, 10), off = arr_offset(n, 11);
            for (int k = 11; k < K; ++k) {
                const int64_t cnt = (int64_t)(n >> k);
                for (int64_t i = tid; i < cnt; i += kThreads) wr[off + i] = wr[off_prev + 2 * i] + wr[off_prev + 2 * i + 1];
                off_prev = off;
                off += cnt;
                __syncthreads();
            }
        }
        __syncthreads();                          // list counts (and workspace levels) visible

        // merge the pass's statistics and update every level still being refined (the decision
        // to skip a level is uniform across the work-group)
        auto update_merged = [&](int k, const Part u) {
            if (tid == 0) update_level(lv[k], u, probe, first, A);
        };
        // the listed values of level k kept by the current estimate (every one in the first
        // pass): totals of the count and of the sums of (value - centre) and its square, in a
        // fixed order (the waves' lists in turn)
        auto list_sums = [&](int k, double centre) {
            const Level L = lv[k];
            const int room = list_room(n, k);
            Acc a;
            acc_reset(a);
            // the waves' lists one after another: entry j of the concatenation
            const double *l = wr + list_offset(n, k);
            const int c0 = min(list_cnt[0][k], room), c1 = min(list_cnt[1][k], room);
            const int c2 = min(list_cnt[2][k], room), c3 = min(list_cnt[3][k], room);
            const int p1 = c0, p2 = p1 + c1, p3 = p2 + c2, c = p3 + c3;
            for (int j0 = 0; j0 < c; j0 += 4 * kThreads) {
                double v[4];                     // four loads in flight, then their sums in order
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * kThreads + tid;
                    const int w = (j >= p1) + (j >= p2) + (j >= p3);
                    const int base = w == 0 ? 0 : w == 1 ? p1 : w == 2 ? p2 : p3;
                    v[u] = j < c ? l[(int64_t)w * room + (j - base)] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = j0 + u * kThreads + tid < c &&
                                    (first || fabs(v[u] - L.shift) <= L.lim);
                    const double e = ok ? v[u] - centre : 0.0;
                    a.n += ok ? 1 : 0;
                    a.s1 += e;
                    a.s2 = fma(e, e, a.s2);
                }
            }
            Part p = {(double)a.n, a.s1, a.s2};
            return block_sums(p, sh);
        };
        // full read: the unlisted values' statistics are the kept totals less the listed kept
        // values (all around the list centre)
        auto keep_unlisted = [&](int k, const Part &tot) {
            bool full = true;
            for (int w = 0; w < kWaves; ++w) full = full && list_cnt[w][k] <= list_room(n, k);
            Part ls = {0.0, 0.0, 0.0};
            if (full) ls = list_sums(k, lv[k].lc);
            if (tid == 0) {
                Level &S = lv[k];
                S.listed = full;
                S.nn = tot.n - ls.n;
                S.ns1 = tot.mean - ls.mean;
                S.ns2 = tot.m2 - ls.m2;
            }
        };
        if (mode == kList) {
            // a list pass: each wave takes levels wave, wave + 4, ... on its own (wave-only
            // reductions, the wave's lane 0 updates the level), one barrier at the end
            for (int k = wave; k < K; k += kWaves) {
                const Level L = lv[k];
                if (!L.active) continue;
                Part u = {0.0, 0.0, 0.0};
                if (k < klist) {
                    // the listed values: the four waves' lists one after another
                    const double *l = wr + list_offset(n, k);
                    const int room = list_room(n, k);
                    const int c0 = min(list_cnt[0][k], room), c1 = min(list_cnt[1][k], room);
                    const int c2 = min(list_cnt[2][k], room), c3 = min(list_cnt[3][k], room);
                    const int p1 = c0, p2 = p1 + c1, p3 = p2 + c2, c = p3 + c3;
                    Acc a;
                    acc_reset(a);
                    for (int j0 = 0; j0 < c; j0 += 4 * 64) {
                        double v[4];             // four loads in flight, then their sums in order
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int j = j0 + q * 64 + lane;
                            const int w = (j >= p1) + (j >= p2) + (j >= p3);
                            const int base = w == 0 ? 0 : w == 1 ? p1 : w == 2 ? p2 : p3;
                            v[q] = j < c ? l[(int64_t)w * room + (j - base)] : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool ok = j0 + q * 64 + lane < c && fabs(v[q] - L.shift) <= L.lim;
                            const double e = ok ? v[q] - L.lc : 0.0;
                            a.n += ok ? 1 : 0;
                            a.s1 += e;
                            a.s2 = fma(e, e, a.s2);
                        }
                    }
                    const Part t = wave_sums(Part{(double)a.n, a.s1, a.s2});
                    const double cnt = L.nn + t.n;
                    if (cnt > 0.0) {
                        const double s1 = L.ns1 + t.mean, s2 = L.ns2 + t.m2;
                        u.n = cnt;
                        u.mean = L.lc + s1 / cnt;
                        u.m2 = fmax(0.0, s2 - s1 * (s1 / cnt));
                    }
                } else {
                    // a level stored whole in the workspace
                    const int64_t cnt = (int64_t)(n >> k);
                    const double *vals = wr + arr_offset(n, k);
                    Acc a;
                    acc_reset(a);
                    for (int64_t i0 = 0; i0 < cnt; i0 += 4 * 64) {
                        double v[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int64_t i = i0 + q * 64 + lane;
                            v[q] = i < cnt ? vals[i] : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) take(a, L, false, i0 + q * 64 + lane < cnt, v[q]);
                    }
                    u = wave_merge(acc_part(a, L.shift));
                }
                if (lane == 0) update_level(lv[k], u, false, false, A);
            }
            __syncthreads();
            continue;
        }
        for (int k = 0; k < klist; ++k) {
            if (!(first || lv[k].active)) continue;
            if (k < 3) {
                const Acc &a = k == 0 ? a0 : k == 1 ? a1 : a2;
                const uint32_t nw = k == 0 ? n0w : k == 1 ? n1w : n2w;
                Part tot;
                const Part u = wave_counted_part(a, nw, lv[k].shift, sh, &tot);
                if (build) keep_unlisted(k, tot);
                update_merged(k, u);
            } else {
                Part p = {0.0, 0.0, 0.0};
                if (my_k == k) p = acc_part(am, lv[k].shift);
                const Part u = block_merge(p, sh);
                if (build) {
                    Part q = {0.0, 0.0, 0.0};
                    if (my_k == k) q = Part{(double)am.n, am.s1, am.s2};
                    keep_unlisted(k, block_sums(q, sh));
                }
                update_merged(k, u);
            }
            __syncthreads();
        }
        if (probe) continue;
        int64_t off = 0;
        for (int k = kArrFirst; k < K; ++k) {
            const int64_t cnt = (int64_t)(n >> k);
            const Level Lk = lv[k];
            if (first || Lk.active) {
                Acc a;
                acc_reset(a);
                for (int64_t i0 = 0; i0 < cnt; i0 += 4 * kThreads) {
                    double v[4];                 // four loads in flight, then their sums in order
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t i = i0 + u * kThreads + tid;
                        v[u] = i < cnt ? wr[off + i] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) take(a, Lk, first, i0 + u * kThreads + tid < cnt, v[u]);
                }
                update_merged(k, block_merge(acc_part(a, Lk.shift), sh));
                __syncthreads();
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
    // levels 9.. of every row (fewer than n_in / 256 values) and the lists of levels 0..8
    *bytes = (int64_t)n_dm * spdm::ws_row_doubles(n_in) * 8 + 256;
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
    a.ws_row = spdm::ws_row_doubles(n_in);
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
