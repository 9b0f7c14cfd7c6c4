// C ABI of the boxcar single-pulse search (declared in include/spd.h): parameter validation,
// construction of each method's level tables, output geometry, workspace layout, and the launch
// sequence on the caller's stream.  Nothing here allocates device memory or synchronises.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "spd.h"
#include "spd_batch.h"
#include "spd_internal.h"

namespace {

using spd::kMaxLevels;
using spd::kMaxLevelWidths;

struct Level {
    int shift = 0;            // boxcars every 2^shift samples
    int base = 0;             // raw offset of unit 0 (BoxDIT carried prefix width)
    int cshift = 0;           // cascade shift from the previous level, in its units
    std::vector<int> units;   // widths in units of 2^shift, ascending (lossy)
    std::vector<int> widths;  // widths in samples, ascending
};

struct Search {
    int method = 0;
    int l_end = 0;
    bool dense = true;        // exhaustive over every width 1..l_end
    std::vector<Level> levels;
    int max_width = 0;
    int fam = 0;              // compiled-in width patterns of the kernel (see family_mask)
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// BoxDIT (Algorithm 1, Section 3.1): iteration k holds L^k_max boxcars on data decimated k
// times; its widths are off_k + m 2^k, m = 1..L^k_max, with off_k = sum_{j<k} 2^j L^j_max.  The
// shifted decimation x^{k+1}[n] = x^k[2n + L^k_max] + x^k[2n + L^k_max + 1] needs L^k_max even.
// Exhaustive search: 256-slot items per wave when the caller leaves it to the library.  Four
// items amortise the window fill over a short row's few items and keep the next item's samples
// in flight; measured on gfx950 they gain 25-40% on rows of at most 16384 slots from L_end 128
// to 512, as long as the launch keeps some 32 waves per compute unit.  Elsewhere one item per
// wave is as fast or faster.
int exh_default_items(int32_t l_end, int32_t n_dm, int32_t n_out) {
    const int64_t waves4 = (int64_t)n_dm * ceil_div(ceil_div(n_out, spd::kExhSlots), 4);
    if (waves4 < 8192) return 1;
    if (l_end >= 128 && l_end <= spd::kExhBlock && n_out <= 16384) return 4;
    return 1;
}

int build_boxdit(const spd_params *p, Search *s) {
    if (!p->boxdit_lmax || p->n_boxdit_lmax < 1) return SPD_EINVAL;
    for (int i = 0; i < p->n_boxdit_lmax; ++i) {
        const int L = p->boxdit_lmax[i];
        if (L < 2 || L > kMaxLevelWidths || (L & 1)) return SPD_EINVAL;
    }
    int64_t off = 0;
    int prevL = 0;
    for (int k = 0;; ++k) {
        if (k >= kMaxLevels) return SPD_EINVAL;
        const int L = p->boxdit_lmax[std::min(k, p->n_boxdit_lmax - 1)];
        if (off + ((int64_t)1 << k) > p->l_end) break;
        Level lv;
        lv.shift = k;
        lv.base = (int)off;
        lv.cshift = k == 0 ? 0 : prevL;
        for (int m = 1; m <= L; ++m) {
            const int64_t w = off + ((int64_t)m << k);
            if (w > p->l_end) break;
            lv.units.push_back(m);
            lv.widths.push_back((int)w);
        }
        s->levels.push_back(lv);
        off += (int64_t)L << k;
        prevL = L;
    }
    return SPD_OK;
}

// IGRID IG(d) with P layers (Section 3.2): step j has base width W = 2^j and boxcars every
// max(1, W/P) samples; the tree traversal to depth d adds widths W + q W/2^d, q < 2^d (Table 1).
// Level 0 holds all steps with W <= P (every sample); level k >= 1 holds the single step with
// W = P 2^k, whose widths are (P + q P/2^d) 2^k.
int build_igrid(const spd_params *p, Search *s) {
    const int d = p->igrid_depth;
    if (d < 0 || d > 4) return SPD_EINVAL;
    const int P = p->igrid_layers ? p->igrid_layers : (1 << (d + 1));
    if (!is_pow2(P) || P < (1 << d) || P > 64) return SPD_EINVAL;
    Level l0;
    std::vector<char> on(2 * P + 1, 0);
    for (int W = 1; W <= P && W <= p->l_end; W <<= 1) {
        const int inc = std::max(1, W >> d);
        for (int q = 0; q < (1 << d); ++q) {
            const int w = W + q * inc;
            if (w < 2 * W && w <= p->l_end) on[w] = 1;
        }
    }
    for (int w = 1; w <= 2 * P; ++w)
        if (on[w]) {
            l0.units.push_back(w);
            l0.widths.push_back(w);
        }
    s->levels.push_back(l0);
    for (int k = 1;; ++k) {
        if ((int64_t)P << k > p->l_end) break;
        if (k >= kMaxLevels) return SPD_EINVAL;
        Level lv;
        lv.shift = k;
        for (int q = 0; q < (1 << d); ++q) {
            const int u = P + q * (P >> d);
            if (((int64_t)u << k) > p->l_end) break;
            lv.units.push_back(u);
            lv.widths.push_back(u << k);
        }
        s->levels.push_back(lv);
    }
    return SPD_OK;
}

int build_search(const spd_params *p, Search *s) {
    if (!p) return SPD_EINVAL;
    if (p->l_end < 1 || p->l_end > SPD_MAX_LEND) return SPD_EINVAL;
    if (!(p->flags & (SPD_WRITE_PLANES | SPD_WRITE_CANDIDATES))) return SPD_EINVAL;
    if (p->flags & ~(uint32_t)(SPD_WRITE_PLANES | SPD_WRITE_CANDIDATES)) return SPD_EINVAL;
    if (!std::isfinite(p->threshold)) return SPD_EINVAL;
    s->method = p->method;
    s->l_end = p->l_end;
    int st = SPD_OK;
    if (p->method == SPD_EXHAUSTIVE) {
        Level lv;
        if (p->widths && p->n_widths > 0) {
            if (p->l_end > SPD_MAX_LIST_LEND) return SPD_EINVAL;
            int prev = 0;
            for (int i = 0; i < p->n_widths; ++i) {
                const int w = p->widths[i];
                if (w <= prev || w > p->l_end) return SPD_EINVAL;
                lv.widths.push_back(w);
                prev = w;
            }
            s->dense = false;
        } else {
            if (p->widths || p->n_widths) return SPD_EINVAL;
            for (int w = 1; w <= p->l_end; ++w) lv.widths.push_back(w);
        }
        lv.units = lv.widths;
        s->levels.push_back(lv);
    } else if (p->method == SPD_BOXDIT) {
        st = build_boxdit(p, s);
        if (st == SPD_OK) {
            bool same = true;
            for (int i = 1; i < p->n_boxdit_lmax; ++i) same = same && p->boxdit_lmax[i] == p->boxdit_lmax[0];
            const int L0 = p->boxdit_lmax[0];
            if (same) s->fam = L0 == 8 ? 4 : L0 == 16 ? 5 : L0 == 32 ? 6 : 0;
        }
    } else if (p->method == SPD_IGRID) {
        st = build_igrid(p, s);
        const int P = p->igrid_layers ? p->igrid_layers : (1 << (p->igrid_depth + 1));
        const int d = p->igrid_depth;
        if (d >= 1 && d <= 3 && P == (1 << (d + 1))) s->fam = d;
        if (d == 0 && P == 1) s->fam = 7;
    } else {
        return SPD_EINVAL;
    }
    if (st != SPD_OK) return st;
    if (s->levels.empty() || s->levels.size() > (size_t)kMaxLevels) return SPD_EINVAL;
    for (const Level &lv : s->levels) {
        if (lv.widths.empty()) return SPD_EINVAL;
        if (p->method != SPD_EXHAUSTIVE &&
            (lv.units.size() > (size_t)kMaxLevelWidths || lv.units.back() > 255))
            return SPD_EINVAL;
        s->max_width = std::max(s->max_width, lv.widths.back());
    }
    return SPD_OK;
}

constexpr int kGroupC = spd::kGroup;
constexpr int kDefaultStepLevels = 4;

// One launch of the cascade kernel: levels k0 .. k0+J-1 over tiles of T units of its input.
struct StepPlan {
    int k0 = 0, J = 0, T = 0, tiles = 0, maxu = 8, lds_bytes = 0, lds_sc = 0;
    int nth = spd::kStepThreads;   // threads per work-group of the single-beam launch
    bool has_out = false;
    int64_t in_len = 0;        // units of the input series per row
    int64_t out_len = 0;       // units handed to the next step per row
    int64_t ld_out = 0;        // row pitch of the handed-on series in the workspace
    int64_t off_out = -1, off_cout = -1;
    spd::StepLevel lv[spd::kStepMaxLevels + 1];
    float rtab[spd::kStepMaxLevels][spd::kMaxLevelWidths] = {{0}};
};

struct Layout {
    spd_plan_info info;
    std::vector<StepPlan> steps;
    int exh_nseg = 0;
    int exh_per = 1;          // 256-slot items per wave
    int64_t n_slabs = 0, slabs_per_wave = 0;
    int n_waves = 0, slab_cap = 0, n_scale = 0;
    int64_t slab_base[kMaxLevels + 1] = {0};
    int tiles_per_row[kMaxLevels] = {0};
    int tile_slots[kMaxLevels] = {0};
    int64_t off_scale = 0, off_mask = 0, off_cnt = 0, off_ent = 0, off_surv = 0, off_msk = 0;
    int64_t off_wtot = 0, off_woff = 0, off_Y = -1, off_W = -1;
    int64_t cnt_off[kMaxLevels] = {0};
    int cnt_stride[kMaxLevels] = {0};
    int64_t off_rec = -1;     // records of the cascade steps (lossy, candidates only)
    int64_t off_amask = -1;   // above-threshold bits of every slot (lossy, candidates only)
    int64_t amask_words = 0;
    int64_t mask_off[kMaxLevels] = {0};
    int mask_wps[kMaxLevels] = {0};
    int64_t scale_ld = 0;
};

// Lay out one step: units each level must form in a tile, LDS buffers, 1/sqrt(L) tables.
// Returns the LDS bytes, or -1 if the step cannot be formed with these J and T.
int plan_step(const Search &s, int k0, int J, int T, StepPlan *st) {
    const int K = (int)s.levels.size() - 1;
    st->k0 = k0;
    st->J = J;
    st->T = T;
    st->has_out = (k0 + J <= K);
    int umax_all = 1;
    for (int j = 0; j < J; ++j) umax_all = std::max(umax_all, s.levels[k0 + j].units.back());
    st->maxu = (int)round_up(umax_all, 4);
    if ((T >> (J - 1)) % spd::kGroup || (st->has_out && (T >> J) < 1)) return -1;
    const int top = st->has_out ? J : J - 1;
    int64_t N[spd::kStepMaxLevels + 1] = {0};
    for (int j = top; j >= 0; --j) {
        int64_t need = 0;
        if (j < J) need = (T >> j) + s.levels[k0 + j].units.back() - 1;
        else need = T >> J;
        if (j < top) need = std::max<int64_t>(need, 2 * N[j + 1] + s.levels[k0 + j + 1].cshift);
        N[j] = j == 0 ? round_up(need, 4) : need;          // the window is loaded as float4
    }
    // One unit buffer and one carry buffer per tile: level j+1 is written over the part of
    // level j that the tile has finished with (the units a batch of groups has read), so the
    // buffers only need to hold the largest level.
    int64_t capv[spd::kStepMaxLevels + 1] = {0};
    int64_t ybuf = 0, cbuf = 0;
    for (int j = 0; j <= top; ++j) {
        spd::StepLevel &L = st->lv[j];
        std::memset(&L, 0, sizeof(L));
        const Level &lv = s.levels[k0 + j];
        L.k = lv.shift;
        L.cshift = j == 0 ? 0 : lv.cshift;
        L.n_units = (int)N[j];
        capv[j] = round_up((j < J) ? std::max<int64_t>(N[j], (T >> j) + st->maxu + 8) : N[j], 4);
        ybuf = std::max(ybuf, capv[j]);
        L.base = lv.base;
        if (j < J) {
            L.umax = lv.units.back();
            L.ufull = (k0 + j + 1 <= K) ? s.levels[k0 + j + 1].cshift : 0;
            for (int u : lv.units) L.evalmask |= 1ull << (u - 1);
            if (s.fam && L.evalmask == spd::family_mask(s.fam, 1)) L.pattern = 1;
            else if (s.fam && L.evalmask == spd::family_mask(s.fam, 2)) L.pattern = 2;
            // 1/sqrt(L) for every unit count of the level, rounded once from FP64
            for (int u = 1; u <= L.umax; ++u)
                st->rtab[j][u - 1] = (float)(1.0 / std::sqrt((double)lv.base + std::ldexp((double)u, lv.shift)));
            if (s.method == SPD_BOXDIT && !(j == 0 && k0 == 0))
                cbuf = std::max<int64_t>(cbuf, round_up(T >> j, 4));
        }
    }
    for (int j = 0; j <= top; ++j) {
        st->lv[j].lds_y = 0;
        st->lv[j].lds_c = (int)ybuf;
        capv[j] = ybuf;
    }
    const int64_t lds = ybuf + cbuf;
    st->lds_bytes = (int)(lds * 4);
    // a halo longer than the tile means the tile is too short for these levels
    if (N[0] - T > T) return -1;
    // every LDS read of the kernel must land on a unit the tile formed:
    //   cascade  y_j[n] <- y_{j-1}[2n + cshift], y_{j-1}[2n + cshift + 1],  n < N_j
    //   banks    y_j[m + u], m < T >> j, u < umax_j;  float4 window reads up to m + umax_j + 7
    for (int j = 1; j <= top; ++j)
        if (2 * (N[j] - 1) + st->lv[j].cshift + 1 >= N[j - 1]) return -1;
    // in-place formation: the halo units of level j+1 (n >= (S_j - cshift) / 2, formed after
    // the last batch of level j) are written below every unit of level j that they read
    for (int j = 1; j <= top; ++j) {
        const int64_t Sp = T >> (j - 1);
        const int64_t cs = st->lv[j].cshift;
        const int64_t n_start = std::max<int64_t>(0, (Sp - cs) >> 1);
        if (N[j] > 2 * n_start + cs) return -1;
    }
    for (int j = 0; j < J; ++j) {
        const int64_t last_used = (T >> j) - 1 + st->lv[j].umax - 1;
        const int64_t um = st->lv[j].umax;
        const int64_t last_read = (T >> j) - kGroupC +
                                  std::max(((um - 1) / 4) * 4 + 7, round_up(um + 3, 4) - 1);
        if (last_used >= N[j] || last_read >= capv[j]) return -1;
    }
    return st->lds_bytes;
}

// ref_out: the output length the tile lengths are sized for (0: n_out).  A batch passes its
// longest beam's, so that every beam gets the same launch geometry.
int make_layout(const spd_params *p, const Search &s, int32_t n_dm, int32_t n_in, int32_t n_out,
                Layout *L, int64_t ref_out = 0) {
    if (n_dm < 1 || n_in < 1 || n_out < 1 || n_out > n_in) return SPD_EINVAL;
    if (ref_out <= 0) ref_out = n_out;
    if (p->rho && (p->n_rho < 1 || p->n_rho > SPD_MAX_LEVELS)) return SPD_EINVAL;
    if (!p->rho && p->n_rho != 0) return SPD_EINVAL;
    if ((int64_t)n_in > (int64_t)INT32_MAX - (1 << 20)) return SPD_EINVAL;
    std::memset(&L->info, 0, sizeof(L->info));
    spd_plan_info &I = L->info;
    const int nlev = (int)s.levels.size();
    const int K = s.levels.back().shift;
    I.n_levels = nlev;
    I.top_level = K;
    I.max_width = s.max_width;
    I.required_halo = s.max_width - 1;
    int64_t off = 0;
    for (int i = 0; i < nlev; ++i) {
        const int k = s.levels[i].shift;
        I.level_shift[i] = k;
        I.level_nwidths[i] = (int)s.levels[i].widths.size();
        I.plane_slots[i] = ceil_div(n_out, (int64_t)1 << k);
        I.plane_pitch[i] = round_up(I.plane_slots[i], 64);
        I.plane_offset[i] = off;
        off += I.plane_pitch[i] * n_dm;
    }
    I.plane_elems = off;

    const bool lossy = s.method != SPD_EXHAUSTIVE;
    int64_t ws = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = ws;
        ws += round_up(std::max<int64_t>(bytes, 1), 256);
        return at;
    };
    if (!lossy) {
        // a wave takes 1, 2 or 4 consecutive 256-slot items; more than one only while every
        // width fits one LDS window, so that the window slides on from item to item
        const int per = p->segment == 0 ? exh_default_items(s.l_end, n_dm, n_out)
                                         : p->segment / spd::kExhSlots;
        if (p->segment != 0 && (p->segment % spd::kExhSlots != 0 ||
                                (per != 1 && per != 2 && per != spd::kExhItemsPerWave)))
            return SPD_EINVAL;
        if (per > 1 && s.l_end > spd::kExhBlock) return SPD_EINVAL;
        if (p->step_levels != 0) return SPD_EINVAL;
        L->exh_nseg = (int)ceil_div(n_out, spd::kExhSlots);
        L->exh_per = per;
        I.segment = spd::kExhSlots * per;
        I.n_segments = (int)ceil_div(L->exh_nseg, per);
        L->tiles_per_row[0] = L->exh_nseg;
        L->tile_slots[0] = spd::kExhSlots;
        L->n_scale = s.l_end;
        L->slab_cap = spd::kExhSlabCap;
    } else {
        // chain of cascade steps, each covering up to kStepMaxLevels levels
        const bool fixed_T = p->segment != 0;
        int T = fixed_T ? p->segment : 4096;
        if (T < 256 || T > 32768 || T % 256) return SPD_EINVAL;
        if (p->step_levels < 0 || p->step_levels > spd::kStepMaxLevels) return SPD_EINVAL;
        // library's choice of levels per launch: 4 (measured on MI355X: moving levels 4 and 5,
        // whose tiles keep few threads busy, into the next launch beats the extra 1/16-sized
        // hand-off through HBM for every compiled-in family)
        const int jmax = p->step_levels ? p->step_levels : kDefaultStepLevels;
        int k0 = 0;
        int64_t in_len = n_in;
        while (k0 <= K) {
            StepPlan st;
            int J = std::min(jmax, K + 1 - k0);
            int Tj = T;
            // a step whose first level has fewer slots than a tile gets a shorter tile (a multiple
            // of 256), since one long tile per row would idle most of its threads; results do not
            // depend on the tile length.  A fixed segment still sets the first launch's tile.
            if (k0 > 0 || !fixed_T) {
                const int64_t want =
                    std::max<int64_t>(256, round_up(ceil_div(ref_out, (int64_t)1 << k0), 256));
                if (want < Tj) {
                    StepPlan trial;
                    int l2 = plan_step(s, k0, J, (int)want, &trial);
                    if (l2 >= 0 && p->rho) l2 += spd::kStepMaxLevels * spd::kMaxLevelWidths * 4;
                    if (l2 >= 0 && l2 <= 60 * 1024) Tj = (int)want;
                }
            }
            int lds = -1;
            for (;;) {
                lds = plan_step(s, k0, J, Tj, &st);
                if (lds >= 0 && p->rho) {
                    // this row's width scales: kStepMaxLevels x kMaxLevelWidths floats after the buffers
                    st.lds_sc = st.lds_bytes / 4;
                    st.lds_bytes += spd::kStepMaxLevels * spd::kMaxLevelWidths * 4;
                    lds = st.lds_bytes;
                }
                if (lds >= 0 && lds <= 60 * 1024) break;
                if (J > 1) {
                    --J;
                } else if (!fixed_T && Tj > 256) {
                    Tj >>= 1;
                    J = std::min(jmax, K + 1 - k0);
                } else {
                    return SPD_EINVAL;
                }
            }
            st.in_len = in_len;
            // IG(1) tiles of at most kSmallTileMax units run on kSmallStepThreads: its light width
            // sets leave the launch bound by the plane writes, which go faster from more, smaller
            // work-groups; the denser sets are faster on kStepThreads
            st.nth = (s.fam == 1 && st.T <= spd::kSmallTileMax) ? spd::kSmallStepThreads
                                                                  : spd::kStepThreads;
            const int64_t slots0 = I.plane_slots[k0];
            int64_t tiles = ceil_div(slots0, st.T);
            if (st.has_out) {
                const int k1 = k0 + st.J;
                const int64_t usable = std::max<int64_t>(0, ((int64_t)n_in - s.levels[k1].base) >> k1);
                tiles = std::max(tiles, ceil_div(usable, st.T >> st.J));
                st.out_len = tiles * (st.T >> st.J);
                st.ld_out = round_up(st.out_len, 64);
            }
            if (tiles * n_dm > INT32_MAX) return SPD_EINVAL;
            st.tiles = (int)tiles;
            for (int j = 0; j < st.J; ++j) {
                L->tiles_per_row[k0 + j] = st.tiles;
                L->tile_slots[k0 + j] = st.T >> j;
                st.lv[j].slots = (int)I.plane_slots[k0 + j];
                st.lv[j].plane_off = I.plane_offset[k0 + j];
                st.lv[j].pitch = I.plane_pitch[k0 + j];
            }
            in_len = st.out_len;
            L->steps.push_back(st);
            k0 += st.J;
        }
        I.segment = L->steps[0].T;
        I.n_segments = L->steps[0].tiles;
        L->slab_cap = spd::kSlabCap;
        for (StepPlan &st : L->steps) {
            if (st.has_out) {
                st.off_out = take((int64_t)n_dm * st.ld_out * 4);
                if (s.method == SPD_BOXDIT) st.off_cout = take((int64_t)n_dm * st.ld_out * 4);
            }
        }
    }
    // the launches of the filter, in stream order
    auto add_launch = [&](int first, int nlv, int64_t in_units, int64_t out_units, int nth,
                          int tile) {
        const int i = I.n_launches++;
        I.launch_first_level[i] = first;
        I.launch_levels[i] = nlv;
        I.launch_in_units[i] = in_units;
        I.launch_out_units[i] = out_units;
        I.launch_threads[i] = nth;
        I.launch_tile[i] = tile;
    };
    if (lossy) {
        const int series = s.method == SPD_BOXDIT ? 2 : 1;   // decimated series (+ carried prefixes)
        for (const StepPlan &st : L->steps)
            add_launch(st.k0, st.J, st.k0 == 0 ? (int64_t)n_in : series * st.in_len,
                       st.has_out ? series * st.out_len : 0, st.nth, st.T);
    } else {
        add_launch(-1, 0, 0, 0, 256, 0);                          // 1/sqrt(L) table
        if (!s.dense) add_launch(-1, 0, 0, 0, 256, 0);            // width mask
        add_launch(0, 1, n_in, 0, 64, 0);
    }
    if (I.n_launches > SPD_MAX_LAUNCHES) return SPD_EINVAL;

    L->slab_base[0] = 0;
    for (int k = 0; k < nlev; ++k)
        L->slab_base[k + 1] = L->slab_base[k] + (int64_t)n_dm * L->tiles_per_row[k];
    L->n_slabs = L->slab_base[nlev];
    for (StepPlan &st : L->steps)
        for (int j = 0; j < st.J; ++j) st.lv[j].slab_base = L->slab_base[st.k0 + j];
    // pre-candidate counts: a cascade launch keeps the counts of its levels for one tile side by
    // side; the exhaustive search has one level
    {
        int64_t cb = 0;
        for (StepPlan &st : L->steps) {
            for (int j = 0; j < st.J; ++j) {
                st.lv[j].cnt_off = cb + j;
                L->cnt_off[st.k0 + j] = cb + j;
                L->cnt_stride[st.k0 + j] = st.J;
            }
            cb += (int64_t)n_dm * st.tiles * st.J;
        }
        if (L->steps.empty()) {
            L->cnt_off[0] = 0;
            L->cnt_stride[0] = 1;
        }
    }
    L->n_waves = (int)std::min<int64_t>(spd::kPeakWaves, L->n_slabs);
    L->slabs_per_wave = ceil_div(L->n_slabs, L->n_waves);
    L->n_waves = (int)ceil_div(L->n_slabs, L->slabs_per_wave);

    // the exhaustive kernel's masked tail group reads up to kExhGroup entries past the tables;
    // with a sigma table every row has its own
    L->scale_ld = (!lossy && p->rho) ? (int64_t)L->n_scale + spd::kExhGroup : 0;
    L->off_scale = take(((int64_t)L->n_scale + spd::kExhGroup) * 4 * (L->scale_ld ? n_dm : 1));
    L->off_mask = take(s.dense ? 4 : (ceil_div(s.l_end, 32) + 4) * 4);
    L->off_cnt = take(L->n_slabs * 4);
    L->off_ent = take(L->n_slabs * L->slab_cap * 4);
    L->off_surv = take(L->n_slabs * 4);
    L->off_msk = take(L->n_slabs * 8);
    L->off_wtot = take((int64_t)L->n_waves * 8);
    L->off_woff = take((int64_t)L->n_waves * 8);
    if (!(p->flags & SPD_WRITE_PLANES)) {
        if (lossy) {
            // candidates only: no planes anywhere; the cascade leaves one bit per group of
            // kGroup slots (any of them above the threshold or not) and the peak finder forms
            // the few slot values it needs again from each step's record
            L->off_rec = take((int64_t)L->steps.size() * (int64_t)sizeof(spd::RecStep));
            int64_t words = 0;
            for (int k = 0; k < nlev; ++k) {
                L->mask_wps[k] = (int)ceil_div(ceil_div(L->tile_slots[k], spd::kGroup), 32);
                L->mask_off[k] = words;
                words += (int64_t)n_dm * L->tiles_per_row[k] * L->mask_wps[k];
            }
            L->off_amask = take(words * 4);
            L->amask_words = words;
            for (StepPlan &st : L->steps)
                for (int j = 0; j < st.J; ++j) {
                    st.lv[j].mask_off = L->mask_off[st.k0 + j];
                    st.lv[j].mask_wps = L->mask_wps[st.k0 + j];
                }
        } else {
            // the exhaustive search is bound by arithmetic: its planes go to the workspace
            L->off_Y = take(I.plane_elems * 4);
            L->off_W = take(I.plane_elems * 2);
        }
    }
    I.workspace_bytes = ws;
    return SPD_OK;
}

thread_local char g_errbuf[256];

int hip_fail(int err) {
    std::snprintf(g_errbuf, sizeof(g_errbuf), "HIP launch failed: %s", spd::hip_error_text(err));
    return SPD_EHIP;
}

}  // namespace

namespace spd {
int record_hip_error(int err) { return hip_fail(err); }
}  // namespace spd

extern "C" {

int spd_abi_version(void) { return SPD_ABI_VERSION; }

const char *spd_error_string(int status) {
    switch (status) {
        case SPD_OK: return "ok";
        case SPD_EINVAL: return "invalid argument";
        case SPD_EALIGN: return "misaligned argument (t0 must be a multiple of 2^K)";
        case SPD_EWORKSPACE: return "workspace missing or smaller than spd_plan_info.workspace_bytes";
        case SPD_EHIP: return g_errbuf[0] ? g_errbuf : "HIP launch failed";
        default: return "unknown status";
    }
}

int spd_plan(const spd_params *params, int32_t n_dm, int32_t n_in, int32_t n_out,
             spd_plan_info *out) {
    if (!out) return SPD_EINVAL;
    Search s;
    int st = build_search(params, &s);
    if (st != SPD_OK) return st;
    Layout L;
    st = make_layout(params, s, n_dm, n_in, n_out, &L);
    if (st != SPD_OK) return st;
    *out = L.info;
    return SPD_OK;
}

int spd_level_widths(const spd_params *params, int32_t level, int32_t *out, int32_t cap,
                     int32_t *n) {
    if (!n || cap < 0 || (cap > 0 && !out)) return SPD_EINVAL;
    Search s;
    const int st = build_search(params, &s);
    if (st != SPD_OK) return st;
    if (level < 0 || level >= (int)s.levels.size()) return SPD_EINVAL;
    const std::vector<int> &w = s.levels[level].widths;
    *n = (int32_t)w.size();
    for (int i = 0; i < (int)w.size() && i < cap; ++i) out[i] = w[i];
    return SPD_OK;
}

}  // extern "C"

namespace {

struct Prepared {
    Search s;
    Layout L;
    char *ws = nullptr;
    float *Y = nullptr;
    uint16_t *W = nullptr;
};

// Shared validation of spd_filter / spd_peaks / spd_search.
int prepare(const spd_params *params, int32_t n_dm, int32_t n_in, int32_t n_out, float *snr,
            uint16_t *width, void *workspace, int64_t workspace_bytes, Prepared *P) {
    int st = build_search(params, &P->s);
    if (st != SPD_OK) return st;
    st = make_layout(params, P->s, n_dm, n_in, n_out, &P->L);
    if (st != SPD_OK) return st;
    const bool want_planes = params->flags & SPD_WRITE_PLANES;
    if (want_planes && (!snr || !width)) return SPD_EINVAL;
    if (!workspace || workspace_bytes < P->L.info.workspace_bytes) return SPD_EWORKSPACE;
    if ((uintptr_t)workspace & 255) return SPD_EALIGN;
    if (want_planes && (((uintptr_t)snr & 15) || ((uintptr_t)width & 7))) return SPD_EALIGN;
    P->ws = static_cast<char *>(workspace);
    P->Y = want_planes ? snr : P->L.off_Y >= 0 ? reinterpret_cast<float *>(P->ws + P->L.off_Y) : nullptr;
    P->W = want_planes ? width : P->L.off_W >= 0 ? reinterpret_cast<uint16_t *>(P->ws + P->L.off_W) : nullptr;
    return SPD_OK;
}

// The fields of a cascade launch's arguments that do not depend on the beam.
void fill_step_shared(const spd_params *params, const Search &s, const StepPlan &st, size_t si,
                      spd::StepArgs *a) {
    std::memset(a, 0, sizeof(*a));
    a->T = st.T;
    a->J = st.J;
    a->has_out = st.has_out;
    a->normalise = si == 0;
    a->carry = s.method == SPD_BOXDIT;
    a->want_cand = (params->flags & SPD_WRITE_CANDIDATES) != 0;
    a->threshold = params->threshold;
    a->rho = params->rho;
    a->ld_rho = params->n_rho;
    a->n_rho = params->n_rho;
    a->lds_sc = st.lds_sc;
    a->write_planes = (params->flags & SPD_WRITE_PLANES) != 0;
    a->nth = st.nth;
    a->rec = nullptr;
    for (int j = 0; j <= st.J && j <= spd::kStepMaxLevels; ++j) a->lv[j] = st.lv[j];
    std::memcpy(a->rtab, st.rtab, sizeof(a->rtab));
}

// HIP events recorded before the first launch and after each launch (spd_filter_timed).
struct LaunchMarks {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> ev;
    int mark() {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return (int)err;
        ev.push_back(e);
        return (int)hipEventRecord(e, stream);
    }
    ~LaunchMarks() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// Tile gating of a search (spd_search_gated): the tile flag map and which tiles a pass keeps.
struct Gate {
    const uint8_t *flag = nullptr;   // [n_row_tiles][n_col_tiles]
    int tile_rows = 0, tile_len = 0, n_col_tiles = 0;
    int mode = 0;                    // peak finder: 1 = unflagged tiles, 2 = flagged tiles
    const int64_t *base = nullptr;   // candidates written before this pass's list
};

int run_filter(const spd_params *params, const Prepared &P, const float *x, int64_t ld,
               int32_t n_dm, int32_t n_in, int32_t n_out, const float *mean, const float *sigma,
               void *hip_stream, LaunchMarks *marks = nullptr, const Gate *gate = nullptr) {
    auto mark = [&]() { return marks ? marks->mark() : 0; };
    if (P.L.off_amask >= 0) {
        // candidates only: the cascade sets only the bits of slots above the threshold (this
        // clearing is not one of the filter's listed launches)
        const int err = spd::launch_fill_u32(reinterpret_cast<uint32_t *>(P.ws + P.L.off_amask),
                                             P.L.amask_words, 0u, hip_stream);
        if (err) return hip_fail(err);
    }
    if (const int err = mark()) return hip_fail(err);
    const Search &s = P.s;
    const Layout &L = P.L;
    const spd_plan_info &I = L.info;
    const bool want_cand = params->flags & SPD_WRITE_CANDIDATES;
    uint32_t *slab_cnt = reinterpret_cast<uint32_t *>(P.ws + L.off_cnt);
    uint32_t *slab_ent = reinterpret_cast<uint32_t *>(P.ws + L.off_ent);
    const int vec_ok = (((uintptr_t)x & 15) == 0) && (ld % 4 == 0);
    if (s.method != SPD_EXHAUSTIVE) {
        const float *in = x;
        int64_t ld_in = ld;
        const float *cin = nullptr;

        for (size_t si = 0; si < L.steps.size(); ++si) {
            const StepPlan &st = L.steps[si];
            spd::StepArgs a;
            fill_step_shared(params, s, st, si, &a);
            a.in = in;
            a.cin = cin;
            a.out = st.has_out ? reinterpret_cast<float *>(P.ws + st.off_out) : nullptr;
            a.cout = (st.has_out && st.off_cout >= 0) ? reinterpret_cast<float *>(P.ws + st.off_cout)
                                                       : nullptr;
            a.mean = mean;
            a.sigma = sigma;
            a.Y = P.Y;
            a.W = P.W;
            a.slab_cnt = slab_cnt;
            a.slab_ent = slab_ent;
            a.ld_in = ld_in;
            a.ld_cin = ld_in;
            a.ld_out = st.ld_out;
            a.n_dm = n_dm;
            a.n_in = n_in;
            a.in_len = (int32_t)st.in_len;
            a.n_tiles = st.tiles;
            a.vec_ok = si == 0 ? vec_ok : 1;
            if (L.off_rec >= 0) a.rec = reinterpret_cast<spd::RecStep *>(P.ws + L.off_rec) + si;
            if (L.off_amask >= 0) a.amask = reinterpret_cast<uint32_t *>(P.ws + L.off_amask);
            const int err = spd::launch_step(a, s.fam, st.lds_bytes, hip_stream);
            if (err) return hip_fail(err);
            if (const int e2 = mark()) return hip_fail(e2);
            in = a.out;
            ld_in = st.ld_out;
            cin = a.cout;
        }
        return SPD_OK;
    }
    float *scale = reinterpret_cast<float *>(P.ws + L.off_scale);
    uint32_t *evalmask = reinterpret_cast<uint32_t *>(P.ws + L.off_mask);
    {
        spd::ScaleArgs a;
        std::memset(&a, 0, sizeof(a));
        a.scale = scale;
        a.n = L.n_scale;
        a.rho = params->rho;
        a.ld_rho = params->n_rho;
        a.n_rho = params->n_rho;
        a.n_rows = n_dm;
        a.row_ld = L.scale_ld;
        const int err = spd::launch_scales(a, hip_stream);
        if (err) return hip_fail(err);
        if (const int e2 = mark()) return hip_fail(e2);
    }
    if (!s.dense) {
        spd::MaskArgs m;
        std::memset(&m, 0, sizeof(m));
        m.evalmask = evalmask;
        m.n_words = (int)ceil_div(s.l_end, 32);
        for (int w : s.levels[0].widths) m.bits[(w - 1) >> 5] |= 1u << ((w - 1) & 31);
        const int err = spd::launch_evalmask(m, hip_stream);
        if (err) return hip_fail(err);
        if (const int e2 = mark()) return hip_fail(e2);
    }
    spd::ExhArgs a;
    std::memset(&a, 0, sizeof(a));
    a.x = x;
    a.ld = ld;
    a.mean = mean;
    a.sigma = sigma;
    a.Y = P.Y;
    a.W = P.W;
    a.scale = scale;
    a.scale_ld = L.scale_ld;
    a.evalmask = evalmask;
    a.slab_cnt = slab_cnt;
    a.slab_ent = slab_ent;
    a.pitch = I.plane_pitch[0];
    a.n_dm = n_dm;
    a.n_in = n_in;
    a.n_out = n_out;
    a.l_end = s.l_end;
    a.n_seg = L.exh_nseg;
    a.segs_per_wave = L.exh_per;
    a.vec_ok = vec_ok;
    a.want_cand = want_cand;
    a.threshold = params->threshold;
    if (gate) {
        a.tile_flag = gate->flag;
        a.tile_rows = gate->tile_rows;
        a.tile_len = gate->tile_len;
        a.n_col_tiles = gate->n_col_tiles;
    }
    const int err = spd::launch_exhaustive(a, s.dense, hip_stream);
    if (err) return hip_fail(err);
    if (const int e2 = mark()) return hip_fail(e2);
    return SPD_OK;
}

spd::PeakArgs peak_args(const spd_params *params, const Prepared &P, int32_t n_dm, int64_t t0,
                        spd_candidate *cand, int64_t cand_cap, int64_t *cand_count) {
    const Layout &L = P.L;
    const spd_plan_info &I = L.info;
    spd::PeakArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Y = P.Y;
    a.W = P.W;
    a.slab_cnt = reinterpret_cast<uint32_t *>(P.ws + L.off_cnt);
    a.slab_ent = reinterpret_cast<uint32_t *>(P.ws + L.off_ent);
    a.surv = reinterpret_cast<uint32_t *>(P.ws + L.off_surv);
    a.mask = reinterpret_cast<uint64_t *>(P.ws + L.off_msk);
    a.wave_tot = reinterpret_cast<int64_t *>(P.ws + L.off_wtot);
    a.wave_off = reinterpret_cast<int64_t *>(P.ws + L.off_woff);
    a.cand = cand;
    a.cand_cap = cand_cap;
    a.cand_count = cand_count;
    a.t0 = t0;
    a.n_slabs = L.n_slabs;
    a.slabs_per_wave = L.slabs_per_wave;
    a.n_waves = L.n_waves;
    a.slab_cap = L.slab_cap;
    a.n_levels = I.n_levels;
    a.n_dm = n_dm;
    a.threshold = params->threshold;
    for (int i = 0; i < I.n_levels; ++i) {
        a.level_shift[i] = I.level_shift[i];
        a.level_slots[i] = (int)I.plane_slots[i];
        a.level_pitch[i] = I.plane_pitch[i];
        a.level_off[i] = I.plane_offset[i];
        a.tiles_per_row[i] = L.tiles_per_row[i];
        a.tile_slots[i] = L.tile_slots[i];
    }
    for (int i = 0; i <= I.n_levels; ++i) a.slab_base[i] = L.slab_base[i];
    for (int i = 0; i < I.n_levels; ++i) {
        a.cnt_off[i] = L.cnt_off[i];
        a.cnt_stride[i] = L.cnt_stride[i];
    }
    a.rec = nullptr;
    if (L.off_amask >= 0) {
        a.amask = reinterpret_cast<const uint32_t *>(P.ws + L.off_amask);
        for (int i = 0; i < I.n_levels; ++i) {
            a.mask_off[i] = L.mask_off[i];
            a.mask_wps[i] = L.mask_wps[i];
        }
    }
    if (L.off_rec >= 0) {
        a.rec = reinterpret_cast<const spd::RecStep *>(P.ws + L.off_rec);
        for (size_t si = 0; si < L.steps.size(); ++si)
            for (int j = 0; j < L.steps[si].J; ++j) {
                a.level_step[L.steps[si].k0 + j] = (int8_t)si;
                a.level_j[L.steps[si].k0 + j] = (int8_t)j;
            }
    }
    return a;
}

int run_peaks(const spd_params *params, const Prepared &P, int32_t n_dm, int64_t t0,
              spd_candidate *cand, int64_t cand_cap, int64_t *cand_count, void *hip_stream,
              const Gate *gate = nullptr) {
    spd::PeakArgs a = peak_args(params, P, n_dm, t0, cand, cand_cap, cand_count);
    if (gate) {
        a.tile_flag = gate->flag;
        a.flag_mode = gate->mode;
        a.tile_rows = gate->tile_rows;
        a.tile_len = gate->tile_len;
        a.n_col_tiles = gate->n_col_tiles;
        a.base_count = gate->base;
    }
    const int err = spd::launch_peaks(a, hip_stream);
    if (err) return hip_fail(err);
    return SPD_OK;
}


// ---------------------------------------------------------------------------------------
// Batches of beams (spd_batch.h)
// ---------------------------------------------------------------------------------------
struct BatchPlan {
    Search s;
    std::vector<Layout> L;
    std::vector<int64_t> ws_off;
    int64_t ws_total = 0;
    int64_t table_bytes = 0;
    int64_t base_off = 0;       // offset of the item_base arrays in the table
    int64_t peak_off = 0;       // offset of the per-beam peak-finder arguments
    int64_t wbase_off = 0;      // offset of the peak finder's wave_base array
    int64_t n_waves = 0;        // peak-finder waves of all beams
    int n_steps = 0;
};

int batch_plan(const spd_params *params, int32_t n_beams, const spd_beam *beams, BatchPlan *B) {
    if (!params || !beams || n_beams < 1 || n_beams > (1 << 16)) return SPD_EINVAL;
    if (params->method == SPD_EXHAUSTIVE || params->rho) return SPD_EINVAL;
    int st = build_search(params, &B->s);
    if (st != SPD_OK) return st;
    B->L.resize(n_beams);
    B->ws_off.resize(n_beams);
    int64_t off = 0, ref_out = 1;
    for (int b = 0; b < n_beams; ++b) ref_out = std::max<int64_t>(ref_out, beams[b].n_out);
    for (int b = 0; b < n_beams; ++b) {
        st = make_layout(params, B->s, beams[b].n_dm, beams[b].n_in, beams[b].n_out, &B->L[b],
                         ref_out);
        if (st != SPD_OK) return st;
        const std::vector<StepPlan> &S = B->L[b].steps;
        const std::vector<StepPlan> &S0 = B->L[0].steps;
        if (S.size() != S0.size()) return SPD_EINVAL;
        for (size_t i = 0; i < S.size(); ++i)
            if (S[i].k0 != S0[i].k0 || S[i].J != S0[i].J || S[i].T != S0[i].T ||
                S[i].lds_bytes != S0[i].lds_bytes)
                return SPD_EINVAL;
        B->ws_off[b] = off;
        off += round_up(B->L[b].info.workspace_bytes, 256);
    }
    B->n_steps = (int)B->L[0].steps.size();
    B->ws_total = off;
    B->base_off = round_up((int64_t)B->n_steps * n_beams * (int64_t)sizeof(spd::BeamView), 256);
    B->peak_off = round_up(B->base_off + (int64_t)B->n_steps * (n_beams + 1) * 8, 256);
    B->wbase_off = round_up(B->peak_off + (int64_t)n_beams * (int64_t)sizeof(spd::PeakArgs), 256);
    B->table_bytes = B->wbase_off + (int64_t)(n_beams + 1) * 8;
    B->n_waves = 0;
    for (int b = 0; b < n_beams; ++b) B->n_waves += B->L[b].n_waves;
    return SPD_OK;
}

// the beam's view of cascade step si: its buffers in the caller's memory and its workspace
spd::BeamView beam_view(const spd_params *params, const BatchPlan &B, const spd_beam &bm, int b,
                        int si, char *ws_base) {
    const Layout &L = B.L[b];
    const StepPlan &st = L.steps[si];
    char *ws = ws_base + B.ws_off[b];
    const bool planes = params->flags & SPD_WRITE_PLANES;
    spd::BeamView v;
    std::memset(&v, 0, sizeof(v));
    if (si == 0) {
        v.in = bm.x;
        v.ld_in = bm.ld;
        v.vec_ok = (((uintptr_t)bm.x & 15) == 0) && (bm.ld % 4 == 0);
    } else {
        const StepPlan &pv = L.steps[si - 1];
        v.in = reinterpret_cast<const float *>(ws + pv.off_out);
        v.cin = pv.off_cout >= 0 ? reinterpret_cast<const float *>(ws + pv.off_cout) : nullptr;
        v.ld_in = pv.ld_out;
        v.vec_ok = 1;
    }
    v.ld_cin = v.ld_in;
    v.out = st.has_out ? reinterpret_cast<float *>(ws + st.off_out) : nullptr;
    v.cout = (st.has_out && st.off_cout >= 0) ? reinterpret_cast<float *>(ws + st.off_cout) : nullptr;
    v.ld_out = st.ld_out;
    v.mean = bm.mean;
    v.sigma = bm.sigma;
    v.Y = planes ? bm.snr : nullptr;           // lossy only: candidates-only stores no planes
    v.W = planes ? bm.width : nullptr;
    v.rec = L.off_rec >= 0 ? reinterpret_cast<spd::RecStep *>(ws + L.off_rec) + si : nullptr;
    v.amask = L.off_amask >= 0 ? reinterpret_cast<uint32_t *>(ws + L.off_amask) : nullptr;
    for (int j = 0; j < st.J; ++j) {
        v.mask_off[j] = st.lv[j].mask_off;
        v.cnt_off[j] = st.lv[j].cnt_off;
    }
    v.slab_cnt = reinterpret_cast<uint32_t *>(ws + L.off_cnt);
    v.slab_ent = reinterpret_cast<uint32_t *>(ws + L.off_ent);
    v.n_dm = bm.n_dm;
    v.n_in = bm.n_in;
    v.in_len = (int32_t)st.in_len;
    v.n_tiles = st.tiles;
    for (int j = 0; j < st.J; ++j) {
        v.plane_off[j] = st.lv[j].plane_off;
        v.pitch[j] = st.lv[j].pitch;
        v.slab_base[j] = st.lv[j].slab_base;
        v.slots[j] = st.lv[j].slots;
    }
    return v;
}

// the single-beam view of beam b of a batch (its layout, workspace and planes)
Prepared beam_prepared(const spd_params *params, const BatchPlan &B, const spd_beam &bm, int b,
                       char *ws_base) {
    Prepared P;
    P.s = B.s;
    P.L = B.L[b];
    P.ws = ws_base + B.ws_off[b];
    const bool planes = params->flags & SPD_WRITE_PLANES;
    P.Y = planes ? bm.snr : nullptr;
    P.W = planes ? bm.width : nullptr;
    return P;
}

int check_beam(const spd_params *params, const BatchPlan &B, const spd_beam &bm, int b) {
    const bool planes = params->flags & SPD_WRITE_PLANES;
    const bool cands = params->flags & SPD_WRITE_CANDIDATES;
    if (!bm.x || !bm.mean || !bm.sigma || bm.ld < bm.n_in) return SPD_EINVAL;
    if (planes && (!bm.snr || !bm.width)) return SPD_EINVAL;
    if (planes && ((((uintptr_t)bm.snr) & 15) || (((uintptr_t)bm.width) & 7))) return SPD_EALIGN;
    if (cands && (bm.cand_cap < 0 || (bm.cand_cap > 0 && !bm.cand) || !bm.cand_count))
        return SPD_EINVAL;
    if (bm.t0 < 0 || (bm.t0 & (((int64_t)1 << B.L[b].info.top_level) - 1))) return SPD_EALIGN;
    return SPD_OK;
}

}  // namespace

extern "C" {

int spd_filter(const spd_params *params, const float *x, int64_t ld, int32_t n_dm, int32_t n_in,
               int32_t n_out, const float *mean, const float *sigma, float *snr, uint16_t *width,
               void *workspace, int64_t workspace_bytes, void *hip_stream) {
    Prepared P;
    int st = prepare(params, n_dm, n_in, n_out, snr, width, workspace, workspace_bytes, &P);
    if (st != SPD_OK) return st;
    if (!x || !mean || !sigma || ld < n_in) return SPD_EINVAL;
    return run_filter(params, P, x, ld, n_dm, n_in, n_out, mean, sigma, hip_stream);
}

int spd_filter_timed(const spd_params *params, const float *x, int64_t ld, int32_t n_dm,
                     int32_t n_in, int32_t n_out, const float *mean, const float *sigma,
                     float *snr, uint16_t *width, void *workspace, int64_t workspace_bytes,
                     void *hip_stream, float *launch_ms, int32_t cap, int32_t *n_launches) {
    if (!n_launches || cap < 0 || (cap > 0 && !launch_ms)) return SPD_EINVAL;
    Prepared P;
    int st = prepare(params, n_dm, n_in, n_out, snr, width, workspace, workspace_bytes, &P);
    if (st != SPD_OK) return st;
    if (!x || !mean || !sigma || ld < n_in) return SPD_EINVAL;
    LaunchMarks marks;
    marks.stream = static_cast<hipStream_t>(hip_stream);
    st = run_filter(params, P, x, ld, n_dm, n_in, n_out, mean, sigma, hip_stream, &marks);
    if (st != SPD_OK) return st;
    const int n = (int)marks.ev.size() - 1;
    hipError_t err = hipEventSynchronize(marks.ev.back());
    if (err != hipSuccess) return hip_fail((int)err);
    for (int i = 0; i < n && i < cap; ++i) {
        err = hipEventElapsedTime(&launch_ms[i], marks.ev[i], marks.ev[i + 1]);
        if (err != hipSuccess) return hip_fail((int)err);
    }
    *n_launches = n;
    return SPD_OK;
}

int spd_peaks(const spd_params *params, int32_t n_dm, int32_t n_in, int32_t n_out, int64_t t0,
              const float *snr, const uint16_t *width, spd_candidate *cand, int64_t cand_cap,
              int64_t *cand_count, void *workspace, int64_t workspace_bytes, void *hip_stream) {
    if (!params || !(params->flags & SPD_WRITE_CANDIDATES)) return SPD_EINVAL;
    Prepared P;
    int st = prepare(params, n_dm, n_in, n_out, const_cast<float *>(snr),
                     const_cast<uint16_t *>(width), workspace, workspace_bytes, &P);
    if (st != SPD_OK) return st;
    if (cand_cap < 0 || (cand_cap > 0 && !cand) || !cand_count) return SPD_EINVAL;
    if (t0 < 0 || (t0 & (((int64_t)1 << P.L.info.top_level) - 1))) return SPD_EALIGN;
    return run_peaks(params, P, n_dm, t0, cand, cand_cap, cand_count, hip_stream);
}

int spd_search(const spd_params *params, const float *x, int64_t ld, int32_t n_dm, int32_t n_in,
               int32_t n_out, int64_t t0, const float *mean, const float *sigma, float *snr,
               uint16_t *width, spd_candidate *cand, int64_t cand_cap, int64_t *cand_count,
               void *workspace, int64_t workspace_bytes, void *hip_stream) {
    Prepared P;
    int st = prepare(params, n_dm, n_in, n_out, snr, width, workspace, workspace_bytes, &P);
    if (st != SPD_OK) return st;
    const bool want_cand = params->flags & SPD_WRITE_CANDIDATES;
    if (!x || !mean || !sigma || ld < n_in) return SPD_EINVAL;
    if (want_cand && (cand_cap < 0 || (cand_cap > 0 && !cand) || !cand_count)) return SPD_EINVAL;
    if (t0 < 0 || (t0 & (((int64_t)1 << P.L.info.top_level) - 1))) return SPD_EALIGN;
    st = run_filter(params, P, x, ld, n_dm, n_in, n_out, mean, sigma, hip_stream);
    if (st != SPD_OK || !want_cand) return st;
    return run_peaks(params, P, n_dm, t0, cand, cand_cap, cand_count, hip_stream);
}

// ---------------------------------------------------------------------------------------
// Tile-gated search (spd.h: spd_gated_plan / spd_search_gated)
// ---------------------------------------------------------------------------------------
static int gated_check(const spd_params *lossy, const spd_params *exh, int32_t n_dm,
                       int32_t n_in, int32_t n_out, int32_t tile_rows, int32_t tile_len,
                       spd_plan_info *li, spd_plan_info *ei) {
    if (!lossy || !exh || lossy->method == SPD_EXHAUSTIVE || exh->method != SPD_EXHAUSTIVE)
        return SPD_EINVAL;
    if (!(lossy->flags & SPD_WRITE_CANDIDATES) || !(exh->flags & SPD_WRITE_CANDIDATES))
        return SPD_EINVAL;
    if (tile_rows < 1 || tile_len < 1024 || tile_len % 1024) return SPD_EINVAL;
    int st = spd_plan(lossy, n_dm, n_in, n_out, li);
    if (st != SPD_OK) return st;
    return spd_plan(exh, n_dm, n_in, n_out, ei);
}

int spd_gated_plan(const spd_params *lossy, const spd_params *exh, int32_t n_dm, int32_t n_in,
                   int32_t n_out, int32_t tile_rows, int32_t tile_len, int64_t *workspace_bytes) {
    if (!workspace_bytes) return SPD_EINVAL;
    spd_plan_info li, ei;
    const int st = gated_check(lossy, exh, n_dm, n_in, n_out, tile_rows, tile_len, &li, &ei);
    if (st != SPD_OK) return st;
    *workspace_bytes = round_up(li.workspace_bytes, 256) + round_up(ei.workspace_bytes, 256);
    return SPD_OK;
}

int spd_search_gated(const spd_params *lossy, const spd_params *exh, const float *x, int64_t ld,
                     int32_t n_dm, int32_t n_in, int32_t n_out, int64_t t0, const float *mean,
                     const float *sigma, const uint8_t *tile_flag, int32_t tile_rows,
                     int32_t tile_len, float *snr, uint16_t *width, float *exh_snr,
                     uint16_t *exh_width, spd_candidate *cand, int64_t cand_cap,
                     int64_t *cand_count, void *workspace, int64_t workspace_bytes,
                     void *hip_stream) {
    spd_plan_info li, ei;
    int st = gated_check(lossy, exh, n_dm, n_in, n_out, tile_rows, tile_len, &li, &ei);
    if (st != SPD_OK) return st;
    if (!tile_flag || !x || !mean || !sigma || ld < n_in) return SPD_EINVAL;
    if (cand_cap < 0 || (cand_cap > 0 && !cand) || !cand_count) return SPD_EINVAL;
    if (t0 < 0 || (t0 & (((int64_t)1 << li.top_level) - 1))) return SPD_EALIGN;
    const int64_t lw = round_up(li.workspace_bytes, 256);
    if (!workspace || workspace_bytes < lw + round_up(ei.workspace_bytes, 256)) return SPD_EWORKSPACE;
    Prepared PL, PE;
    st = prepare(lossy, n_dm, n_in, n_out, snr, width, workspace, lw, &PL);
    if (st != SPD_OK) return st;
    st = prepare(exh, n_dm, n_in, n_out, exh_snr, exh_width, static_cast<char *>(workspace) + lw,
                 workspace_bytes - lw, &PE);
    if (st != SPD_OK) return st;
    Gate g;
    g.flag = tile_flag;
    g.tile_rows = tile_rows;
    g.tile_len = tile_len;
    g.n_col_tiles = (int)ceil_div(n_out, tile_len);
    // the lossy search everywhere; its candidates outside the flagged tiles come first
    st = run_filter(lossy, PL, x, ld, n_dm, n_in, n_out, mean, sigma, hip_stream);
    if (st != SPD_OK) return st;
    g.mode = 1;
    st = run_peaks(lossy, PL, n_dm, t0, cand, cand_cap, cand_count, hip_stream, &g);
    if (st != SPD_OK) return st;
    // the exhaustive set on the flagged tiles only; its candidates follow
    st = run_filter(exh, PE, x, ld, n_dm, n_in, n_out, mean, sigma, hip_stream, nullptr, &g);
    if (st != SPD_OK) return st;
    g.mode = 2;
    g.base = cand_count;
    return run_peaks(exh, PE, n_dm, t0, cand, cand_cap, cand_count, hip_stream, &g);
}

int spd_batch_plan(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                   int64_t *workspace_bytes, int64_t *table_bytes) {
    if (!workspace_bytes || !table_bytes) return SPD_EINVAL;
    BatchPlan B;
    const int st = batch_plan(params, n_beams, beams, &B);
    if (st != SPD_OK) return st;
    *workspace_bytes = std::max<int64_t>(B.ws_total, 256);
    *table_bytes = B.table_bytes;
    return SPD_OK;
}

int spd_batch_table(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                    void *workspace, void *table, int64_t table_bytes) {
    BatchPlan B;
    const int st = batch_plan(params, n_beams, beams, &B);
    if (st != SPD_OK) return st;
    if (!workspace || !table || table_bytes < B.table_bytes) return SPD_EINVAL;
    if ((uintptr_t)workspace & 255) return SPD_EALIGN;
    char *t = static_cast<char *>(table);
    spd::BeamView *views = reinterpret_cast<spd::BeamView *>(t);
    int64_t *base = reinterpret_cast<int64_t *>(t + B.base_off);
    for (int si = 0; si < B.n_steps; ++si) {
        int64_t items = 0;
        for (int b = 0; b < n_beams; ++b) {
            views[(int64_t)si * n_beams + b] =
                beam_view(params, B, beams[b], b, si, static_cast<char *>(workspace));
            base[(int64_t)si * (n_beams + 1) + b] = items;
            items += (int64_t)beams[b].n_dm * B.L[b].steps[si].tiles;
        }
        base[(int64_t)si * (n_beams + 1) + n_beams] = items;
    }
    if (params->flags & SPD_WRITE_CANDIDATES) {
        spd::PeakArgs *pk = reinterpret_cast<spd::PeakArgs *>(t + B.peak_off);
        int64_t *wb = reinterpret_cast<int64_t *>(t + B.wbase_off);
        int64_t waves = 0;
        for (int b = 0; b < n_beams; ++b) {
            const Prepared P = beam_prepared(params, B, beams[b], b, static_cast<char *>(workspace));
            pk[b] = peak_args(params, P, beams[b].n_dm, beams[b].t0, beams[b].cand,
                              beams[b].cand_cap, beams[b].cand_count);
            wb[b] = waves;
            waves += B.L[b].n_waves;
        }
        wb[n_beams] = waves;
    }
    return SPD_OK;
}

int spd_batch_search(const spd_params *params, int32_t n_beams, const spd_beam *beams,
                     const void *table_dev, void *workspace, int64_t workspace_bytes,
                     int32_t grid, void *hip_stream) {
    BatchPlan B;
    int st = batch_plan(params, n_beams, beams, &B);
    if (st != SPD_OK) return st;
    if (!table_dev || grid < 0) return SPD_EINVAL;
    if ((uintptr_t)table_dev & 15) return SPD_EALIGN;
    if (!workspace || workspace_bytes < B.ws_total) return SPD_EWORKSPACE;
    if ((uintptr_t)workspace & 255) return SPD_EALIGN;
    for (int b = 0; b < n_beams; ++b) {
        st = check_beam(params, B, beams[b], b);
        if (st != SPD_OK) return st;
    }
    const char *t = static_cast<const char *>(table_dev);
    for (int b = 0; b < n_beams; ++b) {
        const Layout &L = B.L[b];
        if (L.off_amask < 0) continue;
        const int err = spd::launch_fill_u32(
            reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + B.ws_off[b] + L.off_amask),
            L.amask_words, 0u, hip_stream);
        if (err) return hip_fail(err);
    }
    for (int si = 0; si < B.n_steps; ++si) {
        const StepPlan &sp = B.L[0].steps[si];
        spd::StepBatchArgs a;
        fill_step_shared(params, B.s, sp, si, &a.s);
        a.beams = reinterpret_cast<const spd::BeamView *>(t) + (int64_t)si * n_beams;
        a.item_base = reinterpret_cast<const int64_t *>(t + B.base_off) + (int64_t)si * (n_beams + 1);
        a.n_beams = n_beams;
        int64_t items = 0;
        for (int b = 0; b < n_beams; ++b) items += (int64_t)beams[b].n_dm * B.L[b].steps[si].tiles;
        a.n_items = items;
        const int64_t g = grid > 0 ? std::min<int64_t>(grid, items) : std::min<int64_t>(items, INT32_MAX);
        const int err = spd::launch_step_batch(a, B.s.fam, sp.lds_bytes, (int)g, hip_stream);
        if (err) return hip_fail(err);
    }
    if (!(params->flags & SPD_WRITE_CANDIDATES)) return SPD_OK;
    // the peak finder of every beam: one launch per pass, arguments from the table
    spd::PeakBatchArgs pb;
    pb.tab = reinterpret_cast<const spd::PeakArgs *>(t + B.peak_off);
    pb.wave_base = reinterpret_cast<const int64_t *>(t + B.wbase_off);
    pb.n_waves = B.n_waves;
    pb.n_beams = n_beams;
    const int err = spd::launch_peaks_batch(pb, hip_stream);
    if (err) return hip_fail(err);
    return SPD_OK;
}

}  // extern "C"
