// C ABI of the boxcar single-pulse search (declared in include/spd.h): parameter validation,
// construction of each method's level tables, output geometry, workspace layout, and the launch
// sequence on the caller's stream.  Nothing here allocates device memory or synchronises.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "spd.h"
#include "spd_internal.h"

namespace {

using spd::kLossyChunk;
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
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// BoxDIT (Algorithm 1, Section 3.1): iteration k holds L^k_max boxcars on data decimated k
// times; its widths are off_k + m 2^k, m = 1..L^k_max, with off_k = sum_{j<k} 2^j L^j_max.  The
// shifted decimation x^{k+1}[n] = x^k[2n + L^k_max] + x^k[2n + L^k_max + 1] needs L^k_max even.
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
    } else if (p->method == SPD_IGRID) {
        st = build_igrid(p, s);
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

struct Layout {
    spd_plan_info info;
    int seg = 0, n_seg = 0, max_chunks = 0, lds_bytes = 0;
    int64_t n_slabs = 0, slabs_per_wave = 0;
    int n_waves = 0, slab_cap = 0, n_scale = 0, lds_scale = 0;
    int64_t off_scale = 0, off_mask = 0, off_cnt = 0, off_ent = 0, off_surv = 0, off_msk = 0;
    int64_t off_wtot = 0, off_woff = 0, off_Y = -1, off_W = -1;
    std::vector<int> cap, lds_y, lds_c, scale_off;
};

int make_layout(const spd_params *p, const Search &s, int32_t n_dm, int32_t n_in, int32_t n_out,
                Layout *L) {
    if (n_dm < 1 || n_in < 1 || n_out < 1 || n_out > n_in) return SPD_EINVAL;
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
    if (!lossy) {
        if (p->segment != 0 && p->segment != spd::kExhSlots) return SPD_EINVAL;
        L->seg = spd::kExhSlots;
    } else {
        const int64_t G = std::max<int64_t>(kLossyChunk, (int64_t)4 << K);
        const int64_t full = round_up(n_out, G);
        int64_t seg;
        if (p->segment != 0) {
            if (p->segment < 0 || p->segment % G) return SPD_EINVAL;
            seg = std::min<int64_t>(p->segment, full);
        } else {
            const int64_t want_items = ceil_div(8192, n_dm);          // fill 256 CUs several times
            seg = round_up(ceil_div(n_out, want_items), G);
            const int64_t floor_seg = std::min(full, round_up(4 * (int64_t)s.max_width, G));
            seg = std::max(seg, floor_seg);
            seg = std::min(seg, full);
        }
        if (seg > (1 << 30)) seg = (int64_t)1 << 30;
        L->seg = (int)seg;
    }
    L->n_seg = (int)ceil_div(n_out, L->seg);
    I.segment = L->seg;
    I.n_segments = L->n_seg;
    if ((int64_t)n_dm * L->n_seg > INT32_MAX) return SPD_EINVAL;

    // LDS windows of the cascade kernel
    L->cap.assign(nlev, 0);
    L->lds_y.assign(nlev, 0);
    L->lds_c.assign(nlev, 0);
    L->scale_off.assign(nlev, 0);
    int lds = 0, nscale = 0;
    for (int i = 0; i < nlev; ++i) {
        const Level &lv = s.levels[i];
        L->scale_off[i] = nscale;
        nscale += (int)lv.widths.size();
        if (!lossy) continue;
        const int umax = lv.units.back();
        const int cap = (int)round_up(ceil_div(kLossyChunk, (int64_t)1 << lv.shift) + umax + 16, 4);
        L->cap[i] = cap;
        L->lds_y[i] = lds;
        lds += cap;
        if (s.method == SPD_BOXDIT && i > 0) {
            L->lds_c[i] = lds;
            lds += cap;
        }
    }
    if (lossy) {
        L->lds_scale = lds;                          // 1/sqrt(L) table of the cascade kernel
        lds += (int)round_up(nscale, 4);
    } else {
        nscale = s.l_end;
    }
    L->n_scale = nscale;
    L->lds_bytes = lds * 4;
    if (L->lds_bytes > 60 * 1024) return SPD_EINVAL;
    L->max_chunks = lossy ? (int)ceil_div((int64_t)L->seg + s.max_width + ((int64_t)4 << K),
                                          kLossyChunk) + 4
                          : 0;

    // candidate bookkeeping
    L->slab_cap = lossy ? spd::kSlabCap : spd::kExhSlabCap;
    L->n_slabs = (int64_t)(lossy ? nlev : 1) * n_dm * L->n_seg;
    L->n_waves = (int)std::min<int64_t>(spd::kPeakWaves, L->n_slabs);
    L->slabs_per_wave = ceil_div(L->n_slabs, L->n_waves);
    L->n_waves = (int)ceil_div(L->n_slabs, L->slabs_per_wave);

    int64_t ws = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = ws;
        ws += round_up(std::max<int64_t>(bytes, 1), 256);
        return at;
    };
    // the exhaustive kernel's masked tail group reads up to kExhGroup entries past the tables
    L->off_scale = take(((int64_t)nscale + spd::kExhGroup) * 4);
    L->off_mask = take(s.dense ? 4 : (ceil_div(s.l_end, 32) + 4) * 4);
    L->off_cnt = take(L->n_slabs * 4);
    L->off_ent = take(L->n_slabs * L->slab_cap * 4);
    L->off_surv = take(L->n_slabs * 4);
    L->off_msk = take(L->n_slabs * 8);
    L->off_wtot = take((int64_t)L->n_waves * 8);
    L->off_woff = take((int64_t)L->n_waves * 8);
    if (!(p->flags & SPD_WRITE_PLANES)) {
        L->off_Y = take(I.plane_elems * 4);
        L->off_W = take(I.plane_elems * 2);
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
    P->Y = want_planes ? snr : reinterpret_cast<float *>(P->ws + P->L.off_Y);
    P->W = want_planes ? width : reinterpret_cast<uint16_t *>(P->ws + P->L.off_W);
    return SPD_OK;
}

int run_filter(const spd_params *params, const Prepared &P, const float *x, int64_t ld,
               int32_t n_dm, int32_t n_in, int32_t n_out, const float *mean, const float *sigma,
               void *hip_stream) {
    const Search &s = P.s;
    const Layout &L = P.L;
    const spd_plan_info &I = L.info;
    const bool want_cand = params->flags & SPD_WRITE_CANDIDATES;
    uint32_t *slab_cnt = reinterpret_cast<uint32_t *>(P.ws + L.off_cnt);
    uint32_t *slab_ent = reinterpret_cast<uint32_t *>(P.ws + L.off_ent);
    const int vec_ok = (((uintptr_t)x & 15) == 0) && (ld % 4 == 0);
    const int nlev = I.n_levels;
    if (s.method != SPD_EXHAUSTIVE) {
        spd::LossyArgs a;
        std::memset(&a, 0, sizeof(a));
        a.x = x;
        a.ld = ld;
        a.mean = mean;
        a.sigma = sigma;
        a.Y = P.Y;
        a.W = P.W;
        a.slab_cnt = slab_cnt;
        a.slab_ent = slab_ent;
        a.n_dm = n_dm;
        a.n_in = n_in;
        a.n_out = n_out;
        a.n_levels = nlev;
        a.seg = L.seg;
        a.n_seg = L.n_seg;
        a.max_chunks = L.max_chunks;
        a.vec_ok = vec_ok;
        a.want_cand = want_cand;
        a.n_scale = L.n_scale;
        a.lds_scale = L.lds_scale;
        a.threshold = params->threshold;
        for (int i = 0; i < nlev; ++i) {
            const Level &lv = s.levels[i];
            spd::LevelDesc &D = a.lv[i];
            D.cshift = lv.cshift;
            D.nw = (int)lv.units.size();
            D.umax = lv.units.back();
            D.ufull = (i + 1 < nlev) ? s.levels[i + 1].cshift : 0;
            D.base = lv.base;
            D.cap = L.cap[i];
            D.lds_y = L.lds_y[i];
            D.lds_c = L.lds_c[i];
            D.scale_off = L.scale_off[i];
            D.slots = (int)I.plane_slots[i];
            D.plane_off = I.plane_offset[i];
            D.pitch = I.plane_pitch[i];
            for (size_t j = 0; j < lv.units.size(); ++j) D.units[j] = (uint8_t)lv.units[j];
        }
        const int err = spd::launch_lossy(a, s.method == SPD_BOXDIT, L.lds_bytes, hip_stream);
        if (err) return hip_fail(err);
        return SPD_OK;
    }
    float *scale = reinterpret_cast<float *>(P.ws + L.off_scale);
    uint32_t *evalmask = reinterpret_cast<uint32_t *>(P.ws + L.off_mask);
    {
        spd::ScaleArgs a;
        a.scale = scale;
        a.n = L.n_scale;
        const int err = spd::launch_scales(a, hip_stream);
        if (err) return hip_fail(err);
    }
    if (!s.dense) {
        spd::MaskArgs m;
        std::memset(&m, 0, sizeof(m));
        m.evalmask = evalmask;
        m.n_words = (int)ceil_div(s.l_end, 32);
        for (int w : s.levels[0].widths) m.bits[(w - 1) >> 5] |= 1u << ((w - 1) & 31);
        const int err = spd::launch_evalmask(m, hip_stream);
        if (err) return hip_fail(err);
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
    a.evalmask = evalmask;
    a.slab_cnt = slab_cnt;
    a.slab_ent = slab_ent;
    a.pitch = I.plane_pitch[0];
    a.n_dm = n_dm;
    a.n_in = n_in;
    a.n_out = n_out;
    a.l_end = s.l_end;
    a.n_seg = L.n_seg;
    a.vec_ok = vec_ok;
    a.want_cand = want_cand;
    a.threshold = params->threshold;
    const int err = spd::launch_exhaustive(a, s.dense, hip_stream);
    if (err) return hip_fail(err);
    return SPD_OK;
}

int run_peaks(const spd_params *params, const Prepared &P, int32_t n_dm, int64_t t0,
              spd_candidate *cand, int64_t cand_cap, int64_t *cand_count, void *hip_stream) {
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
    a.n_seg = L.n_seg;
    a.seg = L.seg;
    a.threshold = params->threshold;
    for (int i = 0; i < I.n_levels; ++i) {
        a.level_shift[i] = I.level_shift[i];
        a.level_slots[i] = (int)I.plane_slots[i];
        a.level_pitch[i] = I.plane_pitch[i];
        a.level_off[i] = I.plane_offset[i];
    }
    const int err = spd::launch_peaks(a, hip_stream);
    if (err) return hip_fail(err);
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

}  // extern "C"
