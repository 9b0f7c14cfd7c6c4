// Drives the C-ABI layer's host code (built with the launch stubs) over many parameter sets and
// sizes under AddressSanitizer / UBSan: planning, width tables, the search entry points with
// stand-in device addresses (never dereferenced on the host), batches and the gated search.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "spd.h"
#include "spd_batch.h"

static int failures = 0;
#define CHECK(c)                                                                     \
    do {                                                                             \
        if (!(c)) {                                                                  \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);        \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

static spd_params make(int method, int l_end, int depth, int lmax, uint32_t flags, int seg, int lev) {
    static int32_t lm[1];
    lm[0] = lmax;
    spd_params p = {};
    p.method = method;
    p.l_end = l_end;
    p.igrid_depth = depth;
    p.boxdit_lmax = method == SPD_BOXDIT ? lm : nullptr;
    p.n_boxdit_lmax = method == SPD_BOXDIT ? 1 : 0;
    p.threshold = 5.0f;
    p.flags = flags;
    p.segment = seg;
    p.step_levels = lev;
    return p;
}

int main() {
    // stand-in device addresses: aligned, never dereferenced by the host code
    char *dev = reinterpret_cast<char *>(uintptr_t(1) << 40);
    const int lends[] = {1, 2, 7, 64, 256, 1000, 4096, 8192, 65535};
    const int sizes[][2] = {{1, 1}, {3, 5}, {17, 333}, {64, 4097}, {5, 70001}, {2, 262144}};
    int plans = 0;
    for (int method = 0; method < 3; ++method)
        for (int sub = 0; sub < 4; ++sub)
            for (int l_end : lends)
                for (uint32_t flags = 1; flags <= 3; ++flags)
                    for (auto &sz : sizes) {
                        const int depth = method == SPD_IGRID ? sub : 0;
                        const int lmax = 2 * (sub + 1) * 4;
                        if (method == SPD_EXHAUSTIVE && (sub > 0 || l_end > 8192)) continue;
                        spd_params p = make(method, l_end, depth, lmax, flags, 0, 0);
                        spd_plan_info info;
                        const int n_dm = sz[0], n = sz[1];
                        int st = spd_plan(&p, n_dm, n, n, &info);
                        if (st != SPD_OK) continue;
                        ++plans;
                        CHECK(info.n_levels >= 1 && info.n_levels <= SPD_MAX_LEVELS);
                        for (int i = 0; i < info.n_levels; ++i) {
                            int32_t buf[64], cnt = 0;
                            CHECK(spd_level_widths(&p, i, buf, 64, &cnt) == SPD_OK);
                            CHECK(cnt >= 1);
                        }
                        int64_t cnt_dummy = 0;
                        (void)cnt_dummy;
                        st = spd_search(&p, reinterpret_cast<float *>(dev), n, n_dm, n, n, 0,
                                        reinterpret_cast<float *>(dev), reinterpret_cast<float *>(dev),
                                        reinterpret_cast<float *>(dev), reinterpret_cast<uint16_t *>(dev),
                                        reinterpret_cast<spd_candidate *>(dev), 16,
                                        reinterpret_cast<int64_t *>(dev), dev, info.workspace_bytes,
                                        nullptr);
                        CHECK(st == SPD_OK);
                        // a workspace one byte short is refused before anything is enqueued
                        if (info.workspace_bytes > 0)
                            CHECK(spd_search(&p, reinterpret_cast<float *>(dev), n, n_dm, n, n, 0,
                                             reinterpret_cast<float *>(dev), reinterpret_cast<float *>(dev),
                                             reinterpret_cast<float *>(dev), reinterpret_cast<uint16_t *>(dev),
                                             reinterpret_cast<spd_candidate *>(dev), 16,
                                             reinterpret_cast<int64_t *>(dev), dev,
                                             info.workspace_bytes - 1, nullptr) == SPD_EWORKSPACE);
                    }
    // explicit launch shapes
    for (int seg = 256; seg <= 8192; seg *= 2)
        for (int lev = 1; lev <= 6; ++lev) {
            spd_params p = make(SPD_IGRID, 8192, 1, 0, 3, seg, lev);
            spd_plan_info info;
            if (spd_plan(&p, 8, 100000, 90000, &info) == SPD_OK) ++plans;
        }
    // a batch of uneven beams, candidates only, and its descriptor table in host memory
    {
        spd_params p = make(SPD_BOXDIT, 4096, 0, 16, SPD_WRITE_CANDIDATES, 0, 0);
        std::vector<spd_beam> beams(5);
        for (int b = 0; b < 5; ++b) {
            spd_beam &bm = beams[b];
            bm = spd_beam();
            bm.x = reinterpret_cast<float *>(dev);
            bm.n_dm = 3 + 7 * b;
            bm.n_in = bm.n_out = 5000 + 17001 * b;
            bm.ld = bm.n_in;
            bm.mean = bm.sigma = reinterpret_cast<float *>(dev);
            bm.cand = reinterpret_cast<spd_candidate *>(dev);
            bm.cand_cap = 8;
            bm.cand_count = reinterpret_cast<int64_t *>(dev);
        }
        int64_t ws = 0, tb = 0;
        CHECK(spd_batch_plan(&p, 5, beams.data(), &ws, &tb) == SPD_OK);
        std::vector<char> table(tb);
        CHECK(spd_batch_table(&p, 5, beams.data(), dev, table.data(), tb) == SPD_OK);
        CHECK(spd_batch_search(&p, 5, beams.data(), dev, dev, ws, 0, nullptr) == SPD_OK);
        CHECK(spd_batch_table(&p, 5, beams.data(), dev, table.data(), tb - 1) == SPD_EINVAL);
    }
    // the gated search
    {
        spd_params pl = make(SPD_IGRID, 512, 1, 0, SPD_WRITE_CANDIDATES, 0, 0);
        spd_params pe = make(SPD_EXHAUSTIVE, 512, 0, 0, 3, 0, 0);
        int64_t ws = 0;
        CHECK(spd_gated_plan(&pl, &pe, 100, 9000, 9000, 16, 4096, &ws) == SPD_OK);
        CHECK(spd_search_gated(&pl, &pe, reinterpret_cast<float *>(dev), 9000, 100, 9000, 9000, 0,
                               reinterpret_cast<float *>(dev), reinterpret_cast<float *>(dev),
                               reinterpret_cast<uint8_t *>(dev), 16, 4096, nullptr, nullptr,
                               reinterpret_cast<float *>(dev), reinterpret_cast<uint16_t *>(dev),
                               reinterpret_cast<spd_candidate *>(dev), 4,
                               reinterpret_cast<int64_t *>(dev), dev, ws, nullptr) == SPD_OK);
    }
    std::printf("plans %d, failures %d\n", plans, failures);
    return failures ? 1 : 0;
}
