// Host-only stand-ins for the kernel launchers of spd_kernels.hip, so that the C-ABI layer
// (spd_api.cpp: parameter checks, width tables, tile planning, workspace carving, descriptor
// tables) can be built with g++ under AddressSanitizer / UBSan and driven without a GPU.
// Launches do nothing and report success; family_mask restates the compiled-in width patterns.
#include <cstdint>

#include "spd_internal.h"

namespace spd {
namespace {
constexpr uint64_t ig_l0(int P, int d) {
    uint64_t m = 0;
    for (int W = 1; W <= P; W <<= 1) {
        const int inc = (W >> d) > 1 ? (W >> d) : 1;
        for (int q = 0; q < (1 << d); ++q)
            if (W + q * inc < 2 * W) m |= 1ull << (W + q * inc - 1);
    }
    return m;
}
constexpr uint64_t ig_lk(int P, int d) {
    uint64_t m = 0;
    for (int q = 0; q < (1 << d); ++q) m |= 1ull << (P + q * (P >> d) - 1);
    return m;
}
constexpr uint64_t run(int L) { return L >= 64 ? ~0ull : ((1ull << L) - 1); }
}  // namespace

int launch_scales(const ScaleArgs &, void *) { return 0; }
int launch_evalmask(const MaskArgs &, void *) { return 0; }
int launch_step(const StepArgs &a, int, int lds_bytes, void *) {
    return (a.J < 1 || a.T < 1 || lds_bytes <= 0 || lds_bytes > 64 * 1024) ? 1 : 0;
}
int launch_step_batch(const StepBatchArgs &, int, int lds_bytes, int, void *) {
    return (lds_bytes <= 0 || lds_bytes > 64 * 1024) ? 1 : 0;
}
int launch_exhaustive(const ExhArgs &, bool, void *) { return 0; }
int launch_peaks(const PeakArgs &, void *) { return 0; }
int launch_peaks_batch(const PeakBatchArgs &, void *) { return 0; }
int launch_fill_u32(uint32_t *, int64_t, uint32_t, void *) { return 0; }
const char *hip_error_text(int) { return "stub"; }
uint64_t family_mask(int fam, int pattern) {
    switch (fam) {
        case 1: return pattern == 1 ? ig_l0(4, 1) : ig_lk(4, 1);
        case 2: return pattern == 1 ? ig_l0(8, 2) : ig_lk(8, 2);
        case 3: return pattern == 1 ? ig_l0(16, 3) : ig_lk(16, 3);
        case 4: return run(8);
        case 5: return run(16);
        case 6: return run(32);
        case 7: return 1;
        default: return 0;
    }
}
}  // namespace spd
