// spd_search_noalloc: spd_search with its workspace in a fixed device array of the library,
// for callers that cannot allocate device memory.
//
// The workspace of spd_search (hand-off series of the cascade steps, pre-candidate slabs,
// peak-finder counters and offsets, and the planes when only candidates are requested) lives
// here in `scratch`, one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel: in host code that name is only a stand-in for the symbol.  The
// first call on a device, with that device current, resolves the device address of its copy
// with hipGetSymbolAddress and keeps it; every later call on that device uses the kept address.
//
// Nothing in the workspace needs clearing between calls: every slab count, survivor count,
// mask and per-wave total is written by the launch that produces it before any kernel reads it.
// Calls on one GPU share the array, so calls that overlap in time on one GPU (several streams or
// threads) race on it; such callers serialise their calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "spd.h"

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[SPD_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's copy of `scratch` (resolved once per device), or null with
// *err set to the HIP error.
void *scratch_ptr(int *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = (int)e;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = (int)hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? (int)e : (int)hipErrorInvalidSymbol;
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    *err = 0;
    return g_ptr[dev];
}

}  // namespace

namespace spd {
int record_hip_error(int err);   // spd_api.cpp: keeps the HIP text for spd_error_string
}

extern "C" int spd_search_noalloc(const spd_params *params, const float *x, int64_t ld,
                                  int32_t n_dm, int32_t n_in, int32_t n_out, int64_t t0,
                                  const float *mean, const float *sigma, float *snr,
                                  uint16_t *width, spd_candidate *cand, int64_t cand_cap,
                                  int64_t *cand_count, void *hip_stream) {
    spd_plan_info info;
    int st = spd_plan(params, n_dm, n_in, n_out, &info);
    if (st != SPD_OK) return st;
    if (info.workspace_bytes > (int64_t)SPD_NOALLOC_SCRATCH_BYTES) return SPD_EWORKSPACE;
    int err = 0;
    void *ws = scratch_ptr(&err);
    if (!ws) return spd::record_hip_error(err);
    return spd_search(params, x, ld, n_dm, n_in, n_out, t0, mean, sigma, snr, width, cand,
                      cand_cap, cand_count, ws, (int64_t)SPD_NOALLOC_SCRATCH_BYTES, hip_stream);
}
