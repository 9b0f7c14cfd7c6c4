// Noise statistics per DM trial (declared in include/spd_msd.h): robust mean and standard
// deviation with iterative outlier rejection, for the samples and for every power-of-two
// decimation of them.  One work-group per row, FP64 throughout.  Partial statistics
// (count, mean, sum of squared deviations) are accumulated per thread with single-value updates
// and merged pairwise with Chan, Golub & LeVeque's formula, in a fixed order.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "spd.h"
#include "spd_msd.h"

namespace spdm {

constexpr int kThreads = 256;

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

__device__ __forceinline__ void add(Part &p, double v) {
    p.n += 1.0;
    const double d = v - p.mean;
    p.mean += d / p.n;
    p.m2 += d * (v - p.mean);
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
    Part r = merge(merge(sh[0], sh[1]), merge(sh[2], sh[3]));
    return r;
}

struct MsdArgs {
    const float *x;
    int64_t ld;
    double *ws;          // per row: level k >= 1 series at offset n_in - (n_in >> (k - 1)) ...
    int64_t ws_row;      // doubles per row
    float *mean, *sigma, *rho, *level_sd;
    int32_t n_dm, n_in, levels, max_iter;
    double tau;
};

// value i of the level's series: level 0 reads the samples, later levels the workspace
__device__ __forceinline__ double value(const float *xr, const double *yk, int k, int64_t i) {
    return k == 0 ? (double)xr[i] : yk[i];
}

__global__ __launch_bounds__(kThreads) void msd_kernel(const MsdArgs A) {
    __shared__ Part sh[4];
    const int d = blockIdx.x;
    if (d >= A.n_dm) return;
    const float *xr = A.x + (int64_t)d * A.ld;
    double *wr = A.ws + (int64_t)d * A.ws_row;
    double sd0 = 0.0;
    int64_t off = 0;                 // workspace offset of the current level's series
    const double *prev = nullptr;    // previous level's series (level >= 2)
    for (int k = 0; k < A.levels; ++k) {
        const int64_t n = (int64_t)A.n_in >> k;
        double *yk = wr + off;
        if (k >= 1) {
            for (int64_t i = threadIdx.x; i < n; i += kThreads)
                yk[i] = (k == 1) ? (double)xr[2 * i] + (double)xr[2 * i + 1]
                                 : prev[2 * i] + prev[2 * i + 1];
            __syncthreads();
        }
        // first estimate over every value, then passes with rejection
        Part p = {0.0, 0.0, 0.0};
        for (int64_t i = threadIdx.x; i < n; i += kThreads) add(p, value(xr, yk, k, i));
        Part t = block_merge(p, sh);
        double m = t.mean;
        double sd = t.n > 1.0 ? sqrt(t.m2 / (t.n - 1.0)) : 0.0;
        double kept = t.n;
        for (int it = 0; it < A.max_iter; ++it) {
            const double lim = A.tau * sd;
            Part q = {0.0, 0.0, 0.0};
            for (int64_t i = threadIdx.x; i < n; i += kThreads) {
                const double v = value(xr, yk, k, i);
                if (fabs(v - m) <= lim) add(q, v);
            }
            const Part u = block_merge(q, sh);
            if (u.n == kept || u.n < 2.0) break;
            kept = u.n;
            m = u.mean;
            sd = sqrt(u.m2 / (u.n - 1.0));
        }
        if (k == 0) sd0 = sd;
        if (threadIdx.x == 0) {
            if (k == 0) {
                A.mean[d] = (float)m;
                A.sigma[d] = (float)sd;
            }
            if (A.rho) A.rho[(int64_t)d * A.levels + k] = (float)(sd / (sqrt((double)(1 << k)) * sd0));
            if (A.level_sd) A.level_sd[(int64_t)d * A.levels + k] = (float)sd;
        }
        if (k >= 1) {
            prev = yk;
            off += n;
        }
        __syncthreads();
    }
}

}  // namespace spdm

extern "C" {

int spd_msd_workspace(int32_t n_dm, int32_t n_in, int32_t levels, int64_t *bytes) {
    if (!bytes || n_dm < 1 || n_in < 2 || levels < 1 || levels > SPD_MAX_LEVELS ||
        ((int64_t)n_in >> (levels - 1)) < 2)
        return SPD_EINVAL;
    *bytes = (int64_t)n_dm * n_in * 8 + 256;   // levels 1.. need fewer than n_in doubles per row
    return SPD_OK;
}

int spd_msd(const float *x, int64_t ld, int32_t n_dm, int32_t n_in, int32_t levels, float tau,
            int32_t max_iter, float *mean, float *sigma, float *rho, float *level_sd,
            void *workspace, int64_t workspace_bytes, void *hip_stream) {
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
    a.ws_row = n_in;
    a.mean = mean;
    a.sigma = sigma;
    a.rho = rho;
    a.level_sd = level_sd;
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
