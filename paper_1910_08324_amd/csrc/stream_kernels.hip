// Block ingestion of the streaming search (declared in include/spd_batch.h): a strided copy of
// rows of samples into a beam's device buffer.  One work-group per (row, 4096-column chunk); each
// lane moves four float4 (vector path) or sixteen floats with unit-stride accesses.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "spd.h"
#include "spd_batch.h"

namespace spds {

constexpr int kThreads = 256;
constexpr int kChunk = 4096;        // columns per work-group

template <bool VEC>
__global__ __launch_bounds__(kThreads) void copy_rows_kernel(float *dst, int64_t ld_dst,
                                                             const float *src, int64_t ld_src,
                                                             int32_t n_cols) {
    const int64_t r = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    float *d = dst + r * ld_dst + c0;
    const float *s = src + r * ld_src + c0;
    const int n = (int)min<int64_t>(kChunk, n_cols - c0);
    if (VEC) {
        // n is a multiple of 4 except in the row's last chunk; its tail is copied one by one
        const int n4 = n >> 2;
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = threadIdx.x + u * kThreads;
            if (q < n4) v[u] = reinterpret_cast<const float4 *>(s)[q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = threadIdx.x + u * kThreads;
            if (q < n4) reinterpret_cast<float4 *>(d)[q] = v[u];
        }
        for (int c = 4 * n4 + threadIdx.x; c < n; c += kThreads) d[c] = s[c];
    } else {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = threadIdx.x + u * kThreads;
            if (c < n) v[u] = s[c];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = threadIdx.x + u * kThreads;
            if (c < n) d[c] = v[u];
        }
    }
}

}  // namespace spds

extern "C" int spd_copy_rows(float *dst, int64_t ld_dst, const float *src, int64_t ld_src,
                             int32_t n_rows, int32_t n_cols, void *hip_stream) {
    if (n_rows < 0 || n_cols < 0 || n_rows > 65535) return SPD_EINVAL;
    if (n_rows == 0 || n_cols == 0) return SPD_OK;
    if (!dst || !src || ld_dst < n_cols || ld_src < n_cols) return SPD_EINVAL;
    const bool vec = (((uintptr_t)dst | (uintptr_t)src) & 15) == 0 && ((ld_dst | ld_src) & 3) == 0;
    const dim3 grid((unsigned)((n_cols + spds::kChunk - 1) / spds::kChunk), (unsigned)n_rows);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (vec)
        hipLaunchKernelGGL(spds::copy_rows_kernel<true>, grid, dim3(spds::kThreads), 0, st, dst,
                           ld_dst, src, ld_src, n_cols);
    else
        hipLaunchKernelGGL(spds::copy_rows_kernel<false>, grid, dim3(spds::kThreads), 0, st, dst,
                           ld_dst, src, ld_src, n_cols);
    return hipGetLastError() == hipSuccess ? SPD_OK : SPD_EHIP;
}
