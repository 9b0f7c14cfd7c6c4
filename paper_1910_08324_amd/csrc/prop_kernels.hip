// Learned tile proposal on gfx950 (declared in include/spd_proposal.h): GPU tile generator,
// DIT-level features, and the forward / backward / Adam kernels of a three-layer 5-tap
// convolutional network in bfloat16 on MFMA (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.
//
// Activations are stored channel-last and padded: act[row][pos'][32] with pos' = pos + 2 and
// zero positions 0, 1, 258..261, so the 5 taps of output position p read the contiguous
// 5 x C_in values starting at act[row][p][0].  A convolution is then, per row, the GEMM
//     D[co][p] = sum_k W[co][k] B[k][p],   B[k][p] = act_flat[row][p C_in + k],  k = t C_in + ci,
// one 32 (channels) x 32 (positions) MFMA tile per wave and 16 values of k per instruction.
// The weight gradient is the same product with positions as the reduction index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "spd.h"
#include "spd_proposal.h"

namespace spdp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int ROWS = SPD_PROP_TILE_ROWS;
constexpr int LEN = SPD_PROP_TILE_LEN;
constexpr int POS = SPD_PROP_POS;
constexpr int RP = SPD_PROP_ROW_POS;
constexpr int FCH = SPD_PROP_FEAT_CH;
constexpr int CH = SPD_PROP_CH;
constexpr int TAPS = SPD_PROP_TAPS;
constexpr int KW1 = 48;                 // padded k of layer 1 (5 taps x 8 channels = 40)
constexpr int KW = TAPS * CH;           // 160
constexpr int MAX_PART_WAVES = 1024;    // waves of the weight-gradient passes

// bfloat16: the upper half of an IEEE binary32, rounded to nearest even
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two 32x32 -> 64-bit
// products, with the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------------------
struct Words {
    uint32_t a0, a1, a2, a3;
};

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &z0, float &z1) {
    float u = ((float)a + 1.0f) * 0x1p-32f;
    u = fminf(u, 1.0f);
    const float v = (float)b * 0x1p-32f;
    const float rad = sqrtf(-2.0f * logf(u));
    const float ang = 6.28318530717958647692f * v;
    z0 = rad * cosf(ang);
    z1 = rad * sinf(ang);
}

struct TileArgs {
    float *x;
    uint64_t seed;
    int64_t first_tile;
    int32_t n_tiles;
};

// one work-group per row; 256 threads x 4 blocks of 4 samples
__global__ __launch_bounds__(256) void tiles_kernel(const TileArgs A) {
    const int i = blockIdx.x / ROWS;
    const int r = blockIdx.x - i * ROWS;
    if (i >= A.n_tiles) return;
    const int64_t t = A.first_tile + i;
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)((uint64_t)t >> 32);
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    // pulse parameters of the tile (the same in every thread)
    const Words h = philox(0u, 0xFFFFFFFFu, tlo, thi, k0, k1);
    const int n_p = (int)(((uint64_t)h.a0 * 3u) >> 32);
    int prow[2] = {-1, -1}, pst[2] = {0, 0}, pw[2] = {0, 0};
    float pamp[2] = {0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (j < n_p) {
            const Words q = philox((uint32_t)(j + 1), 0xFFFFFFFFu, tlo, thi, k0, k1);
            prow[j] = (int)(((uint64_t)q.a0 * ROWS) >> 32);
            const int S = 1 + (int)(((uint64_t)q.a1 * 64u) >> 32);
            const float u = (float)((double)q.a2 * 0x1p-32);
            const float snr = (float)(6.0 + 24.0 * (double)u);
            pw[j] = S;
            pst[j] = (int)(((uint64_t)q.a3 * (uint64_t)(LEN - S + 1)) >> 32);
            pamp[j] = (float)((double)snr / sqrt((double)S));
        }
    }
    float *xr = A.x + (int64_t)blockIdx.x * LEN;
    for (int b = threadIdx.x; b < LEN / 4; b += 256) {
        const Words w = philox((uint32_t)b, (uint32_t)r, tlo, thi, k0, k1);
        float z[4];
        box_muller(w.a0, w.a1, z[0], z[1]);
        box_muller(w.a2, w.a3, z[2], z[3]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (prow[j] == r) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int s = 4 * b + q;
                    if (s >= pst[j] && s < pst[j] + pw[j]) z[q] += pamp[j];
                }
            }
        }
        *reinterpret_cast<float4 *>(xr + 4 * b) = make_float4(z[0], z[1], z[2], z[3]);
    }
}

// ---------------------------------------------------------------------------------------
// Features: thread p of a row's work-group sums level-4 unit p (16 samples); coarser levels
// are pairwise sums across lanes (butterflies of 2, 4, 8, 16 lanes, inside one wave).
// ---------------------------------------------------------------------------------------
struct FeatArgs {
    const float *x;
    int64_t ld;
    const float *mean;
    const float *sigma;
    uint16_t *feat;
    int32_t n_rows;
};

__global__ __launch_bounds__(256) void features_kernel(const FeatArgs A) {
    const int r = blockIdx.x;
    const int p = threadIdx.x;
    if (r >= A.n_rows) return;
    const float *xr = A.x + (int64_t)r * A.ld + 16 * p;
    const float mu = A.mean[r];
    const float inv = 1.0f / A.sigma[r];
    float y4 = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4 *>(xr + 4 * q);
        y4 += (v.x - mu) * inv;
        y4 += (v.y - mu) * inv;
        y4 += (v.z - mu) * inv;
        y4 += (v.w - mu) * inv;
    }
    const float y5 = y4 + __shfl_xor(y4, 1);
    const float y6 = y5 + __shfl_xor(y5, 2);
    const float y7 = y6 + __shfl_xor(y6, 4);
    const float y8 = y7 + __shfl_xor(y7, 8);
    // unit variance under white noise: divide level k by 2^(k/2)
    const uint16_t c0 = to_bf16(y4 * 0.25f);
    const uint16_t c1 = to_bf16(y5 * 0.17677669529663688f);
    const uint16_t c2 = to_bf16(y6 * 0.125f);
    const uint16_t c3 = to_bf16(y7 * 0.088388347648318441f);
    const uint16_t c4 = to_bf16(y8 * 0.0625f);
    uint16_t *fr = A.feat + (int64_t)r * RP * FCH;
    *reinterpret_cast<uint4 *>(fr + (p + 2) * FCH) =
        make_uint4((uint32_t)c0 | ((uint32_t)c1 << 16), (uint32_t)c2 | ((uint32_t)c3 << 16),
                   (uint32_t)c4, 0u);
    if (p < RP - POS) {
        const int pad = p < 2 ? p : POS + p;          // positions 0, 1, 258 .. 261
        *reinterpret_cast<uint4 *>(fr + pad * FCH) = make_uint4(0u, 0u, 0u, 0u);
    }
}

// ---------------------------------------------------------------------------------------
// Weights in bfloat16 for the MFMA operands: forward rows W[co][t C_in + ci] (layer 1 padded
// to k = 48), and for the input gradient the flipped transpose Wt[ci][t' 32 + co] =
// W[co][4 - t'][ci].
// ---------------------------------------------------------------------------------------
struct WB {
    uint16_t *w1, *w2, *w3, *w2t, *w3t;
};

__global__ void prep_weights_kernel(const float *params, WB o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < CH * KW1) {
        const int co = i / KW1, k = i - co * KW1;
        o.w1[i] = k < TAPS * FCH ? to_bf16(params[SPD_PROP_OFF_W1 + co * TAPS * FCH + k]) : 0;
    }
    if (i < CH * KW) {
        o.w2[i] = to_bf16(params[SPD_PROP_OFF_W2 + i]);
        o.w3[i] = to_bf16(params[SPD_PROP_OFF_W3 + i]);
        const int ci = i / KW, k = i - ci * KW;
        const int tp = k / CH, co = k - tp * CH;
        const int src = co * KW + (TAPS - 1 - tp) * CH + ci;
        o.w2t[i] = to_bf16(params[SPD_PROP_OFF_W2 + src]);
        o.w3t[i] = to_bf16(params[SPD_PROP_OFF_W3 + src]);
    }
}

// ---------------------------------------------------------------------------------------
// Convolution as an MFMA GEMM.  MODE 0: out = relu(conv + bias).  MODE 1 (input gradient):
// out = conv(dz, Wt) where prev > 0, else 0.  Work-group = half a row (128 positions), one
// 32 x 32 output tile per wave.
// ---------------------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t *in;        // [rows][RP][CI]
    const uint16_t *w;         // [32][KS 16]
    const float *bias;         // MODE 0
    const uint16_t *prev;      // MODE 1: activations whose ReLU masks the gradient
    uint16_t *out;             // [rows][RP][32]
    int32_t rows;
};

template <int CI, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const ConvArgs A) {
    constexpr int KS = (TAPS * CI + 15) / 16;
    constexpr int KWC = KS * 16;
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int r = blockIdx.x >> 1;
    const int half = blockIdx.x & 1;
    if (r >= A.rows) return;
    const int p0 = half * 128 + wave * 32;
    const int h = l >> 5;
    const int n = l & 31;
    const uint16_t *inr = A.in + (int64_t)r * RP * CI;
    bf16x8 wa[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) wa[s] = load8(A.w + n * KWC + 16 * s + 8 * h);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const bf16x8 b = load8(inr + (p0 + n) * CI + 16 * s + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[s], b, acc, 0, 0, 0);
    }
    // D[co][pos]: lane l, register i -> co = 8 (i / 4) + 4 h + i % 4, pos = p0 + n
    const int64_t ro = ((int64_t)r * RP + p0 + n + 2) * CH;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        uint16_t hv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 8 * g + 4 * h + j;
            float v = acc[4 * g + j];
            if (MODE == 0) {
                v = fmaxf(v + A.bias[co], 0.0f);
            } else {
                v = from_bf16(A.prev[ro + co]) > 0.0f ? v : 0.0f;
            }
            hv[j] = to_bf16(v);
        }
        *reinterpret_cast<uint2 *>(A.out + ro + 8 * g + 4 * h) =
            make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16),
                       (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
    }
    // zero pads of the output row: positions 0, 1 (first half) and 258 .. 261 (second half)
    if (half == 0 && wave == 0 && l < 16) {
        *reinterpret_cast<uint2 *>(A.out + (int64_t)r * RP * CH + 4 * l) = make_uint2(0u, 0u);
    }
    if (half == 1 && wave == 3 && l < 32) {
        *reinterpret_cast<uint2 *>(A.out + ((int64_t)r * RP + POS + 2) * CH + 4 * l) =
            make_uint2(0u, 0u);
    }
}

// ---------------------------------------------------------------------------------------
// Read-out, tile logit (log-mean-exp over the tile's positions) and, when training, the loss
// and the gradient of the read-out: one work-group per tile, thread p takes position p of
// all 64 rows.
// ---------------------------------------------------------------------------------------
struct HeadArgs {
    const uint16_t *a3;
    const float *params;
    const float *labels;       // null: inference
    float *s;                  // [rows][POS] scores
    float *logits;             // may be null
    float *loss_t;             // [n_tiles]
    float *hpart;              // [n_tiles][33]: d wh, d bh
    uint16_t *dz3;             // [rows][RP][32]
    int32_t n_tiles;
};

__device__ __forceinline__ float block_max(float v, float *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__device__ __forceinline__ float block_sum(float v, float *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__device__ __forceinline__ void load_act(const uint16_t *p, float a[CH]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p + 8 * q);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            a[8 * q + 2 * e] = __uint_as_float(w[e] << 16);
            a[8 * q + 2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
        }
    }
}

__global__ __launch_bounds__(256) void head_kernel(const HeadArgs A) {
    __shared__ float sh[4];
    const int t = blockIdx.x;
    const int p = threadIdx.x;
    if (t >= A.n_tiles) return;
    const float *wh = A.params + SPD_PROP_OFF_WH;
    const float bh = A.params[SPD_PROP_OFF_BH];
    float w[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) w[c] = wh[c];
    float mx = -__builtin_huge_valf();
    for (int j = 0; j < ROWS; ++j) {
        const int64_t row = (int64_t)t * ROWS + j;
        float a[CH];
        load_act(A.a3 + (row * RP + p + 2) * CH, a);
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < CH; ++c) s += w[c] * a[c];
        s += bh;
        A.s[row * POS + p] = s;
        mx = fmaxf(mx, s);
    }
    mx = block_max(mx, sh);
    float se = 0.0f;
    for (int j = 0; j < ROWS; ++j) se += expf(A.s[((int64_t)t * ROWS + j) * POS + p] - mx);
    se = block_sum(se, sh);
    const float lse = mx + logf(se);
    const float logit = lse - 9.70406052783923f;               // log(64 * 256)
    if (p == 0 && A.logits) A.logits[t] = logit;
    if (!A.labels) return;
    const float y = A.labels[t];
    const float sig = 1.0f / (1.0f + expf(-logit));
    const float dlogit = (sig - y) / (float)A.n_tiles;
    if (p == 0) A.loss_t[t] = fmaxf(logit, 0.0f) + log1pf(expf(-fabsf(logit))) - y * logit;
    float gw[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) gw[c] = 0.0f;
    float gb = 0.0f;
    for (int j = 0; j < ROWS; ++j) {
        const int64_t row = (int64_t)t * ROWS + j;
        const float ds = expf(A.s[row * POS + p] - lse) * dlogit;
        float a[CH];
        load_act(A.a3 + (row * RP + p + 2) * CH, a);
        uint32_t packed[CH / 2];
#pragma unroll
        for (int c = 0; c < CH; c += 2) {
            const float d0 = a[c] > 0.0f ? ds * w[c] : 0.0f;
            const float d1 = a[c + 1] > 0.0f ? ds * w[c + 1] : 0.0f;
            packed[c / 2] = (uint32_t)to_bf16(d0) | ((uint32_t)to_bf16(d1) << 16);
            gw[c] += ds * a[c];
            gw[c + 1] += ds * a[c + 1];
        }
        gb += ds;
        uint16_t *dzp = A.dz3 + (row * RP + p + 2) * CH;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<uint4 *>(dzp + 8 * q) =
                make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
        if (p < RP - POS) {
            const int pad = p < 2 ? p : POS + p;
            uint16_t *zp = A.dz3 + (row * RP + pad) * CH;
#pragma unroll
            for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4 *>(zp + 8 * q) = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    float *hp = A.hpart + (int64_t)t * (CH + 1);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const float v = block_sum(gw[c], sh);
        if (p == 0) hp[c] = v;
    }
    const float vb = block_sum(gb, sh);
    if (p == 0) hp[CH] = vb;
}

// ---------------------------------------------------------------------------------------
// Weight gradient: dW[co][k] = sum over rows and positions of dz[row][p][co] in[row][p C_in + k]
// (and the bias gradient sum of dz), as MFMA products with positions as the reduction index.
// Each wave accumulates a fixed set of rows and writes one partial; the partials are reduced in
// a fixed order afterwards.
// ---------------------------------------------------------------------------------------
struct WgArgs {
    const uint16_t *dz;        // [rows][RP][32]
    const uint16_t *in;        // [rows][RP][CI]
    float *part;               // [n_waves][32 KR + 32]
    int32_t rows;
    int32_t n_waves;
};

template <int CI>
__global__ __launch_bounds__(256) void wgrad_kernel(const WgArgs A) {
    constexpr int KR = TAPS * CI;
    constexpr int NT = (KR + 31) / 32;
    const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (wv >= A.n_waves) return;
    const int h = l >> 5;
    const int n = l & 31;
    f32x16 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[nt][i] = 0.0f;
    float bsum = 0.0f;
    for (int r = wv; r < A.rows; r += A.n_waves) {
        const uint16_t *dzr = A.dz + (int64_t)r * RP * CH;
        const uint16_t *inr = A.in + (int64_t)r * RP * CI;
        for (int ps = 0; ps < POS / 16; ++ps) {
            const int pb = 16 * ps + 8 * h;
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint16_t v = dzr[(pb + j + 2) * CH + n];
                a[j] = __builtin_bit_cast(__bf16, v);
                bsum += from_bf16(v);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int k = nt * 32 + n;
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint16_t v = k < KR ? inr[(pb + j) * CI + k] : (uint16_t)0;
                    b[j] = __builtin_bit_cast(__bf16, v);
                }
                acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nt], 0, 0, 0);
            }
        }
    }
    float *pw = A.part + (int64_t)wv * (CH * KR + CH);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int k = nt * 32 + n;
        if (k < KR) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int co = 8 * (i / 4) + 4 * h + (i % 4);
                pw[co * KR + k] = acc[nt][i];
            }
        }
    }
    const float other = __shfl_down(bsum, 32);
    if (l < 32) pw[CH * KR + l] = bsum + other;
}

// ---------------------------------------------------------------------------------------
// Fixed-order reduction of the partials into the gradient vector, and the mean loss.
// ---------------------------------------------------------------------------------------
struct RedArgs {
    const float *part1, *part2, *part3, *hpart, *loss_t;
    float *grads;
    float *loss;
    int32_t n_waves, n_tiles;
};

// Sum of src[w * stride] over w in [w0, w1), in increasing w, with 8 loads in flight.
__device__ __forceinline__ float ordered_sum(const float *src, int64_t stride, int w0, int w1) {
    float g = 0.0f;
    int w = w0;
    for (; w + 8 <= w1; w += 8) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[(int64_t)(w + q) * stride];
#pragma unroll
        for (int q = 0; q < 8; ++q) g += v[q];
    }
    for (; w < w1; ++w) g += src[(int64_t)w * stride];
    return g;
}

// A work-group takes RED_PARAMS gradient entries; each entry's partials are cut into RED_CHUNKS
// consecutive ranges summed in order by separate threads, and the range sums are added in order.
constexpr int RED_PARAMS = 8;
constexpr int RED_CHUNKS = 32;

__global__ __launch_bounds__(256) void reduce_kernel(const RedArgs A) {
    __shared__ float part[RED_CHUNKS][RED_PARAMS];
    __shared__ float lsum[256];
    const int j = threadIdx.x % RED_PARAMS;
    const int c = threadIdx.x / RED_PARAMS;
    const int i = blockIdx.x * RED_PARAMS + j;
    const float *src = nullptr;
    int stride = 0, idx = 0, count = A.n_waves;
    if (i < SPD_PROP_OFF_B1) {
        src = A.part1; stride = CH * 40 + CH; idx = i;
    } else if (i < SPD_PROP_OFF_W2) {
        src = A.part1; stride = CH * 40 + CH; idx = CH * 40 + (i - SPD_PROP_OFF_B1);
    } else if (i < SPD_PROP_OFF_B2) {
        src = A.part2; stride = CH * KW + CH; idx = i - SPD_PROP_OFF_W2;
    } else if (i < SPD_PROP_OFF_W3) {
        src = A.part2; stride = CH * KW + CH; idx = CH * KW + (i - SPD_PROP_OFF_B2);
    } else if (i < SPD_PROP_OFF_B3) {
        src = A.part3; stride = CH * KW + CH; idx = i - SPD_PROP_OFF_W3;
    } else if (i < SPD_PROP_OFF_WH) {
        src = A.part3; stride = CH * KW + CH; idx = CH * KW + (i - SPD_PROP_OFF_B3);
    } else if (i <= SPD_PROP_OFF_BH) {
        src = A.hpart; stride = CH + 1; idx = i - SPD_PROP_OFF_WH; count = A.n_tiles;
    }
    const int w0 = (int)((int64_t)c * count / RED_CHUNKS);
    const int w1 = (int)((int64_t)(c + 1) * count / RED_CHUNKS);
    part[c][j] = src ? ordered_sum(src + idx, stride, w0, w1) : 0.0f;
    __syncthreads();
    if (c == 0 && i < SPD_PROP_NPARAMS) {
        float g = 0.0f;
        for (int q = 0; q < RED_CHUNKS; ++q) g += part[q][j];
        A.grads[i] = g;
    }
    if (blockIdx.x == 0) {
        // mean loss: 256 ordered ranges of the tiles, then the range sums in order
        const int t0 = (int)((int64_t)threadIdx.x * A.n_tiles / 256);
        const int t1 = (int)((int64_t)(threadIdx.x + 1) * A.n_tiles / 256);
        lsum[threadIdx.x] = ordered_sum(A.loss_t, 1, t0, t1);
        __syncthreads();
        if (threadIdx.x == 0) {
            float L = 0.0f;
            for (int q = 0; q < 256; ++q) L += lsum[q];
            A.loss[0] = L / (float)A.n_tiles;
        }
    }
}

struct AdamArgs {
    float *p;
    const float *g;
    float *m, *v;
    float lr, c1, c2;          // c1 = 1 / (1 - beta1^step), c2 = 1 / (1 - beta2^step)
};

__global__ void adam_kernel(const AdamArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= SPD_PROP_NPARAMS) return;
    const float g = A.g[i];
    const float m = 0.9f * A.m[i] + 0.1f * g;
    const float v = 0.999f * A.v[i] + 0.001f * g * g;
    A.m[i] = m;
    A.v[i] = v;
    A.p[i] -= A.lr * (m * A.c1) / (sqrtf(v * A.c2) + 1e-8f);
}

// ---------------------------------------------------------------------------------------
// Per-tile maximum over a search's planes, and labels.
// ---------------------------------------------------------------------------------------
struct TileMaxArgs {
    const float *snr;
    float *out;
    int64_t off[SPD_MAX_LEVELS];
    int64_t pitch[SPD_MAX_LEVELS];
    int64_t slots[SPD_MAX_LEVELS];
    int32_t n_levels, rows_per_tile, n_tiles;
    int32_t vec_ok;            // planes 16-byte aligned: float4 loads
};

// A float (never NaN here) as a signed integer of the same order: non-negative floats keep their
// bits, negative ones have the 31 magnitude bits inverted.  The map is its own inverse.
__device__ __forceinline__ int32_t order_key(int32_t bits) { return bits >= 0 ? bits : bits ^ 0x7FFFFFFF; }

__global__ void tile_init_kernel(int32_t *key, int32_t n_tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) key[t] = order_key(__float_as_int(-__builtin_huge_valf()));
}

// one work-group per DM row: the row's maximum over every level, merged into its tile's entry
// with an integer atomic maximum on the order key
__global__ __launch_bounds__(256) void tile_max_kernel(const TileMaxArgs A, int32_t *key) {
    __shared__ float sh[4];
    const int d = blockIdx.x;
    if (d >= A.n_tiles * A.rows_per_tile) return;
    float mx = -__builtin_huge_valf();
    for (int lv = 0; lv < A.n_levels; ++lv) {
        const float *Y = A.snr + A.off[lv] + (int64_t)d * A.pitch[lv];
        const int64_t n = A.slots[lv];
        const int64_t n4 = A.vec_ok ? n >> 2 : 0;
        for (int64_t q = threadIdx.x; q < n4; q += 256) {
            const float4 v = reinterpret_cast<const float4 *>(Y)[q];
            mx = fmaxf(mx, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
        }
        for (int64_t s = 4 * n4 + threadIdx.x; s < n; s += 256) mx = fmaxf(mx, Y[s]);
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) atomicMax(key + d / A.rows_per_tile, order_key(__float_as_int(mx)));
}

__global__ void tile_fin_kernel(int32_t *key, int32_t n_tiles) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) reinterpret_cast<float *>(key)[t] = __int_as_float(order_key(key[t]));
}

__global__ void labels_kernel(const float *e, const float *l, int32_t n, float thr, float m,
                              float *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float prod = m * l[i];
    out[i] = (e[i] > thr && e[i] > prod) ? 1.0f : 0.0f;
}

// tile (r, c) of an n_row x n_col grid: logits in column order (c n_row + r, as the features of
// one column of tiles after another give them), flags in row order (r n_col + c)
__global__ void flags_kernel(const float *logits, int32_t n_row, int32_t n_col, float thr,
                             uint8_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_row * n_col) return;
    const int64_t r = i / n_col, c = i - r * n_col;
    flags[i] = logits[c * n_row + r] > thr ? 1 : 0;
}

// ---------------------------------------------------------------------------------------
// Fused inference: one work-group per row runs the three convolutions with the activations in
// LDS (features 4.2 KB, two activation buffers of 21 KB), then the read-out; only the
// features come from HBM.  Each row leaves its read-out maximum and sum of exp(s - max); a
// second kernel combines a tile's 64 rows into the logit.  The MFMA sequence is the unfused
// kernels' one, so the activations are bitwise the same.
// ---------------------------------------------------------------------------------------
struct InferArgs {
    const uint16_t *feat;
    WB wb;
    const float *params;
    float *row_max;            // [rows]
    float *row_sum;            // [rows]
    int32_t rows;
};

// Activation rows in LDS: padded position pp keeps its 32 channels (four 16-byte chunks) in a
// row of 40 bf16 (80 bytes).  16-byte loads of one chunk by any 8 or 16 consecutive positions
// (the MFMA operand and the read-out) then fall in distinct LDS banks, with 32 or 64 banks;
// a 64-byte stride puts four positions on the same banks.
constexpr int ACT_LD = CH + 8;
__device__ __forceinline__ int act_at(int pp, int c) { return pp * ACT_LD + (c << 3); }

// The weights of one layer as this lane feeds them to the MFMA (A operand: output channel n =
// lane % 32, k = 16 s + 8 (lane / 32) .. + 7), held in registers across the rows of a launch.
template <int CI>
struct LayerW {
    static constexpr int KS = (TAPS * CI + 15) / 16;
    bf16x8 w[KS];
    __device__ __forceinline__ void load(const uint16_t *wg, int l) {
        const int h = l >> 5, n = l & 31;
#pragma unroll
        for (int s = 0; s < KS; ++s) w[s] = load8(wg + n * (KS * 16) + 16 * s + 8 * h);
    }
};

// one layer of a row held in LDS: out = relu(W in + b), 2 tiles of 32 positions per wave, their
// two accumulation chains interleaved so that consecutive MFMAs are independent.  The layer-1
// input (8 features per position, 16 bytes) is a plain row; wider inputs are padded.  bias: the
// layer's 32 biases in LDS.
template <int CI>
__device__ __forceinline__ void conv_lds(const uint16_t *in, const LayerW<CI> &W, const float *bias,
                                         uint16_t *out, int wave, int l) {
    constexpr int KS = LayerW<CI>::KS;
    static_assert(CI == FCH || CI == CH, "layer inputs are the features or an activation row");
    const int h = l >> 5;
    const int n = l & 31;
    f32x16 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            // k = 16 s + 8 h: tap s / 2, channels 16 (s % 2) + 8 h .. + 7 of position p0 + n + tap
            const int p0 = wave * 64 + t * 32;
            const uint16_t *src = CI == CH ? in + act_at(p0 + n + (s >> 1), 2 * (s & 1) + h)
                                           : in + (p0 + n) * CI + 16 * s + 8 * h;
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W.w[s], load8(src), acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int po = wave * 64 + t * 32 + n + 2;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 bv = *reinterpret_cast<const float4 *>(bias + 8 * g + 4 * h);
            const float bb[4] = {bv.x, bv.y, bv.z, bv.w};
            uint16_t hv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) hv[j] = to_bf16(fmaxf(acc[t][4 * g + j] + bb[j], 0.0f));
            *reinterpret_cast<uint2 *>(out + act_at(po, g) + 4 * h) =
                make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16),
                           (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
        }
    }
}

// Persistent: each work-group takes rows blockIdx.x, + gridDim.x, ... with the weights in
// registers for the whole launch, and fetches the next row's features while it computes the
// current one.
__global__ __launch_bounds__(256) void infer_kernel(const InferArgs A) {
    constexpr int NF = RP * FCH / 8;                 // 16-byte pieces of a row's features
    static_assert(NF > 256 && NF <= 512, "a row's features take one or two pieces per thread");
    __shared__ __attribute__((aligned(16))) uint16_t f[RP * FCH];
    __shared__ __attribute__((aligned(16))) uint16_t a[RP * ACT_LD];
    __shared__ __attribute__((aligned(16))) uint16_t b[RP * ACT_LD];
    __shared__ __attribute__((aligned(16))) float bias[3 * CH];
    __shared__ float red[8];
    if ((int)blockIdx.x >= A.rows) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int l = tid & 63;
    LayerW<FCH> W1;
    LayerW<CH> W2, W3;
    W1.load(A.wb.w1, l);
    W2.load(A.wb.w2, l);
    W3.load(A.wb.w3, l);
    if (tid < 3 * CH) {
        const int j = tid / CH, c = tid - j * CH;
        const int off = j == 0 ? SPD_PROP_OFF_B1 : (j == 1 ? SPD_PROP_OFF_B2 : SPD_PROP_OFF_B3);
        bias[tid] = A.params[off + c];
    }
    // zero pads of the activation buffers (positions 0, 1, 258 .. 261); the layers never write them
    for (int i = tid; i < 6 * CH / 8; i += 256) {
        const int pos = i / (CH / 8), part = i - pos * (CH / 8);
        const int pp = pos < 2 ? pos : POS + pos;
        *reinterpret_cast<uint4 *>(a + act_at(pp, part)) = make_uint4(0u, 0u, 0u, 0u);
        *reinterpret_cast<uint4 *>(b + act_at(pp, part)) = make_uint4(0u, 0u, 0u, 0u);
    }
    const float *wh = A.params + SPD_PROP_OFF_WH;
    const float bh = A.params[SPD_PROP_OFF_BH];
    uint4 fp0 = make_uint4(0u, 0u, 0u, 0u), fp1 = fp0;
    auto fetch = [&](int r) {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.feat + (int64_t)r * RP * FCH);
        fp0 = src[tid];
        if (tid + 256 < NF) fp1 = src[tid + 256];
    };
    fetch(blockIdx.x);
    for (int r = blockIdx.x; r < A.rows; r += gridDim.x) {
        reinterpret_cast<uint4 *>(f)[tid] = fp0;
        if (tid + 256 < NF) reinterpret_cast<uint4 *>(f)[tid + 256] = fp1;
        __syncthreads();
        if (r + (int)gridDim.x < A.rows) fetch(r + gridDim.x);
        conv_lds<FCH>(f, W1, bias, a, wave, l);
        __syncthreads();
        conv_lds<CH>(a, W2, bias + CH, b, wave, l);
        __syncthreads();
        conv_lds<CH>(b, W3, bias + 2 * CH, a, wave, l);
        __syncthreads();
        // read-out of position tid, then the row's max and sum of exp(s - max)
        float act[CH];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = *reinterpret_cast<const uint4 *>(a + act_at(tid + 2, q));
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                act[8 * q + 2 * e] = __uint_as_float(w[e] << 16);
                act[8 * q + 2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
            }
        }
        float sv = 0.0f;
#pragma unroll
        for (int c = 0; c < CH; ++c) sv += wh[c] * act[c];
        sv += bh;
        const float mx = block_max(sv, red);
        const float se = block_sum(expf(sv - mx), red + 4);
        if (tid == 0) {
            A.row_max[r] = mx;
            A.row_sum[r] = se;
        }
        __syncthreads();                    // f and a are rewritten for the next row
    }
}

__global__ void infer_combine_kernel(const float *row_max, const float *row_sum, int32_t n_tiles,
                                     float *logits) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    float M = -__builtin_huge_valf();
    for (int j = 0; j < ROWS; ++j) M = fmaxf(M, row_max[t * ROWS + j]);
    float Z = 0.0f;
    for (int j = 0; j < ROWS; ++j) Z += row_sum[t * ROWS + j] * expf(row_max[t * ROWS + j] - M);
    logits[t] = M + logf(Z) - 9.70406052783923f;
}

// ---------------------------------------------------------------------------------------
// Workspace layout for n_tiles tiles.
// ---------------------------------------------------------------------------------------
struct Layout {
    int64_t wb, a1, a2, a3, dz3, dz2, dz1, s, loss_t, hpart, part1, part2, part3, total;
    int n_waves;
};

inline int64_t up256(int64_t v) { return (v + 255) & ~(int64_t)255; }

Layout layout(int32_t n_tiles) {
    Layout L;
    const int64_t rows = (int64_t)n_tiles * ROWS;
    const int64_t act = rows * RP * CH * 2;
    L.n_waves = (int)(rows < MAX_PART_WAVES ? rows : MAX_PART_WAVES);
    int64_t o = 0;
    auto take = [&](int64_t b) { const int64_t at = o; o += up256(b); return at; };
    L.wb = take((int64_t)(CH * KW1 + 4 * CH * KW) * 2);
    L.a1 = take(act);
    L.a2 = take(act);
    L.a3 = take(act);
    L.dz3 = take(act);
    L.dz2 = take(act);
    L.dz1 = take(act);
    L.s = take(rows * POS * 4);
    L.loss_t = take((int64_t)n_tiles * 4);
    L.hpart = take((int64_t)n_tiles * (CH + 1) * 4);
    L.part1 = take((int64_t)L.n_waves * (CH * 40 + CH) * 4);
    L.part2 = take((int64_t)L.n_waves * (CH * KW + CH) * 4);
    L.part3 = take((int64_t)L.n_waves * (CH * KW + CH) * 4);
    L.total = o;
    return L;
}

struct Bufs {
    WB wb;
    uint16_t *a1, *a2, *a3, *dz3, *dz2, *dz1;
    float *s, *loss_t, *hpart, *part1, *part2, *part3;
};

Bufs bufs(const Layout &L, void *ws) {
    char *b = static_cast<char *>(ws);
    Bufs B;
    uint16_t *w = reinterpret_cast<uint16_t *>(b + L.wb);
    B.wb.w1 = w;
    B.wb.w2 = w + CH * KW1;
    B.wb.w3 = B.wb.w2 + CH * KW;
    B.wb.w2t = B.wb.w3 + CH * KW;
    B.wb.w3t = B.wb.w2t + CH * KW;
    B.a1 = reinterpret_cast<uint16_t *>(b + L.a1);
    B.a2 = reinterpret_cast<uint16_t *>(b + L.a2);
    B.a3 = reinterpret_cast<uint16_t *>(b + L.a3);
    B.dz3 = reinterpret_cast<uint16_t *>(b + L.dz3);
    B.dz2 = reinterpret_cast<uint16_t *>(b + L.dz2);
    B.dz1 = reinterpret_cast<uint16_t *>(b + L.dz1);
    B.s = reinterpret_cast<float *>(b + L.s);
    B.loss_t = reinterpret_cast<float *>(b + L.loss_t);
    B.hpart = reinterpret_cast<float *>(b + L.hpart);
    B.part1 = reinterpret_cast<float *>(b + L.part1);
    B.part2 = reinterpret_cast<float *>(b + L.part2);
    B.part3 = reinterpret_cast<float *>(b + L.part3);
    return B;
}

thread_local char g_err[160];

int fail(hipError_t e) {
    snprintf(g_err, sizeof(g_err), "HIP launch failed: %s", hipGetErrorString(e));
    return SPD_EHIP;
}

#define SPDP_LAUNCH(...)                                   \
    do {                                                   \
        hipLaunchKernelGGL(__VA_ARGS__);                   \
        const hipError_t e_ = hipGetLastError();           \
        if (e_ != hipSuccess) return fail(e_);             \
    } while (0)

int check_ws(int32_t n_tiles, const void *ws, int64_t ws_bytes, Layout *L) {
    if (n_tiles < 1 || n_tiles > (1 << 20)) return SPD_EINVAL;
    *L = layout(n_tiles);
    if (!ws || ws_bytes < L->total) return SPD_EWORKSPACE;
    if ((uintptr_t)ws & 255) return SPD_EALIGN;
    return SPD_OK;
}

// forward through the three layers and the read-out (labels: training mode)
int run_forward(const float *params, const uint16_t *feat, int32_t n_tiles, const float *labels,
                float *logits, const Layout &L, const Bufs &B, hipStream_t st) {
    const int rows = n_tiles * ROWS;
    SPDP_LAUNCH(prep_weights_kernel, dim3((CH * KW + 255) / 256), dim3(256), 0, st, params, B.wb);
    ConvArgs c;
    memset(&c, 0, sizeof(c));
    c.rows = rows;
    c.in = feat;
    c.w = B.wb.w1;
    c.bias = params + SPD_PROP_OFF_B1;
    c.out = B.a1;
    SPDP_LAUNCH((conv_kernel<FCH, 0>), dim3(2 * rows), dim3(256), 0, st, c);
    c.in = B.a1;
    c.w = B.wb.w2;
    c.bias = params + SPD_PROP_OFF_B2;
    c.out = B.a2;
    SPDP_LAUNCH((conv_kernel<CH, 0>), dim3(2 * rows), dim3(256), 0, st, c);
    c.in = B.a2;
    c.w = B.wb.w3;
    c.bias = params + SPD_PROP_OFF_B3;
    c.out = B.a3;
    SPDP_LAUNCH((conv_kernel<CH, 0>), dim3(2 * rows), dim3(256), 0, st, c);
    HeadArgs h;
    h.a3 = B.a3;
    h.params = params;
    h.labels = labels;
    h.s = B.s;
    h.logits = logits;
    h.loss_t = B.loss_t;
    h.hpart = B.hpart;
    h.dz3 = B.dz3;
    h.n_tiles = n_tiles;
    SPDP_LAUNCH(head_kernel, dim3(n_tiles), dim3(256), 0, st, h);
    (void)L;
    return SPD_OK;
}

}  // namespace spdp

using namespace spdp;

extern "C" {

int spd_tiles_generate(uint64_t seed, int64_t first_tile, int32_t n_tiles, float *x,
                       void *hip_stream) {
    if (n_tiles < 1 || n_tiles > (1 << 24) || first_tile < 0 || !x) return SPD_EINVAL;
    TileArgs a{x, seed, first_tile, n_tiles};
    SPDP_LAUNCH(tiles_kernel, dim3((unsigned)n_tiles * ROWS), dim3(256), 0,
                static_cast<hipStream_t>(hip_stream), a);
    return SPD_OK;
}

int spd_prop_features(const float *x, int64_t ld, int32_t n_rows, const float *mean,
                      const float *sigma, uint16_t *feat, void *hip_stream) {
    if (!x || !mean || !sigma || !feat || n_rows < 1 || ld < LEN || (ld & 3)) return SPD_EINVAL;
    if (((uintptr_t)x & 15) || ((uintptr_t)feat & 15)) return SPD_EALIGN;
    FeatArgs a{x, ld, mean, sigma, feat, n_rows};
    SPDP_LAUNCH(features_kernel, dim3(n_rows), dim3(256), 0, static_cast<hipStream_t>(hip_stream), a);
    return SPD_OK;
}

int spd_prop_workspace(int32_t n_tiles, int64_t *bytes) {
    if (!bytes || n_tiles < 1 || n_tiles > (1 << 20)) return SPD_EINVAL;
    *bytes = layout(n_tiles).total;
    return SPD_OK;
}

int spd_prop_forward(const float *params, const uint16_t *feat, int32_t n_tiles, float *logits,
                     void *workspace, int64_t workspace_bytes, void *hip_stream) {
    Layout L;
    const int st = check_ws(n_tiles, workspace, workspace_bytes, &L);
    if (st != SPD_OK) return st;
    if (!params || !feat || !logits) return SPD_EINVAL;
    if ((uintptr_t)feat & 15) return SPD_EALIGN;
    const Bufs B = bufs(L, workspace);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int rows = n_tiles * ROWS;
    SPDP_LAUNCH(prep_weights_kernel, dim3((CH * KW + 255) / 256), dim3(256), 0, s, params, B.wb);
    InferArgs a;
    a.feat = feat;
    a.wb = B.wb;
    a.params = params;
    a.row_max = B.s;
    a.row_sum = B.s + rows;
    a.rows = rows;
    // persistent grid: as many work-groups as the device keeps resident at once, at most one per row
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, infer_kernel, 256, 0) != hipSuccess)
        return fail(hipGetLastError());
    const int grid = std::max(1, std::min(rows, cus * std::max(1, per_cu)));
    SPDP_LAUNCH(infer_kernel, dim3(grid), dim3(256), 0, s, a);
    SPDP_LAUNCH(infer_combine_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0, s, a.row_max,
                a.row_sum, n_tiles, logits);
    return SPD_OK;
}

int spd_prop_backward(const float *params, const uint16_t *feat, const float *labels,
                      int32_t n_tiles, float *logits, float *grads, float *loss,
                      void *workspace, int64_t workspace_bytes, void *hip_stream) {
    Layout L;
    int st = check_ws(n_tiles, workspace, workspace_bytes, &L);
    if (st != SPD_OK) return st;
    if (!params || !feat || !labels || !grads || !loss) return SPD_EINVAL;
    const Bufs B = bufs(L, workspace);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    st = run_forward(params, feat, n_tiles, labels, logits, L, B, s);
    if (st != SPD_OK) return st;
    const int rows = n_tiles * ROWS;
    const int wg_blocks = (L.n_waves + 3) / 4;
    WgArgs w;
    w.rows = rows;
    w.n_waves = L.n_waves;
    // layer 3: weights, then the gradient at layer 2's output
    w.dz = B.dz3;
    w.in = B.a2;
    w.part = B.part3;
    SPDP_LAUNCH(wgrad_kernel<CH>, dim3(wg_blocks), dim3(256), 0, s, w);
    ConvArgs c;
    memset(&c, 0, sizeof(c));
    c.rows = rows;
    c.in = B.dz3;
    c.w = B.wb.w3t;
    c.prev = B.a2;
    c.out = B.dz2;
    SPDP_LAUNCH((conv_kernel<CH, 1>), dim3(2 * rows), dim3(256), 0, s, c);
    // layer 2
    w.dz = B.dz2;
    w.in = B.a1;
    w.part = B.part2;
    SPDP_LAUNCH(wgrad_kernel<CH>, dim3(wg_blocks), dim3(256), 0, s, w);
    c.in = B.dz2;
    c.w = B.wb.w2t;
    c.prev = B.a1;
    c.out = B.dz1;
    SPDP_LAUNCH((conv_kernel<CH, 1>), dim3(2 * rows), dim3(256), 0, s, c);
    // layer 1 (no gradient at the features)
    w.dz = B.dz1;
    w.in = feat;
    w.part = B.part1;
    SPDP_LAUNCH(wgrad_kernel<FCH>, dim3(wg_blocks), dim3(256), 0, s, w);
    RedArgs r{B.part1, B.part2, B.part3, B.hpart, B.loss_t, grads, loss, L.n_waves, n_tiles};
    SPDP_LAUNCH(reduce_kernel, dim3((SPD_PROP_NPARAMS + RED_PARAMS - 1) / RED_PARAMS), dim3(256), 0, s, r);
    return SPD_OK;
}

int spd_prop_adam(float *params, const float *grads, float *m, float *v, int32_t step, float lr,
                  void *hip_stream) {
    if (!params || !grads || !m || !v || step < 1) return SPD_EINVAL;
    AdamArgs a;
    a.p = params;
    a.g = grads;
    a.m = m;
    a.v = v;
    a.lr = lr;
    a.c1 = (float)(1.0 / (1.0 - pow(0.9, step)));
    a.c2 = (float)(1.0 / (1.0 - pow(0.999, step)));
    SPDP_LAUNCH(adam_kernel, dim3((SPD_PROP_NPARAMS + 255) / 256), dim3(256), 0,
                static_cast<hipStream_t>(hip_stream), a);
    return SPD_OK;
}

int spd_tile_max(const float *snr, const spd_plan_info *info, int32_t n_dm, int32_t rows_per_tile,
                 float *tile_max, void *hip_stream) {
    if (!snr || !info || !tile_max || rows_per_tile < 1 || n_dm < rows_per_tile ||
        n_dm % rows_per_tile || info->n_levels < 1 || info->n_levels > SPD_MAX_LEVELS)
        return SPD_EINVAL;
    TileMaxArgs a;
    memset(&a, 0, sizeof(a));
    a.snr = snr;
    a.out = tile_max;
    a.n_levels = info->n_levels;
    a.rows_per_tile = rows_per_tile;
    a.n_tiles = n_dm / rows_per_tile;
    a.vec_ok = ((uintptr_t)snr & 15) == 0;
    for (int i = 0; i < info->n_levels; ++i) {
        a.off[i] = info->plane_offset[i];
        a.pitch[i] = info->plane_pitch[i];
        a.slots[i] = info->plane_slots[i];
        if ((a.off[i] | a.pitch[i]) & 3) a.vec_ok = 0;
    }
    // the output holds the order keys until the last pass turns them back into floats
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int32_t *key = reinterpret_cast<int32_t *>(tile_max);
    const dim3 tg((a.n_tiles + 255) / 256);
    SPDP_LAUNCH(tile_init_kernel, tg, dim3(256), 0, st, key, a.n_tiles);
    SPDP_LAUNCH(tile_max_kernel, dim3(n_dm), dim3(256), 0, st, a, key);
    SPDP_LAUNCH(tile_fin_kernel, tg, dim3(256), 0, st, key, a.n_tiles);
    return SPD_OK;
}

int spd_prop_labels(const float *exh_max, const float *lossy_max, int32_t n_tiles,
                    float threshold, float margin, float *labels, void *hip_stream) {
    if (!exh_max || !lossy_max || !labels || n_tiles < 1) return SPD_EINVAL;
    const float m = (float)(1.0 + (double)margin);
    SPDP_LAUNCH(labels_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0,
                static_cast<hipStream_t>(hip_stream), exh_max, lossy_max, n_tiles, threshold, m,
                labels);
    return SPD_OK;
}

int spd_prop_flags(const float *logits, int32_t n_row_tiles, int32_t n_col_tiles,
                   float logit_threshold, uint8_t *flags, void *hip_stream) {
    if (!logits || !flags || n_row_tiles < 1 || n_col_tiles < 1 ||
        (int64_t)n_row_tiles * n_col_tiles > INT32_MAX)
        return SPD_EINVAL;
    const int64_t n = (int64_t)n_row_tiles * n_col_tiles;
    SPDP_LAUNCH(flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                static_cast<hipStream_t>(hip_stream), logits, n_row_tiles, n_col_tiles,
                logit_threshold, flags);
    return SPD_OK;
}

}  // extern "C"
