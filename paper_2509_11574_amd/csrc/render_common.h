// Device helpers shared by the forward and backward render kernels.
#pragma once

#include "gps_internal.h"

namespace gps {

struct GParams {
    const float* mean;
    const float* log_scale;
    const float* quat;
    const float* opacity_logit;
    const float* rgb;
};

struct GGrads {
    float* mean;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* rgb;
};

// Block-wide exclusive scan of one unsigned per thread (NT a multiple of 64).
template <int NT>
__device__ __forceinline__ unsigned int block_excl_scan(unsigned int val, unsigned int* total)
{
    __shared__ unsigned int wsum[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned int x = val;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    unsigned int before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        unsigned int s = wsum[k];
        if (k < wid) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + x - val;
}

// Block-wide float sum (deterministic: DPP within waves, then waves in order).
template <int NT>
__device__ __forceinline__ float block_sum(float v)
{
    __shared__ float wsum[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += wsum[k];
    __syncthreads();
    return t;
}

// Tile rectangle of a projected record: tiles [x0, x1] x [y0, y1] (empty if x0 > x1).
__device__ __forceinline__ void rec_rect(float4 r2, int* x0, int* x1, int* y0, int* y1)
{
    unsigned int a = __float_as_uint(r2.z), b = __float_as_uint(r2.w);
    *x0 = (int)(a & 0xffffu);
    *x1 = (int)(a >> 16) - 1;
    *y0 = (int)(b & 0xffffu);
    *y1 = (int)(b >> 16) - 1;
}

__device__ __forceinline__ float pack_rect(int lo, int hi_plus1)
{
    return __uint_as_float((unsigned int)lo | ((unsigned int)hi_plus1 << 16));
}

}  // namespace gps
