// One Adam update of a scalar (shared by the Adam kernel and the backward kernel
// that applies Adam in its epilogue, so that both give bitwise the same result).
#pragma once

#include <hip/hip_runtime.h>

namespace gps {

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                         float eps, float ibc1, float ibc2)
{
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * g * g;
    const float mh = m * ibc1, vh = v * ibc2;
    p -= lr * mh / (sqrtf(vh) + eps);
}

// beta^t for an integer t >= 0 by repeated squaring in binary64: at most 2 log2 t
// products, so a relative error below 1e-14, far under the binary32 rounding of the
// bias correction it feeds (a few dozen instructions instead of a general pow).
__device__ __forceinline__ double pow_uint(double b, unsigned int t)
{
    double r = 1.0, p = b;
    for (; t; t >>= 1) {
        if (t & 1u) r *= p;
        p *= p;
    }
    return r;
}

// Bias corrections 1 / (1 - beta^t), in double (1 - beta^t loses digits in
// binary32 for small t).
__device__ __forceinline__ void adam_bias(int t, float b1, float b2, float* ibc1, float* ibc2)
{
    const unsigned int ut = t > 0 ? (unsigned int)t : 0u;
    *ibc1 = (float)(1.0 / (1.0 - pow_uint((double)b1, ut)));
    *ibc2 = (float)(1.0 / (1.0 - pow_uint((double)b2, ut)));
}

}  // namespace gps
