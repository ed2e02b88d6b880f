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

// Bias corrections 1 / (1 - beta^t), in double (1 - beta^t loses digits in
// binary32 for small t).
__device__ __forceinline__ void adam_bias(int t, float b1, float b2, float* ibc1, float* ibc2)
{
    *ibc1 = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
    *ibc2 = (float)(1.0 / (1.0 - pow((double)b2, (double)t)));
}

}  // namespace gps
