// Streaming kernels of known HBM traffic, for scaling the hardware's memory
// counters (not part of the method): one reads n floats and writes one float
// per block, the other writes n floats and reads nothing.  Each element is
// touched once, in 16-byte vector accesses where the pointer allows it.
#include "render_common.h"

namespace gps {

constexpr int kStreamBlk = 256;
constexpr int kStreamGrid = 4096;

__global__ void __launch_bounds__(kStreamBlk) k_stream_read(const float* __restrict__ x, size_t n,
                                                            float* __restrict__ out)
{
    const size_t stride = (size_t)gridDim.x * kStreamBlk;
    const size_t t = (size_t)blockIdx.x * kStreamBlk + threadIdx.x;
    float acc = 0.0f;
    const size_t n4 = ((reinterpret_cast<uintptr_t>(x) & 15u) == 0u) ? n / 4 : 0;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (size_t i = t; i < n4; i += stride) {
        const float4 v = x4[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    for (size_t i = 4 * n4 + t; i < n; i += stride) acc += x[i];
    acc = block_sum<kStreamBlk>(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kStreamBlk) k_stream_write(float* __restrict__ y, size_t n, float v)
{
    const size_t stride = (size_t)gridDim.x * kStreamBlk;
    const size_t t = (size_t)blockIdx.x * kStreamBlk + threadIdx.x;
    const size_t n4 = ((reinterpret_cast<uintptr_t>(y) & 15u) == 0u) ? n / 4 : 0;
    float4* y4 = reinterpret_cast<float4*>(y);
    for (size_t i = t; i < n4; i += stride) y4[i] = make_float4(v, v, v, v);
    for (size_t i = 4 * n4 + t; i < n; i += stride) y[i] = v;
}

}  // namespace gps

using namespace gps;

extern "C" int32_t gps_stream_blocks(void) { return kStreamGrid; }

extern "C" gps_status gps_stream_read(const float* x, size_t n, float* out, void* stream)
{
    if (!x || !out || n == 0) return GPS_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_stream_read, dim3(kStreamGrid), dim3(kStreamBlk), 0, (hipStream_t)stream, x, n, out);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

extern "C" gps_status gps_stream_write(float* y, size_t n, float v, void* stream)
{
    if (!y || n == 0) return GPS_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_stream_write, dim3(kStreamGrid), dim3(kStreamBlk), 0, (hipStream_t)stream, y, n, v);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}
