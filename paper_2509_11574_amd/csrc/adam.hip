// Fused Adam over all parameter groups in one launch (per-attribute learning
// rates of Appendix C are supplied by the caller).  HBM-streaming: every
// scalar reads param, grad, m, v and writes param, m, v (28 bytes).  Groups
// whose arrays are 16-byte aligned with n % 4 == 0 are processed as float4.
#include "adam_math.h"
#include "gps_internal.h"
#include "launch.h"
#include "prof.h"

namespace gps {

constexpr int kMaxGroups = 8;

struct AdamArgs {
    float* p[kMaxGroups];
    const float* g[kMaxGroups];
    float* m[kMaxGroups];
    float* v[kMaxGroups];
    float lr[kMaxGroups];
    long long start[kMaxGroups + 1];  // prefix of work items (float4 or scalar units)
    int vec[kMaxGroups];
    long long n[kMaxGroups];
    int ng;
    int step;
    const int* step_ctr;
    float b1, b2, eps;
};

__global__ void __launch_bounds__(256) k_adam(AdamArgs a)
{
    // bias corrections, computed once per block and shared through LDS
    __shared__ float sbc[2];
    if (threadIdx.x == 0) adam_bias(a.step_ctr ? (*a.step_ctr + 1) : a.step, a.b1, a.b2, &sbc[0], &sbc[1]);
    __syncthreads();
    const float ibc1 = sbc[0], ibc2 = sbc[1];
    const long long total = a.start[a.ng];
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (long long)gridDim.x * 256ll) {
        int k = 0;
#pragma unroll 1
        while (k + 1 < a.ng && i >= a.start[k + 1]) ++k;
        const long long j = i - a.start[k];
        const float lr = a.lr[k];
        if (a.vec[k]) {
            float4 p = reinterpret_cast<float4*>(a.p[k])[j];
            const float4 g = reinterpret_cast<const float4*>(a.g[k])[j];
            float4 m = reinterpret_cast<float4*>(a.m[k])[j];
            float4 v = reinterpret_cast<float4*>(a.v[k])[j];
            adam_one(p.x, g.x, m.x, v.x, lr, a.b1, a.b2, a.eps, ibc1, ibc2);
            adam_one(p.y, g.y, m.y, v.y, lr, a.b1, a.b2, a.eps, ibc1, ibc2);
            adam_one(p.z, g.z, m.z, v.z, lr, a.b1, a.b2, a.eps, ibc1, ibc2);
            adam_one(p.w, g.w, m.w, v.w, lr, a.b1, a.b2, a.eps, ibc1, ibc2);
            reinterpret_cast<float4*>(a.p[k])[j] = p;
            reinterpret_cast<float4*>(a.m[k])[j] = m;
            reinterpret_cast<float4*>(a.v[k])[j] = v;
        } else {
            float p = a.p[k][j], m = a.m[k][j], v = a.v[k][j];
            adam_one(p, a.g[k][j], m, v, lr, a.b1, a.b2, a.eps, ibc1, ibc2);
            a.p[k][j] = p;
            a.m[k][j] = m;
            a.v[k][j] = v;
        }
    }
}

// One lane, vector memory path (the address depends on the lane id).
__global__ void __launch_bounds__(64) k_step_incr(int* ctr)
{
    if (threadIdx.x == 0) ctr[threadIdx.x] += 1;
}

gps_status launch_adam(const gps_adam_group* groups, int n_groups, int step, int* step_counter, float b1, float b2,
                       float eps, hipStream_t s)
{
    AdamArgs a;
    a.ng = n_groups;
    a.step = step;
    a.step_ctr = step_counter;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.start[0] = 0;
    for (int k = 0; k < n_groups; ++k) {
        const gps_adam_group& gr = groups[k];
        a.p[k] = gr.param;
        a.g[k] = gr.grad;
        a.m[k] = gr.m;
        a.v[k] = gr.v;
        a.lr[k] = gr.lr;
        a.n[k] = gr.n;
        const bool aligned = ((uintptr_t)gr.param | (uintptr_t)gr.grad | (uintptr_t)gr.m | (uintptr_t)gr.v) % 16 == 0;
        a.vec[k] = aligned && gr.n % 4 == 0;
        a.start[k + 1] = a.start[k] + (a.vec[k] ? gr.n / 4 : gr.n);
    }
    const long long total = a.start[n_groups];
    if (total > 0) {
        long long blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        GPS_LAUNCH(K_ADAM, s, k_adam, dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    if (step_counter) GPS_LAUNCH(K_STEP_INCR, s, k_step_incr, dim3(1), dim3(64), 0, s, step_counter);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
