// Gaussian removal (Sec. 3.2.2, Eq. 8): a stable compaction of the Gaussian
// set (and of companion arrays such as the Adam moments) that drops the
// Gaussians whose opacity is too low or whose largest scale is too large or
// too small.  The decisions compare stored parameters with thresholds on the
// logit and log-scale axes (binary32), so they are exact and order-free.
//   k_remove_count    per block of 256 Gaussians: how many are kept
//   k_remove_scan     one block: block offsets, kept total (the output row stride)
//   k_remove_scatter  per Gaussian: its rows of every set to its kept position
#include <cmath>

#include "gps_internal.h"
#include "launch.h"
#include "prof.h"
#include "render_common.h"

namespace gps {

constexpr int kRemoveSets = 4;

struct RemovalArgs {
    const float* in[kRemoveSets][5];  // per set: mean, log_scale, quat, opacity_logit, rgb
    float* out[kRemoveSets][5];
    int n_sets, M;
    float t_logit, t_hi, t_lo;        // logit(min_opacity), ln(max_scale), ln(min_scale)
    unsigned int* blk_cnt;
    unsigned int* blk_off;
    unsigned int* total;
    int* out_count;
};

__device__ __forceinline__ bool keep_gaussian(const RemovalArgs& a, int g)
{
    const float o = a.in[0][3][g];
    const float* l = a.in[0][1];
    const float lmax = fmaxf(fmaxf(l[g], l[a.M + g]), l[2 * a.M + g]);
    return !(o < a.t_logit) && !(lmax > a.t_hi) && !(lmax < a.t_lo);
}

__global__ void __launch_bounds__(256) k_remove_count(RemovalArgs a)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    const unsigned int k = (g < a.M && keep_gaussian(a, g)) ? 1u : 0u;
    unsigned int tot;
    block_excl_scan<256>(k, &tot);
    if (threadIdx.x == 0) a.blk_cnt[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_remove_scan(RemovalArgs a, int nblk)
{
    __shared__ unsigned int wsum[16];
    __shared__ unsigned int carry_s;
    if (threadIdx.x == 0) carry_s = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + threadIdx.x;
        const unsigned int c = i < nblk ? a.blk_cnt[i] : 0u;
        unsigned int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        unsigned int before = 0u, total = 0u;
        for (int k = 0; k < 16; ++k) {
            if (k < wid) before += wsum[k];
            total += wsum[k];
        }
        const unsigned int carry = carry_s;
        if (i < nblk) a.blk_off[i] = carry + before + x - c;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *a.total = carry_s;
        if (a.out_count) *a.out_count = (int)carry_s;
    }
}

__global__ void __launch_bounds__(256) k_remove_scatter(RemovalArgs a)
{
    constexpr int kRows[5] = {3, 3, 4, 1, 3};
    const int g = blockIdx.x * 256 + threadIdx.x;
    const bool k = g < a.M && keep_gaussian(a, g);
    unsigned int tot;
    const unsigned int excl = block_excl_scan<256>(k ? 1u : 0u, &tot);
    if (!k) return;
    const size_t pos = a.blk_off[blockIdx.x] + excl;
    const size_t nk = *a.total;  // row stride of the outputs
    for (int s = 0; s < a.n_sets; ++s)
#pragma unroll
        for (int f = 0; f < 5; ++f)
            for (int r = 0; r < kRows[f]; ++r)
                a.out[s][f][(size_t)r * nk + pos] = a.in[s][f][(size_t)r * a.M + g];
}

size_t removal_workspace_bytes(int M)
{
    const size_t nblk = M > 0 ? (size_t)(M + 255) / 256 : 1;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(4 * nblk) * 2 + 256;
}

gps_status launch_remove_gaussians(const gps_removal_cfg* cfg, const gps_gaussians* sets_in, gps_gaussians* sets_out,
                                   int n_sets, int* out_count, char* ws, hipStream_t s)
{
    RemovalArgs a;
    a.n_sets = n_sets;
    a.M = sets_in[0].count;
    a.t_logit = (float)std::log((double)cfg->min_opacity / (1.0 - (double)cfg->min_opacity));
    a.t_hi = (float)std::log((double)cfg->max_scale);
    a.t_lo = (float)std::log((double)cfg->min_scale);
    for (int k = 0; k < n_sets; ++k) {
        const gps_gaussians& gi = sets_in[k];
        gps_gaussians& go = sets_out[k];
        a.in[k][0] = gi.mean, a.in[k][1] = gi.log_scale, a.in[k][2] = gi.quat, a.in[k][3] = gi.opacity_logit,
        a.in[k][4] = gi.rgb;
        a.out[k][0] = go.mean, a.out[k][1] = go.log_scale, a.out[k][2] = go.quat, a.out[k][3] = go.opacity_logit,
        a.out[k][4] = go.rgb;
    }
    const int nblk = a.M > 0 ? (a.M + 255) / 256 : 0;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nb = nblk > 0 ? (size_t)nblk : 1;
    a.blk_cnt = reinterpret_cast<unsigned int*>(ws);
    a.blk_off = reinterpret_cast<unsigned int*>(ws + al(4 * nb));
    a.total = reinterpret_cast<unsigned int*>(ws + 2 * al(4 * nb));
    a.out_count = out_count;
    if (nblk > 0) GPS_LAUNCH(K_REMOVE, s, k_remove_count, dim3(nblk), dim3(256), 0, s, a);
    GPS_LAUNCH(K_REMOVE, s, k_remove_scan, dim3(1), dim3(1024), 0, s, a, nblk);
    if (nblk > 0) GPS_LAUNCH(K_REMOVE, s, k_remove_scatter, dim3(nblk), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
