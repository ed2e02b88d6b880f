// Point-to-plane ICP camera tracking (Sec. 3.2.1, "Camera tracking", Eq. 5).
//   k_depth_down   one level of the depth hierarchy: mean of the valid depths of
//                  each 2x2 block (binary64 sum and division, rounded once)
//   k_icp_pairs    per pixel of the current level: back-projection, projective
//                  association into the previous frame's raycast depth, the
//                  model vertex and vertex-map normal there, the point-to-plane
//                  residual r and its Jacobian J = (N, p x N) for a left
//                  perturbation of the camera-to-world pose; at most 1024
//                  blocks of 256 lanes, each lane taking every (256 x blocks)-th
//                  pixel; per block the 29 sums (upper triangle of J J^T, J r,
//                  r^2, count) in a fixed order
//   k_icp_total    one block: the block sums in binary64, in a fixed order
//   k_icp_solve    one lane: Cholesky solve of H xi = -g in binary64 and the
//                  update T_{g,k} <- Exp(xi) T_{g,k} of the device pose
// No atomics: the system is bitwise reproducible.  Every stage reads the pose
// from device memory, so a tracking loop can be replayed as a graph.
#include <cmath>
#include <mutex>

#include "gps_internal.h"
#include "launch.h"
#include "prof.h"
#include "se3.h"

namespace gps {

constexpr int kIcpTerms = 29;  // 21 (H, upper triangle, row-major) + 6 (g) + E + count
constexpr int kIcpMaxBlocks = 1024;  // widest grid of k_icp_pairs (four blocks per compute unit)

// Block sums of the allocation-free reduce (gps_icp_reduce_noalloc): room for the
// widest grid, so every level size fits.  One copy per GPU, held until the process
// ends; each call overwrites the entries it reads, so nothing is cleared.  Host code
// takes its address from icp_scratch(), never from this name.
static __device__ __align__(256) float scratch[kIcpTerms * kIcpMaxBlocks];
static_assert(sizeof(scratch) == GPS_ICP_SCRATCH_BYTES, "the header states the scratch size");

__global__ void __launch_bounds__(256) k_depth_down(const float* __restrict__ in, int W, int H,
                                                    float* __restrict__ out, int Wo, int Ho)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= Wo * Ho) return;
    const int i = p % Wo, j = p / Wo;
    const float* r0 = in + (size_t)(2 * j) * W + 2 * i;
    const float* r1 = r0 + W;
    const float v[4] = {r0[0], r0[1], r1[0], r1[1]};
    double s = 0.0;
    int n = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (v[k] > 0.0f) {
            s += (double)v[k];
            ++n;
        }
    out[p] = n > 0 ? (float)(s / (double)n) : 0.0f;
}

struct IcpArgs {
    // previous frame: intrinsics, pose (world -> camera), raycast depth
    float pfx, pfy, pcx, pcy;
    float pR[9], pt[3];
    int pW, pH;
    const float* pdepth;
    // current level: intrinsics, depth; the pose comes from `pose`
    float fx, fy, cx, cy;
    int W, H;
    const float* depth;
    const float* pose;  // [12]: R row-major, t (world -> camera)
    float dist2;
    float* part;        // [kIcpTerms][nblk]
    int nblk;
};

__device__ __forceinline__ float wave_sum_f(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ void prev_point(const IcpArgs& a, int i, int j, float d, float x[3])
{
    x[0] = ((float)i - a.pcx) / a.pfx * d;
    x[1] = ((float)j - a.pcy) / a.pfy * d;
    x[2] = d;
}

__global__ void __launch_bounds__(256) k_icp_pairs(IcpArgs a)
{
    __shared__ float red[kIcpTerms][4];
    // Relative pose current camera -> previous camera, formed in binary64 from the
    // two world-to-camera poses so that the association and the residual are
    // computed without world coordinates: q = R_rel X + t_rel.
    double Rc[9], tc[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = (double)a.pose[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) tc[k] = (double)a.pose[9 + k];
    float Rrel[9], trel[3], Rct[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double tr = (double)a.pt[r];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // (R_p R_c^T)[r][c] = sum_k R_p[r][k] R_c[c][k]
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) s += (double)a.pR[3 * r + k] * Rc[3 * c + k];
            Rrel[3 * r + c] = (float)s;
            tr -= s * tc[c];
            Rct[3 * r + c] = (float)Rc[3 * c + r];
        }
        trel[r] = (float)tr;
    }
    float v[kIcpTerms];
#pragma unroll
    for (int k = 0; k < kIcpTerms; ++k) v[k] = 0.0f;
    // each lane takes the pixels p, p + 256 * gridDim.x, ... (a fixed assignment, so
    // the sums have a fixed order)
    const int n = a.W * a.H;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n; p += 256 * gridDim.x) {
        const float d = a.depth[p];
        const int i = p % a.W, j = p / a.W;
        bool ok = d > 0.0f;
        float X[3] = {((float)i - a.cx) / a.fx * d, ((float)j - a.cy) / a.fy * d, d};
        float q[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < 3; ++r) q[r] = Rrel[3 * r] * X[0] + Rrel[3 * r + 1] * X[1] + Rrel[3 * r + 2] * X[2] + trel[r];
        ok = ok && q[2] > 0.0f;
        int ua = 0, vb = 0;
        if (ok) {
            const float u = a.pfx * q[0] / q[2] + a.pcx, w = a.pfy * q[1] / q[2] + a.pcy;
            ok = u >= 0.5f && u < (float)a.pW - 1.5f && w >= 0.5f && w < (float)a.pH - 1.5f;  // neighbours in the image
            ua = (int)floorf(u + 0.5f);
            vb = (int)floorf(w + 0.5f);
            ok = ok && ua >= 1 && ua <= a.pW - 2 && vb >= 1 && vb <= a.pH - 2;
        }
        float Xs[3], Nc[3];
        if (ok) {
            const int s = vb * a.pW + ua;
            const float dc = a.pdepth[s], dl = a.pdepth[s - 1], dr = a.pdepth[s + 1], du = a.pdepth[s - a.pW],
                        dd = a.pdepth[s + a.pW];
            ok = dc > 0.0f && dl > 0.0f && dr > 0.0f && du > 0.0f && dd > 0.0f;
            if (ok) {
                float xl[3], xr[3], xu[3], xd[3];
                prev_point(a, ua, vb, dc, Xs);
                prev_point(a, ua - 1, vb, dl, xl);
                prev_point(a, ua + 1, vb, dr, xr);
                prev_point(a, ua, vb - 1, du, xu);
                prev_point(a, ua, vb + 1, dd, xd);
                const float ex[3] = {xr[0] - xl[0], xr[1] - xl[1], xr[2] - xl[2]};
                const float ey[3] = {xd[0] - xu[0], xd[1] - xu[1], xd[2] - xu[2]};
                Nc[0] = ex[1] * ey[2] - ex[2] * ey[1];
                Nc[1] = ex[2] * ey[0] - ex[0] * ey[2];
                Nc[2] = ex[0] * ey[1] - ex[1] * ey[0];
                const float nn = Nc[0] * Nc[0] + Nc[1] * Nc[1] + Nc[2] * Nc[2];
                ok = nn > 0.0f;
                const float inv = ok ? 1.0f / sqrtf(nn) : 0.0f;
                // the sign of N cancels in J J^T and J r: no turn towards the camera is needed
                Nc[0] *= inv;
                Nc[1] *= inv;
                Nc[2] *= inv;
            }
        }
        if (ok) {
            const float df[3] = {q[0] - Xs[0], q[1] - Xs[1], q[2] - Xs[2]};
            ok = df[0] * df[0] + df[1] * df[1] + df[2] * df[2] <= a.dist2;
            if (ok) {
                const float r = df[0] * Nc[0] + df[1] * Nc[1] + df[2] * Nc[2];
                // world normal N = R_p^T N_c; world point p = R_c^T (X - t_c)
                float Nw[3], P[3];
                const float xt[3] = {X[0] - a.pose[9], X[1] - a.pose[10], X[2] - a.pose[11]};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Nw[k] = a.pR[k] * Nc[0] + a.pR[3 + k] * Nc[1] + a.pR[6 + k] * Nc[2];
                    P[k] = Rct[3 * k] * xt[0] + Rct[3 * k + 1] * xt[1] + Rct[3 * k + 2] * xt[2];
                }
                const float J[6] = {Nw[0], Nw[1], Nw[2], P[1] * Nw[2] - P[2] * Nw[1], P[2] * Nw[0] - P[0] * Nw[2],
                                    P[0] * Nw[1] - P[1] * Nw[0]};
                int k = 0;
#pragma unroll
                for (int r0 = 0; r0 < 6; ++r0)
#pragma unroll
                    for (int c0 = r0; c0 < 6; ++c0) v[k++] += J[r0] * J[c0];
#pragma unroll
                for (int r0 = 0; r0 < 6; ++r0) v[21 + r0] += J[r0] * r;
                v[27] += r * r;
                v[28] += 1.0f;
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kIcpTerms; ++k) {
        const float s = wave_sum_f(v[k]);
        if (lane == 0) red[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < kIcpTerms) {
        const int k = threadIdx.x;
        a.part[(size_t)k * a.nblk + blockIdx.x] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

// Wavefront w sums the terms w and w + 16 over the block partials (both in one
// pass, so their loads overlap): lane l takes blocks l, l + 64, ... in binary64,
// then a fixed butterfly across the lanes.
__global__ void __launch_bounds__(1024) k_icp_total(const float* __restrict__ part, int nblk, double* __restrict__ sys)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int k0 = wid, k1 = wid + 16;
    const bool two = k1 < kIcpTerms;
    const float* p0 = part + (size_t)k0 * nblk;
    const float* p1 = part + (size_t)(two ? k1 : k0) * nblk;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int b = lane; b < nblk; b += 64) {
        s0 += (double)p0[b];
        s1 += (double)p1[b];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
    }
    if (lane == 0) {
        sys[k0] = s0;
        if (two) sys[k1] = s1;
    }
}

// The same sums (each wavefront's two terms, the same order), kept in LDS as well,
// then the Gauss-Newton step of k_icp_solve by the block's first lane: one launch
// for the system and the step instead of two.
__device__ void icp_solve_one(const double* sys, const float* pose, float* res);

__global__ void __launch_bounds__(1024) k_icp_total_solve(const float* __restrict__ part, int nblk,
                                                          double* __restrict__ sys, float* __restrict__ pose,
                                                          float* __restrict__ out_xi)
{
    __shared__ double ssys[kIcpTerms];
    __shared__ float res[18];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int k0 = wid, k1 = wid + 16;
    const bool two = k1 < kIcpTerms;
    const float* p0 = part + (size_t)k0 * nblk;
    const float* p1 = part + (size_t)(two ? k1 : k0) * nblk;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int b = lane; b < nblk; b += 64) {
        s0 += (double)p0[b];
        s1 += (double)p1[b];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
    }
    if (lane == 0) {
        sys[k0] = s0;
        ssys[k0] = s0;
        if (two) {
            sys[k1] = s1;
            ssys[k1] = s1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) icp_solve_one(ssys, pose, res);
    __syncthreads();
    // one value per lane (vector stores)
    if (threadIdx.x < 12) pose[threadIdx.x] = res[threadIdx.x];
    if (out_xi && threadIdx.x < 6) out_xi[threadIdx.x] = res[12 + threadIdx.x];
}

// The Gauss-Newton step: res = (new pose (12), xi (6)); the pose is kept when fewer
// than 6 pairs remain or H is not positive definite (xi = 0 then).
__device__ void icp_solve_one(const double* sys, const float* pose, float* res)
{
    double L[36], y[6], xi[6];
    bool ok = sys[28] >= 6.0;
    // H from its upper triangle, Cholesky H = L L^T
    double Hm[36];
    int k = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) {
            Hm[6 * r + c] = sys[k];
            Hm[6 * c + r] = sys[k];
            ++k;
        }
    // (fully unrolled so that the arrays stay in registers; a non-positive pivot
    // clears `ok` and is replaced by 1 to finish the factorisation harmlessly)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = Hm[6 * j + j];
#pragma unroll
        for (int m = 0; m < j; ++m) s -= L[6 * j + m] * L[6 * j + m];
        if (!(s > 0.0)) {
            ok = false;
            s = 1.0;
        }
        L[6 * j + j] = sqrt(s);
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double u = Hm[6 * i + j];
#pragma unroll
            for (int m = 0; m < j; ++m) u -= L[6 * i + m] * L[6 * j + m];
            L[6 * i + j] = u / L[6 * j + j];
        }
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) xi[m] = 0.0;
    if (ok) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {  // L y = -g
            double u = -sys[21 + i];
#pragma unroll
            for (int m = 0; m < i; ++m) u -= L[6 * i + m] * y[m];
            y[i] = u / L[6 * i + i];
        }
#pragma unroll
        for (int i = 5; i >= 0; --i) {  // L^T xi = y
            double u = y[i];
#pragma unroll
            for (int m = i + 1; m < 6; ++m) u -= L[6 * m + i] * xi[m];
            xi[i] = u / L[6 * i + i];
        }
        double Rx[9], tx[3];
        se3_exp_d(xi, Rx, tx);
        // camera to world: R_g = R_c^T, t_g = -R_c^T t_c; then R_g' = Rx R_g, t_g' = Rx t_g + tx
        double Rg[9], tg[3], Rg2[9], tg2[3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Rg[3 * r + c] = (double)pose[3 * c + r];
        for (int r = 0; r < 3; ++r)
            tg[r] = -(Rg[3 * r] * (double)pose[9] + Rg[3 * r + 1] * (double)pose[10] + Rg[3 * r + 2] * (double)pose[11]);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c)
                Rg2[3 * r + c] = Rx[3 * r] * Rg[c] + Rx[3 * r + 1] * Rg[3 + c] + Rx[3 * r + 2] * Rg[6 + c];
            tg2[r] = Rx[3 * r] * tg[0] + Rx[3 * r + 1] * tg[1] + Rx[3 * r + 2] * tg[2] + tx[r];
        }
        // back to world to camera: R_c = R_g'^T, t_c = -R_g'^T t_g'
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) res[3 * r + c] = (float)Rg2[3 * c + r];
            res[9 + r] = (float)-(Rg2[r] * tg2[0] + Rg2[3 + r] * tg2[1] + Rg2[6 + r] * tg2[2]);
        }
    } else {
        for (int m = 0; m < 12; ++m) res[m] = pose[m];
    }
    for (int m = 0; m < 6; ++m) res[12 + m] = (float)xi[m];
}

__global__ void __launch_bounds__(64) k_icp_solve(const double* __restrict__ sys, float* __restrict__ pose,
                                                  float* __restrict__ out_xi)
{
    __shared__ float res[18];
    if (threadIdx.x == 0) icp_solve_one(sys, pose, res);
    __syncthreads();
    // one value per lane (vector stores)
    if (threadIdx.x < 12) pose[threadIdx.x] = res[threadIdx.x];
    if (out_xi && threadIdx.x < 6) out_xi[threadIdx.x] = res[12 + threadIdx.x];
}

// Device address of `scratch` on the current device, looked up once per device.
gps_status icp_scratch(char** out, size_t* bytes)
{
    static std::mutex mu;
    static void* addr[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GPS_ERR_HIP;
    if (dev < 0 || dev >= 64) return GPS_ERR_UNSUPPORTED_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GPS_ERR_HIP;
        addr[dev] = p;
    }
    *out = static_cast<char*>(addr[dev]);
    *bytes = sizeof(scratch);
    return GPS_OK;
}

// Bytes of block sums k_icp_pairs writes for a level of W x H pixels.
size_t icp_partial_bytes(int W, int H)
{
    const size_t want = ((size_t)W * H + 255) / 256;
    return (size_t)kIcpTerms * sizeof(float) * (want < kIcpMaxBlocks ? want : kIcpMaxBlocks);
}

size_t icp_workspace_bytes(int W, int H)
{
    const size_t nblk = ((size_t)W * H + 255) / 256;
    return ((kIcpTerms * 4 * nblk + 255) & ~(size_t)255) + 256;
}

gps_status launch_depth_downsample(const float* in, int W, int H, float* out, hipStream_t s)
{
    const int Wo = W / 2, Ho = H / 2;
    const int n = Wo * Ho;
    if (n > 0) GPS_LAUNCH(K_ICP, s, k_depth_down, dim3((n + 255) / 256), dim3(256), 0, s, in, W, H, out, Wo, Ho);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

gps_status launch_icp_reduce(const gps_camera& prev, const float* prev_depth, const gps_camera& lvl,
                             const float* depth, const float* pose, float dist_thresh, double* sys, char* ws,
                             hipStream_t s, float* step_pose, float* step_xi)
{
    IcpArgs a;
    a.pfx = prev.fx, a.pfy = prev.fy, a.pcx = prev.cx, a.pcy = prev.cy;
    for (int k = 0; k < 9; ++k) a.pR[k] = prev.R[k];
    for (int k = 0; k < 3; ++k) a.pt[k] = prev.t[k];
    a.pW = prev.width, a.pH = prev.height;
    a.pdepth = prev_depth;
    a.fx = lvl.fx, a.fy = lvl.fy, a.cx = lvl.cx, a.cy = lvl.cy;
    a.W = lvl.width, a.H = lvl.height;
    a.depth = depth;
    a.pose = pose;
    a.dist2 = dist_thresh * dist_thresh;
    // at most kIcpMaxBlocks blocks; larger levels loop inside the block
    const size_t want = ((size_t)lvl.width * lvl.height + 255) / 256;
    a.nblk = (int)(want < kIcpMaxBlocks ? want : kIcpMaxBlocks);
    a.part = reinterpret_cast<float*>(ws);
    GPS_LAUNCH(K_ICP, s, k_icp_pairs, dim3(a.nblk), dim3(256), 0, s, a);
    if (step_pose)  // the step in the same launch as the system's sum (gps_icp_step)
        GPS_LAUNCH(K_ICP, s, k_icp_total_solve, dim3(1), dim3(1024), 0, s, a.part, a.nblk, sys, step_pose, step_xi);
    else
        GPS_LAUNCH(K_ICP, s, k_icp_total, dim3(1), dim3(1024), 0, s, a.part, a.nblk, sys);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

gps_status launch_icp_solve(const double* sys, float* pose, float* out_xi, hipStream_t s)
{
    GPS_LAUNCH(K_ICP, s, k_icp_solve, dim3(1), dim3(64), 0, s, sys, pose, out_xi);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
