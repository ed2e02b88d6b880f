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
    const float* in[kRemoveSets][6];  // per set: mean, log_scale, quat, opacity_logit, rgb, SH bands
    float* out[kRemoveSets][6];
    int sh_rows;                      // rows of the SH bands (3 K; 0 without)
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
    for (int s = 0; s < a.n_sets; ++s) {
#pragma unroll
        for (int f = 0; f < 5; ++f)
            for (int r = 0; r < kRows[f]; ++r)
                a.out[s][f][(size_t)r * nk + pos] = a.in[s][f][(size_t)r * a.M + g];
        for (int r = 0; r < a.sh_rows; ++r) a.out[s][5][(size_t)r * nk + pos] = a.in[s][5][(size_t)r * a.M + g];
    }
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
        a.in[k][5] = gi.sh;
        a.out[k][5] = go.sh;
    }
    a.sh_rows = 3 * sh_count(sets_in[0].sh_degree);
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

// ------------------------------------------------------------------ insertion
// Gaussian insertion (Sec. 3.2.2, Eq. 6; Appendix A).
//   k_insert_flags  per pixel: mask (bit 0) and sample (bit 1) flags and the
//                   mask depth (the depth on mask pixels, 0 elsewhere); per
//                   block of 256 pixels, the number taken
//   k_insert_bits   per 8x8 pixel block: a 64-bit word of its mask pixels
//   k_insert_scan   one block: block offsets, total taken -> out_count
//   k_insert_place  per taken pixel: its row-major output position
//   k_insert_init   per new Gaussian: its surface point, normal, scale (the
//                   three nearest mask vertices over the whole mask), rotation

struct InsertArgs {
    DevCam cam;
    const float* render_rgb;
    const float* frame_rgb;
    const float* weight;
    const float* depth;
    const float* rnd;
    float* out[6];  // mean, log_scale, quat, opacity_logit, rgb, SH bands: planar [rows][capacity]
    int sh_rows;    // rows of the SH bands (3 K; 0 without): new Gaussians start with zeros there
    int* out_pixel;
    int* out_count;
    int capacity;
    int nbx, nby;  // 8x8 pixel blocks per row and column
    float t_c, t_w, t_frac, scale_cap, flat_ratio, logit_opacity;
    unsigned int* flags;
    unsigned long long* bits;  // per 8x8 block: bit (8 row + column) set on mask pixels
    unsigned int* blk_cnt;
    unsigned int* blk_off;
    unsigned int* total;
    int* list;     // pixel of each output position
    float* mdepth; // depth of the mask pixels, 0 elsewhere
};

__global__ void __launch_bounds__(256) k_insert_flags(InsertArgs a)
{
    const int n = a.cam.W * a.cam.H;
    const int p = blockIdx.x * 256 + threadIdx.x;
    unsigned int f = 0u;
    if (p < n) {
        const size_t HW = (size_t)n;
        const float e = (fabsf(a.render_rgb[p] - a.frame_rgb[p]) + fabsf(a.render_rgb[HW + p] - a.frame_rgb[HW + p])) +
                        fabsf(a.render_rgb[2 * HW + p] - a.frame_rgb[2 * HW + p]);
        const bool mask = a.depth[p] > 0.0f && e > a.t_c && a.weight[p] < a.t_w;
        f = (mask ? 1u : 0u) | ((mask && a.rnd[p] < a.t_frac) ? 2u : 0u);
        a.flags[p] = f;
        a.mdepth[p] = mask ? a.depth[p] : 0.0f;
    }
    unsigned int tot;
    block_excl_scan<256>((f >> 1) & 1u, &tot);
    if (threadIdx.x == 0) a.blk_cnt[blockIdx.x] = tot;
}

// One wavefront per 8x8 pixel block: lane 8 r + c holds pixel (8 bx + c, 8 by + r).
__global__ void __launch_bounds__(256) k_insert_bits(InsertArgs a)
{
    const int blk = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (blk >= a.nbx * a.nby) return;  // uniform per wavefront
    const int bx = blk % a.nbx, by = blk / a.nbx;
    const int px = bx * 8 + (lane & 7), py = by * 8 + (lane >> 3);
    const bool m = px < a.cam.W && py < a.cam.H && a.mdepth[(size_t)py * a.cam.W + px] > 0.0f;
    const unsigned long long word = __ballot(m);
    if (lane == 0) a.bits[blk] = word;
}

__global__ void __launch_bounds__(1024) k_insert_scan(InsertArgs a, int nblk)
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

// Camera-frame point of pixel (i, j) at depth d.
__device__ __forceinline__ void cam_point(const DevCam& c, int i, int j, float d, float x[3])
{
    x[0] = ((float)i - c.cx) / c.fx * d;
    x[1] = ((float)j - c.cy) / c.fy * d;
    x[2] = d;
}

// The normal and the neighbour distances are rotation- and translation-free, so
// they are formed from camera-frame differences (no world-coordinate
// cancellation in binary32); only the mean and the normal are rotated to the
// world frame, x_w = R^T (x_c - t).
// Per pixel: the output position of each sampled pixel (row-major order) into
// the list, so that the initialisation runs one lane per new Gaussian.
__global__ void __launch_bounds__(256) k_insert_place(InsertArgs a)
{
    const int n = a.cam.W * a.cam.H;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool take = p < n && (a.flags[p] & 2u);
    unsigned int tot;
    const unsigned int excl = block_excl_scan<256>(take ? 1u : 0u, &tot);
    if (!take) return;
    const unsigned int pos = a.blk_off[blockIdx.x] + excl;
    if (pos < (unsigned int)a.capacity) a.list[pos] = p;
}

// Per new Gaussian (position pos < min(sampled, capacity)).
__global__ void __launch_bounds__(256) k_insert_init(InsertArgs a)
{
    const int W = a.cam.W, H = a.cam.H, n = W * H;
    const unsigned int pos = blockIdx.x * 256 + threadIdx.x;
    if (pos >= *a.total || pos >= (unsigned int)a.capacity) return;
    const int p = a.list[pos];
    const int i = p % W, j = p / W;
    const DevCam& c = a.cam;
    float X[3];
    cam_point(c, i, j, a.depth[p], X);
    // normal: central differences of the vertex map, facing the camera (at -X)
    float nc[3] = {-X[0], -X[1], -X[2]};
    if (i > 0 && i < W - 1 && j > 0 && j < H - 1 && a.depth[p - 1] > 0.0f && a.depth[p + 1] > 0.0f &&
        a.depth[p - W] > 0.0f && a.depth[p + W] > 0.0f) {
        float xm[3], xp[3], ym[3], yp[3];
        cam_point(c, i - 1, j, a.depth[p - 1], xm);
        cam_point(c, i + 1, j, a.depth[p + 1], xp);
        cam_point(c, i, j - 1, a.depth[p - W], ym);
        cam_point(c, i, j + 1, a.depth[p + W], yp);
        const float dx[3] = {xp[0] - xm[0], xp[1] - xm[1], xp[2] - xm[2]};
        const float dy[3] = {yp[0] - ym[0], yp[1] - ym[1], yp[2] - ym[2]};
        const float cr[3] = {dx[1] * dy[2] - dx[2] * dy[1], dx[2] * dy[0] - dx[0] * dy[2], dx[0] * dy[1] - dx[1] * dy[0]};
        if (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] > 0.0f) {
            nc[0] = cr[0];
            nc[1] = cr[1];
            nc[2] = cr[2];
        }
    }
    const float inl = 1.0f / sqrtf(nc[0] * nc[0] + nc[1] * nc[1] + nc[2] * nc[2]);
    const float sg = (nc[0] * X[0] + nc[1] * X[1] + nc[2] * X[2]) > 0.0f ? -inl : inl;
#pragma unroll
    for (int k = 0; k < 3; ++k) nc[k] *= sg;
    float nv[3], V[3];
    const float xt[3] = {X[0] - c.t[0], X[1] - c.t[1], X[2] - c.t[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        nv[k] = c.R[k] * nc[0] + c.R[3 + k] * nc[1] + c.R[6 + k] * nc[2];
        V[k] = c.R[k] * xt[0] + c.R[3 + k] * xt[1] + c.R[6 + k] * xt[2];
    }
    // The three nearest other mask vertices over the whole mask (Appendix A), by
    // rings of 8x8 blocks around the query's block.  A pixel column c beyond the
    // scanned window holds only points of the half-space fx x - (c - cx) z <= 0
    // (or >= 0), so no unscanned vertex is nearer than the distance from X to the
    // nearest such plane: the search stops once the third distance is within it.
    // A third distance above sqrt(3) scale_cap gives s1 = scale_cap whatever the
    // exact neighbours are, so the rings stop there as well once three are held.
    const float r2max = 3.0f * a.scale_cap * a.scale_cap;
    float b0 = INFINITY, b1 = INFINITY, b2 = INFINITY;  // squared distances, ascending
    int cnt = 0;
    const int bi = i >> 3, bj = j >> 3;
    // Distance from X (on the ray of pixel column i, depth Z) to the plane through the
    // camera centre holding the rays of column c: |i - c| Z / |(fx, c - cx)| (the
    // integer difference is exact, so the bound has no cancellation); rows alike.
    auto plane_dist = [&](int q, int cq, float f, float cc) {
        const float k = (float)cq - cc;
        return (float)abs(q - cq) * X[2] / sqrtf(f * f + k * k);
    };
    // lower bound of the distance from X to any point of pixel columns [c0, c1], rows [r0, r1]
    auto box_bound = [&](int c0, int c1, int r0, int r1) {
        float lx = 0.0f, ly = 0.0f;
        if (c0 > i) lx = plane_dist(i, c0, c.fx, c.cx);
        else if (c1 < i) lx = plane_dist(i, c1, c.fx, c.cx);
        if (r0 > j) ly = plane_dist(j, r0, c.fy, c.cy);
        else if (r1 < j) ly = plane_dist(j, r1, c.fy, c.cy);
        return fmaxf(lx, ly) * (1.0f - 1e-4f);  // rounding margin: never above the true bound
    };
    for (int r = 0;; ++r) {
        const int bx0 = bi - r, bx1 = bi + r, by0 = bj - r, by1 = bj + r;
        for (int by = max(by0, 0); by <= min(by1, a.nby - 1); ++by) {
            const bool full = by == by0 || by == by1;  // top and bottom rows of the ring: every block
            for (int bx = bx0; bx <= bx1; bx = full ? bx + 1 : (bx == bx0 ? bx1 : bx1 + 1)) {
                if (bx < 0 || bx >= a.nbx) continue;
                const int c0 = bx * 8, r0 = by * 8;
                if (cnt >= 3) {
                    const float lb = box_bound(c0, min(c0 + 7, W - 1), r0, min(r0 + 7, H - 1));
                    if (lb * lb >= b2) continue;
                }
                unsigned long long word = a.bits[(size_t)by * a.nbx + bx];
                while (word) {
                    const int k = __ffsll((long long)word) - 1;
                    word &= word - 1ull;
                    const int ii = c0 + (k & 7), jj = r0 + (k >> 3);
                    if (ii == i && jj == j) continue;
                    float U[3];
                    cam_point(c, ii, jj, a.mdepth[(size_t)jj * W + ii], U);
                    const float d2 = (U[0] - X[0]) * (U[0] - X[0]) + (U[1] - X[1]) * (U[1] - X[1]) +
                                     (U[2] - X[2]) * (U[2] - X[2]);
                    ++cnt;
                    if (d2 < b2) {
                        if (d2 < b1) {
                            b2 = b1;
                            if (d2 < b0) {
                                b1 = b0;
                                b0 = d2;
                            } else {
                                b1 = d2;
                            }
                        } else {
                            b2 = d2;
                        }
                    }
                }
            }
        }
        // distance bound of everything outside the scanned window
        const int x0 = max(bx0, 0) * 8, x1 = min(bx1 * 8 + 7, W - 1);
        const int y0 = max(by0, 0) * 8, y1 = min(by1 * 8 + 7, H - 1);
        float bound = INFINITY;
        if (x0 > 0) bound = fminf(bound, box_bound(0, x0 - 1, j, j));
        if (x1 < W - 1) bound = fminf(bound, box_bound(x1 + 1, W - 1, j, j));
        if (y0 > 0) bound = fminf(bound, box_bound(i, i, 0, y0 - 1));
        if (y1 < H - 1) bound = fminf(bound, box_bound(i, i, y1 + 1, H - 1));
        if (bound == INFINITY) break;                       // the whole image is scanned
        if (cnt >= 3 && b2 <= bound * bound) break;         // exact: nothing unscanned is nearer
        if (cnt >= 3 && bound * bound >= r2max) break;      // the third is beyond sqrt(3) cap: capped
    }
    float s1 = a.scale_cap;
    if (cnt > 0) {
        const int m = cnt < 3 ? cnt : 3;
        const float sum = m == 1 ? b0 : (m == 2 ? b0 + b1 : (b0 + b1) + b2);
        s1 = fminf(a.scale_cap, sqrtf(sum / (float)m));  // root mean square distance
    }
    // shortest-arc rotation taking the local z axis onto the normal; for a normal
    // near -z the scalar part 1 + n_z is formed as (n_x^2 + n_y^2) / (1 - n_z), its
    // value on the unit sphere, so that the rounding of the normalisation cannot
    // leave a spurious 1 + n_z against vanishing n_x, n_y
    const float nxy2 = nv[0] * nv[0] + nv[1] * nv[1];
    float q[4] = {nv[2] < 0.0f ? nxy2 / (1.0f - nv[2]) : 1.0f + nv[2], -nv[1], nv[0], 0.0f};
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    if (qn > 0.0f) {
        q[0] /= qn;
        q[1] /= qn;
        q[2] /= qn;
    } else {
        q[0] = 0.0f;
        q[1] = 1.0f;
        q[2] = 0.0f;
    }
    const size_t C = (size_t)a.capacity, HW = (size_t)n;
#pragma unroll
    for (int k = 0; k < 3; ++k) a.out[0][k * C + pos] = V[k];
    a.out[1][pos] = logf(s1);
    a.out[1][C + pos] = logf(s1);
    a.out[1][2 * C + pos] = logf(a.flat_ratio * s1);
#pragma unroll
    for (int k = 0; k < 4; ++k) a.out[2][k * C + pos] = q[k];
    a.out[3][pos] = a.logit_opacity;
#pragma unroll
    for (int k = 0; k < 3; ++k) a.out[4][k * C + pos] = a.frame_rgb[k * HW + p];
    for (int r = 0; r < a.sh_rows; ++r) a.out[5][r * C + pos] = 0.0f;
    if (a.out_pixel) a.out_pixel[pos] = p;
}

size_t insertion_workspace_bytes(int W, int H)
{
    const size_t n = (size_t)W * H, nblk = n > 0 ? (n + 255) / 256 : 1;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nbits = (size_t)((W + 7) / 8) * ((H + 7) / 8);
    return 3 * al(4 * n) + 2 * al(4 * nblk) + 256 + al(8 * nbits);
}

gps_status launch_insert_gaussians(const gps_insert_cfg* cfg, const DevCam& cam, const float* render_rgb,
                                   const float* frame_rgb, const float* weight, const float* sdf_depth,
                                   const float* rnd, gps_gaussians* out, int* out_pixel, int* out_count, char* ws,
                                   hipStream_t s)
{
    InsertArgs a;
    a.cam = cam;
    a.render_rgb = render_rgb;
    a.frame_rgb = frame_rgb;
    a.weight = weight;
    a.depth = sdf_depth;
    a.rnd = rnd;
    a.out[0] = out->mean, a.out[1] = out->log_scale, a.out[2] = out->quat, a.out[3] = out->opacity_logit,
    a.out[4] = out->rgb;
    a.out[5] = out->sh;
    a.sh_rows = 3 * sh_count(out->sh_degree);
    a.out_pixel = out_pixel;
    a.out_count = out_count;
    a.capacity = out->count;
    a.nbx = (cam.W + 7) / 8;
    a.nby = (cam.H + 7) / 8;
    a.t_c = (float)(3.0 * (double)cfg->delta_c);
    a.t_w = cfg->delta_w;
    a.t_frac = cfg->fraction;
    a.scale_cap = cfg->scale_cap;
    a.flat_ratio = cfg->flat_ratio;
    a.logit_opacity = (float)std::log((double)cfg->opacity / (1.0 - (double)cfg->opacity));
    const size_t n = (size_t)cam.W * cam.H;
    const int nblk = (int)((n + 255) / 256);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nb = nblk > 0 ? (size_t)nblk : 1;
    a.flags = reinterpret_cast<unsigned int*>(ws);
    a.blk_cnt = reinterpret_cast<unsigned int*>(ws + al(4 * n));
    a.blk_off = reinterpret_cast<unsigned int*>(ws + al(4 * n) + al(4 * nb));
    a.total = reinterpret_cast<unsigned int*>(ws + al(4 * n) + 2 * al(4 * nb));
    a.list = reinterpret_cast<int*>(ws + al(4 * n) + 2 * al(4 * nb) + 256);
    a.mdepth = reinterpret_cast<float*>(ws + 2 * al(4 * n) + 2 * al(4 * nb) + 256);
    a.bits = reinterpret_cast<unsigned long long*>(ws + 3 * al(4 * n) + 2 * al(4 * nb) + 256);
    const int nbits = a.nbx * a.nby;
    if (nblk > 0) GPS_LAUNCH(K_INSERT, s, k_insert_flags, dim3(nblk), dim3(256), 0, s, a);
    if (nbits > 0) GPS_LAUNCH(K_INSERT, s, k_insert_bits, dim3((nbits + 3) / 4), dim3(256), 0, s, a);
    GPS_LAUNCH(K_INSERT, s, k_insert_scan, dim3(1), dim3(1024), 0, s, a, nblk);
    const size_t cap = (size_t)a.capacity < n ? (size_t)a.capacity : n;
    if (nblk > 0 && cap > 0) {
        GPS_LAUNCH(K_INSERT, s, k_insert_place, dim3(nblk), dim3(256), 0, s, a);
        GPS_LAUNCH(K_INSERT, s, k_insert_init, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
