// TSDF + colour fusion and SDF raycast (Sec. 3.1 first pass, Sec. 3.2.1).
//
// Fusion is one lane per lattice point, lanes along x so that the volume
// arrays stream coalesced; only points in the frustum with a valid depth
// sample read and write the volume, so traffic is 8 B/point outside the
// truncation band and 32 B/point inside it (read + write).
//
// The raycast is one lane per pixel.  The march decides the crossing sample in
// binary32 with a fixed evaluation order (the same order every implementation
// of this path uses, so the crossing index is reproducible), and skips samples
// whose 2x2x2 stencil lies in an 8^3 brick whose minimum signed distance is
// positive -- such samples cannot be a crossing, so skipping them does not
// change which sample is found.
#include <algorithm>
#include <cmath>

#include "gps_internal.h"
#include "launch.h"
#include "prof.h"

namespace gps {

// ----------------------------------------------------------------- fusion
struct FuseArgs {
    int nx, ny, nz;
    float ox, oy, oz, voxel, mu, wmax;
    unsigned int N;
    DevCam cam;
    const float* depth;
    const float* img;
    float* tsdf;
    float* w;
    float* col;
    float* cw;
};

__global__ void __launch_bounds__(256) k_fuse(FuseArgs a)
{
    const unsigned int idx = blockIdx.x * 256u + threadIdx.x;
    if (idx >= a.N) return;
    const unsigned int x = idx % (unsigned)a.nx;
    const unsigned int r = idx / (unsigned)a.nx;
    const unsigned int y = r % (unsigned)a.ny;
    const unsigned int z = r / (unsigned)a.ny;
    const DevCam& c = a.cam;
    float zc, eta;
    int i, j;
    {
#pragma clang fp contract(off)
        float p0 = d32_lattice(a.ox, a.voxel, (int)x);
        float p1 = d32_lattice(a.oy, a.voxel, (int)y);
        float p2 = d32_lattice(a.oz, a.voxel, (int)z);
        float xc = d32_row(c.R, c.t, 0, p0, p1, p2);
        float yc = d32_row(c.R, c.t, 1, p0, p1, p2);
        zc = d32_row(c.R, c.t, 2, p0, p1, p2);
        if (!(zc > 0.0f)) return;
        float u = c.fx * xc;
        u = u / zc;
        u = u + c.cx;
        float v = c.fy * yc;
        v = v / zc;
        v = v + c.cy;
        float fu = floorf(u + 0.5f);
        float fv = floorf(v + 0.5f);
        if (!(fu >= 0.0f && fu < (float)c.W && fv >= 0.0f && fv < (float)c.H)) return;
        i = (int)fu;
        j = (int)fv;
        float d = a.depth[(size_t)j * c.W + i];
        if (!(d > 0.0f)) return;
        eta = d - zc;
        if (eta < -a.mu) return;
    }
    const bool band = fabsf(eta) <= a.mu;
    const float f = fminf(1.0f, eta / a.mu);
    const float w = a.w[idx];
    const float tv = a.tsdf[idx];
    a.tsdf[idx] = (w * tv + f) / (w + 1.0f);
    a.w[idx] = fminf(w + 1.0f, a.wmax);
    if (band) {
        const float wc = a.cw[idx];
        const size_t HW = (size_t)c.W * c.H;
        const size_t p = (size_t)j * c.W + i;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float obs = a.img[ch * HW + p];
            float* cp = a.col + (size_t)ch * a.N + idx;
            *cp = (wc * *cp + obs) / (wc + 1.0f);
        }
        a.cw[idx] = fminf(wc + 1.0f, a.wmax);
    }
}

gps_status launch_fuse(const gps_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                       hipStream_t s)
{
    FuseArgs a;
    a.nx = vol->nx;
    a.ny = vol->ny;
    a.nz = vol->nz;
    a.ox = vol->origin[0];
    a.oy = vol->origin[1];
    a.oz = vol->origin[2];
    a.voxel = vol->voxel;
    a.mu = vol->trunc;
    a.wmax = vol->max_weight;
    a.N = (unsigned int)((size_t)vol->nx * vol->ny * vol->nz);
    a.cam = dev_cam(*cam);
    a.depth = depth;
    a.img = rgb;
    a.tsdf = vol->tsdf;
    a.w = vol->weight;
    a.col = vol->rgb;
    a.cw = vol->rgb_weight;
    unsigned int blocks = (a.N + 255u) / 256u;
    GPS_LAUNCH(K_FUSE, s, k_fuse, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

// ------------------------------------------------------------ brick minimum
// bmin[b] = min tsdf over lattice points [8b, 8b+8] (clipped), i.e. every
// 2x2x2 stencil whose base point lies in brick b.
struct BrickArgs {
    int nx, ny, nz, bx, by, bz;
    const float* tsdf;
    float* bmin;
};

// Brick minima: one wavefront per 8^3 brick, over its 9^3 lattice points (the
// brick and the first plane of its +x, +y, +z neighbours: every 2x2x2 sample
// stencil based in the brick), four bricks per block.
__global__ void __launch_bounds__(256) k_brick_min(BrickArgs a)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= a.bx * a.by * a.bz) return;
    const int bxi = b % a.bx, byi = (b / a.bx) % a.by, bzi = b / (a.bx * a.by);
    const int x0 = bxi * kBrick, y0 = byi * kBrick, z0 = bzi * kBrick;
    float m = INFINITY;
    for (int k = lane; k < 9 * 9 * 9; k += 64) {
        const int dx = k % 9, dy = (k / 9) % 9, dz = k / 81;
        const int x = x0 + dx, y = y0 + dy, z = z0 + dz;
        if (x < a.nx && y < a.ny && z < a.nz) m = fminf(m, a.tsdf[x + (size_t)a.nx * (y + (size_t)a.ny * z)]);
    }
    m = -wave_max(-m);
    if (lane == 0) a.bmin[b] = m;
}

// Superbricks of kSuper^3 = 64 bricks: the minimum of their bricks' minima (one
// wavefront each, a lane per brick), so a superbrick above the threshold has
// every sample stencil based in it positive.
constexpr int kSuper = 4;

__global__ void __launch_bounds__(256) k_super_min(const float* __restrict__ bmin, float* __restrict__ smin, int bx,
                                                   int by, int bz, int sx, int sy, int sz)
{
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= sx * sy * sz) return;
    const int jx = t % sx, jy = (t / sx) % sy, jz = t / (sx * sy);
    const int x = jx * kSuper + (lane & 3), y = jy * kSuper + ((lane >> 2) & 3), z = jz * kSuper + (lane >> 4);
    float m = (x < bx && y < by && z < bz) ? bmin[x + bx * (y + by * z)] : INFINITY;
    m = -wave_max(-m);
    if (lane == 0) smin[t] = m;
}

// ---------------------------------------------------------------- raycast
struct RayArgs {
    int n[3];
    float origin[3];
    float voxel, inv_voxel, h, inv_h, z_near;
    int bx, by, bz;
    int sx, sy;  // superbricks along x and y
    int max_steps;
    const float* tsdf;
    const float* rgb;
    const float* bmin;  // may be null
    const float* smin;  // superbrick minima (null with bmin)
    size_t N;
    int n_views;
    DevCam cams[GPS_MAX_VIEWS];
    float* out_depth[GPS_MAX_VIEWS];
    float* out_rgb[GPS_MAX_VIEWS];
};

// binary32 trilinear of the tsdf (decision arithmetic); returns +1 outside.
__device__ __forceinline__ float dec_trilinear(const RayArgs& a, const float g[3], int* inside)
{
#pragma clang fp contract(off)
    float b[3], fr[3];
    int bi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        b[k] = floorf(g[k]);
        fr[k] = g[k] - b[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!(b[k] >= 0.0f && b[k] <= (float)(a.n[k] - 2))) {
            *inside = 0;
            return 1.0f;
        }
        bi[k] = (int)b[k];
    }
    *inside = 1;
    const size_t sx = 1, sy = (size_t)a.n[0], sz = (size_t)a.n[0] * a.n[1];
    const float* p = a.tsdf + bi[0] + sy * bi[1] + sz * bi[2];
    float v000 = p[0], v100 = p[sx], v010 = p[sy], v110 = p[sy + sx];
    float v001 = p[sz], v101 = p[sz + sx], v011 = p[sz + sy], v111 = p[sz + sy + sx];
    float c00 = d32_lerp(v000, v100, fr[0]);
    float c10 = d32_lerp(v010, v110, fr[0]);
    float c01 = d32_lerp(v001, v101, fr[0]);
    float c11 = d32_lerp(v011, v111, fr[0]);
    float c0 = d32_lerp(c00, c10, fr[1]);
    float c1 = d32_lerp(c01, c11, fr[1]);
    return d32_lerp(c0, c1, fr[2]);
}

// Trilinear of a field with the stencil clamped into the lattice (values).
__device__ __forceinline__ float val_trilinear(const RayArgs& a, const float* f, const float p[3])
{
    int bi[3];
    float fr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float g = (p[k] - a.origin[k]) * a.inv_voxel;
        float b = floorf(g);
        b = fminf(fmaxf(b, 0.0f), (float)(a.n[k] - 2));
        fr[k] = fminf(fmaxf(g - b, 0.0f), 1.0f);
        bi[k] = (int)b;
    }
    const size_t sy = (size_t)a.n[0], sz = (size_t)a.n[0] * a.n[1];
    const float* q = f + bi[0] + sy * bi[1] + sz * bi[2];
    float c00 = q[0] + fr[0] * (q[1] - q[0]);
    float c10 = q[sy] + fr[0] * (q[sy + 1] - q[sy]);
    float c01 = q[sz] + fr[0] * (q[sz + 1] - q[sz]);
    float c11 = q[sz + sy] + fr[0] * (q[sz + sy + 1] - q[sz + sy]);
    float c0 = c00 + fr[1] * (c10 - c00);
    float c1 = c01 + fr[1] * (c11 - c01);
    return c0 + fr[2] * (c1 - c0);
}

__global__ void __launch_bounds__(256) k_raycast(RayArgs a)
{
    const int view = blockIdx.z;
    const DevCam& c = a.cams[view];
    const int col = blockIdx.x * 16 + (threadIdx.x & 15);
    const int row = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (col >= c.W || row >= c.H) return;
    const size_t HW = (size_t)c.W * c.H;
    const size_t pix = (size_t)row * c.W + col;
    float* od = a.out_depth[view];
    float* oc = a.out_rgb[view];

    float o[3], dh[3], lam0, lam1, rn;
    int nsteps;
    {
#pragma clang fp contract(off)
        float rx = ((float)col - c.cx) / c.fx;
        float ry = ((float)row - c.cy) / c.fy;
        float dir[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = c.R[0 * 3 + k] * c.t[0];
            float u = c.R[1 * 3 + k] * c.t[1];
            s = s + u;
            float w = c.R[2 * 3 + k] * c.t[2];
            s = s + w;
            o[k] = -s;
            float s2 = c.R[0 * 3 + k] * rx;
            float u2 = c.R[1 * 3 + k] * ry;
            s2 = s2 + u2;
            s2 = s2 + c.R[2 * 3 + k];
            dir[k] = s2;
        }
        float rn2 = rx * rx;
        float ry2 = ry * ry;
        rn2 = rn2 + ry2;
        rn2 = rn2 + 1.0f;
        rn = sqrtf(rn2);
#pragma unroll
        for (int k = 0; k < 3; ++k) dh[k] = dir[k] / rn;
        lam0 = a.z_near * rn;
        lam1 = INFINITY;
        bool miss = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float lo = a.origin[k];
            float span = a.voxel * (float)(a.n[k] - 1);
            float hi = lo + span;
            if (dh[k] != 0.0f) {
                float t1 = (lo - o[k]) / dh[k];
                float t2 = (hi - o[k]) / dh[k];
                float tmn = t1 < t2 ? t1 : t2;
                float tmx = t1 < t2 ? t2 : t1;
                if (tmn > lam0) lam0 = tmn;
                if (tmx < lam1) lam1 = tmx;
            } else if (o[k] < lo || o[k] > hi) {
                miss = true;
            }
        }
        if (miss || !(lam0 < lam1)) {
            od[pix] = 0.0f;
            oc[pix] = 0.0f;
            oc[HW + pix] = 0.0f;
            oc[2 * HW + pix] = 0.0f;
            return;
        }
        float span_l = lam1 - lam0;
        float ns = floorf(span_l / a.h);
        // the lattice diagonal bounds the march; this only guards the float->int conversion
        nsteps = ns < (float)a.max_steps ? (int)ns : a.max_steps;
    }

    // Lattice-space ray for brick exits (values only, never decides a crossing).
    float g0[3], gd[3], igd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g0[k] = (o[k] - a.origin[k]) * a.inv_voxel;
        gd[k] = dh[k] * a.inv_voxel;
        igd[k] = gd[k] != 0.0f ? 1.0f / gd[k] : 0.0f;
    }

    float Fprev = 0.0f;
    int prev_inside = 0, prev_skipped = 0;
    int hit = -1;
    float Fhit = 0.0f;
    for (int s = 0; s <= nsteps; ++s) {
        float g[3];
        {
#pragma clang fp contract(off)
            float kf = (float)s;
            float lam = kf * a.h;
            lam = lam0 + lam;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float q = lam * dh[k];
                q = o[k] + q;
                q = q - a.origin[k];
                g[k] = q * a.inv_voxel;
            }
        }
        if (a.bmin) {
            float b0 = floorf(g[0]), b1 = floorf(g[1]), b2 = floorf(g[2]);
            if (b0 >= 0.0f && b1 >= 0.0f && b2 >= 0.0f && b0 <= (float)(a.n[0] - 2) && b1 <= (float)(a.n[1] - 2) &&
                b2 <= (float)(a.n[2] - 2)) {
                const int i0 = (int)b0 >> 3, i1 = (int)b1 >> 3, i2 = (int)b2 >> 3;
                const int j0 = i0 / kSuper, j1 = i1 / kSuper, j2 = i2 / kSuper;
                int edge = 0, bb[3];
                if (a.smin[j0 + a.sx * (j1 + a.sy * j2)] > kBrickPositive) {
                    edge = kBrick * kSuper;  // the whole superbrick is positive
                    bb[0] = j0;
                    bb[1] = j1;
                    bb[2] = j2;
                } else if (a.bmin[i0 + a.bx * (i1 + a.by * i2)] > kBrickPositive) {
                    edge = kBrick;
                    bb[0] = i0;
                    bb[1] = i1;
                    bb[2] = i2;
                }
                if (edge) {
                    // Every sample whose base lies in this box is positive.  Samples at least
                    // one step before the ray's exit from the box are inside it (the exit and
                    // the step count are values only: the step of margin covers their rounding).
                    float lam_exit = INFINITY;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        if (gd[k] > 0.0f)
                            lam_exit = fminf(lam_exit, ((float)((bb[k] + 1) * edge) - g0[k]) * igd[k]);
                        else if (gd[k] < 0.0f)
                            lam_exit = fminf(lam_exit, ((float)(bb[k] * edge) - g0[k]) * igd[k]);
                    }
                    int s_last = (int)floorf((lam_exit - lam0) * a.inv_h) - 1;
                    if (s_last > nsteps) s_last = nsteps;
                    if (s_last < s) s_last = s;
                    s = s_last;
                    Fprev = 1.0f;  // known positive; recomputed if it brackets the crossing
                    prev_inside = 1;
                    prev_skipped = 1;
                    continue;
                }
            }
        }
        int inside;
        float F = dec_trilinear(a, g, &inside);
        if (s >= 1 && Fprev > 0.0f && F <= 0.0f) {
            hit = s;
            Fhit = F;
            break;
        }
        Fprev = F;
        prev_inside = inside;
        prev_skipped = 0;
    }
    if (hit < 0) {
        od[pix] = 0.0f;
        oc[pix] = 0.0f;
        oc[HW + pix] = 0.0f;
        oc[2 * HW + pix] = 0.0f;
        return;
    }
    float la, lb;
    {
#pragma clang fp contract(off)
        float kf = (float)(hit - 1);
        la = kf * a.h;
        la = lam0 + la;
        float kb = (float)hit;
        lb = kb * a.h;
        lb = lam0 + lb;
    }
    if (prev_skipped) {
        // the bracketing sample was skipped: evaluate it (it is positive)
        float g[3];
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float q = la * dh[k];
                q = o[k] + q;
                q = q - a.origin[k];
                g[k] = q * a.inv_voxel;
            }
        }
        Fprev = dec_trilinear(a, g, &prev_inside);
    }
    const float Fa = prev_inside ? Fprev : 1.0f;
    const float lam_star = la + a.h * Fa / (Fa - Fhit);
    float V[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = o[k] + lam_star * dh[k];
    const float zc = c.R[6] * V[0] + c.R[7] * V[1] + c.R[8] * V[2] + c.t[2];
    (void)lb;
    od[pix] = zc;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) oc[ch * HW + pix] = val_trilinear(a, a.rgb + ch * a.N, V);
}

gps_status launch_raycast(const gps_volume* vol, const gps_camera* cams, int n_views, float* const* out_depth,
                          float* const* out_rgb, float z_near, float step, hipStream_t s)
{
    RayArgs a;
    a.n[0] = vol->nx;
    a.n[1] = vol->ny;
    a.n[2] = vol->nz;
    for (int k = 0; k < 3; ++k) a.origin[k] = vol->origin[k];
    a.voxel = vol->voxel;
    a.inv_voxel = 1.0f / vol->voxel;
    a.h = step > 0.0f ? step : vol->voxel * 0.5f;
    a.z_near = z_near;
    {
        const double diag = vol->voxel * std::sqrt((double)vol->nx * vol->nx + (double)vol->ny * vol->ny +
                                                   (double)vol->nz * vol->nz);
        a.max_steps = (int)std::min(diag / a.h + 4.0, 1.0e8);
    }
    a.inv_h = 1.0f / a.h;
    a.bx = (vol->nx + kBrick - 1) / kBrick;
    a.by = (vol->ny + kBrick - 1) / kBrick;
    a.bz = (vol->nz + kBrick - 1) / kBrick;
    a.sx = (a.bx + kSuper - 1) / kSuper;
    a.sy = (a.by + kSuper - 1) / kSuper;
    const int sz = (a.bz + kSuper - 1) / kSuper;
    a.tsdf = vol->tsdf;
    a.rgb = vol->rgb;
    a.bmin = vol->brick_min;
    a.smin = vol->brick_min ? vol->brick_min + (size_t)a.bx * a.by * a.bz : nullptr;
    a.N = (size_t)vol->nx * vol->ny * vol->nz;
    a.n_views = n_views;
    int maxW = 0, maxH = 0;
    for (int v = 0; v < n_views; ++v) {
        a.cams[v] = dev_cam(cams[v]);
        a.out_depth[v] = out_depth[v];
        a.out_rgb[v] = out_rgb[v];
        if (cams[v].width > maxW) maxW = cams[v].width;
        if (cams[v].height > maxH) maxH = cams[v].height;
    }
    if (vol->brick_min) {
        BrickArgs b{vol->nx, vol->ny, vol->nz, a.bx, a.by, a.bz, vol->tsdf, vol->brick_min};
        GPS_LAUNCH(K_BRICK_MIN, s, k_brick_min, dim3((a.bx * a.by * a.bz + 3) / 4), dim3(256), 0, s, b);
        const int ns = a.sx * a.sy * sz;
        GPS_LAUNCH(K_BRICK_MIN, s, k_super_min, dim3((ns + 3) / 4), dim3(256), 0, s, vol->brick_min,
                   vol->brick_min + (size_t)a.bx * a.by * a.bz, a.bx, a.by, a.bz, a.sx, a.sy, sz);
        if (hipGetLastError() != hipSuccess) return GPS_ERR_HIP;
    }
    dim3 grid((maxW + 15) / 16, (maxH + 15) / 16, n_views);
    GPS_LAUNCH(K_RAYCAST, s, k_raycast, grid, dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
