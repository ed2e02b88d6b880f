// Device code shared by the dense lattice (sdf.hip) and the voxel-block hash
// (hash.hip): the fusion update of one lattice point and the per-pixel ray march,
// the latter templated on how lattice values are read (a Field), so that both
// stores take the same binary32 decisions and evaluate the same values.
#pragma once

#include <cmath>

#include "gps_internal.h"

namespace gps {

// ----------------------------------------------------------------- fusion
struct FuseCtx {
    float ox, oy, oz, voxel, mu, wmax;
    DevCam cam;
    const float* depth;
    const float* img;
};

// Fusion of lattice point (x, y, z) (Sec. 3.2.1 "SDF fusion"): nearest pixel of
// its projection, eta = d - z; points with eta < -mu are left alone; otherwise the
// truncated value min(1, eta / mu) is averaged in with a capped weight, and the
// colour inside |eta| <= mu with its own weight.  The point's values sit at `idx`
// of the planes; the three colour planes are `stride` apart.
__device__ __forceinline__ void fuse_point(const FuseCtx& a, int x, int y, int z, size_t idx, size_t stride,
                                           float* __restrict__ tsdf, float* __restrict__ wt,
                                           float* __restrict__ col, float* __restrict__ cwt)
{
    const DevCam& c = a.cam;
    float zc, eta;
    int i, j;
    {
#pragma clang fp contract(off)
        float p0 = d32_lattice(a.ox, a.voxel, x);
        float p1 = d32_lattice(a.oy, a.voxel, y);
        float p2 = d32_lattice(a.oz, a.voxel, z);
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
    const float w = wt[idx];
    const float tv = tsdf[idx];
    tsdf[idx] = (w * tv + f) / (w + 1.0f);
    wt[idx] = fminf(w + 1.0f, a.wmax);
    if (band) {
        const float wc = cwt[idx];
        const size_t HW = (size_t)c.W * c.H;
        const size_t p = (size_t)j * c.W + i;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float obs = a.img[ch * HW + p];
            float* cp = col + (size_t)ch * stride + idx;
            *cp = (wc * *cp + obs) / (wc + 1.0f);
        }
        cwt[idx] = fminf(wc + 1.0f, a.wmax);
    }
}

// ---------------------------------------------------------------- raycast
// Geometry of a march: the region's lattice (points 0 .. n-1 per axis at
// origin + voxel * index), the step and the views.
struct MarchArgs {
    int n[3];
    float origin[3];
    float voxel, inv_voxel, h, inv_h, z_near;
    int max_steps;
    int n_views;
    DevCam cams[GPS_MAX_VIEWS];
    float* out_depth[GPS_MAX_VIEWS];
    float* out_rgb[GPS_MAX_VIEWS];
};

// A Field provides
//   void fetch8(int plane, const int b[3], float q[8]) const
//       the values of plane 0 (tsdf) or 1..3 (colour) at the 2x2x2 stencil based
//       at lattice point b (q[dx + 2 dy + 4 dz]; b and b + 1 inside the lattice);
//   bool skip_box(const int b[3], float lo[3], float hi[3]) const
//       true when every sample whose stencil base lies in the box [lo, hi) (lattice
//       coordinates, containing b) reads positive; the box is then skipped;
//   bool depth_range(int view, int col, int row, float* zlo, float* zhi) const
//       true when every sample of the pixel's ray outside the camera depths
//       [zlo, zhi] reads positive (zlo > zhi: all of them); false: no such bound.

// binary32 trilinear of the tsdf (decision arithmetic); +1 where the stencil
// leaves the lattice.
template <class Fld>
__device__ __forceinline__ float dec_trilinear(const MarchArgs& a, const Fld& fld, const float g[3], int* inside)
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
    float q[8];
    fld.fetch8(0, bi, q);
    float c00 = d32_lerp(q[0], q[1], fr[0]);
    float c10 = d32_lerp(q[2], q[3], fr[0]);
    float c01 = d32_lerp(q[4], q[5], fr[0]);
    float c11 = d32_lerp(q[6], q[7], fr[0]);
    float c0 = d32_lerp(c00, c10, fr[1]);
    float c1 = d32_lerp(c01, c11, fr[1]);
    return d32_lerp(c0, c1, fr[2]);
}

// Trilinear of a plane with the stencil clamped into the lattice (values).
template <class Fld>
__device__ __forceinline__ float val_trilinear(const MarchArgs& a, const Fld& fld, int plane, const float p[3])
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
    float q[8];
    fld.fetch8(plane, bi, q);
    float c00 = q[0] + fr[0] * (q[1] - q[0]);
    float c10 = q[2] + fr[0] * (q[3] - q[2]);
    float c01 = q[4] + fr[0] * (q[5] - q[4]);
    float c11 = q[6] + fr[0] * (q[7] - q[6]);
    float c0 = c00 + fr[1] * (c10 - c00);
    float c1 = c01 + fr[1] * (c11 - c01);
    return c0 + fr[2] * (c1 - c0);
}

// One pixel's ray (Sec. 3.1 first pass): march with step h from depth z_near
// inside the lattice box until the trilinear signed distance turns from positive
// to non-positive (binary32 decisions, fixed order), refine by the secant, and
// write the camera depth of the crossing and its trilinear colour (0 on a miss).
template <class Fld>
__device__ __forceinline__ void march_pixel(const MarchArgs& a, const Fld& fld, int view, int col, int row)
{
    const DevCam& c = a.cams[view];
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

    // A depth interval outside which every sample reads positive: the march covers
    // its samples only (two steps of margin on each side cover the rounding of the
    // bounds, which are values only).  The sample before the first one marched is
    // then known positive, as after a skipped box.
    int s_first = 0;
    {
        float zlo, zhi;
        if (fld.depth_range(view, col, row, &zlo, &zhi)) {
            if (!(zlo <= zhi)) {
                nsteps = -1;
            } else {
                const float shi = ceilf((zhi * rn - lam0) * a.inv_h) + 2.0f;
                const float slo = floorf((zlo * rn - lam0) * a.inv_h) - 2.0f;
                if (shi < (float)nsteps) nsteps = shi < 0.0f ? -1 : (int)shi;
                if (slo > 0.0f) s_first = slo < (float)(nsteps + 1) ? (int)slo : nsteps + 1;
            }
        }
    }

    // Lattice-space ray for box exits (values only, never decides a crossing).
    float g0[3], gd[3], igd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g0[k] = (o[k] - a.origin[k]) * a.inv_voxel;
        gd[k] = dh[k] * a.inv_voxel;
        igd[k] = gd[k] != 0.0f ? 1.0f / gd[k] : 0.0f;
    }

    float Fprev = 0.0f;
    int prev_inside = 0, prev_skipped = 0;
    if (s_first > 0) {
        Fprev = 1.0f;
        prev_inside = 1;
        prev_skipped = 1;
    }
    int hit = -1;
    float Fhit = 0.0f;
    for (int s = s_first; s <= nsteps; ++s) {
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
        {
            const float b0 = floorf(g[0]), b1 = floorf(g[1]), b2 = floorf(g[2]);
            if (b0 >= 0.0f && b1 >= 0.0f && b2 >= 0.0f && b0 <= (float)(a.n[0] - 2) && b1 <= (float)(a.n[1] - 2) &&
                b2 <= (float)(a.n[2] - 2)) {
                const int bi[3] = {(int)b0, (int)b1, (int)b2};
                float lo[3], hi[3];
                if (fld.skip_box(bi, lo, hi)) {
                    // Every sample whose base lies in this box is positive.  Samples at least
                    // one step before the ray's exit from the box are inside it (the exit and
                    // the step count are values only: the step of margin covers their rounding).
                    float lam_exit = INFINITY;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        if (gd[k] > 0.0f)
                            lam_exit = fminf(lam_exit, (hi[k] - g0[k]) * igd[k]);
                        else if (gd[k] < 0.0f)
                            lam_exit = fminf(lam_exit, (lo[k] - g0[k]) * igd[k]);
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
        float F = dec_trilinear(a, fld, g, &inside);
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
    float la;
    {
#pragma clang fp contract(off)
        float kf = (float)(hit - 1);
        la = kf * a.h;
        la = lam0 + la;
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
        Fprev = dec_trilinear(a, fld, g, &prev_inside);
    }
    const float Fa = prev_inside ? Fprev : 1.0f;
    const float lam_star = la + a.h * Fa / (Fa - Fhit);
    float V[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = o[k] + lam_star * dh[k];
    const float zc = c.R[6] * V[0] + c.R[7] * V[1] + c.R[8] * V[2] + c.t[2];
    od[pix] = zc;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) oc[ch * HW + pix] = val_trilinear(a, fld, 1 + ch, V);
}

inline void march_setup(MarchArgs* a, int nx, int ny, int nz, const float origin[3], float voxel, float z_near,
                        float step, const gps_camera* cams, int n_views, float* const* out_depth,
                        float* const* out_rgb, int* maxW, int* maxH)
{
    a->n[0] = nx;
    a->n[1] = ny;
    a->n[2] = nz;
    for (int k = 0; k < 3; ++k) a->origin[k] = origin[k];
    a->voxel = voxel;
    a->inv_voxel = 1.0f / voxel;
    a->h = step > 0.0f ? step : voxel * 0.5f;
    a->z_near = z_near;
    {
        const double diag = voxel * std::sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
        const double ms = diag / a->h + 4.0;
        a->max_steps = (int)(ms < 1.0e8 ? ms : 1.0e8);
    }
    a->inv_h = 1.0f / a->h;
    a->n_views = n_views;
    *maxW = 0;
    *maxH = 0;
    for (int v = 0; v < n_views; ++v) {
        a->cams[v] = dev_cam(cams[v]);
        a->out_depth[v] = out_depth[v];
        a->out_rgb[v] = out_rgb[v];
        if (cams[v].width > *maxW) *maxW = cams[v].width;
        if (cams[v].height > *maxH) *maxH = cams[v].height;
    }
}

}  // namespace gps
