// Device helpers shared by the forward and backward render kernels.
#pragma once

#include "gps_internal.h"
#include "sh.h"

namespace gps {

struct GParams {
    const float* mean;
    const float* log_scale;
    const float* quat;
    const float* opacity_logit;
    const float* rgb;
    const float* sh;  // [3][sh_k][M] or null
    int sh_k;         // SH coefficients per channel: 0, 3, 8 or 15
};

struct GGrads {
    float* mean;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* rgb;
    float* sh;
};

// The colour of Gaussian g seen from camera c: rgb plus the SH bands at the unit
// direction from the camera centre o = -R^T t to the centre mu.
__device__ __forceinline__ void view_colour(const GParams& gp, int M, int g, const DevCam& c, float m0, float m1,
                                            float m2, float col[3])
{
    col[0] = gp.rgb[g];
    col[1] = gp.rgb[M + g];
    col[2] = gp.rgb[2 * M + g];
    if (gp.sh_k == 0) return;
    const float v0 = m0 + (c.R[0] * c.t[0] + c.R[3] * c.t[1] + c.R[6] * c.t[2]);
    const float v1 = m1 + (c.R[1] * c.t[0] + c.R[4] * c.t[1] + c.R[7] * c.t[2]);
    const float v2 = m2 + (c.R[2] * c.t[0] + c.R[5] * c.t[1] + c.R[8] * c.t[2]);
    const float ir = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
    float Y[kShMaxK];
    if (gp.sh_k == 15) sh_basis<15>(v0 * ir, v1 * ir, v2 * ir, Y);
    else if (gp.sh_k == 8) sh_basis<8>(v0 * ir, v1 * ir, v2 * ir, Y);
    else sh_basis<3>(v0 * ir, v1 * ir, v2 * ir, Y);
    const int K = gp.sh_k;
    for (int ch = 0; ch < 3; ++ch) {
        float acc = col[ch];
        for (int k = 0; k < K; ++k) acc += gp.sh[((size_t)ch * K + k) * M + g] * Y[k];
        col[ch] = acc;
    }
}

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

// Tile rectangle [tx0, tx1] x [ty0, ty1] of a projected Gaussian from its centre
// (mx, my) and padded pixel half-extents (rxp, ryp).  Every kernel that needs
// the rectangle evaluates this same function on the same stored floats, so
// they all agree on it.  Returns false when no pixel of the image is covered.
struct TileRect {
    int tx0, tx1, ty0, ty1;
};

__device__ __forceinline__ bool rect_of(float mx, float my, float rxp, float ryp, int W, int H, int tw, int th,
                                        TileRect* r)
{
    const float xlo = fmaxf(mx - rxp, 0.0f), xhi = fminf(mx + rxp, (float)(W - 1));
    const float ylo = fmaxf(my - ryp, 0.0f), yhi = fminf(my + ryp, (float)(H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return false;
    const int px0 = (int)ceilf(xlo), px1 = (int)floorf(xhi), py0 = (int)ceilf(ylo), py1 = (int)floorf(yhi);
    if (px0 > px1 || py0 > py1) return false;
    r->tx0 = px0 / tw;
    r->tx1 = px1 / tw;
    r->ty0 = py0 / th;
    r->ty1 = py1 / th;
    return true;
}

// Pixel-to-lane layout of a tile: each wavefront covers a WW x WH block of the
// tile (8x8 for one pixel per lane, 8x16 for two, 16x16 for four), so that a
// Gaussian touching one corner of the tile activates few wavefronts.
template <int TW, int TH, int PPT>
struct TileLayout {
    static constexpr int NT = TW * TH / PPT;
    static constexpr int NW = NT / 64;
    static constexpr int WW = (PPT == 4) ? 16 : 8;
    static constexpr int WH = 64 * PPT / WW;
    static constexpr int NWX = TW / WW;
    static constexpr int LROWS = 64 / WW;  // rows between a lane's successive pixels
    static_assert(NW * 64 == NT && NWX * WW == TW && (NW / NWX) * WH == TH, "tile layout");
    __device__ static int wave_x0(int wid) { return (wid % NWX) * WW; }
    __device__ static int wave_y0(int wid) { return (wid / NWX) * WH; }
    __device__ static int lane_x(int lane) { return lane % WW; }
    __device__ static int lane_y(int lane) { return lane / WW; }
};

// Whether a record's opacity can reach alpha_min at some pixel of a rectangle
// of pixels [x0, x0 + w - 1] x [y0, y0 + h - 1] (the support ellipse of Eq. 3
// against the rectangle, not its bounding box).  The per-pixel test is
// l2s + A dx^2 + B dx dy + C dy^2 >= log2(alpha_min) with the record's
// binary32 coefficients (A, C < 0, B^2 < 4AC: a concave quadratic).  Its largest
// value over a box is 0 when the box holds the centre, else on an edge, where
// it is the one-variable maximum clamped to the edge: dy = -B dx / (2C) on the
// edges of fixed dx, dx = -B dy / (2A) on those of fixed dy.  The box is the
// rectangle grown by one pixel on every side and the threshold is lowered by a
// small slack, so that every pixel passing the rounded per-pixel test (which
// lies within one pixel of the exact ellipse) is in a rectangle that passes.
struct SupportTest {
    float mx, my, A, B, C, kx, ky, need;
    __device__ SupportTest(const float4& r0, const float4& r1, float l2amin)
        : mx(r0.x), my(r0.y), A(r0.z), B(r0.w), C(r1.x)
    {
        kx = -0.5f * B * __builtin_amdgcn_rcpf(A);
        ky = -0.5f * B * __builtin_amdgcn_rcpf(C);
        need = (l2amin - r1.y) * 1.0001f - 1e-4f;  // log2(alpha_min / sigma), with slack
    }
    __device__ float at(float dx, float dy) const { return dx * (A * dx + B * dy) + C * dy * dy; }
    __device__ bool meets(float x0, float y0, float w, float h) const
    {
        const float X0 = (x0 - 1.0f) - mx, X1 = (x0 + w) - mx;
        const float Y0 = (y0 - 1.0f) - my, Y1 = (y0 + h) - my;
        if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return true;
        const float e0 = at(X0, fminf(fmaxf(ky * X0, Y0), Y1));
        const float e1 = at(X1, fminf(fmaxf(ky * X1, Y0), Y1));
        const float e2 = at(fminf(fmaxf(kx * Y0, X0), X1), Y0);
        const float e3 = at(fminf(fmaxf(kx * Y1, X0), X1), Y1);
        return !(fmaxf(fmaxf(e0, e1), fmaxf(e2, e3)) < need);  // a NaN keeps the record
    }
};

// Wavefronts of a tile (origin tx0, ty0) whose pixel rectangle the record's
// support meets: bit w for wavefront w.  A wavefront outside the support has
// opacity below alpha_min at every one of its pixels, so it may skip the record.
template <class Lay>
__device__ __forceinline__ unsigned int wave_support_mask(const float4& r0, const float4& r1, float l2amin, int tx0,
                                                          int ty0)
{
    static_assert(Lay::NW <= 32, "wavefront mask fits 32 bits");
    const SupportTest st(r0, r1, l2amin);
    unsigned int mk = 0u;
#pragma unroll
    for (int wv = 0; wv < Lay::NW; ++wv) {
        const float x0 = (float)(tx0 + Lay::wave_x0(wv)), y0 = (float)(ty0 + Lay::wave_y0(wv));
        if (st.meets(x0, y0, (float)Lay::WW, (float)Lay::WH)) mk |= 1u << wv;
    }
    return mk;
}

// Tile configurations (tile width, height, staged batch, pixels per lane) for
// which both compositing kernels are instantiated.  A 32-pixel-wide tile reads
// each row of a float image plane as one whole 128-byte line.
#define GPS_TILE_CONFIGS(X) \
    X(8, 8, 128, 1)         \
    X(8, 8, 256, 1)         \
    X(8, 8, 512, 1)         \
    X(16, 16, 128, 1)       \
    X(16, 16, 256, 1)       \
    X(16, 16, 128, 2)       \
    X(16, 16, 256, 2)       \
    X(16, 16, 512, 2)       \
    X(16, 16, 128, 4)       \
    X(16, 16, 256, 4)       \
    X(16, 16, 512, 4)       \
    X(16, 32, 128, 1)       \
    X(16, 32, 128, 2)       \
    X(16, 32, 256, 2)       \
    X(16, 32, 128, 4)       \
    X(16, 32, 256, 4)       \
    X(16, 32, 512, 4)       \
    X(32, 16, 128, 2)       \
    X(32, 16, 256, 2)

}  // namespace gps
