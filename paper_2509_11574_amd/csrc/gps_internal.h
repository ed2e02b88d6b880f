// Internal definitions shared by the HIP translation units of libgps.
// Device layouts, the workspace map, the binary32 decision arithmetic and
// wavefront helpers.  Nothing here is part of the public ABI (include/gps.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gps.h"

namespace gps {

constexpr int kBrick = 8;             // empty-space-skipping brick edge (lattice points)
constexpr float kBrickPositive = 1e-3f;  // a brick whose minimum exceeds this reads positive
constexpr int kSortCap = 8192;        // longest tile list sorted in LDS (64 KiB of keys)
constexpr int kRecFloats = 12;        // projected record: 48 bytes
constexpr int kAdj = 10;              // screen-space adjoints per instance
constexpr int kBlk = 256;             // threads per block of the per-Gaussian kernels
constexpr int kFlush = 32;            // records between flushes of the backward's per-wavefront partials

// ---------------------------------------------------------------------------
// Camera / view tables passed by value as kernel arguments.
// ---------------------------------------------------------------------------
struct DevCam {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    int W, H;
};

inline DevCam dev_cam(const gps_camera& c)
{
    DevCam d;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
    d.W = c.width;
    d.H = c.height;
    return d;
}

struct DevView {
    DevCam cam;
    int tiles_x, tiles_y, tile_base;
    int pix_base;  // offset of this view's pixels in the per-pixel workspace plane
    const float* base_rgb;
    const float* base_depth;
    const float* target_rgb;
    const float* target_depth;
    float* out_rgb;
    float* out_depth;
    const float* g_rgb;    // explicit upstream adjoints (backward), or null
    const float* g_depth;
    const float* pose_xi;  // [6] left perturbation applied at upload, or null
    float* out_aux;        // [H][W] T_final / W_G copy for the caller, or null
};

struct ViewTable {
    int n;
    int n_tiles;  // over all views
    DevView v[GPS_MAX_VIEWS];
};

// Renderer constants.
struct RParams {
    float eps, lambda, dil, amin, amax, Tmin, znear;
    int mode;
    int M;          // Gaussians
    int V;          // views
    int nvg;        // V * M
    int tile_w, tile_h;
    unsigned long long cap;  // instance capacity
};

// ---------------------------------------------------------------------------
// Workspace map.  The header occupies the first 1 KiB.
// ---------------------------------------------------------------------------
struct WsHeader {
    int status;                    // sticky gps_status of device-side failures
    int adam_step;                 // optional Adam step counter
    unsigned long long n_inst;     // instances emitted by the last forward
    unsigned long long n_fallback; // tiles sorted by the global-memory fallback
    unsigned long long cap;        // instance capacity of the last forward
    unsigned long long pairs_eval;     // (pixel, instance) opacity evaluations of every forward since reset
    unsigned long long pairs_contrib;  // of those, pairs composited (alpha >= alpha_min, before a stop)
    float loss;
    int n_views;
    int n_tiles;
    unsigned int n_large;          // tiles longer than one wavefront sorts (block sort)
    float view_stats[GPS_MAX_VIEWS][4];  // per view: colour L1 sum, depth L1 sum, |Omega|, pad
};

struct WsLayout {
    size_t total;
    size_t hdr, vtab, tilemax, tile_cnt, tile_start, tile_queue, tile_loss, tile_pairs, pix_aux, rec, cnt, off,
        blk_sum, blk_off,
        keys, inst_vg, partial, pose_part;
    int n_tiles, nvg, nblk_vg, nblk_g;
    unsigned long long cap;
};

struct WsPtrs {
    WsHeader* hdr;
    float* tilemax;
    unsigned int* tile_cnt;     // [kCntSplit][n_tiles]: instances that pass the depth cull, per sub-counter;
                                // after the tile scan, the start of each sub-counter's range
    unsigned int* tile_start;   // n_tiles + 1
    unsigned int* tile_queue;   // tiles in processing order (longest first)
    float4* tile_loss;          // per tile: colour L1 sum, depth L1 sum, |Omega| count, 0
    uint2* tile_pairs;          // per tile: evaluated and composited (pixel, instance) pairs
    float* pix_aux;             // per pixel: T_final (sorted) or W_G (sort-free)
    float4* rec;                // 3 float4 per view-Gaussian
    unsigned int* cnt;
    unsigned int* off;
    unsigned int* blk_sum;
    unsigned int* blk_off;
    unsigned long long* keys;   // (depth bits << 32) | view-Gaussian, grouped by tile
    unsigned int* inst_vg;      // per slot: the instance's rank in its tile sub-counter (count -> emit)
    float* partial;             // [cap][kAdj]
    float* pose_part;           // [nblk_g][V][6]
};

inline WsPtrs ws_ptrs(char* ws, const WsLayout& L)
{
    WsPtrs p;
    p.hdr = reinterpret_cast<WsHeader*>(ws + L.hdr);
    p.tilemax = reinterpret_cast<float*>(ws + L.tilemax);
    p.tile_cnt = reinterpret_cast<unsigned int*>(ws + L.tile_cnt);
    p.tile_start = reinterpret_cast<unsigned int*>(ws + L.tile_start);
    p.tile_queue = reinterpret_cast<unsigned int*>(ws + L.tile_queue);
    p.tile_loss = reinterpret_cast<float4*>(ws + L.tile_loss);
    p.tile_pairs = reinterpret_cast<uint2*>(ws + L.tile_pairs);
    p.pix_aux = reinterpret_cast<float*>(ws + L.pix_aux);
    p.rec = reinterpret_cast<float4*>(ws + L.rec);
    p.cnt = reinterpret_cast<unsigned int*>(ws + L.cnt);
    p.off = reinterpret_cast<unsigned int*>(ws + L.off);
    p.blk_sum = reinterpret_cast<unsigned int*>(ws + L.blk_sum);
    p.blk_off = reinterpret_cast<unsigned int*>(ws + L.blk_off);
    p.keys = reinterpret_cast<unsigned long long*>(ws + L.keys);
    p.inst_vg = reinterpret_cast<unsigned int*>(ws + L.inst_vg);
    p.partial = reinterpret_cast<float*>(ws + L.partial);
    p.pose_part = reinterpret_cast<float*>(ws + L.pose_part);
    return p;
}

// ---------------------------------------------------------------------------
// binary32 decision arithmetic.  Each statement is one IEEE operation; the
// library is compiled with -ffp-contract=on (only a*b+c written as ONE
// expression may fuse) and these helpers additionally forbid contraction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float d32_row(const float* R, const float* t, int r, float p0, float p1, float p2)
{
#pragma clang fp contract(off)
    float a = R[3 * r + 0] * p0;
    float b = R[3 * r + 1] * p1;
    float s = a + b;
    float c = R[3 * r + 2] * p2;
    s = s + c;
    s = s + t[r];
    return s;
}

__device__ __forceinline__ float d32_lattice(float origin, float voxel, int idx)
{
#pragma clang fp contract(off)
    float f = (float)idx;
    float v = voxel * f;
    return origin + v;
}

__device__ __forceinline__ float d32_lerp(float a, float b, float f)
{
#pragma clang fp contract(off)
    float d = b - a;
    float e = f * d;
    return a + e;
}

// ---------------------------------------------------------------------------
// Opacity of a projected Gaussian at a pixel, Eq. 3:
//   alpha = sigma * exp(-0.5 * (a dx^2 + 2 b dx dy + c dy^2)).
// The projection stores the conic pre-scaled for a base-2 exponential,
//   A' = -0.5 log2(e) a,  B' = -log2(e) b,  C' = -0.5 log2(e) c,
// and log2(sigma), so that
//   alpha = exp2(A' dx^2 + B' dx dy + C' dy^2 + log2 sigma)
// costs three products, three fused multiply-adds and one v_exp_f32.  The
// squares dx^2, dx dy, dy^2 are kept: the backward reuses them.  The
// operations are written out with explicit fused multiply-adds so that the
// forward and the backward kernels evaluate bit-identical values (the
// backward recomputes the transmittance and must stop at the same Gaussian).
// ---------------------------------------------------------------------------
struct AlphaEval {
    float raw;  // alpha before the cap
    float dx, dy, dxx, dxy, dyy;
};

__device__ __forceinline__ AlphaEval eval_alpha(float px, float py, float mx, float my, float A, float B, float C,
                                                float log2_sigma)
{
#pragma clang fp contract(off)
    AlphaEval r;
    r.dx = px - mx;
    r.dy = py - my;
    r.dxx = r.dx * r.dx;
    r.dxy = r.dx * r.dy;
    r.dyy = r.dy * r.dy;
    const float pw = __builtin_fmaf(A, r.dxx, __builtin_fmaf(B, r.dxy, __builtin_fmaf(C, r.dyy, log2_sigma)));
    r.raw = __builtin_amdgcn_exp2f(pw);
    return r;
}

// ---------------------------------------------------------------------------
// Wavefront (64 lanes) helpers.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND_ZERO = true>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO));
}

// Sum over the 64 lanes; the total is valid in lane 63 only.
__device__ __forceinline__ float wave_sum_to_lane63(float v)
{
    v += dpp_f<0x111>(v);  // row_shr:1
    v += dpp_f<0x112>(v);  // row_shr:2
    v += dpp_f<0x114>(v);  // row_shr:4
    v += dpp_f<0x118>(v);  // row_shr:8   -> lane 15 of each row holds its row sum
    v += dpp_f<0x142, 0xa, 0xf, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xc, 0xf, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sums each of ten per-lane values over each 16-lane row of the wavefront and
// stores the row totals at dst[row * 10 + q] (LDS, 40 floats).  A transpose-
// reduction within rows, DPP only: the pairs (q, q+5) are exchanged between
// lanes i and i^8 (row_ror:8), then pairs of the five results between i and
// 7-i within each half-row (row_half_mirror), then between i and i^2 and i^1
// (quad_perm).  Each exchange keeps one value of the pair, sends the other and
// adds the partner's: 15 + 7 + 4 + 3 = 29 VALU operations, against 40 for ten
// independent row reductions.  Lane bits (b3 b2 b1 b0) of the row then hold
// value (b1 ? 2 : 0) + b2 + 5 b3 when b0 = 0 and value 4 + 5 b3 when b0 = 1 (written
// from the lanes with b1 = b2 = 0).  Every lane must be active; the summation
// order is fixed.
__device__ __forceinline__ void wave_rows_sum10_store(const float (&g)[10], float* dst, int lane)
{
    const int i = lane & 15;
    const bool s3 = (i & 8) != 0, s2 = (i & 4) != 0, s1 = (i & 2) != 0, s0 = (i & 1) != 0;
    float h[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) h[q] = (s3 ? g[q + 5] : g[q]) + dpp_f<0x128>(s3 ? g[q] : g[q + 5]);  // row_ror:8
    const float p0 = (s2 ? h[1] : h[0]) + dpp_f<0x141>(s2 ? h[0] : h[1]);  // row_half_mirror
    const float p1 = (s2 ? h[3] : h[2]) + dpp_f<0x141>(s2 ? h[2] : h[3]);
    const float p2 = h[4] + dpp_f<0x141>(h[4]);
    const float r0 = (s1 ? p1 : p0) + dpp_f<0x4E>(s1 ? p0 : p1);  // quad_perm [2,3,0,1]
    const float r1 = p2 + dpp_f<0x4E>(p2);
    const float f = (s0 ? r1 : r0) + dpp_f<0xB1>(s0 ? r0 : r1);  // quad_perm [1,0,3,2]
    const int idx = s0 ? 4 + 5 * (int)s3 : (s1 ? 2 : 0) + (int)s2 + 5 * (int)s3;
    if (!s0 || (!s1 && !s2)) dst[(lane >> 4) * 10 + idx] = f;
}

// Sum over the 64 lanes, result uniform across the wave.
__device__ __forceinline__ float wave_sum(float v)
{
    v = wave_sum_to_lane63(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ bool wave_any(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) != 0ull;
}

__device__ __forceinline__ int find_view(const ViewTable& vt, int tile)
{
    int v = 0;
#pragma unroll 1
    for (int k = 1; k < vt.n; ++k)
        if (tile >= vt.v[k].tile_base) v = k;
    return v;
}


}  // namespace gps
