// Forward render: EWA projection, tile binning, per-tile depth sort and
// compositing over the SDF base image, with the loss fused into the
// compositing epilogue (Sec. 3.1 second pass, Eq. 1-4, Eq. 7).
//
// Kernel sequence (one launch each, all grids sized from host-known shapes,
// so the sequence is graph-capturable):
//   k_tilemax      per screen tile: max of the SDF depth (invalid = +inf); launched
//                  with the view-table upload, not per forward
//   k_project      per (view, Gaussian): projected record and the number of
//                  screen tiles its support box covers (one slot per tile);
//                  also clears the per-tile counters of this forward
//   k_scan_blocks  one block: offsets of the per-block slot counts
//   k_expand<0>    block-cooperative walk of the tile rectangles: per-tile
//                  counts of the instances that pass the exact depth cull
//   k_scan_tiles   one block: tile ranges
//   k_expand<1>    the same walk: (depth, view-Gaussian) keys scattered into tile ranges
//   k_tile_sort_*  per tile: bitonic sort of its keys in LDS (one wavefront
//                  for tiles of <= 512 instances, a 256-lane block above)
//   k_composite_fwd<TW,TH,B,PPT>  (composite_fwd.hip) per tile: LDS-staged
//                  batches of B records, wavefronts skip records whose support
//                  misses their pixels, front-to-back compositing, loss
//                  partial per tile
//   k_loss_reduce  one block: per-view and total loss
#include "binning.h"
#include "launch.h"
#include "prof.h"
#include "render_common.h"
#include "se3.h"

namespace gps {

// ---------------------------------------------------- tile depth maxima
// Per screen tile: the maximum of the SDF base depth (invalid = +inf), taken
// when the view table is uploaded (the base images are fixed until the next upload).
__global__ void __launch_bounds__(256) k_tilemax(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w)
{
    const ViewTable& vt = *vtp;
    const int tile = blockIdx.x;
    const int v = find_view(vt, tile);
    const DevView& V = vt.v[v];
    const int lt = tile - V.tile_base;
    const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
    float m = -INFINITY;
    for (int k = threadIdx.x; k < rp.tile_w * rp.tile_h; k += 256) {
        int x = tx * rp.tile_w + k % rp.tile_w, y = ty * rp.tile_h + k / rp.tile_w;
        if (x < V.cam.W && y < V.cam.H) {
            float d = V.base_depth[(size_t)y * V.cam.W + x];
            m = fmaxf(m, d > 0.0f ? d : INFINITY);
        }
    }
    m = wave_max(m);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) w.tilemax[tile] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Per-forward resets (run by the first kernel of the forward, over its whole
// grid): the per-tile sub-counters and the forward's header counters.
__device__ __forceinline__ void forward_resets(const ViewTable& vt, const RParams& rp, const WsPtrs& w)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    for (int i = gid; i < kCntSplit * vt.n_tiles; i += nth) w.tile_cnt[i] = 0u;
    if (gid == 0) {
        w.hdr->n_inst = 0ull;
        w.hdr->n_fallback = 0ull;
        w.hdr->n_views = rp.V;
    }
}

// ---------------------------------------------------------------- project
// EWA projection of one Gaussian into one view (Eq. 3; 3DGS convention):
//   p_c = R mu + t, Sigma_3D = R_q diag(s^2) R_q^T, J the pinhole Jacobian,
//   Sigma_2D = (J R) Sigma_3D (J R)^T + dilation I, conic = Sigma_2D^-1.
// Record of 12 floats: r0 = (m_x, m_y, A', B'), r1 = (C', log2 sigma, z, red),
// r2 = (green, blue, half-width, half-height of the support box), the colour
// being the one seen from this view (rgb plus the SH bands), where
// (A', B', C') = (-0.5 a, -b, -0.5 c) log2(e) for the conic (a, b, c), the
// opacity then being exp2(A' dx^2 + B' dx dy + C' dy^2 + log2 sigma).
// The support ellipse where sigma exp(-q/2) >= alpha_min has the bounding box
// m +- sqrt(kappa Sigma_xx), sqrt(kappa Sigma_yy), kappa = 2 ln(sigma/alpha_min);
// it is padded by one pixel and turned into a tile rectangle.
struct ProjOut {
    float4 r0, r1, r2;
    bool valid;
};

__device__ __forceinline__ ProjOut project_one(const DevView& V, const RParams& rp, const GParams& gp, int g)
{
    ProjOut o;
    o.valid = false;
    o.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
    o.r1 = make_float4(0.f, 0.f, 0.f, 0.f);
    o.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int M = rp.M;
    const DevCam& c = V.cam;
    const float m0 = gp.mean[g], m1 = gp.mean[M + g], m2 = gp.mean[2 * M + g];
    const float z = d32_row(c.R, c.t, 2, m0, m1, m2);  // depth key (binary32 decision)
    if (!(z >= rp.znear)) return o;
    const float x = c.R[0] * m0 + c.R[1] * m1 + c.R[2] * m2 + c.t[0];
    const float y = c.R[3] * m0 + c.R[4] * m1 + c.R[5] * m2 + c.t[1];
    float qw = gp.quat[g], qx = gp.quat[M + g], qy = gp.quat[2 * M + g], qz = gp.quat[3 * M + g];
    const float qinv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qinv;
    qx *= qinv;
    qy *= qinv;
    qz *= qinv;
    float Rq[9];
    Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
    Rq[1] = 2.f * (qx * qy - qw * qz);
    Rq[2] = 2.f * (qx * qz + qw * qy);
    Rq[3] = 2.f * (qx * qy + qw * qz);
    Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
    Rq[5] = 2.f * (qy * qz - qw * qx);
    Rq[6] = 2.f * (qx * qz - qw * qy);
    Rq[7] = 2.f * (qy * qz + qw * qx);
    Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);
    const float s0 = __expf(gp.log_scale[g]), s1 = __expf(gp.log_scale[M + g]), s2 = __expf(gp.log_scale[2 * M + g]);
    float Mm[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Mm[3 * r + 0] = Rq[3 * r + 0] * s0;
        Mm[3 * r + 1] = Rq[3 * r + 1] * s1;
        Mm[3 * r + 2] = Rq[3 * r + 2] * s2;
    }
    // W = J R (2x3)
    const float iz = 1.0f / z;
    const float J00 = c.fx * iz, J02 = -c.fx * x * iz * iz, J11 = c.fy * iz, J12 = -c.fy * y * iz * iz;
    float W0[3], W1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        W0[k] = J00 * c.R[k] + J02 * c.R[6 + k];
        W1[k] = J11 * c.R[3 + k] + J12 * c.R[6 + k];
    }
    // U = W Mm (2x3); Sigma_2D = U U^T
    float U0[3], U1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        U0[k] = W0[0] * Mm[k] + W0[1] * Mm[3 + k] + W0[2] * Mm[6 + k];
        U1[k] = W1[0] * Mm[k] + W1[1] * Mm[3 + k] + W1[2] * Mm[6 + k];
    }
    const float A = U0[0] * U0[0] + U0[1] * U0[1] + U0[2] * U0[2] + rp.dil;
    const float B = U0[0] * U1[0] + U0[1] * U1[1] + U0[2] * U1[2];
    const float C = U1[0] * U1[0] + U1[1] * U1[1] + U1[2] * U1[2] + rp.dil;
    const float det = A * C - B * B;
    if (!(det > 0.0f)) return o;
    const float idet = 1.0f / det;
    const float sig = 1.0f / (1.0f + __expf(-gp.opacity_logit[g]));
    if (!(sig > rp.amin)) return o;
    const float mx = c.fx * x * iz + c.cx, my = c.fy * y * iz + c.cy;
    const float kappa = 2.0f * __logf(sig / rp.amin);
    // support half-extents padded by one pixel (covers the rounding of the opacity test)
    const float rxp = sqrtf(kappa * A) + 1.0f, ryp = sqrtf(kappa * C) + 1.0f;
    if (!(rxp < 1e7f) || !(ryp < 1e7f) || !(fabsf(mx) < 1e7f) || !(fabsf(my) < 1e7f)) return o;
    // conic (a, b, c) = (C, -B, A) / det, pre-scaled for the base-2 exponential
    constexpr float kL2E = 1.4426950408889634f;
    o.r0 = make_float4(mx, my, (-0.5f * kL2E) * (C * idet), kL2E * (B * idet));
    float col[3];
    view_colour(gp, M, g, c, m0, m1, m2, col);
    o.r1 = make_float4((-0.5f * kL2E) * (A * idet), __log2f(sig), z, col[0]);
    o.r2 = make_float4(col[1], col[2], rxp, ryp);
    o.valid = true;
    return o;
}

__global__ void __launch_bounds__(kBlk) k_project(const ViewTable* __restrict__ vtp, RParams rp, GParams gp, WsPtrs w)
{
    const ViewTable& vt = *vtp;
    forward_resets(vt, rp, w);
    const int vg = blockIdx.x * kBlk + threadIdx.x;
    unsigned int count = 0;
    if (vg < rp.nvg) {
        const int v = vg / rp.M, g = vg - v * rp.M;
        const DevView& V = vt.v[v];
        ProjOut p = project_one(V, rp, gp, g);
        w.rec[3 * (size_t)vg + 0] = p.r0;
        w.rec[3 * (size_t)vg + 1] = p.r1;
        w.rec[3 * (size_t)vg + 2] = p.r2;
        TileRect r;
        if (p.valid && rect_of(p.r0.x, p.r0.y, p.r2.z, p.r2.w, V.cam.W, V.cam.H, rp.tile_w, rp.tile_h, &r))
            count = (unsigned int)((r.tx1 - r.tx0 + 1) * (r.ty1 - r.ty0 + 1));  // one slot per covered tile
        w.cnt[vg] = count;
    }
    unsigned int tot;
    block_excl_scan<kBlk>(count, &tot);
    if (threadIdx.x == 0) w.blk_sum[blockIdx.x] = tot;
}

// ------------------------------------------------------------------- scan
// One block of 1024 lanes: exclusive scan of the per-block instance counts and
// of the per-tile counts; capacity check.
__device__ unsigned long long scan_array_1024(const unsigned int* in, unsigned int* out, int n, int write_total)
{
    __shared__ unsigned int wsum[16];
    __shared__ unsigned long long carry_s;
    if (threadIdx.x == 0) carry_s = 0ull;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < n; base += 4096) {
        unsigned int v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int i = base + threadIdx.x * 4 + k;
            v[k] = i < n ? in[i] : 0u;
            sum += v[k];
        }
        unsigned int x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            unsigned int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        unsigned int before = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wid) before += wsum[k];
            tot += wsum[k];
        }
        unsigned long long carry = carry_s;
        unsigned int run = (unsigned int)carry + before + x - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int i = base + threadIdx.x * 4 + k;
            if (i < n) out[i] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + tot;
        __syncthreads();
    }
    unsigned long long total = carry_s;
    if (write_total && threadIdx.x == 0) out[n] = (unsigned int)total;
    __syncthreads();
    return total;
}

__global__ void __launch_bounds__(1024) k_scan_blocks(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w,
                                                     int nblk_vg, int n_tiles, int resets)
{
    if (resets) forward_resets(*vtp, rp, w);  // no projection launch (no Gaussians): the resets are here
    unsigned long long total = scan_array_1024(w.blk_sum, w.blk_off, nblk_vg, 0);
    if (threadIdx.x == 0) {
        w.hdr->n_inst = total;
        w.hdr->cap = rp.cap;
        w.hdr->n_tiles = n_tiles;
        if (total > rp.cap) atomicCAS(&w.hdr->status, 0, GPS_ERR_CAPACITY);
    }
}

// Also orders the tiles for the compositing kernels, longest first:
// tiles are bucketed by floor(log2(count + 1)) and the buckets laid out in
// descending order.  The order inside a bucket is arbitrary; it affects only
// which block processes a tile, never a result.
__global__ void __launch_bounds__(1024) k_scan_tiles(RParams rp, WsPtrs w, int n_tiles)
{
    if (w.hdr->n_inst > rp.cap) return;
    __shared__ unsigned int wsum[16], hist[33], cur[33];
    __shared__ unsigned int carry_s, n_large;
    if (threadIdx.x < 33) hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        carry_s = 0u;
        n_large = 0u;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned int last_tot[4] = {0u, 0u, 0u, 0u};  // the lane's tile lengths in the last chunk
    // One pass per chunk of 4 tiles per lane: the sub-counts are read once, their
    // totals scanned over the block (chunks carried in order) into the tile
    // ranges, each sub-counter replaced by the start of its range inside its
    // tile's range, and the tile lengths counted into the histogram.
    for (int base = 0; base < n_tiles; base += 4 * 1024) {
        unsigned int c[4][kCntSplit], tot[4], sum = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = base + threadIdx.x * 4 + i;
            tot[i] = 0u;
#pragma unroll
            for (int k = 0; k < kCntSplit; ++k) {
                c[i][k] = t < n_tiles ? w.tile_cnt[(size_t)k * n_tiles + t] : 0u;
                tot[i] += c[i][k];
            }
            sum += tot[i];
        }
        unsigned int x = sum;
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
        unsigned int run = carry + before + x - sum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = base + threadIdx.x * 4 + i;
            if (t < n_tiles) {
                w.tile_start[t] = run;
                unsigned int r = run;
#pragma unroll
                for (int k = 0; k < kCntSplit; ++k) {
                    w.tile_cnt[(size_t)k * n_tiles + t] = r;
                    r += c[i][k];
                }
                atomicAdd(&hist[31 - __clz(tot[i] + 1u)], 1u);
                if (tot[i] >= kLongTile) atomicAdd(&n_large, 1u);
            }
            last_tot[i] = tot[i];
            run += tot[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + total;
        __syncthreads();
    }
    // Longest-first order: buckets floor(log2(count + 1)) laid out in descending order.
    if (threadIdx.x == 0) {
        w.tile_start[n_tiles] = carry_s;
        w.hdr->n_large = n_large;
        unsigned int o = 0;
        for (int bkt = 32; bkt >= 0; --bkt) {
            cur[bkt] = o;
            o += hist[bkt];
        }
    }
    __syncthreads();
    if (n_tiles <= 4 * 1024) {
        // one chunk: this lane's four tile lengths are still in registers
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = threadIdx.x * 4 + i;
            if (t < n_tiles) w.tile_queue[atomicAdd(&cur[31 - __clz(last_tot[i] + 1u)], 1u)] = (unsigned int)t;
        }
        return;
    }
    for (int i = threadIdx.x; i < n_tiles; i += 1024) {
        const unsigned int pos = atomicAdd(&cur[31 - __clz(w.tile_start[i + 1] - w.tile_start[i] + 1u)], 1u);
        w.tile_queue[pos] = (unsigned int)i;
    }
}

// ------------------------------------------------------------ count / emit
// Block-cooperative expansion of the instances of kExpG consecutive
// view-Gaussians (a share of one projection block of kBlk): the block's kBlk
// lanes walk the concatenation of their tile rectangles together (instance i
// belongs to the Gaussian whose prefix range holds i, found by binary search in
// LDS), so one large Gaussian, or a run of dense ones, is spread over several
// lanes per Gaussian instead of serialising one lane.  Slots are numbered per
// projection block: instance i of projection block b has slot blk_off[b] + i,
// whichever expansion block handles it.
//   COUNT:  tiles that the support ellipse meets (SupportTest) and that pass
//           the exact depth cull get one of their kCntSplit sub-counters
//           (chosen by block index) incremented; the count before the increment
//           (the instance's rank in that sub-counter) is parked in inst_vg[slot];
//           the per-view-Gaussian slot offsets are written.
//   EMIT:   the same instances (the culls are the same binary32 tests on the
//           same values, the block index the same) write the key
//           (depth bits << 32) | view-Gaussian at the sub-counter's start + rank,
//           with no atomics, and zero the instance partials of every slot.  A
//           tile holds at most one instance of a view-Gaussian, and slots grow
//           with the view-Gaussian index, so the keys sort as (depth, slot) would;
//           the backward recovers the slot from the view-Gaussian's offset and the
//           tile's place in its rectangle.
template <bool EMIT>
__global__ void __launch_bounds__(kBlk) k_expand(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w)
{
    constexpr int kSplit = kBlk / kExpG;  // expansion blocks per projection block
    const ViewTable& vt = *vtp;
    __shared__ unsigned int pre[kExpG + 1];
    __shared__ float4 sbox[kExpG];  // mx, my, rxp, ryp
    __shared__ float4 scon[kExpG];  // the exponent's coefficients A, B, C and log2 sigma
    __shared__ float sz[kExpG];
    __shared__ int4 sview[kExpG];   // tile_base, tiles_x, W, H
    const int pb = blockIdx.x / kSplit;
    const int g0 = (blockIdx.x % kSplit) * kExpG;  // first lane (Gaussian) of this block's share
    const int vg = pb * kBlk + threadIdx.x;         // lane k: Gaussian k of the projection block
    const int k = threadIdx.x - g0;
    // The count, the record of this block's share (written by the projection for every
    // view-Gaussian) and the block's slot base are loaded together with the capacity
    // check, before any of them is waited for.
    const bool mine = k >= 0 && k < kExpG && vg < rp.nvg;
    const unsigned long long n_inst = w.hdr->n_inst;
    const unsigned int c = vg < rp.nvg ? w.cnt[vg] : 0u;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    if (mine) {
        r0 = w.rec[3 * (size_t)vg];
        r1 = w.rec[3 * (size_t)vg + 1];
        r2 = w.rec[3 * (size_t)vg + 2];
    }
    const unsigned int base = w.blk_off[pb];
    if (n_inst > rp.cap) return;
    unsigned int tot;
    const unsigned int excl = block_excl_scan<kBlk>(c, &tot);  // prefix within the projection block
    if (k >= 0 && k < kExpG) {
        pre[k] = excl;
        if (k == kExpG - 1) pre[kExpG] = excl + c;
        if (c > 0) {
            sbox[k] = make_float4(r0.x, r0.y, r2.z, r2.w);
            scon[k] = make_float4(r0.z, r0.w, r1.x, r1.y);
            sz[k] = r1.z;
            const DevView& V = vt.v[vg / rp.M];
            sview[k] = make_int4(V.tile_base, V.tiles_x, V.cam.W, V.cam.H);
        }
        if (!EMIT && vg < rp.nvg) w.off[vg] = base + excl;
    }
    // sub-counter of this block: the same block index, so the same sub-counter, in both passes
    const size_t sub = (size_t)(blockIdx.x % kCntSplit) * vt.n_tiles;
    __syncthreads();
    const unsigned int first = pre[0], last = pre[kExpG];
    const float l2amin = __log2f(rp.amin);
    for (unsigned int i = first + threadIdx.x; i < last; i += kBlk) {
        int lo = 0, hi = kExpG;  // pre[lo] <= i < pre[hi]
#pragma unroll
        for (int step = 0; step < kExpGLog2; ++step) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        const unsigned int j = i - pre[lo];
        const float4 bx = sbox[lo];
        const int4 vw = sview[lo];
        TileRect r;
        if (!rect_of(bx.x, bx.y, bx.z, bx.w, vw.z, vw.w, rp.tile_w, rp.tile_h, &r)) continue;
        const unsigned int wdt = (unsigned int)(r.tx1 - r.tx0 + 1);
        const int tix = r.tx0 + (int)(j % wdt), tiy = r.ty0 + (int)(j / wdt);
        const int tile = vw.x + tiy * vw.y + tix;
        const float z = sz[lo];
        const unsigned int slot = base + i;
        if (EMIT) {
            // The per-Gaussian reduce sums every slot of a Gaussian: all slots start at
            // zero (culled ones, and those the backward's tiles stop before, stay so).
            float* pz = w.partial + (size_t)slot * kAdj;
#pragma unroll
            for (int q = 0; q < kAdj; ++q) pz[q] = 0.0f;
        }
        // the support ellipse must meet the tile (its box may only overlap it)
        const float4 cn = scon[lo];
        const SupportTest st(make_float4(bx.x, bx.y, cn.x, cn.y), make_float4(cn.z, cn.w, 0.0f, 0.0f), l2amin);
        if (!st.meets((float)(tix * rp.tile_w), (float)(tiy * rp.tile_h), (float)rp.tile_w, (float)rp.tile_h)) continue;
        if (!(z < w.tilemax[tile] + rp.eps)) continue;  // exact tile-level depth cull
        if (!EMIT) {
            w.inst_vg[slot] = atomicAdd(w.tile_cnt + sub + tile, 1u);
        } else {
            // key: depth bits, then the view-Gaussian (within a tile it orders as the slot does)
            const unsigned int pos = w.tile_cnt[sub + tile] + w.inst_vg[slot];
            if (pos < w.tile_start[tile + 1])
                w.keys[pos] = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned int)(pb * kBlk + g0 + lo);
        }
    }
}

// -------------------------------------------------------------- tile sort
// Tiles of fewer than kLongTile keys are sorted in registers by the first
// wavefront of their compositing block (wave_sort_tile, binning.h).
// k_tile_sort_large: one block per longer tile (bitonic network in LDS, the
// same compare-exchange order); tiles longer than kSortCap use the same network
// in global memory.

__device__ __forceinline__ void cas_lds(unsigned long long* sh, int i, int j)
{
    const unsigned long long a = sh[i], b = sh[j];
    if (a > b) {
        sh[i] = b;
        sh[j] = a;
    }
}

// One block sorts the n >= kLongTile keys starting at keys[s].
__device__ void sort_tile_block(const WsPtrs& w, unsigned int s, int n)
{
    int P = 1;
    while (P < n) P <<= 1;
    unsigned long long* key = w.keys + s;
    if (n <= kSortCap) {
        extern __shared__ unsigned long long sh[];  // kSortCap keys (dynamic LDS)
        for (int i = threadIdx.x; i < P; i += 256) sh[i] = i < n ? key[i] : ~0ull;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            const int half = k >> 1;
            for (int c = threadIdx.x; c < P / 2; c += 256) {
                const int blk = c / half, wi = c - blk * half;
                cas_lds(sh, blk * k + wi, blk * k + k - 1 - wi);
            }
            __syncthreads();
            for (int jj = k >> 2; jj > 0; jj >>= 1) {
                for (int c = threadIdx.x; c < P / 2; c += 256) {
                    const int i = (c / jj) * 2 * jj + (c % jj);
                    cas_lds(sh, i, i + jj);
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < n; i += 256) key[i] = sh[i];
    } else {
        // Rare: a tile longer than the LDS holds.  Same network in global
        // memory; elements at or past n act as +inf and are never touched.
        if (threadIdx.x == 0) atomicAdd(&w.hdr->n_fallback, 1ull);
        for (int k = 2; k <= P; k <<= 1) {
            const int half = k >> 1;
            for (int c = threadIdx.x; c < P / 2; c += 256) {
                const int blk = c / half, wi = c - blk * half;
                const int i = blk * k + wi, j = blk * k + k - 1 - wi;
                if (j < n) {
                    unsigned long long a = key[i], b = key[j];
                    if (a > b) {
                        key[i] = b;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
            for (int jj = k >> 2; jj > 0; jj >>= 1) {
                for (int c = threadIdx.x; c < P / 2; c += 256) {
                    const int i = (c / jj) * 2 * jj + (c % jj), j = i + jj;
                    if (j < n) {
                        unsigned long long a = key[i], b = key[j];
                        if (a > b) {
                            key[i] = b;
                            key[j] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
}

// The tiles of at least kLongTile keys lead the longest-first tile queue (the
// tile scan counts them), so block b takes queue position b; past them, blocks
// exit after one header read.
__global__ void __launch_bounds__(256) k_tile_sort_large(RParams rp, WsPtrs w)
{
    if (w.hdr->n_inst > rp.cap || blockIdx.x >= w.hdr->n_large) return;
    const int tile = (int)w.tile_queue[blockIdx.x];
    const unsigned int s = w.tile_start[tile], e = w.tile_start[tile + 1];
    const int n = (int)(e - s);
    if ((unsigned int)n >= kLongTile) sort_tile_block(w, s, n);
}

// ------------------------------------------------------------ loss reduce
__global__ void __launch_bounds__(1024) k_loss_reduce(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w, float* out_loss,
                                                     int has_loss)
{
    const ViewTable& vt = *vtp;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // Per view: the colour L1 sum, depth L1 sum and |Omega| over its tiles, each
    // summed per lane, then per wavefront (DPP), then over the wavefronts in order
    // by one thread: one barrier for all views.
    __shared__ float4 red[GPS_MAX_VIEWS][16];
    for (int v = 0; v < vt.n; ++v) {
        const DevView& V = vt.v[v];
        const int nt = V.tiles_x * V.tiles_y;
        float a = 0.0f, b = 0.0f, c = 0.0f;
        for (int t = threadIdx.x; t < nt; t += 1024) {
            const float4 q = w.tile_loss[V.tile_base + t];
            a += q.x;
            b += q.y;
            c += q.z;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        if (lane == 0) red[v][wid] = make_float4(a, b, c, 0.0f);
    }
    // Evaluated / composited pair counts of this forward, summed over the tiles in
    // a fixed order and added to the cumulative counters of the header.
    unsigned long long pe = 0ull, pc = 0ull;
    if (w.hdr->n_inst <= rp.cap) {
        for (int t = threadIdx.x; t < vt.n_tiles; t += 1024) {
            const uint2 q = w.tile_pairs[t];
            pe += q.x;
            pc += q.y;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        pe += __shfl_xor(pe, o, 64);
        pc += __shfl_xor(pc, o, 64);
    }
    __shared__ unsigned long long spe[16], spc[16];
    if (lane == 0) {
        spe[wid] = pe;
        spc[wid] = pc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float L = 0.0f;
        for (int v = 0; v < vt.n; ++v) {
            float a = 0.0f, b = 0.0f, c = 0.0f;
            for (int k = 0; k < 16; ++k) {
                a += red[v][k].x;
                b += red[v][k].y;
                c += red[v][k].z;
            }
            w.hdr->view_stats[v][0] = a;
            w.hdr->view_stats[v][1] = b;
            w.hdr->view_stats[v][2] = c;
            w.hdr->view_stats[v][3] = 0.0f;
            const float npx = 3.0f * (float)vt.v[v].cam.W * (float)vt.v[v].cam.H;
            L += a / npx + (c > 0.0f ? rp.lambda * b / c : 0.0f);
        }
        unsigned long long te = 0ull, tc = 0ull;
        for (int k = 0; k < 16; ++k) {
            te += spe[k];
            tc += spc[k];
        }
        w.hdr->pairs_eval += te;
        w.hdr->pairs_contrib += tc;
        L = L / (float)vt.n;
        w.hdr->loss = has_loss ? L : 0.0f;
        if (out_loss && has_loss) *out_loss = L;
    }
}

// ------------------------------------------------------------ view table
// Copies the by-value view table into the workspace, so that a replayed
// sequence of kernels reads whatever table was uploaded last.
// A view with pose_xi is written with the camera Exp(xi) T_cw (binary64
// composition, rounded once to binary32).
__global__ void __launch_bounds__(256) k_upload_views(ViewTable vt, ViewTable* dst)
{
    const unsigned int* src = reinterpret_cast<const unsigned int*>(&vt);
    unsigned int* d = reinterpret_cast<unsigned int*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(ViewTable) / 4); i += 256) d[i] = src[i];
    __syncthreads();
    const int v = threadIdx.x;
    if (v < vt.n && vt.v[v].pose_xi) {
        double xi[6], E[9], e[3];
        for (int k = 0; k < 6; ++k) xi[k] = (double)vt.v[v].pose_xi[k];
        se3_exp_d(xi, E, e);
        const DevCam& c = vt.v[v].cam;
        DevCam& o = dst->v[v].cam;
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k)
                o.R[3 * r + k] = (float)(E[3 * r] * c.R[k] + E[3 * r + 1] * c.R[3 + k] + E[3 * r + 2] * c.R[6 + k]);
            o.t[r] = (float)(E[3 * r] * c.t[0] + E[3 * r + 1] * c.t[1] + E[3 * r + 2] * c.t[2] + e[r]);
        }
    }
}

// The table upload, then (with_tilemax) the tile depth maxima of its views.
gps_status launch_views_upload(const ViewTable& vt, const RParams& rp, const WsLayout& L, char* ws, int with_tilemax,
                               hipStream_t s)
{
    ViewTable* dvt = reinterpret_cast<ViewTable*>(ws + L.vtab);
    GPS_LAUNCH(K_UPLOAD, s, k_upload_views, dim3(1), dim3(256), 0, s, vt, dvt);
    if (with_tilemax && L.n_tiles > 0)
        GPS_LAUNCH(K_TILEMAX, s, k_tilemax, dim3(L.n_tiles), dim3(256), 0, s, dvt, rp, ws_ptrs(ws, L));
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

// ----------------------------------------------------------------- launch
gps_status launch_render_fwd(const gps_render_cfg* cfg, const RParams& rp, const gps_gaussians* g,
                             const ViewTable& vt, const WsLayout& L, char* ws, float* out_loss, hipStream_t s)
{
    WsPtrs w = ws_ptrs(ws, L);
    GParams gp{g->mean, g->log_scale, g->quat, g->opacity_logit, g->rgb, g->sh_degree > 0 ? g->sh : nullptr,
               sh_count(g->sh_degree)};
    int has_loss = 1;
    for (int v = 0; v < vt.n; ++v)
        if (!vt.v[v].target_rgb) has_loss = 0;
    // the kernels read the view table from the workspace
    const ViewTable* dvt = reinterpret_cast<const ViewTable*>(ws + L.vtab);
    if (!(cfg->flags & GPS_RENDER_VIEWS_PRESET)) {
        const gps_status st = launch_views_upload(vt, rp, L, ws, 1, s);
        if (st != GPS_OK) return st;
    }
    if (L.nblk_vg > 0) GPS_LAUNCH(K_PROJECT, s, k_project, dim3(L.nblk_vg), dim3(kBlk), 0, s, dvt, rp, gp, w);
    GPS_LAUNCH(K_SCAN, s, k_scan_blocks, dim3(1), dim3(1024), 0, s, dvt, rp, w, L.nblk_vg, L.n_tiles,
               L.nblk_vg > 0 ? 0 : 1);
    if (L.nblk_vg > 0)
        GPS_LAUNCH(K_TILE_COUNT, s, k_expand<false>, dim3(L.nblk_vg * (kBlk / kExpG)), dim3(kBlk), 0, s, dvt, rp, w);
    GPS_LAUNCH(K_SCAN_TILES, s, k_scan_tiles, dim3(1), dim3(1024), 0, s, rp, w, L.n_tiles);
    if (L.nblk_vg > 0)
        GPS_LAUNCH(K_EMIT, s, k_expand<true>, dim3(L.nblk_vg * (kBlk / kExpG)), dim3(kBlk), 0, s, dvt, rp, w);
    if (rp.mode != 2)  // the unsorted sort-free blend keeps the emission order
        GPS_LAUNCH(K_TILE_SORT_LARGE, s, k_tile_sort_large, dim3(L.n_tiles), dim3(256),
                   kSortCap * sizeof(unsigned long long), s, rp, w);
    if (!dispatch_cfwd(cfg, dvt, rp, w, L.n_tiles, s)) return GPS_ERR_UNSUPPORTED_CONFIG;
    GPS_LAUNCH(K_LOSS_REDUCE, s, k_loss_reduce, dim3(1), dim3(1024), 0, s, dvt, rp, w, out_loss, has_loss);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
