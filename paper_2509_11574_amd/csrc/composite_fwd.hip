// Forward compositing (Sec. 3.1 second pass, Eq. 1-4, Eq. 7): per screen
// tile, LDS-staged batches of B depth-sorted records; each wavefront skips the
// records whose support ellipse misses its pixels and composites the rest front to
// back over the SDF base colour and depth, with the loss partial of the tile
// written in the epilogue.
#include "binning.h"
#include "launch.h"
#include "prof.h"
#include "render_common.h"

namespace gps {

// ---------------------------------------------------------- composite fwd
// One record at one pixel: the opacity test (alpha >= alpha_min), the
// transmittance stop (sorted mode) and the accumulation of colour and depth.
// `live` is the depth test of Eq. 1-2; a pixel that stops gets thr = -inf.
template <int MODE>
__device__ __forceinline__ void composite_step(bool live, float raw, const float4& r1, const float4& r2,
                                               const RParams& rp, float& T, float& thr, float& ac0, float& ac1,
                                               float& ac2, float& ad, unsigned int& n_eval,
                                               unsigned int& n_contrib, unsigned long long& live_mask)
{
    bool use;
    if (MODE == 0) {
        const float a = fminf(raw, rp.amax);
        const bool ok = live && a >= rp.amin;
        const float Tn = T * (1.0f - a);
        const bool stop = ok && Tn < rp.Tmin;  // 3DGS transmittance stop
        use = ok && !stop;
        const float wgt = use ? a * T : 0.0f;
        ac0 = __builtin_fmaf(wgt, r1.w, ac0);
        ac1 = __builtin_fmaf(wgt, r2.x, ac1);
        ac2 = __builtin_fmaf(wgt, r2.y, ac2);
        ad = __builtin_fmaf(wgt, r1.z, ad);
        T = use ? Tn : T;
        thr = stop ? -INFINITY : thr;
    } else {
        use = live && raw >= rp.amin;
        const float a = use ? raw : 0.0f;
        T += a;  // W_G
        ac0 = __builtin_fmaf(a, r1.w, ac0);
        ac1 = __builtin_fmaf(a, r2.x, ac1);
        ac2 = __builtin_fmaf(a, r2.y, ac2);
        ad = __builtin_fmaf(a, r1.z, ad);
    }
    const unsigned long long lm = __builtin_amdgcn_ballot_w64(live);
    live_mask |= lm;
    n_eval += (unsigned int)__builtin_popcountll(lm);
    n_contrib += use ? 1u : 0u;  // per lane, summed over the wavefront in the epilogue
}

template <int TW, int TH, int B, int PPT, int MODE>
__global__ void __launch_bounds__(TW * TH / PPT) k_composite_fwd(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w)
{
    const ViewTable& vt = *vtp;
    using Lay = TileLayout<TW, TH, PPT>;
    constexpr int NT = Lay::NT;
    __shared__ float4 srec[3 * B];
    __shared__ unsigned int smask[B];  // wavefront mask per staged record (32-bit: no byte stores in LDS)
    // One block per tile, in queue order (longest tile lists first): the
    // hardware dispatches blocks in index order as resources free up, which
    // balances tiles of very different lengths without any global counter.  The
    // queue entry is read together with the capacity check (one round trip) and
    // checked against the tile count.
    const unsigned long long n_inst = w.hdr->n_inst;
    const unsigned int queued = w.tile_queue[blockIdx.x];
    if ((n_inst > rp.cap) | (queued >= (unsigned int)vt.n_tiles)) return;
    const int tile = (int)queued;
    const int v = find_view(vt, tile);
    const DevView& V = vt.v[v];
    const int lt = tile - V.tile_base;
    const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
    const int Wd = V.cam.W, Ht = V.cam.H;
    const size_t HW = (size_t)Wd * Ht;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wx0 = tx * TW + Lay::wave_x0(wid), wy0 = ty * TH + Lay::wave_y0(wid);
    const int px = wx0 + Lay::lane_x(lane);
    const int py0 = wy0 + Lay::lane_y(lane);
    const float fpx = (float)px;
    const float l2amin = __log2f(rp.amin);  // the support test of the staged records

    // thr: the depth test of Eq. 1-2 passes while d_i < D_t + eps.  The list is
    // depth-ordered, so once a record fails it every later record fails too; a
    // pixel that stops for another reason (outside the image, transmittance
    // below T_min) gets thr = -inf, so the one comparison carries every stop.
    float thr[PPT], T[PPT], ac0[PPT], ac1[PPT], ac2[PPT], ad[PPT];
    unsigned int n_eval = 0, n_contrib = 0;  // per wavefront (uniform) / per lane
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int py = py0 + k * Lay::LROWS;
        const bool inb = px < Wd && py < Ht;
        float dt = inb ? V.base_depth[(size_t)py * Wd + px] : 0.0f;
        float dcull = dt > 0.0f ? dt : INFINITY;
        thr[k] = inb ? dcull + rp.eps : -INFINITY;
        T[k] = MODE == 0 ? 1.0f : 0.0f;
        ac0[k] = ac1[k] = ac2[k] = ad[k] = 0.0f;
    }
    const unsigned int s = w.tile_start[tile], e = w.tile_start[tile + 1];
    // Depth order: lists shorter than kLongTile are sorted here, in registers of
    // the first wavefront (the longer ones by k_tile_sort_large before this
    // kernel); the barrier publishes the sorted keys to the block.  MODE 2 (the
    // sort-free blend without the sort) takes the list in emission order.
    if (MODE != 2 && e - s > 1u && e - s < kLongTile) {
        if (wid == 0) wave_sort_tile(w.keys + s, (int)(e - s), lane);
        __syncthreads();
    }
    const int tx0 = tx * TW, ty0 = ty * TH;
    bool wave_alive = true;  // some pixel of this wavefront still takes records
    for (unsigned int b = s; b < e; b += B) {
        if (__syncthreads_count(wave_alive && lane == 0) == 0) break;
        // Stage B records; each also gets the set of wavefronts whose pixels its
        // support ellipse meets (the test runs once per record, not once per record
        // and wavefront).
        for (int j = threadIdx.x; j < B; j += NT) {
            unsigned int mk = 0u;
            if (b + j < e) {
                unsigned int vg = (unsigned int)w.keys[b + j];
                if (vg >= (unsigned int)rp.nvg) vg = 0u;  // guard: never read outside the records
                const float4* r = w.rec + 3 * (size_t)vg;
                const float4 r0 = r[0], r1 = r[1], r2 = r[2];
                srec[3 * j + 0] = r0;
                srec[3 * j + 1] = r1;
                srec[3 * j + 2] = r2;
                mk = wave_support_mask<Lay>(r0, r1, l2amin, tx0, ty0);
            }
            smask[j] = mk;
        }
        __syncthreads();
        const int n = (int)min((unsigned int)B, e - b);
        for (int c0 = 0; c0 < n && wave_alive; c0 += 64) {
            // The records of this chunk whose support meets this wavefront; the
            // others have opacity below alpha_min at all its pixels.
            const int jl = c0 + lane;
            unsigned long long m = __builtin_amdgcn_ballot_w64(jl < n && ((smask[jl] >> wid) & 1u));
            // Records are taken two at a time: the opacities of both are independent
            // of the transmittance, so their evaluation overlaps; the compositing then
            // applies them in list order.  When the set has an odd count the second is
            // a copy of the first that no lane takes (its depth test is forced false).
            while (m) {
                const int ja = c0 + (int)__builtin_ctzll(m);
                m &= m - 1ull;
                const bool hb = m != 0ull;
                const int jb = hb ? c0 + (int)__builtin_ctzll(m) : ja;
                if (hb) m &= m - 1ull;
                const float4 a0 = srec[3 * ja], a1 = srec[3 * ja + 1], a2 = srec[3 * ja + 2];
                const float4 b0 = srec[3 * jb], b1 = srec[3 * jb + 1], b2 = srec[3 * jb + 2];
                unsigned long long live_a = 0ull, live_b = 0ull;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const float fpy = (float)(py0 + k * Lay::LROWS);
                    const AlphaEval ea = eval_alpha(fpx, fpy, a0.x, a0.y, a0.z, a0.w, a1.x, a1.y);
                    const AlphaEval eb = eval_alpha(fpx, fpy, b0.x, b0.y, b0.z, b0.w, b1.x, b1.y);
                    const bool la = a1.z < thr[k];  // depth test of Eq. 1-2
                    composite_step<MODE>(la, ea.raw, a1, a2, rp, T[k], thr[k], ac0[k], ac1[k], ac2[k], ad[k],
                                         n_eval, n_contrib, live_a);
                    const bool lb = hb && b1.z < thr[k];  // after a's update: a may have stopped the pixel
                    composite_step<MODE>(lb, eb.raw, b1, b2, rp, T[k], thr[k], ac0[k], ac1[k], ac2[k], ad[k],
                                         n_eval, n_contrib, live_b);
                }
                // A record that no lane passes ends the wavefront's list: every later
                // record is deeper (not so in an unsorted list, MODE 2).
                if (MODE != 2 && (!live_a || (hb && !live_b))) {
                    wave_alive = false;
                    break;
                }
            }
        }
    }

    // epilogue: outputs and the fused loss partial of this tile.  The inputs of every
    // pixel of the lane are loaded before the first store (addresses outside the image
    // clamped to pixel 0, absent target planes read from the base images, the values
    // then dropped), so the epilogue waits for one round trip.
    float lc = 0.0f, ld = 0.0f, lo = 0.0f;
    float edt[PPT], ec0[PPT], ec1[PPT], ec2[PPT], et0[PPT], et1[PPT], et2[PPT], etd[PPT];
    {
        const float* trgb = V.target_rgb ? V.target_rgb : V.base_rgb;
        const float* tdep = V.target_depth ? V.target_depth : V.base_depth;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int py = py0 + k * Lay::LROWS;
            const size_t p = (px < Wd && py < Ht) ? (size_t)py * Wd + px : 0;
            edt[k] = V.base_depth[p];
            ec0[k] = V.base_rgb[p];
            ec1[k] = V.base_rgb[HW + p];
            ec2[k] = V.base_rgb[2 * HW + p];
            et0[k] = trgb[p];
            et1[k] = trgb[HW + p];
            et2[k] = trgb[2 * HW + p];
            etd[k] = tdep[p];
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int py = py0 + k * Lay::LROWS;
        if (!(px < Wd && py < Ht)) continue;
        const size_t p = (size_t)py * Wd + px;
        const float dt = edt[k];
        const bool dvalid = dt > 0.0f;
        float Cs[3], Ds;
        const float ct0 = ec0[k], ct1 = ec1[k], ct2 = ec2[k];
        if (MODE == 0) {
            Cs[0] = __builtin_fmaf(T[k], ct0, ac0[k]);
            Cs[1] = __builtin_fmaf(T[k], ct1, ac1[k]);
            Cs[2] = __builtin_fmaf(T[k], ct2, ac2[k]);
            Ds = dvalid ? __builtin_fmaf(T[k], dt, ad[k]) : 0.0f;
        } else {
            const float inv = 1.0f / (1.0f + T[k]);
            Cs[0] = (ct0 + ac0[k]) * inv;
            Cs[1] = (ct1 + ac1[k]) * inv;
            Cs[2] = (ct2 + ac2[k]) * inv;
            Ds = dvalid ? (dt + ad[k]) * inv : 0.0f;
        }
        V.out_rgb[p] = Cs[0];
        V.out_rgb[HW + p] = Cs[1];
        V.out_rgb[2 * HW + p] = Cs[2];
        V.out_depth[p] = Ds;
        w.pix_aux[(size_t)V.pix_base + p] = T[k];
        if (V.out_aux) V.out_aux[p] = T[k];
        if (V.target_rgb) {
            lc += fabsf(Cs[0] - et0[k]) + fabsf(Cs[1] - et1[k]) + fabsf(Cs[2] - et2[k]);
            if (V.target_depth) {
                const float dobs = etd[k];
                if (dobs > 0.0f && dvalid) {
                    ld += fabsf(Ds - dobs);
                    lo += 1.0f;
                }
            }
        }
    }
    // One barrier: wave sums (DPP) of the three loss partials, the pair counts
    // (already uniform per wavefront), then the wavefronts in order by one thread.
    constexpr int NW = Lay::NW;
    __shared__ float sred[NW][3];
    __shared__ unsigned int scnt[NW][2];
    lc = wave_sum(lc);
    ld = wave_sum(ld);
    lo = wave_sum(lo);
    for (int o = 32; o > 0; o >>= 1) n_contrib += __shfl_xor(n_contrib, o, 64);
    if (lane == 0) {
        sred[wid][0] = lc;
        sred[wid][1] = ld;
        sred[wid][2] = lo;
        scnt[wid][0] = n_eval;
        scnt[wid][1] = n_contrib;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.0f, bsum = 0.0f, c = 0.0f;
        unsigned int te = 0u, tc = 0u;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            a += sred[k][0];
            bsum += sred[k][1];
            c += sred[k][2];
            te += scnt[k][0];
            tc += scnt[k][1];
        }
        w.tile_loss[tile] = make_float4(a, bsum, c, 0.0f);
        w.tile_pairs[tile] = make_uint2(te, tc);  // summed by k_loss_reduce
    }
}

// ----------------------------------------------------------------- launch
template <int TW, int TH, int B, int PPT, int MODE>
static void launch_cfwd_mode(const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles, hipStream_t s)
{
    GPS_LAUNCH(K_COMPOSITE_FWD, s, (k_composite_fwd<TW, TH, B, PPT, MODE>), dim3(n_tiles), dim3(TW * TH / PPT), 0, s,
               vt, rp, w);
}

template <int TW, int TH, int B, int PPT>
static void launch_cfwd(const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles, hipStream_t s)
{
    if (rp.mode == 0) launch_cfwd_mode<TW, TH, B, PPT, 0>(vt, rp, w, n_tiles, s);
    else if (rp.mode == 1) launch_cfwd_mode<TW, TH, B, PPT, 1>(vt, rp, w, n_tiles, s);
    else launch_cfwd_mode<TW, TH, B, PPT, 2>(vt, rp, w, n_tiles, s);
}

bool dispatch_cfwd(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                   hipStream_t s)
{
#define X(tw, th, b, ppt)                                                                                  \
    if (cfg->tile_w == tw && cfg->tile_h == th && cfg->batch == b && cfg->pix_per_thread == ppt) {       \
        launch_cfwd<tw, th, b, ppt>(vt, rp, w, n_tiles, s);                                             \
        return true;                                                                                     \
    }
    GPS_TILE_CONFIGS(X)
#undef X
    return false;
}

bool tile_config_supported(const gps_render_cfg* cfg)
{
#define X(tw, th, b, ppt) \
    if (cfg->tile_w == tw && cfg->tile_h == th && cfg->batch == b && cfg->pix_per_thread == ppt) return true;
    GPS_TILE_CONFIGS(X)
#undef X
    return false;
}

}  // namespace gps
