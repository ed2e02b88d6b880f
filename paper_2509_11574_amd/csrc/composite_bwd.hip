// Backward compositing: the analytic gradient of the forward compositing
// kernel.  Per tile it recomputes the front-to-back traversal of every pixel
// (transmittance T_i and the prefix colour and depth), forms the adjoints of
// each contributor's centre, conic, opacity, colour and depth (the first six in
// the base-2 form of the opacity), reduces them over the tile's pixels (a DPP
// transpose-reduction within each 16-lane row, LDS across rows and wavefronts,
// fixed order) and writes one 10-float partial per (tile, Gaussian) instance
// into that instance's slot: the view-Gaussian's first slot plus the tile's
// place in its tile rectangle.  Instances after the point where every pixel of
// the tile has stopped keep the zeros the emission wrote.  No floating-point
// atomics.
#include "launch.h"
#include "prof.h"
#include "render_common.h"

namespace gps {

__device__ __forceinline__ float sgnf(float x) { return (float)((x > 0.0f) - (x < 0.0f)); }

template <int TW, int TH, int B, int PPT, int MODE>
__global__ void __launch_bounds__(TW * TH / PPT)
    k_composite_bwd(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w, int explicit_up, const float* loss_scale)
{
    const ViewTable& vt = *vtp;
    using Lay = TileLayout<TW, TH, PPT>;
    constexpr int NT = Lay::NT;
    constexpr int NW = Lay::NW;
    __shared__ float4 srec[3 * B];
    __shared__ unsigned int sslot[B];
    __shared__ unsigned int smask[B];  // wavefront mask per staged record (32-bit: no byte stores in LDS)
    constexpr int S = kFlush;                // records per flush of the per-wavefront partials
    // Per record: NW wavefronts x 4 row partials x kAdj, padded so that successive
    // records start 10 banks apart (the flush reads (record, component) pairs).
    constexpr int kRecStride = NW * 4 * kAdj + ((10 - (NW * 4 * kAdj) % 32) + 32) % 32;
    __shared__ float slab[S * kRecStride];
    // Bit j of swritten[w]: wavefront w wrote its partial of window record j.  One
    // 64-bit word per wavefront, written by its lane 0: flags of different
    // wavefronts never share an LDS dword (sub-dword stores from different
    // wavefronts into one dword are not used anywhere).
    __shared__ unsigned long long swritten[NW];
    // One block per tile, in queue order (longest tile lists first).  The queue entry is
    // read together with the capacity check (one round trip) and checked against the
    // tile count.
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

    float sc = 1.0f;
    if (!explicit_up && loss_scale) sc = *loss_scale;
    const float invV = 1.0f / (float)rp.V;
    const float om = w.hdr->view_stats[v][2];

    // Per pixel: the upstream adjoint G = (dL/dC*, dL/dD*), CG = G . (C*, D*) and
    // the running PG = G . P_i, where P_i is the composited prefix through
    // Gaussian i.  The remainder term of dL/dalpha_i only ever needs
    // G . (C* - P_i) = CG - PG, so the prefix colours are not kept.
    // thr as in the forward: -inf once a pixel has stopped for a reason other
    // than the depth test (which every deeper record fails as well).
    float thr[PPT], T[PPT], G0[PPT], G1[PPT], G2[PPT], GD[PPT], CG[PPT], PG[PPT], invW[PPT];
    // Every per-pixel load is issued before any is used, so the prologue waits for one
    // round trip: addresses outside the image are clamped to pixel 0 and an absent
    // depth plane is read from the base depth, the values then being dropped.
    bool inb[PPT];
    float ldt[PPT], lc0[PPT], lc1[PPT], lc2[PPT], lds[PPT], lx0[PPT], lx1[PPT], lx2[PPT], lxd[PPT], laux[PPT];
    {
        const float* xrgb = explicit_up ? V.g_rgb : V.target_rgb;
        const float* xdep = explicit_up ? V.g_depth : V.target_depth;
        const float* xdl = xdep ? xdep : V.base_depth;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int py = py0 + k * Lay::LROWS;
            inb[k] = px < Wd && py < Ht;
            const size_t p = inb[k] ? (size_t)py * Wd + px : 0;
            ldt[k] = V.base_depth[p];
            lc0[k] = V.out_rgb[p];
            lc1[k] = V.out_rgb[HW + p];
            lc2[k] = V.out_rgb[2 * HW + p];
            lds[k] = V.out_depth[p];
            laux[k] = MODE != 0 ? w.pix_aux[(size_t)V.pix_base + p] : 0.0f;
            lx0[k] = xrgb[p];
            lx1[k] = xrgb[HW + p];
            lx2[k] = xrgb[2 * HW + p];
            lxd[k] = xdl[p];
        }
        const bool has_xdep = xdep != nullptr;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const float dt = inb[k] ? ldt[k] : 0.0f;
            const bool dvalid = dt > 0.0f;
            thr[k] = inb[k] ? (dvalid ? dt : INFINITY) + rp.eps : -INFINITY;
            T[k] = 1.0f;
            PG[k] = 0.0f;
            G0[k] = G1[k] = G2[k] = GD[k] = 0.0f;
            float cs0 = 0.0f, cs1 = 0.0f, cs2 = 0.0f, ds = 0.0f;
            invW[k] = 1.0f;
            if (inb[k]) {
                cs0 = lc0[k];
                cs1 = lc1[k];
                cs2 = lc2[k];
                ds = lds[k];
                if (MODE != 0) invW[k] = 1.0f / (1.0f + laux[k]);
                if (explicit_up) {
                    G0[k] = lx0[k];
                    G1[k] = lx1[k];
                    G2[k] = lx2[k];
                    GD[k] = (has_xdep && dvalid) ? lxd[k] : 0.0f;
                } else {
                    const float cn = sc * invV / (3.0f * (float)HW);
                    G0[k] = cn * sgnf(cs0 - lx0[k]);
                    G1[k] = cn * sgnf(cs1 - lx1[k]);
                    G2[k] = cn * sgnf(cs2 - lx2[k]);
                    if (has_xdep && dvalid && om > 0.0f) {
                        const float dobs = lxd[k];
                        if (dobs > 0.0f) GD[k] = sc * invV * rp.lambda / om * sgnf(ds - dobs);
                    }
                }
            }
            CG[k] = G0[k] * cs0 + G1[k] * cs1 + G2[k] * cs2 + GD[k] * ds;
        }
    }

    const unsigned int s = w.tile_start[tile], e = w.tile_start[tile + 1];
    const int tx0 = tx * TW, ty0 = ty * TH;
    bool wave_alive = true;  // some pixel of this wavefront still takes records
    for (unsigned int b = s; b < e; b += B) {
        if (__syncthreads_count(wave_alive && lane == 0) == 0) break;
        for (int j = threadIdx.x; j < B; j += NT) {
            unsigned int mk = 0u, slot = 0xffffffffu;
            if (b + j < e) {
                unsigned int vg = (unsigned int)w.keys[b + j];
                if (vg >= (unsigned int)rp.nvg) vg = 0u;  // guard: never read outside the records
                const float4* r = w.rec + 3 * (size_t)vg;
                const float4 r0 = r[0], r1 = r[1], r2 = r[2];
                const unsigned int o = w.off[vg];
                srec[3 * j + 0] = r0;
                srec[3 * j + 1] = r1;
                srec[3 * j + 2] = r2;
                mk = wave_support_mask<Lay>(r0, r1, l2amin, tx0, ty0);
                // the instance's slot: its view-Gaussian's first slot plus this tile's
                // place in the tile rectangle (the rectangle the expansion walked)
                TileRect rr;
                if (rect_of(r0.x, r0.y, r2.z, r2.w, Wd, Ht, rp.tile_w, rp.tile_h, &rr))
                    slot = o + (unsigned int)((ty - rr.ty0) * (rr.tx1 - rr.tx0 + 1) + (tx - rr.tx0));
            }
            smask[j] = mk;
            sslot[j] = slot;
        }
        __syncthreads();
        const int n = (int)min((unsigned int)B, e - b);
        int alive_now = 1;
        for (int j0 = 0; j0 < n && alive_now; j0 += S) {
            const int j1 = min(j0 + S, n);
            // Records of this window whose support meets this wavefront (as in the forward).
            const int jl = j0 + lane;
            unsigned long long m =
                __builtin_amdgcn_ballot_w64(wave_alive && lane < S && jl < j1 && ((smask[jl] >> wid) & 1u));
            unsigned long long written = 0ull;  // window records whose partial this wavefront wrote
            while (m) {
                const int jw = (int)__builtin_ctzll(m);
                m &= m - 1ull;
                const int j = j0 + jw;
                const float4 r0 = srec[3 * j], r1 = srec[3 * j + 1], r2 = srec[3 * j + 2];
                const float c0 = r1.w, c1 = r2.x, c2 = r2.y, zi = r1.z;
                // the forward's decisions, in the same order and arithmetic
                bool lane_live = false, lane_use = false;  // over the lane's pixels
                AlphaEval ae[PPT];
                float av[PPT], Tn[PPT];
                bool use[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const bool live = zi < thr[k];
                    lane_live = lane_live || live;
                    ae[k] = eval_alpha(fpx, (float)(py0 + k * Lay::LROWS), r0.x, r0.y, r0.z, r0.w, r1.x, r1.y);
                    if (MODE == 0) {
                        av[k] = fminf(ae[k].raw, rp.amax);
                        const bool ok = live && av[k] >= rp.amin;
                        Tn[k] = T[k] * (1.0f - av[k]);
                        const bool stop = ok && Tn[k] < rp.Tmin;
                        use[k] = ok && !stop;
                        thr[k] = stop ? -INFINITY : thr[k];
                    } else {
                        av[k] = ae[k].raw;
                        Tn[k] = 0.0f;
                        use[k] = live && av[k] >= rp.amin;
                    }
                    lane_use = lane_use || use[k];
                }
                const unsigned long long any_live = __builtin_amdgcn_ballot_w64(lane_live);
                if (__builtin_amdgcn_ballot_w64(lane_use)) {
                    // Adjoints of the contributing lanes; the others carry zero
                    // weight, so no accumulator needs clearing.
                    float g[kAdj];
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        const float direct = G0[k] * c0 + G1[k] * c1 + G2[k] * c2 + GD[k] * zi;  // G . (c_i, d_i)
                        float wgt, dal;
                        bool apath;
                        if (MODE == 0) {
                            wgt = use[k] ? av[k] * T[k] : 0.0f;  // w_i = alpha_i T_i
                            PG[k] = __builtin_fmaf(wgt, direct, PG[k]);
                            // dL/dalpha_i = T_i G.(c_i,d_i) - G.(C* - P_i) / (1 - alpha_i)
                            dal = T[k] * direct - (CG[k] - PG[k]) * __builtin_amdgcn_rcpf(1.0f - av[k]);
                            apath = use[k] && ae[k].raw <= rp.amax;  // a capped opacity has no gradient
                            T[k] = use[k] ? Tn[k] : T[k];
                        } else {
                            wgt = use[k] ? av[k] * invW[k] : 0.0f;  // d C* / d c_i = alpha_i / (1 + W_G)
                            dal = invW[k] * (direct - CG[k]);
                            apath = use[k];
                        }
                        // alpha = exp2(pw): d alpha / d pw = alpha ln 2; the constant
                        // factors are applied once per Gaussian.
                        const float u = apath ? dal * av[k] : 0.0f;
                        const float t0 = u * ae[k].dx;
                        const float t1 = u * ae[k].dy;
                        if (k == 0) {
                            g[0] = t0;
                            g[1] = t1;
                            g[2] = u * ae[k].dxx;
                            g[3] = u * ae[k].dxy;
                            g[4] = u * ae[k].dyy;
                            g[5] = u;
                            g[6] = wgt * G0[k];
                            g[7] = wgt * G1[k];
                            g[8] = wgt * G2[k];
                            g[9] = wgt * GD[k];
                        } else {
                            g[0] += t0;
                            g[1] += t1;
                            g[2] = __builtin_fmaf(u, ae[k].dxx, g[2]);
                            g[3] = __builtin_fmaf(u, ae[k].dxy, g[3]);
                            g[4] = __builtin_fmaf(u, ae[k].dyy, g[4]);
                            g[5] += u;
                            g[6] = __builtin_fmaf(wgt, G0[k], g[6]);
                            g[7] = __builtin_fmaf(wgt, G1[k], g[7]);
                            g[8] = __builtin_fmaf(wgt, G2[k], g[8]);
                            g[9] = __builtin_fmaf(wgt, GD[k], g[9]);
                        }
                    }
                    wave_rows_sum10_store(g, slab + jw * kRecStride + wid * 4 * kAdj, lane);
                    written |= 1ull << jw;
                }
                if (MODE != 2 && !any_live) {  // this record and all deeper ones fail every pixel
                                               // (an unsorted list, MODE 2, goes on)
                    wave_alive = false;
                    break;
                }
            }
            if (lane == 0) swritten[wid] = written;
            alive_now = __syncthreads_count(wave_alive && lane == 0);
            // one thread per (record, component): sum the wavefront partials in order
            for (int t = threadIdx.x; t < (j1 - j0) * kAdj; t += NT) {
                const int jr = t / kAdj, q = t - jr * kAdj;
                float acc = 0.0f;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww)
                    if ((swritten[ww] >> jr) & 1ull) {
                        const float* sp = slab + jr * kRecStride + ww * 4 * kAdj + q;
                        acc += (sp[0] + sp[kAdj]) + (sp[2 * kAdj] + sp[3 * kAdj]);
                    }
                const unsigned int slot = sslot[j0 + jr];
                if (slot < rp.cap) w.partial[(size_t)slot * kAdj + q] = acc;
            }
            __syncthreads();
        }
        if (!alive_now) break;
    }
}

// ------------------------------------------- per-Gaussian backward (sort-free)
// The backward of the sort-free blend (Eq. 1, 2, 4) as Appendix B organises it:
// each Gaussian accumulates its own adjoints in-thread over the pixels it covers,
// with no atomics.  The blend's adjoints are independent per (pixel, Gaussian)
// (they need only the pixel's C*, D*, W_G and upstream adjoint), so the pixels are
// grouped by screen tile: one block per tile stages the tile's per-pixel state in
// LDS once, then each wavefront takes the tile's Gaussians one at a time and its
// lanes sweep the Gaussian's support rectangle inside the tile 64 pixels at a
// time, summing in registers; one wave reduction per (Gaussian, tile) gives the
// instance partial, written into its slot.  Nothing per pixel is re-read from
// memory for every Gaussian.
template <int TW, int TH>
__global__ void __launch_bounds__(256) k_composite_bwd_pg(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w,
                                                         int explicit_up, const float* loss_scale)
{
    constexpr int NP = TW * TH;
    const ViewTable& vt = *vtp;
    static_assert(TW <= 64, "a step of 64 lanes covers at least one box row");
    __shared__ float4 s_g[NP];  // (dL/dC*, dL/dD*) / (1 + W_G)
    __shared__ float2 s_x[NP];  // G.(C*, D*) / (1 + W_G), D_t + eps (-inf outside the image)
    __shared__ float s_red[4][4 * kAdj];  // per wavefront: the ten row totals of its four rows
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
    const int tx0 = tx * TW, ty0 = ty * TH;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    {
        float sc = 1.0f;
        if (!explicit_up && loss_scale) sc = *loss_scale;
        const float invV = 1.0f / (float)rp.V;
        const float om = w.hdr->view_stats[v][2];
        for (int i = threadIdx.x; i < NP; i += 256) {
            const int px = tx0 + i % TW, py = ty0 + i / TW;
            float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
            float2 x = make_float2(0.f, -INFINITY);
            if (px < Wd && py < Ht) {
                const size_t p = (size_t)py * Wd + px;
                const float dt = V.base_depth[p];
                const bool dvalid = dt > 0.0f;
                const float cs0 = V.out_rgb[p], cs1 = V.out_rgb[HW + p], cs2 = V.out_rgb[2 * HW + p];
                const float ds = V.out_depth[p];
                float G0, G1, G2, GD = 0.0f;
                if (explicit_up) {
                    G0 = V.g_rgb[p];
                    G1 = V.g_rgb[HW + p];
                    G2 = V.g_rgb[2 * HW + p];
                    GD = (V.g_depth && dvalid) ? V.g_depth[p] : 0.0f;
                } else {
                    const float cn = sc * invV / (3.0f * (float)HW);
                    G0 = cn * sgnf(cs0 - V.target_rgb[p]);
                    G1 = cn * sgnf(cs1 - V.target_rgb[HW + p]);
                    G2 = cn * sgnf(cs2 - V.target_rgb[2 * HW + p]);
                    if (V.target_depth && dvalid && om > 0.0f) {
                        const float dobs = V.target_depth[p];
                        if (dobs > 0.0f) GD = sc * invV * rp.lambda / om * sgnf(ds - dobs);
                    }
                }
                const float invW = 1.0f / (1.0f + w.pix_aux[(size_t)V.pix_base + p]);
                const float CG = G0 * cs0 + G1 * cs1 + G2 * cs2 + GD * ds;
                g = make_float4(G0 * invW, G1 * invW, G2 * invW, GD * invW);
                x = make_float2(CG * invW, (dvalid ? dt : INFINITY) + rp.eps);
            }
            s_g[i] = g;
            s_x[i] = x;
        }
    }
    __syncthreads();
    const unsigned int s = w.tile_start[tile], e = w.tile_start[tile + 1];
    for (unsigned int j = s + (unsigned int)wid; j < e; j += 4u) {
        unsigned int vg = (unsigned int)w.keys[j];
        if (vg >= (unsigned int)rp.nvg) vg = 0u;  // guard: never read outside the records
        const float4* r = w.rec + 3 * (size_t)vg;
        const float4 r0 = r[0], r1 = r[1], r2 = r[2];
        const float zi = r1.z, c0 = r1.w, c1 = r2.x, c2 = r2.y;
        // the record's support box (padded, it holds every pixel with alpha >= alpha_min)
        // inside this tile and the image
        const int x0 = max(max((int)ceilf(r0.x - r2.z), tx0), 0);
        const int x1 = min(min((int)floorf(r0.x + r2.z), tx0 + TW - 1), Wd - 1);
        const int y0 = max(max((int)ceilf(r0.y - r2.w), ty0), 0);
        const int y1 = min(min((int)floorf(r0.y + r2.w), ty0 + TH - 1), Ht - 1);
        float g[kAdj];
#pragma unroll
        for (int q = 0; q < kAdj; ++q) g[q] = 0.0f;
        if (x0 <= x1 && y0 <= y1) {
            const int bw = x1 - x0 + 1, bh = y1 - y0 + 1;
            const int dr = 64 / bw, dc = 64 - dr * bw;  // a step of 64 pixels in rows and columns
            int row = lane / bw, col = lane - (lane / bw) * bw;
            while (row < bh) {
                const int px = x0 + col, py = y0 + row;
                const int li = (py - ty0) * TW + (px - tx0);
                const float4 G = s_g[li];
                const float2 X = s_x[li];
                const AlphaEval ae = eval_alpha((float)px, (float)py, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y);
                const bool use = zi < X.y && ae.raw >= rp.amin;  // depth test (Eq. 1-2), alpha_min
                const float a = use ? ae.raw : 0.0f;
                const float direct = G.x * c0 + G.y * c1 + G.z * c2 + G.w * zi;
                const float u = a * (direct - X.x);  // alpha dL/dalpha
                g[0] = __builtin_fmaf(u, ae.dx, g[0]);
                g[1] = __builtin_fmaf(u, ae.dy, g[1]);
                g[2] = __builtin_fmaf(u, ae.dxx, g[2]);
                g[3] = __builtin_fmaf(u, ae.dxy, g[3]);
                g[4] = __builtin_fmaf(u, ae.dyy, g[4]);
                g[5] += u;
                g[6] = __builtin_fmaf(a, G.x, g[6]);  // dC*/dc_i = alpha / (1 + W_G)
                g[7] = __builtin_fmaf(a, G.y, g[7]);
                g[8] = __builtin_fmaf(a, G.z, g[8]);
                g[9] = __builtin_fmaf(a, G.w, g[9]);
                row += dr;
                col += dc;
                if (col >= bw) {
                    col -= bw;
                    ++row;
                }
            }
        }
        // The ten sums over the wavefront: a DPP transpose-reduction within each 16-lane row,
        // then lane q adds the four row totals of component q in a fixed order.  The LDS
        // words are this wavefront's own; the fences order its stores and loads.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        wave_rows_sum10_store(g, s_red[wid], lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float mine = 0.0f;  // lane q keeps component q
        if (lane < kAdj)
            mine = (s_red[wid][lane] + s_red[wid][kAdj + lane]) + (s_red[wid][2 * kAdj + lane] + s_red[wid][3 * kAdj + lane]);
        // the instance's slot: its view-Gaussian's first slot plus this tile's place in
        // the tile rectangle (the rectangle the expansion walked)
        TileRect rr;
        if (lane < kAdj && rect_of(r0.x, r0.y, r2.z, r2.w, Wd, Ht, rp.tile_w, rp.tile_h, &rr)) {
            const unsigned int slot =
                w.off[vg] + (unsigned int)((ty - rr.ty0) * (rr.tx1 - rr.tx0 + 1) + (tx - rr.tx0));
            if (slot < rp.cap) w.partial[(size_t)slot * kAdj + lane] = mine;
        }
    }
}

template <int TW, int TH>
static void launch_cbwd_pg(const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles, int explicit_up,
                           const float* loss_scale, hipStream_t s)
{
    GPS_LAUNCH(K_COMPOSITE_BWD, s, (k_composite_bwd_pg<TW, TH>), dim3(n_tiles), dim3(256), 0, s, vt, rp, w,
               explicit_up, loss_scale);
}

// The per-Gaussian backward of the sort-free blend (GPS_RENDER_BWD_PER_GAUSSIAN).
bool dispatch_cbwd_pg(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                      int explicit_up, const float* loss_scale, hipStream_t s)
{
    if (cfg->tile_w == 8 && cfg->tile_h == 8) launch_cbwd_pg<8, 8>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else if (cfg->tile_w == 16 && cfg->tile_h == 16)
        launch_cbwd_pg<16, 16>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else if (cfg->tile_w == 16 && cfg->tile_h == 32)
        launch_cbwd_pg<16, 32>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else if (cfg->tile_w == 32 && cfg->tile_h == 16)
        launch_cbwd_pg<32, 16>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else return false;
    return true;
}

// ----------------------------------------------------------------- launch
template <int TW, int TH, int B, int PPT, int MODE>
static void launch_cbwd_mode(const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles, int explicit_up,
                             const float* loss_scale, hipStream_t s)
{
    GPS_LAUNCH(K_COMPOSITE_BWD, s, (k_composite_bwd<TW, TH, B, PPT, MODE>), dim3(n_tiles), dim3(TW * TH / PPT), 0, s,
               vt, rp, w, explicit_up, loss_scale);
}

template <int TW, int TH, int B, int PPT>
static void launch_cbwd(const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles, int explicit_up,
                        const float* loss_scale, hipStream_t s)
{
    if (rp.mode == 0) launch_cbwd_mode<TW, TH, B, PPT, 0>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else if (rp.mode == 1) launch_cbwd_mode<TW, TH, B, PPT, 1>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
    else launch_cbwd_mode<TW, TH, B, PPT, 2>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);
}

bool dispatch_cbwd(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                   int explicit_up, const float* loss_scale, hipStream_t s)
{
#define X(tw, th, b, ppt)                                                                              \
    if (cfg->tile_w == tw && cfg->tile_h == th && cfg->batch == b && cfg->pix_per_thread == ppt) {   \
        launch_cbwd<tw, th, b, ppt>(vt, rp, w, n_tiles, explicit_up, loss_scale, s);                 \
        return true;                                                                                 \
    }
    GPS_TILE_CONFIGS(X)
#undef X
    return false;
}

}  // namespace gps
