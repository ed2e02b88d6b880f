// Backward render (analytic gradient of the forward render).
//
//   k_composite_bwd  (composite_bwd.hip) per tile: one 10-float partial per
//       (tile, Gaussian) instance, written into that instance's slot.
//   k_gauss_bwd   per Gaussian: sum its instance partials (a contiguous slot
//       range per view, summed in order), apply the EWA chain rule to the
//       parameters and form the per-Gaussian pose terms, reduced per block.
//   k_pose_reduce per view: sum the block pose partials in order.
//   The per-Gaussian backward of the sort-free blend (GPS_RENDER_BWD_PER_GAUSSIAN)
//   replaces k_composite_bwd by k_composite_bwd_pg (composite_bwd.hip).
//   With Adam in the epilogue (gps_render_bwd_adam), k_gauss_bwd also applies
//   the Adam step to its Gaussian and k_pose_reduce advances the step counter.
// No floating-point atomics: results are bitwise reproducible.
#include "adam_math.h"
#include "launch.h"
#include "prof.h"
#include "render_common.h"
#include "se3.h"

namespace gps {

// ------------------------------------------------------------- gauss bwd
constexpr unsigned int kCoopSlots = 32;  // more slots than this: summed by the whole wavefront
constexpr unsigned int kSlotGroup = 8;   // slots loaded together by one lane

// EWA chain rule of one Gaussian in one view.  The summed instance partials are
// first turned into A[10] = dL/d(mx, my, a, b, c), sigma dL/dsigma, dL/d(r, g, b, d),
// where (a, b, c) is the conic and b multiplies 2 dx dy.
// Adam applied in the epilogue of k_gauss_bwd: the attribute groups (mean,
// log-scale, quaternion, opacity logit, rgb, and the SH bands when there are
// any), each with its learning rate.
struct AdamFuse {
    float* p[6];
    float* m[6];
    float* v[6];
    float lr[6];
    const int* step_ctr;
    int step;
    float b1, b2, eps;
    int on;
};

// SHK: SH coefficients per channel (0, 3, 8 or 15).  The colour adjoint of each
// view (A[6..8]) goes to rgb and, times the basis at that view's direction, to the
// coefficients; through the direction d = (mu - o) / |mu - o| it moves the centre by
// (I - d d^T) / |mu - o| times the basis gradient weighted by the coefficients, and
// the camera centre moves by -R^T rho under the left perturbation, so rho takes R
// times the same vector.
template <int SHK>
__global__ void __launch_bounds__(kBlk) k_gauss_bwd(const ViewTable* __restrict__ vtp, RParams rp, GParams gp, GGrads gg,
                                                    WsPtrs w, AdamFuse af)
{
    const ViewTable& vt = *vtp;
    const int M = rp.M;
    const int g = blockIdx.x * kBlk + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool live = g < M;
    // After a capacity overflow the forward stopped before it wrote the slot offsets
    // and partials: no slot is read, every gradient is zero and the Adam step of the
    // epilogue is skipped, so parameters and moments stay as they were.
    const bool over = w.hdr->n_inst > rp.cap;
    float gmean[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0.0f, grgb[3] = {0, 0, 0};
    constexpr int NSH = SHK > 0 ? 3 * SHK : 1;
    float gsh[NSH];
#pragma unroll
    for (int k = 0; k < NSH; ++k) gsh[k] = 0.0f;
    __shared__ float pred[kBlk / 64][6];

    // Every load that does not depend on another is issued here, before any of them is
    // waited for: the slot count and offset of the first view, the Adam state of the
    // five parameter groups (14 scalars) and the parameters.  The slot sums then wait
    // for one round trip, and the Adam loads overlap them.
    const unsigned int cnt0 = live ? w.cnt[g] : 0u, off0 = live ? w.off[g] : 0u;
    constexpr int kAdamRows[5] = {3, 3, 4, 1, 3};
    float ap[14], am[14], av[14];
    const bool adam_here = live && af.on && !over;
    if (live && af.on) {
        int j = 0;
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int r = 0; r < kAdamRows[a]; ++r, ++j) {
                const size_t i = (size_t)r * M + g;
                ap[j] = af.p[a][i];
                am[j] = af.m[a][i];
                av[j] = af.v[a][i];
            }
    }
    float m0 = 0, m1 = 0, m2 = 0, qw = 1, qx = 0, qy = 0, qz = 0, qn = 1, s[3] = {1, 1, 1}, sig = 0.5f;
    float Rq[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (live) {
        m0 = gp.mean[g];
        m1 = gp.mean[M + g];
        m2 = gp.mean[2 * M + g];
        qw = gp.quat[g];
        qx = gp.quat[M + g];
        qy = gp.quat[2 * M + g];
        qz = gp.quat[3 * M + g];
        qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        const float qi = 1.0f / qn;
        qw *= qi;
        qx *= qi;
        qy *= qi;
        qz *= qi;
        Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
        Rq[1] = 2.f * (qx * qy - qw * qz);
        Rq[2] = 2.f * (qx * qz + qw * qy);
        Rq[3] = 2.f * (qx * qy + qw * qz);
        Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
        Rq[5] = 2.f * (qy * qz - qw * qx);
        Rq[6] = 2.f * (qx * qz - qw * qy);
        Rq[7] = 2.f * (qy * qz + qw * qx);
        Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);
        s[0] = __expf(gp.log_scale[g]);
        s[1] = __expf(gp.log_scale[M + g]);
        s[2] = __expf(gp.log_scale[2 * M + g]);
        sig = 1.0f / (1.0f + __expf(-gp.opacity_logit[g]));
    }
    // Mm = Rq diag(s), Sigma_3D = Mm Mm^T
    float Mm[9], S3[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Rq[3 * r + c] * s[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) S3[3 * r + c] = Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2];

    // Adam's bias corrections, per lane (no barrier, so no wait for the loads above)
    float ibc1 = 1.0f, ibc2 = 1.0f;
    if (adam_here) adam_bias(af.step_ctr ? (*af.step_ctr + 1) : af.step, af.b1, af.b2, &ibc1, &ibc2);

    for (int v = 0; v < vt.n; ++v) {
        float pose[6] = {0, 0, 0, 0, 0, 0};
        const size_t vg = (size_t)v * M + g;
        const unsigned int cl = v == 0 ? cnt0 : (live ? w.cnt[vg] : 0u);
        const unsigned int ol = v == 0 ? off0 : (live ? w.off[vg] : 0u);
        unsigned int cnt = over ? 0u : cl;
        const unsigned int o = cnt ? ol : 0u;
        if ((unsigned long long)o + cnt > w.hdr->n_inst) cnt = 0u;  // guard: stay inside the emitted slots
        // Slots of tiles removed by the depth cull were zeroed by the emission, so the
        // whole contiguous range is summed (in a fixed order).
        float A[kAdj];
#pragma unroll
        for (int q = 0; q < kAdj; ++q) A[q] = 0.0f;
        // A Gaussian with more than kCoopSlots slots is summed by its whole wavefront
        // (lanes take its slots in strides of 64, then a fixed-order wave sum), so the
        // few Gaussians that cover many tiles do not hold their wavefront up.
        unsigned long long big = __ballot(cnt > kCoopSlots);
        while (big) {
            const int b = __ffsll(big) - 1;
            const unsigned int ob = (unsigned int)__shfl((int)o, b, 64), cb = (unsigned int)__shfl((int)cnt, b, 64);
            float acc[kAdj];
#pragma unroll
            for (int q = 0; q < kAdj; ++q) acc[q] = 0.0f;
            for (unsigned int k = (unsigned int)lane; k < cb; k += 64) {
                const float* ps = w.partial + (size_t)(ob + k) * kAdj;
#pragma unroll
                for (int q = 0; q < kAdj; ++q) acc[q] += ps[q];
            }
#pragma unroll
            for (int q = 0; q < kAdj; ++q) {
                const float t = wave_sum(acc[q]);
                if (lane == b) A[q] = t;
            }
            big &= big - 1ull;
        }
        if (cnt > 0 && cnt <= kCoopSlots) {
            // The lane's slots in groups of kSlotGroup: the loads of a group are issued
            // together, so a group costs one round trip (a position past the count reads
            // the group's first slot again and adds zero); the slots are still added in
            // order (adding +0.0 to a sum that starts at +0.0 leaves it unchanged).
            const float* part = w.partial + (size_t)o * kAdj;
            for (unsigned int k0 = 0; k0 < cnt; k0 += kSlotGroup) {
                float sv[kSlotGroup][kAdj];
#pragma unroll
                for (unsigned int i = 0; i < kSlotGroup; ++i) {
                    const bool has = k0 + i < cnt;
                    const float* ps = part + (size_t)(has ? k0 + i : k0) * kAdj;
#pragma unroll
                    for (int q = 0; q < kAdj; ++q) sv[i][q] = ps[q];
#pragma unroll
                    for (int q = 0; q < kAdj; ++q) sv[i][q] = has ? sv[i][q] : 0.0f;
                }
#pragma unroll
                for (unsigned int i = 0; i < kSlotGroup; ++i)
#pragma unroll
                    for (int q = 0; q < kAdj; ++q) A[q] += sv[i][q];
            }
        }
        if (cnt > 0) {
            // The compositing kernel accumulates, with u = dL/dalpha * alpha, the sums
            // of u dx, u dy, u dx^2, u dx dy, u dy^2 and u, where alpha = exp2(pw),
            // pw = A' dx^2 + B' dx dy + C' dy^2 + log2 sigma and (A', B', C') =
            // (-0.5 a, -b, -0.5 c) log2 e.  Since d alpha / d pw = alpha ln 2 and
            // ln 2 log2 e = 1: dL/dm = conic (sum u dx, sum u dy) (applied below, once the
            // conic is known), dL/da = -0.5 A[2], dL/db = -A[3], dL/dc = -0.5 A[4], and
            // dL/dsigma sigma = A[5].
            A[2] *= -0.5f;
            A[3] = -A[3];
            A[4] *= -0.5f;
            const DevCam& c = vt.v[v].cam;
            const float* R = c.R;
            const float x = R[0] * m0 + R[1] * m1 + R[2] * m2 + c.t[0];
            const float y = R[3] * m0 + R[4] * m1 + R[5] * m2 + c.t[1];
            const float z = d32_row(c.R, c.t, 2, m0, m1, m2);
            const float iz = 1.0f / z, iz2 = iz * iz;
            const float J00 = c.fx * iz, J02 = -c.fx * x * iz2, J11 = c.fy * iz, J12 = -c.fy * y * iz2;
            float Wm[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Wm[k] = J00 * R[k] + J02 * R[6 + k];
                Wm[3 + k] = J11 * R[3 + k] + J12 * R[6 + k];
            }
            // conic from Sigma_2D = W S3 W^T + dil
            float WS[6];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    WS[3 * r + k] = Wm[3 * r] * S3[k] + Wm[3 * r + 1] * S3[3 + k] + Wm[3 * r + 2] * S3[6 + k];
            const float SA = WS[0] * Wm[0] + WS[1] * Wm[1] + WS[2] * Wm[2] + rp.dil;
            const float SB = WS[0] * Wm[3] + WS[1] * Wm[4] + WS[2] * Wm[5];
            const float SC = WS[3] * Wm[3] + WS[4] * Wm[4] + WS[5] * Wm[5] + rp.dil;
            const float idet = 1.0f / (SA * SC - SB * SB);
            const float qa = SC * idet, qb = -SB * idet, qc = SA * idet;
            {
                const float sx = A[0], sy = A[1];  // sum u dx, sum u dy
                A[0] = qa * sx + qb * sy;          // dL/dm_x
                A[1] = qb * sx + qc * sy;          // dL/dm_y
            }

            grgb[0] += A[6];
            grgb[1] += A[7];
            grgb[2] += A[8];
            float rho_sh[3] = {0.0f, 0.0f, 0.0f};
            if constexpr (SHK > 0) {
                const float v0 = m0 + (R[0] * c.t[0] + R[3] * c.t[1] + R[6] * c.t[2]);
                const float v1 = m1 + (R[1] * c.t[0] + R[4] * c.t[1] + R[7] * c.t[2]);
                const float v2 = m2 + (R[2] * c.t[0] + R[5] * c.t[1] + R[8] * c.t[2]);
                const float ir = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
                const float d0 = v0 * ir, d1 = v1 * ir, d2 = v2 * ir;
                float Y[SHK], wk[SHK];
                sh_basis<SHK>(d0, d1, d2, Y);
#pragma unroll
                for (int k = 0; k < SHK; ++k) {
                    gsh[k] += A[6] * Y[k];
                    gsh[SHK + k] += A[7] * Y[k];
                    gsh[2 * SHK + k] += A[8] * Y[k];
                    wk[k] = A[6] * gp.sh[(size_t)k * M + g] + A[7] * gp.sh[(size_t)(SHK + k) * M + g] +
                            A[8] * gp.sh[(size_t)(2 * SHK + k) * M + g];
                }
                float gd[3];
                sh_weighted_grad<SHK>(d0, d1, d2, wk, gd);
                const float dd = d0 * gd[0] + d1 * gd[1] + d2 * gd[2];
                const float u0 = (gd[0] - d0 * dd) * ir, u1 = (gd[1] - d1 * dd) * ir, u2 = (gd[2] - d2 * dd) * ir;
                gmean[0] += u0;
                gmean[1] += u1;
                gmean[2] += u2;
                rho_sh[0] = R[0] * u0 + R[1] * u1 + R[2] * u2;
                rho_sh[1] = R[3] * u0 + R[4] * u1 + R[5] * u2;
                rho_sh[2] = R[6] * u0 + R[7] * u1 + R[8] * u2;
            }
            gop += A[5] * (1.0f - sig);  // dL/dsigma * sigma (1 - sigma)
            // G2 = -Q Gq Q with Gq = [[A2, A3/2], [A3/2, A4]]
            const float h = 0.5f * A[3];
            const float T00 = qa * A[2] + qb * h, T01 = qa * h + qb * A[4];
            const float T10 = qb * A[2] + qc * h, T11 = qb * h + qc * A[4];
            const float G00 = -(T00 * qa + T01 * qb), G01 = -(T00 * qb + T01 * qc), G11 = -(T10 * qb + T11 * qc);
            // G3 = W^T G2 W ; GW = 2 G2 W S3
            float G2W[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                G2W[k] = G00 * Wm[k] + G01 * Wm[3 + k];
                G2W[3 + k] = G01 * Wm[k] + G11 * Wm[3 + k];
            }
            float G3[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) G3[3 * r + k] = Wm[r] * G2W[k] + Wm[3 + r] * G2W[3 + k];
            float GW[6];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    GW[3 * r + k] = 2.0f * (G2W[3 * r] * S3[k] + G2W[3 * r + 1] * S3[3 + k] + G2W[3 * r + 2] * S3[6 + k]);
            // G_J = GW R^T  (only J00, J02, J11, J12 depend on p_c)
            const float GJ00 = GW[0] * R[0] + GW[1] * R[1] + GW[2] * R[2];
            const float GJ02 = GW[0] * R[6] + GW[1] * R[7] + GW[2] * R[8];
            const float GJ11 = GW[3] * R[3] + GW[4] * R[4] + GW[5] * R[5];
            const float GJ12 = GW[3] * R[6] + GW[4] * R[7] + GW[5] * R[8];
            const float iz3 = iz2 * iz;
            float gpx = GJ02 * (-c.fx * iz2) + A[0] * c.fx * iz;
            float gpy = GJ12 * (-c.fy * iz2) + A[1] * c.fy * iz;
            float gpz = GJ00 * (-c.fx * iz2) + GJ02 * (2.0f * c.fx * x * iz3) + GJ11 * (-c.fy * iz2) +
                        GJ12 * (2.0f * c.fy * y * iz3) - A[0] * c.fx * x * iz2 - A[1] * c.fy * y * iz2 + A[9];
            gmean[0] += R[0] * gpx + R[3] * gpy + R[6] * gpz;
            gmean[1] += R[1] * gpx + R[4] * gpy + R[7] * gpz;
            gmean[2] += R[2] * gpx + R[5] * gpy + R[8] * gpz;
            // Sigma_3D = Mm Mm^T: G_Mm = 2 G3 Mm
            float GM[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    GM[3 * r + k] = 2.0f * (G3[3 * r] * Mm[k] + G3[3 * r + 1] * Mm[3 + k] + G3[3 * r + 2] * Mm[6 + k]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                gls[k] += (Rq[k] * GM[k] + Rq[3 + k] * GM[3 + k] + Rq[6 + k] * GM[6 + k]) * s[k];
            float GR[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) GR[3 * r + k] = GM[3 * r + k] * s[k];
            float dq[4];
            dq[0] = 2.f * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
            dq[1] = 2.f * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.f * qx * GR[4] - qw * GR[5] + qz * GR[6] +
                           qw * GR[7] - 2.f * qx * GR[8]);
            dq[2] = 2.f * (-2.f * qy * GR[0] + qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] +
                           qz * GR[7] - 2.f * qy * GR[8]);
            dq[3] = 2.f * (-2.f * qz * GR[0] - qw * GR[1] + qx * GR[2] + qw * GR[3] - 2.f * qz * GR[4] +
                           qy * GR[5] + qx * GR[6] + qy * GR[7]);
            const float dot = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
            const float iqn = 1.0f / qn;
            gq[0] += (dq[0] - qw * dot) * iqn;
            gq[1] += (dq[1] - qx * dot) * iqn;
            gq[2] += (dq[2] - qy * dot) * iqn;
            gq[3] += (dq[3] - qz * dot) * iqn;
            // pose: rho gets g_p; phi gets p_c x g_p + 2 vee(Gc Sc - Sc Gc)
            //   Sc = R S3 R^T, Gc = J^T G2 J (J has zeros at (0,1), (1,0))
            float RS[9], Sc[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) RS[3 * r + k] = R[3 * r] * S3[k] + R[3 * r + 1] * S3[3 + k] + R[3 * r + 2] * S3[6 + k];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) Sc[3 * r + k] = RS[3 * r] * R[3 * k] + RS[3 * r + 1] * R[3 * k + 1] + RS[3 * r + 2] * R[3 * k + 2];
            const float J[6] = {J00, 0.0f, J02, 0.0f, J11, J12};
            float Gc[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    Gc[3 * r + k] = J[r] * (G00 * J[k] + G01 * J[3 + k]) + J[3 + r] * (G01 * J[k] + G11 * J[3 + k]);
            float K[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    K[3 * r + k] = (Gc[3 * r] * Sc[k] + Gc[3 * r + 1] * Sc[3 + k] + Gc[3 * r + 2] * Sc[6 + k]) -
                                   (Sc[3 * r] * Gc[k] + Sc[3 * r + 1] * Gc[3 + k] + Sc[3 * r + 2] * Gc[6 + k]);
            pose[0] = gpx + rho_sh[0];
            pose[1] = gpy + rho_sh[1];
            pose[2] = gpz + rho_sh[2];
            pose[3] = y * gpz - z * gpy + 2.0f * K[7];
            pose[4] = z * gpx - x * gpz + 2.0f * K[2];
            pose[5] = x * gpy - y * gpx + 2.0f * K[3];
        }
        // block partial of the pose gradient of view v (fixed order)
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float t = wave_sum(pose[q]);
            if ((threadIdx.x & 63) == 0) pred[threadIdx.x >> 6][q] = t;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
            float t = 0.0f;
#pragma unroll
            for (int ww = 0; ww < kBlk / 64; ++ww) t += pred[ww][threadIdx.x];
            w.pose_part[((size_t)blockIdx.x * rp.V + v) * 6 + threadIdx.x] = t;
        }
        __syncthreads();
    }
    if (live && gg.mean) {
        gg.mean[g] = gmean[0];
        gg.mean[M + g] = gmean[1];
        gg.mean[2 * M + g] = gmean[2];
        gg.log_scale[g] = gls[0];
        gg.log_scale[M + g] = gls[1];
        gg.log_scale[2 * M + g] = gls[2];
        gg.quat[g] = gq[0];
        gg.quat[M + g] = gq[1];
        gg.quat[2 * M + g] = gq[2];
        gg.quat[3 * M + g] = gq[3];
        gg.opacity_logit[g] = gop;
        gg.rgb[g] = grgb[0];
        gg.rgb[M + g] = grgb[1];
        gg.rgb[2 * M + g] = grgb[2];
        if constexpr (SHK > 0) {
#pragma unroll
            for (int k = 0; k < 3 * SHK; ++k) gg.sh[(size_t)k * M + g] = gsh[k];
        }
    }
    if (adam_here) {
        // this lane's Gaussian only: its parameters and moments were read above by this
        // lane alone
        const float* gr[5] = {gmean, gls, gq, &gop, grgb};
        int j = 0;
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int r = 0; r < kAdamRows[a]; ++r, ++j) {
                const size_t i = (size_t)r * M + g;
                adam_one(ap[j], gr[a][r], am[j], av[j], af.lr[a], af.b1, af.b2, af.eps, ibc1, ibc2);
                af.p[a][i] = ap[j];
                af.m[a][i] = am[j];
                af.v[a][i] = av[j];
            }
        if constexpr (SHK > 0) {
#pragma unroll
            for (int r = 0; r < 3 * SHK; ++r) {
                const size_t i = (size_t)r * M + g;
                float p = af.p[5][i], m = af.m[5][i], v = af.v[5][i];
                adam_one(p, gsh[r], m, v, af.lr[5], af.b1, af.b2, af.eps, ibc1, ibc2);
                af.p[5][i] = p;
                af.m[5][i] = m;
                af.v[5][i] = v;
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_pose_reduce(const ViewTable* __restrict__ vtp, RParams rp, WsPtrs w, int nblk,
                                                     float* dpose, int* step_ctr)
{
    // the Adam step counter of a backward with Adam in its epilogue (one lane,
    // vector memory path: the address depends on the lane id); not advanced after
    // a capacity overflow, where the epilogue skipped the update
    if (step_ctr && blockIdx.x == 0 && threadIdx.x == 0 && w.hdr->n_inst <= rp.cap) step_ctr[threadIdx.x] += 1;
    if (!dpose) return;  // launched for the counter alone
    // One block per view: the six components summed per lane over the blocks (in
    // strides), per wavefront (DPP), then over the four wavefronts in order.
    const int v = blockIdx.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ float red[4][6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        float t = 0.0f;
        for (int b = threadIdx.x; b < nblk; b += 256) t += w.pose_part[((size_t)b * rp.V + v) * 6 + q];
        t = wave_sum(t);
        if (lane == 0) red[wid][q] = t;
    }
    __syncthreads();
    const float* xi = vtp->v[v].pose_xi;
    if (!xi) {
        if (threadIdx.x < 6)
            dpose[v * 6 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                         red[3][threadIdx.x];
    } else if (threadIdx.x == 0) {
        // the view was rendered from Exp(xi) T: the gradient with respect to xi is
        // J_l(xi)^T times the gradient of the left perturbation at that pose
        double gz[6], xd[6], J[36];
        for (int q = 0; q < 6; ++q) {
            gz[q] = (double)(((red[0][q] + red[1][q]) + red[2][q]) + red[3][q]);
            xd[q] = (double)xi[q];
        }
        se3_left_jacobian_d(xd, J);
        for (int c = 0; c < 6; ++c) {
            double a = 0.0;
            for (int r = 0; r < 6; ++r) a += J[6 * r + c] * gz[r];
            dpose[v * 6 + c] = (float)a;
        }
    }
}

// ----------------------------------------------------------------- launch
gps_status launch_render_bwd(const gps_render_cfg* cfg, const RParams& rp, const gps_gaussians* g,
                             const ViewTable& vt, const WsLayout& L, char* ws, int explicit_upstream,
                             const float* loss_scale, gps_gaussians* grads, float* dpose, const gps_adam_fused* adam,
                             hipStream_t s)
{
    WsPtrs w = ws_ptrs(ws, L);
    const int shk = sh_count(g->sh_degree);
    GParams gp{g->mean, g->log_scale, g->quat, g->opacity_logit, g->rgb, shk ? g->sh : nullptr, shk};
    GGrads gg{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (grads)
        gg = GGrads{grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->rgb,
                    shk ? grads->sh : nullptr};
    AdamFuse af{};
    af.on = adam != nullptr;
    if (adam) {
        float* const pp[5] = {g->mean, g->log_scale, g->quat, g->opacity_logit, g->rgb};
        float* const mm[5] = {adam->m.mean, adam->m.log_scale, adam->m.quat, adam->m.opacity_logit, adam->m.rgb};
        float* const vv[5] = {adam->v.mean, adam->v.log_scale, adam->v.quat, adam->v.opacity_logit, adam->v.rgb};
        const float lr[5] = {adam->lr_mean, adam->lr_log_scale, adam->lr_quat, adam->lr_opacity, adam->lr_rgb};
        for (int k = 0; k < 5; ++k) {
            af.p[k] = pp[k];
            af.m[k] = mm[k];
            af.v[k] = vv[k];
            af.lr[k] = lr[k];
        }
        af.p[5] = shk ? g->sh : nullptr;
        af.m[5] = shk ? adam->m.sh : nullptr;
        af.v[5] = shk ? adam->v.sh : nullptr;
        af.lr[5] = adam->lr_sh;
        af.step_ctr = adam->step_counter;
        af.step = adam->step;
        af.b1 = adam->beta1;
        af.b2 = adam->beta2;
        af.eps = adam->eps;
    }
    const ViewTable* dvt = reinterpret_cast<const ViewTable*>(ws + L.vtab);
    if (!(cfg->flags & GPS_RENDER_VIEWS_PRESET)) {
        gps_status st = launch_views_upload(vt, rp, L, ws, 0, s);
        if (st != GPS_OK) return st;
    }
    if (cfg->flags & GPS_RENDER_BWD_PER_GAUSSIAN) {
        if (rp.mode == 0) return GPS_ERR_UNSUPPORTED_CONFIG;
        if (!dispatch_cbwd_pg(cfg, dvt, rp, w, L.n_tiles, explicit_upstream, loss_scale, s))
            return GPS_ERR_UNSUPPORTED_CONFIG;
    } else if (!dispatch_cbwd(cfg, dvt, rp, w, L.n_tiles, explicit_upstream, loss_scale, s)) {
        return GPS_ERR_UNSUPPORTED_CONFIG;
    }
    if (L.nblk_g > 0) {
        if (shk == 15)
            GPS_LAUNCH(K_GAUSS_BWD, s, k_gauss_bwd<15>, dim3(L.nblk_g), dim3(kBlk), 0, s, dvt, rp, gp, gg, w, af);
        else if (shk == 8)
            GPS_LAUNCH(K_GAUSS_BWD, s, k_gauss_bwd<8>, dim3(L.nblk_g), dim3(kBlk), 0, s, dvt, rp, gp, gg, w, af);
        else if (shk == 3)
            GPS_LAUNCH(K_GAUSS_BWD, s, k_gauss_bwd<3>, dim3(L.nblk_g), dim3(kBlk), 0, s, dvt, rp, gp, gg, w, af);
        else
            GPS_LAUNCH(K_GAUSS_BWD, s, k_gauss_bwd<0>, dim3(L.nblk_g), dim3(kBlk), 0, s, dvt, rp, gp, gg, w, af);
    }
    int* ctr = adam ? adam->step_counter : nullptr;
    // one block per view (an empty set sums no block partials: dpose = 0), or one
    // block for the step counter alone
    if (dpose || ctr)
        GPS_LAUNCH(K_POSE_REDUCE, s, k_pose_reduce, dim3(dpose ? vt.n : 1), dim3(256), 0, s, dvt, rp, w, L.nblk_g,
                   dpose, ctr);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
