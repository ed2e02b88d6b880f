// SE(3) helpers in binary64 for the device (camera pose updates).
// xi = (rho, phi): translation part first, then the rotation vector.
#pragma once
#include <hip/hip_runtime.h>

namespace gps {

// Exp of xi = (rho, phi) in SE(3) (Rodrigues' formula for the rotation, the left
// Jacobian of SO(3) for the translation).
__device__ inline void se3_exp_d(const double xi[6], double R[9], double t[3])
{
    const double wx = xi[3], wy = xi[4], wz = xi[5];
    const double th2 = wx * wx + wy * wy + wz * wz, th = sqrt(th2);
    const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    double A, B, C;
    if (th < 1e-6) {  // series of sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double V[9];
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = I + A * K[k] + B * K2[k];
        V[k] = I + B * K[k] + C * K2[k];
    }
    for (int r = 0; r < 3; ++r) t[r] = V[3 * r] * xi[0] + V[3 * r + 1] * xi[1] + V[3 * r + 2] * xi[2];
}

// Left Jacobian of SE(3) at xi: J = sum_n ad(xi)^n / (n + 1)!, ad(xi) =
// [[phi^, rho^], [0, phi^]] (hat = cross-product matrix), so that
// Exp(xi + e) = Exp(J e) Exp(xi) to first order in e.  The series is summed to
// 40 terms, which is below binary64 rounding for |phi| up to 2 pi.
__device__ inline void se3_left_jacobian_d(const double xi[6], double J[36])
{
    double ad[36], P[36], Q[36];
    for (int k = 0; k < 36; ++k) ad[k] = 0.0;
    const double hp[9] = {0.0, -xi[5], xi[4], xi[5], 0.0, -xi[3], -xi[4], xi[3], 0.0};
    const double hr[9] = {0.0, -xi[2], xi[1], xi[2], 0.0, -xi[0], -xi[1], xi[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ad[6 * r + c] = hp[3 * r + c];
            ad[6 * r + 3 + c] = hr[3 * r + c];
            ad[6 * (r + 3) + 3 + c] = hp[3 * r + c];
        }
    for (int k = 0; k < 36; ++k) {
        P[k] = (k % 7 == 0) ? 1.0 : 0.0;  // ad^0 / 1!
        J[k] = P[k];
    }
    for (int n = 1; n < 40; ++n) {
        // P <- P ad / (n + 1): ad^n / (n + 1)!
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) {
                double a = 0.0;
                for (int k = 0; k < 6; ++k) a += P[6 * r + k] * ad[6 * k + c];
                Q[6 * r + c] = a / (double)(n + 1);
            }
        for (int k = 0; k < 36; ++k) {
            P[k] = Q[k];
            J[k] += P[k];
        }
    }
}

}  // namespace gps
