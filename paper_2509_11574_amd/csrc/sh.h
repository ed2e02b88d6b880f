// View-dependent colour (Sec. 3.1: SH coefficients per Gaussian, following 3DGS):
// the real spherical harmonics of bands 1..3 at a unit direction d, in the 3DGS
// basis and order (m = -l..l within a band, Condon-Shortley phase, sine terms for
// m < 0), and their partial derivatives with respect to d's components taken as
// independent.  K = 3, 8 or 15 basis functions for degree 1, 2, 3.
#pragma once

#include <hip/hip_runtime.h>

namespace gps {

constexpr int kShMaxK = 15;

__host__ __device__ constexpr int sh_count(int degree) { return (degree + 1) * (degree + 1) - 1; }

template <int K>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float Y[K])
{
    constexpr float c1 = 0.48860251190291992f;
    Y[0] = -c1 * y;
    Y[1] = c1 * z;
    Y[2] = -c1 * x;
    if constexpr (K > 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[3] = 1.0925484305920792f * x * y;
        Y[4] = -1.0925484305920792f * y * z;
        Y[5] = 0.31539156525252005f * (2.0f * zz - xx - yy);
        Y[6] = -1.0925484305920792f * x * z;
        Y[7] = 0.54627421529603959f * (xx - yy);
        if constexpr (K > 8) {
            Y[8] = -0.59004358992664352f * y * (3.0f * xx - yy);
            Y[9] = 2.8906114426405538f * x * y * z;
            Y[10] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
            Y[11] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[12] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
            Y[13] = 1.4453057213202769f * z * (xx - yy);
            Y[14] = -0.59004358992664352f * x * (xx - 3.0f * yy);
        }
    }
}

// g = sum_k w[k] dY_k/dd (the gradient of sum_k w[k] Y_k(d) with d's components free).
template <int K>
__device__ __forceinline__ void sh_weighted_grad(float x, float y, float z, const float w[K], float g[3])
{
    constexpr float c1 = 0.48860251190291992f;
    g[0] = -c1 * w[2];
    g[1] = -c1 * w[0];
    g[2] = c1 * w[1];
    if constexpr (K > 3) {
        const float a = 1.0925484305920792f, b = 0.31539156525252005f, e = 0.54627421529603959f;
        g[0] += a * y * w[3] - 2.0f * b * x * w[5] - a * z * w[6] + 2.0f * e * x * w[7];
        g[1] += a * x * w[3] - a * z * w[4] - 2.0f * b * y * w[5] - 2.0f * e * y * w[7];
        g[2] += -a * y * w[4] + 4.0f * b * z * w[5] - a * x * w[6];
        if constexpr (K > 8) {
            const float xx = x * x, yy = y * y, zz = z * z;
            const float k0 = -0.59004358992664352f, k1 = 2.8906114426405538f, k2 = -0.45704579946446572f,
                        k3 = 0.37317633259011540f, k5 = 1.4453057213202769f;
            g[0] += 6.0f * k0 * x * y * w[8] + k1 * y * z * w[9] - 2.0f * k2 * x * y * w[10] -
                    6.0f * k3 * x * z * w[11] + k2 * (4.0f * zz - 3.0f * xx - yy) * w[12] + 2.0f * k5 * x * z * w[13] +
                    k0 * (3.0f * xx - 3.0f * yy) * w[14];
            g[1] += k0 * (3.0f * xx - 3.0f * yy) * w[8] + k1 * x * z * w[9] + k2 * (4.0f * zz - xx - 3.0f * yy) * w[10] -
                    6.0f * k3 * y * z * w[11] - 2.0f * k2 * x * y * w[12] - 2.0f * k5 * y * z * w[13] -
                    6.0f * k0 * x * y * w[14];
            g[2] += k1 * x * y * w[9] + 8.0f * k2 * y * z * w[10] + k3 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[11] +
                    8.0f * k2 * x * z * w[12] + k5 * (xx - yy) * w[13];
        }
    }
}

}  // namespace gps
