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
#include "sdf_common.h"

namespace gps {

// ----------------------------------------------------------------- fusion
struct FuseArgs {
    FuseCtx ctx;
    int nx, ny;
    unsigned int N;
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
    fuse_point(a.ctx, (int)x, (int)y, (int)z, idx, a.N, a.tsdf, a.w, a.col, a.cw);
}

gps_status launch_fuse(const gps_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                       hipStream_t s)
{
    FuseArgs a;
    a.nx = vol->nx;
    a.ny = vol->ny;
    a.ctx.ox = vol->origin[0];
    a.ctx.oy = vol->origin[1];
    a.ctx.oz = vol->origin[2];
    a.ctx.voxel = vol->voxel;
    a.ctx.mu = vol->trunc;
    a.ctx.wmax = vol->max_weight;
    a.N = (unsigned int)((size_t)vol->nx * vol->ny * vol->nz);
    a.ctx.cam = dev_cam(*cam);
    a.ctx.depth = depth;
    a.ctx.img = rgb;
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

// Brick minima over the 9^3 lattice points of each brick (the brick and the first
// plane of its +x, +y, +z neighbours: every 2x2x2 sample stencil based in the brick).
// One block per row of bricks along x: each lane takes lattice columns x (lanes along
// x, so every load of the block reads whole rows of the lattice) and the minimum over
// the 9 x 9 (y, z) points of its column, kept in LDS; then each brick takes the
// minimum over its 9 columns.  Rows of up to kRowCols columns; longer ones use the
// per-brick kernel below.
constexpr int kRowCols = 4096;

__global__ void __launch_bounds__(256) k_brick_min_rows(BrickArgs a)
{
    __shared__ float scol[kRowCols];
    const int byi = (int)blockIdx.x % a.by, bzi = (int)blockIdx.x / a.by;
    const int y0 = byi * kBrick, z0 = bzi * kBrick;
    const int ny = min(kBrick + 1, a.ny - y0), nz = min(kBrick + 1, a.nz - z0);
    for (int x = threadIdx.x; x < a.nx; x += 256) {
        // the 81 loads of a column are issued before the first is used (a point past
        // the lattice edge reads the column's first point again)
        float v[kBrick + 1][kBrick + 1];
#pragma unroll
        for (int dz = 0; dz < kBrick + 1; ++dz)
#pragma unroll
            for (int dy = 0; dy < kBrick + 1; ++dy) {
                const int yy = y0 + (dy < ny ? dy : 0), zz = z0 + (dz < nz ? dz : 0);
                v[dz][dy] = a.tsdf[x + (size_t)a.nx * ((size_t)yy + (size_t)a.ny * (size_t)zz)];
            }
        float m = INFINITY;
#pragma unroll
        for (int dz = 0; dz < kBrick + 1; ++dz)
#pragma unroll
            for (int dy = 0; dy < kBrick + 1; ++dy) m = fminf(m, v[dz][dy]);
        scol[x] = m;
    }
    __syncthreads();
    for (int bxi = threadIdx.x; bxi < a.bx; bxi += 256) {
        const int x0 = bxi * kBrick, x1 = min(x0 + kBrick, a.nx - 1);
        float m = INFINITY;
        for (int x = x0; x <= x1; ++x) m = fminf(m, scol[x]);
        a.bmin[bxi + (size_t)a.bx * (byi + (size_t)a.by * bzi)] = m;
    }
}

// The same minima, one wavefront per 8^3 brick, four bricks per block (rows longer
// than kRowCols).
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
// The dense lattice as a Field of the march: planar arrays indexed
// x + nx (y + ny z); samples based in an 8^3 brick (or a 32^3 superbrick) whose
// minimum is positive are skipped.
struct DenseField {
    int n[3];
    size_t N;
    const float* tsdf;
    const float* rgb;
    const float* bmin;  // may be null
    const float* smin;  // superbrick minima (null with bmin)
    int bx, by, sx, sy;
    // The last brick found not positive (and its superbrick not positive), or -1:
    // successive samples of a ray mostly stay in one brick, whose answer does not
    // change during a raycast, so its minima are not read again.
    mutable int cbrick = -1;

    __device__ __forceinline__ void fetch8(int plane, const int b[3], float q[8]) const
    {
        const float* f = plane == 0 ? tsdf : rgb + (size_t)(plane - 1) * N;
        const size_t sy_ = (size_t)n[0], sz_ = (size_t)n[0] * n[1];
        const float* p = f + b[0] + sy_ * b[1] + sz_ * b[2];
        q[0] = p[0];
        q[1] = p[1];
        q[2] = p[sy_];
        q[3] = p[sy_ + 1];
        q[4] = p[sz_];
        q[5] = p[sz_ + 1];
        q[6] = p[sz_ + sy_];
        q[7] = p[sz_ + sy_ + 1];
    }

    __device__ __forceinline__ bool depth_range(int, int, int, float*, float*) const { return false; }

    __device__ __forceinline__ bool skip_box(const int b[3], float lo[3], float hi[3]) const
    {
        if (!bmin) return false;
        const int i0 = b[0] >> 3, i1 = b[1] >> 3, i2 = b[2] >> 3;
        const int bi = i0 + bx * (i1 + by * i2);
        if (bi == cbrick) return false;
        const int j0 = i0 / kSuper, j1 = i1 / kSuper, j2 = i2 / kSuper;
        // both minima are read before either is tested (one round trip)
        const float ms = smin[j0 + sx * (j1 + sy * j2)], mb = bmin[bi];
        int edge, bb[3];
        if (ms > kBrickPositive) {
            edge = kBrick * kSuper;  // the whole superbrick is positive
            bb[0] = j0;
            bb[1] = j1;
            bb[2] = j2;
        } else if (mb > kBrickPositive) {
            edge = kBrick;
            bb[0] = i0;
            bb[1] = i1;
            bb[2] = i2;
        } else {
            cbrick = bi;
            return false;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = (float)(bb[k] * edge);
            hi[k] = (float)((bb[k] + 1) * edge);
        }
        return true;
    }
};

__global__ void __launch_bounds__(256) k_raycast(MarchArgs a, DenseField fld)
{
    const int view = blockIdx.z;
    const DevCam& c = a.cams[view];
    const int col = blockIdx.x * 16 + (threadIdx.x & 15);
    const int row = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (col >= c.W || row >= c.H) return;
    const DenseField f = fld;  // this lane's copy (it keeps the last brick found not positive)
    march_pixel(a, f, view, col, row);
}

gps_status launch_raycast(const gps_volume* vol, const gps_camera* cams, int n_views, float* const* out_depth,
                          float* const* out_rgb, float z_near, float step, hipStream_t s)
{
    MarchArgs a;
    int maxW, maxH;
    march_setup(&a, vol->nx, vol->ny, vol->nz, vol->origin, vol->voxel, z_near, step, cams, n_views, out_depth,
                out_rgb, &maxW, &maxH);
    DenseField f;
    f.n[0] = vol->nx;
    f.n[1] = vol->ny;
    f.n[2] = vol->nz;
    f.N = (size_t)vol->nx * vol->ny * vol->nz;
    f.tsdf = vol->tsdf;
    f.rgb = vol->rgb;
    f.bx = (vol->nx + kBrick - 1) / kBrick;
    f.by = (vol->ny + kBrick - 1) / kBrick;
    const int bz = (vol->nz + kBrick - 1) / kBrick;
    f.sx = (f.bx + kSuper - 1) / kSuper;
    f.sy = (f.by + kSuper - 1) / kSuper;
    const int sz = (bz + kSuper - 1) / kSuper;
    f.bmin = vol->brick_min;
    f.smin = vol->brick_min ? vol->brick_min + (size_t)f.bx * f.by * bz : nullptr;
    if (vol->brick_min) {
        BrickArgs b{vol->nx, vol->ny, vol->nz, f.bx, f.by, bz, vol->tsdf, vol->brick_min};
        if (vol->nx <= kRowCols)
            GPS_LAUNCH(K_BRICK_MIN, s, k_brick_min_rows, dim3(f.by * bz), dim3(256), 0, s, b);
        else
            GPS_LAUNCH(K_BRICK_MIN, s, k_brick_min, dim3((f.bx * f.by * bz + 3) / 4), dim3(256), 0, s, b);
        const int ns = f.sx * f.sy * sz;
        GPS_LAUNCH(K_BRICK_MIN, s, k_super_min, dim3((ns + 3) / 4), dim3(256), 0, s, vol->brick_min,
                   vol->brick_min + (size_t)f.bx * f.by * bz, f.bx, f.by, bz, f.sx, f.sy, sz);
        if (hipGetLastError() != hipSuccess) return GPS_ERR_HIP;
    }
    dim3 grid((maxW + 15) / 16, (maxH + 15) / 16, n_views);
    GPS_LAUNCH(K_RAYCAST, s, k_raycast, grid, dim3(256), 0, s, a, f);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
