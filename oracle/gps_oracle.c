/*
 * gps_oracle.c -- plain, slow reference implementation of the Gaussian-plus-SDF
 * mapping path of "Gaussian-plus-SDF SLAM: High-fidelity 3D Reconstruction at
 * 150+ fps" (Peng, Zhou, Shao; arXiv 2509.11574).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: it is used by the test-suite, by the smoke check and by the CPU
 * baseline leg of the benchmark, and by nothing else.  It shares no source,
 * header, table or helper with the HIP implementation.
 *
 * What it computes, with the passage of the paper each part follows:
 *   orc_fuse         TSDF + colour fusion of one RGB-D frame       (Sec. 3.2.1, "SDF fusion")
 *   orc_raycast      per-pixel ray march to the zero crossing,
 *                    trilinear colour C_t and projected depth D_t  (Sec. 3.1, first pass)
 *   orc_project      EWA splat of each Gaussian: 2D mean, 2D
 *                    covariance, conic, opacity, depth             (Sec. 3.1, Eq. 3; 3DGS convention)
 *   orc_render       second pass: Gaussians over the SDF base.
 *                    mode 0: depth-sorted front-to-back "over"
 *                            compositing (the "With sort" renderer
 *                            of Table 7)
 *                    mode 1: the paper's sort-free weighted blend  (Sec. 3.1, Eq. 1, 2, 4)
 *   orc_loss         L1 photometric loss (Eq. 7) plus an L1 depth term
 *   orc_render_bwd   analytic gradient of the render with respect to
 *                    every Gaussian parameter and the 6-DoF pose
 *   orc_adam         Adam update with the per-attribute learning
 *                    rates of Appendix C
 *   orc_alloc_blocks voxel blocks a frame allocates in the block
 *                    hash of the SDF (Sec. 3.2.1, "SDF fusion":
 *                    the SDF lives in a hash table of voxel blocks,
 *                    following InfiniTAM); orc_fuse with a block
 *                    mask is fusion into the allocated blocks only
 *
 * Precision.  Every value is computed in binary64.  Where floating point
 * decides an integer -- the nearest pixel a voxel projects to during fusion,
 * the ray-march sample at which the SDF changes sign, the depth key that orders
 * Gaussians and the depth-cull test -- the decision is taken in binary32 with the
 * evaluation order written out below ("binary32 decision arithmetic"), which is
 * the precision of the GPU kernels.  This file is compiled with
 * -ffp-contract=off so that every binary32 statement rounds once.
 * Decisions that go through exp() (the 1/255 opacity test, the opacity cap and
 * the transmittance stop) cannot be reproduced bit for bit across math
 * libraries; for those the renderer reports, per pixel, a flag when a value fell
 * within a small relative margin of its threshold, so that a comparison can set
 * such pixels aside and count them.
 *
 * Readings taken where the paper is silent are documented at each function.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Threads.  Pixels (raycast, render) and lattice points (fusion) are computed
 * independently of each other, so their loops run on OpenMP threads; every
 * output is the same whatever the thread count.  The backward computes each
 * pixel's contributors in parallel and then adds the pixels' adjoints into the
 * per-Gaussian sums serially, in pixel order, so its sums are the same as
 * well.  orc_set_threads(n) sets the thread count (n <= 0 keeps the current
 * one); it returns the count in effect.
 */
int32_t orc_set_threads(int32_t n)
{
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
}

/* ------------------------------------------------------------------------- */
/* Plain data passed in from Python (ctypes mirrors these exactly).           */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9]; /* world -> camera rotation, row-major */
    float t[3]; /* world -> camera translation         */
} orc_cam;

typedef struct {
    int32_t nx, ny, nz;
    float origin[3]; /* world position of lattice point (0,0,0) */
    float voxel;     /* lattice spacing (m)                      */
    float trunc;     /* truncation distance mu (m)               */
    float max_weight;
} orc_grid;

typedef struct {
    int32_t count;           /* M */
    const float* mean;       /* [3][M] */
    const float* log_scale;  /* [3][M] */
    const float* quat;       /* [4][M]  (w, x, y, z), not necessarily unit */
    const float* opacity_logit; /* [M] */
    const float* rgb;        /* [3][M]  degree-0 colour */
    int32_t sh_degree;       /* 0..3: view-dependent bands 1..sh_degree */
    const float* sh;         /* [3][K][M], K = (sh_degree+1)^2 - 1; NULL when sh_degree = 0 */
} orc_gauss;

typedef struct {
    int32_t mode;       /* 0: sorted over-compositing, 1: sort-free blend (Eq. 1-4) */
    float eps_cull;     /* epsilon of the depth test of Eq. 1-2                      */
    float lambda_depth; /* weight of the depth L1 term                               */
    float dilation;     /* low-pass term added to the diagonal of Sigma_2D (px^2)     */
    float alpha_min;    /* 1/255 (Eq. 3 text)                                         */
    float alpha_max;    /* opacity cap of sorted mode                                 */
    float T_min;        /* transmittance stop of sorted mode (0 disables)             */
    float z_near;       /* near-plane cull of Gaussian centres                        */
} orc_cfg;

/* Projected Gaussian (one view). */
typedef struct {
    int32_t valid;
    double pc[3];     /* centre in the camera frame                */
    double m[2];      /* projected centre (pixels)                 */
    double cov[3];    /* Sigma_2D: xx, xy, yy                      */
    double conic[3];  /* Sigma_2D^-1: a (xx), b (xy), c (yy)       */
    double sigma;     /* maximum opacity = sigmoid(logit)          */
    double depth;     /* d_i = camera z of the centre              */
    float depth32;    /* the same depth in binary32, the sort key  */
    double box[4];    /* support bounding box: xmin, xmax, ymin, ymax */
    double col[3];    /* colour seen from this camera (degree 0 plus the SH bands) */
    double dir[3];    /* unit direction from the camera centre to the centre       */
    double dist;      /* distance from the camera centre to the centre             */
    /* intermediates reused by the adjoint */
    double qn[4], qnorm, s[3], Rq[9], S3[9], J[6], W[6];
} orc_proj;

/* ------------------------------------------------------------------------- */
/* binary32 decision arithmetic                                               */
/*                                                                            */
/* One statement per IEEE operation; compiled without contraction.            */
/* ------------------------------------------------------------------------- */

/* Row r of R p + t, evaluated as (((R_r0 p0) + (R_r1 p1)) + (R_r2 p2)) + t_r. */
static float d32_row(const float* R, const float* t, int r, float p0, float p1, float p2)
{
    float a = R[3 * r + 0] * p0;
    float b = R[3 * r + 1] * p1;
    float s = a + b;
    float c = R[3 * r + 2] * p2;
    s = s + c;
    s = s + t[r];
    return s;
}

/* Lattice point position, origin + voxel * index, per axis. */
static float d32_lattice(float origin, float voxel, int idx)
{
    float f = (float)idx;
    float v = voxel * f;
    return origin + v;
}

static float d32_lerp(float a, float b, float f)
{
    float d = b - a;
    float e = f * d;
    return a + e;
}

/* ------------------------------------------------------------------------- */
/* Small binary64 helpers                                                     */
/* ------------------------------------------------------------------------- */

static void cam_apply64(const orc_cam* cam, const double p[3], double out[3])
{
    for (int r = 0; r < 3; ++r)
        out[r] = (double)cam->R[3 * r + 0] * p[0] + (double)cam->R[3 * r + 1] * p[1] +
                 (double)cam->R[3 * r + 2] * p[2] + (double)cam->t[r];
}

static double sigmoid64(double x) { return 1.0 / (1.0 + exp(-x)); }

static size_t grid_index(const orc_grid* g, int x, int y, int z)
{
    return (size_t)x + (size_t)g->nx * ((size_t)y + (size_t)g->ny * (size_t)z);
}

/* ========================================================================= */
/* O1 -- TSDF + colour fusion  (Sec. 3.2.1 "SDF fusion", following the        */
/* InfiniTAM / KinectFusion projective update).                               */
/*                                                                            */
/* For every lattice point p: project into the frame, take the depth d of the */
/* nearest pixel, eta = d - z (projective signed distance along the optical   */
/* axis).  Points with eta < -mu are occluded and left untouched.  Otherwise  */
/* the truncated value f = min(1, eta/mu) is averaged into the voxel with its */
/* weight, the weight saturating at max_weight.  The colour is averaged, with */
/* its own weight, only inside the band |eta| <= mu.                          */
/* Readings: the paper names the method but not its constants; the weight cap */
/* and the separate colour weight are readings.                               */
/* ========================================================================= */
/* The update of one lattice point (x, y, z) by one frame: tsdf, weight, the    */
/* three colour values and the colour weight are read and written through the  */
/* given pointers (the point's entries, wherever they are stored).             */
static void fuse_point(const orc_grid* g, const orc_cam* cam, const float* depth, const float* img, int x, int y,
                       int z, double* tsdf, double* weight, double* r, double* gr, double* b, double* rgb_weight)
{
    const int W = cam->width, H = cam->height;
    const float mu32 = g->trunc;
    const float negmu32 = -mu32;
    const double mu = (double)g->trunc;
    const double wmax = (double)g->max_weight;
    /* decision: which pixel, and whether the voxel is updated (binary32) */
    float p0 = d32_lattice(g->origin[0], g->voxel, x);
    float p1 = d32_lattice(g->origin[1], g->voxel, y);
    float p2 = d32_lattice(g->origin[2], g->voxel, z);
    float xc = d32_row(cam->R, cam->t, 0, p0, p1, p2);
    float yc = d32_row(cam->R, cam->t, 1, p0, p1, p2);
    float zc = d32_row(cam->R, cam->t, 2, p0, p1, p2);
    if (!(zc > 0.0f)) return;
    float u = cam->fx * xc;
    u = u / zc;
    u = u + cam->cx;
    float v = cam->fy * yc;
    v = v / zc;
    v = v + cam->cy;
    float fu = floorf(u + 0.5f);
    float fv = floorf(v + 0.5f);
    if (!(fu >= 0.0f && fu < (float)W && fv >= 0.0f && fv < (float)H)) return;
    int i = (int)fu, j = (int)fv;
    float d = depth[(size_t)j * W + i];
    if (!(d > 0.0f)) return;
    float eta32 = d - zc;
    if (eta32 < negmu32) return;
    int in_band = fabsf(eta32) <= mu32;

    /* values (binary64) */
    double p[3] = {(double)g->origin[0] + (double)g->voxel * x, (double)g->origin[1] + (double)g->voxel * y,
                   (double)g->origin[2] + (double)g->voxel * z};
    double pc[3];
    cam_apply64(cam, p, pc);
    double eta = (double)d - pc[2];
    double f = eta / mu;
    if (f > 1.0) f = 1.0;
    double w = *weight;
    *tsdf = (w * *tsdf + f) / (w + 1.0);
    *weight = (w + 1.0 < wmax) ? w + 1.0 : wmax;
    if (in_band) {
        double wc = *rgb_weight;
        double* col[3] = {r, gr, b};
        for (int c = 0; c < 3; ++c) {
            double obs = (double)img[(size_t)c * W * H + (size_t)j * W + i];
            *col[c] = (wc * *col[c] + obs) / (wc + 1.0);
        }
        *rgb_weight = (wc + 1.0 < wmax) ? wc + 1.0 : wmax;
    }
}

void orc_fuse(const orc_grid* g, double* tsdf, double* weight, double* rgb, double* rgb_weight,
              const orc_cam* cam, const float* depth, const float* img, const uint8_t* block_mask,
              int32_t block)
{
    const int nbx = block > 0 ? (g->nx + block - 1) / block : 0;
    const int nby = block > 0 ? (g->ny + block - 1) / block : 0;
    const size_t N = (size_t)g->nx * g->ny * g->nz;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                /* with a block mask, only lattice points of allocated blocks exist */
                if (block_mask &&
                    !block_mask[(size_t)(x / block) + (size_t)nbx * ((size_t)(y / block) + (size_t)nby * (z / block))])
                    continue;
                size_t idx = grid_index(g, x, y, z);
                fuse_point(g, cam, depth, img, x, y, z, tsdf + idx, weight + idx, rgb + idx, rgb + N + idx,
                           rgb + 2 * N + idx, rgb_weight + idx);
            }
}

/* The same update for a list of n lattice points only (lattice indices idx[k] =  */
/* x + nx (y + ny z)); their values are stored compactly: tsdf[k], weight[k],    */
/* rgb[c * n + k], rgb_weight[k].  For checking a long sequence of frames at     */
/* sampled points without the whole lattice.                                     */
void orc_fuse_points(const orc_grid* g, const int64_t* idx, int64_t n, double* tsdf, double* weight, double* rgb,
                     double* rgb_weight, const orc_cam* cam, const float* depth, const float* img)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t q = idx[k];
        const int x = (int)(q % g->nx), y = (int)((q / g->nx) % g->ny), z = (int)(q / ((int64_t)g->nx * g->ny));
        fuse_point(g, cam, depth, img, x, y, z, tsdf + k, weight + k, rgb + k, rgb + n + k, rgb + 2 * n + k,
                   rgb_weight + k);
    }
}

/* ========================================================================= */
/* O1b -- voxel-block allocation (Sec. 3.2.1 "SDF fusion": the SDF and colour */
/* live in a global hash table of voxel blocks, following InfiniTAM).         */
/*                                                                            */
/* The lattice is split into blocks of `block`^3 points (block b covers the   */
/* points [block*b, block*b + block) per axis).  A frame allocates, for every */
/* pixel (i, j) with depth d > 0, the blocks that contain the points of its   */
/* ray at camera depths z_k = d + k * voxel, k = -K .. K, K = ceil(mu/voxel)  */
/* (the truncation band around the measured surface, one sample per voxel     */
/* length), for z_k > 0 and inside the lattice's blocks.  Fusion then updates */
/* the allocated blocks only; every other lattice point keeps tsdf 1,         */
/* weight 0 and colour 0, which is what the raycast reads there.              */
/* Readings: the paper names the structure, not its constants -- the block    */
/* edge (8) and the sample spacing are the InfiniTAM conventions, the band is */
/* the truncation distance.  The block index of a sample is decided in       */
/* binary32 with the order written below.                                     */
/* mask: nbx*nby*nbz bytes (x fastest), set to 1 for every block allocated;   */
/* existing entries are kept (allocation accumulates over frames).            */
/* ========================================================================= */
void orc_alloc_blocks(const orc_grid* g, const orc_cam* cam, const float* depth, int32_t block, uint8_t* mask)
{
    const int W = cam->width, H = cam->height;
    const int nb[3] = {(g->nx + block - 1) / block, (g->ny + block - 1) / block, (g->nz + block - 1) / block};
    const int K = (int)ceil((double)g->trunc / (double)g->voxel);
    const float bsz = g->voxel * (float)block;
    const float* R = cam->R;
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            float d = depth[(size_t)j * W + i];
            if (!(d > 0.0f)) continue;
            float xn = (float)i - cam->cx;
            xn = xn / cam->fx;
            float yn = (float)j - cam->cy;
            yn = yn / cam->fy;
            for (int k = -K; k <= K; ++k) {
                float dz = (float)k * g->voxel;
                float z = d + dz;
                if (!(z > 0.0f)) continue;
                float xc = xn * z;
                float yc = yn * z;
                float q0 = xc - cam->t[0];
                float q1 = yc - cam->t[1];
                float q2 = z - cam->t[2];
                int b[3], ok = 1;
                for (int a = 0; a < 3; ++a) {
                    float s = R[0 * 3 + a] * q0;
                    float u = R[1 * 3 + a] * q1;
                    s = s + u;
                    float w = R[2 * 3 + a] * q2;
                    s = s + w;
                    float r = s - g->origin[a];
                    r = r / bsz;
                    float f = floorf(r);
                    if (!(f >= 0.0f && f < (float)nb[a])) {
                        ok = 0;
                        break;
                    }
                    b[a] = (int)f;
                }
                if (!ok) continue;
                size_t idx = (size_t)b[0] + (size_t)nb[0] * ((size_t)b[1] + (size_t)nb[1] * (size_t)b[2]);
#pragma omp atomic write
                mask[idx] = 1;
            }
        }
}

/* ========================================================================= */
/* O2 -- SDF raycast (Sec. 3.1 first pass; Sec. 3.2.1).                       */
/*                                                                            */
/* Each pixel's ray marches through the volume with a fixed step until the    */
/* interpolated signed distance changes sign from positive to non-positive;   */
/* the crossing is refined by the secant between the two bracketing samples.  */
/* The colour C_t is the trilinear interpolation of the eight voxel colours   */
/* around the surface point V, and D_t is the camera depth of V.  A ray with   */
/* no crossing gives D_t = 0 (invalid) and C_t = 0.                           */
/* Readings: step = voxel/2, near bound z_near, lattice values at integer      */
/* positions, samples whose 2x2x2 stencil leaves the lattice read as +1.       */
/* ========================================================================= */

/* binary32 trilinear of one scalar field at lattice coordinate g (binary32). */
static float d32_trilinear(const orc_grid* gr, const float* f, const float g[3], int* inside)
{
    float b[3], fr[3];
    int bi[3];
    for (int a = 0; a < 3; ++a) {
        b[a] = floorf(g[a]);
        fr[a] = g[a] - b[a];
    }
    const int n[3] = {gr->nx, gr->ny, gr->nz};
    for (int a = 0; a < 3; ++a) {
        if (!(b[a] >= 0.0f && b[a] <= (float)(n[a] - 2))) {
            *inside = 0;
            return 1.0f;
        }
        bi[a] = (int)b[a];
    }
    *inside = 1;
#define V32(dx, dy, dz) f[grid_index(gr, bi[0] + (dx), bi[1] + (dy), bi[2] + (dz))]
    float c00 = d32_lerp(V32(0, 0, 0), V32(1, 0, 0), fr[0]);
    float c10 = d32_lerp(V32(0, 1, 0), V32(1, 1, 0), fr[0]);
    float c01 = d32_lerp(V32(0, 0, 1), V32(1, 0, 1), fr[0]);
    float c11 = d32_lerp(V32(0, 1, 1), V32(1, 1, 1), fr[0]);
#undef V32
    float c0 = d32_lerp(c00, c10, fr[1]);
    float c1 = d32_lerp(c01, c11, fr[1]);
    return d32_lerp(c0, c1, fr[2]);
}

/* binary64 trilinear with the stencil clamped into the lattice (continuous). */
static double trilinear64(const orc_grid* gr, const float* f, const double p[3])
{
    const int n[3] = {gr->nx, gr->ny, gr->nz};
    int bi[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double gg = (p[a] - (double)gr->origin[a]) / (double)gr->voxel;
        double b = floor(gg);
        if (b < 0.0) b = 0.0;
        if (b > (double)(n[a] - 2)) b = (double)(n[a] - 2);
        double fa = gg - b;
        if (fa < 0.0) fa = 0.0;
        if (fa > 1.0) fa = 1.0;
        bi[a] = (int)b;
        fr[a] = fa;
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wgt = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) *
                             (dz ? fr[2] : 1.0 - fr[2]);
                acc += wgt * (double)f[grid_index(gr, bi[0] + dx, bi[1] + dy, bi[2] + dz)];
            }
    return acc;
}

/* Exposed for the library pin (torch grid_sample). */
double orc_trilinear(const orc_grid* gr, const float* f, double x, double y, double z)
{
    double p[3] = {x, y, z};
    return trilinear64(gr, f, p);
}

/*
 * Raycast a list of pixels (pix[k] = row * width + col; pix == NULL means every
 * pixel in row-major order, npix must then equal width*height).
 * out_depth[k], out_rgb[c*npix + k]; out_hit_k[k] = index of the sample that
 * closed the crossing, or -1 for a miss (optional).
 */
void orc_raycast(const orc_grid* g, const float* tsdf, const float* rgb, const orc_cam* cam,
                 float z_near, float step, int32_t npix, const int32_t* pix, double* out_depth,
                 double* out_rgb, int32_t* out_hit_k)
{
    const size_t N = (size_t)g->nx * g->ny * g->nz;
    const int n[3] = {g->nx, g->ny, g->nz};
    const float* R = cam->R;
    const float h = (step > 0.0f) ? step : g->voxel * 0.5f;
    const float inv_voxel = 1.0f / g->voxel;

    /* camera centre o = -R^T t (binary32) */
    float o32[3];
    for (int a = 0; a < 3; ++a) {
        float s = R[0 * 3 + a] * cam->t[0];
        float u = R[1 * 3 + a] * cam->t[1];
        s = s + u;
        float w = R[2 * 3 + a] * cam->t[2];
        s = s + w;
        o32[a] = -s;
    }
    double o64[3];
    for (int a = 0; a < 3; ++a)
        o64[a] = -((double)R[0 * 3 + a] * cam->t[0] + (double)R[1 * 3 + a] * cam->t[1] +
                   (double)R[2 * 3 + a] * cam->t[2]);

#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t k = 0; k < npix; ++k) {
        int32_t p = pix ? pix[k] : k;
        int col = p % cam->width, row = p / cam->width;
        out_depth[k] = 0.0;
        for (int c = 0; c < 3; ++c) out_rgb[(size_t)c * npix + k] = 0.0;
        if (out_hit_k) out_hit_k[k] = -1;

        /* ---- binary32 march: decides whether and where the ray hits ---- */
        float rx = ((float)col - cam->cx) / cam->fx;
        float ry = ((float)row - cam->cy) / cam->fy;
        float dir[3];
        for (int a = 0; a < 3; ++a) {
            float s = R[0 * 3 + a] * rx;
            float u = R[1 * 3 + a] * ry;
            s = s + u;
            s = s + R[2 * 3 + a];
            dir[a] = s;
        }
        float rn2 = rx * rx;
        float ry2 = ry * ry;
        rn2 = rn2 + ry2;
        rn2 = rn2 + 1.0f;
        float rn = sqrtf(rn2);
        float dh[3];
        for (int a = 0; a < 3; ++a) dh[a] = dir[a] / rn;
        float lam0 = z_near * rn, lam1 = INFINITY;
        int miss = 0;
        for (int a = 0; a < 3; ++a) {
            float lo = g->origin[a];
            float span = g->voxel * (float)(n[a] - 1);
            float hi = lo + span;
            if (dh[a] != 0.0f) {
                float t1 = (lo - o32[a]) / dh[a];
                float t2 = (hi - o32[a]) / dh[a];
                float tmn = t1 < t2 ? t1 : t2;
                float tmx = t1 < t2 ? t2 : t1;
                if (tmn > lam0) lam0 = tmn;
                if (tmx < lam1) lam1 = tmx;
            } else if (o32[a] < lo || o32[a] > hi) {
                miss = 1;
            }
        }
        if (miss || !(lam0 < lam1)) continue;
        float span_l = lam1 - lam0;
        float nsteps_f = floorf(span_l / h);
        int nsteps = (int)nsteps_f;
        float Fprev = 0.0f;
        int prev_inside = 0;
        int hit = -1;
        for (int s = 0; s <= nsteps; ++s) {
            float kf = (float)s;
            float lam = kf * h;
            lam = lam0 + lam;
            float gg[3];
            for (int a = 0; a < 3; ++a) {
                float q = lam * dh[a];
                q = o32[a] + q;
                q = q - g->origin[a];
                gg[a] = q * inv_voxel;
            }
            int inside;
            float F = d32_trilinear(g, tsdf, gg, &inside);
            if (s >= 1 && Fprev > 0.0f && F <= 0.0f) {
                hit = s;
                break;
            }
            Fprev = F;
            prev_inside = inside;
        }
        if (hit < 0) continue;

        /* ---- binary64 values at the decided crossing ---- */
        double rx64 = ((double)col - cam->cx) / cam->fx;
        double ry64 = ((double)row - cam->cy) / cam->fy;
        double dir64[3], rn64 = sqrt(rx64 * rx64 + ry64 * ry64 + 1.0);
        for (int a = 0; a < 3; ++a)
            dir64[a] = ((double)R[0 * 3 + a] * rx64 + (double)R[1 * 3 + a] * ry64 + (double)R[2 * 3 + a]) / rn64;
        double l0 = (double)z_near * rn64;
        for (int a = 0; a < 3; ++a) {
            double lo = (double)g->origin[a];
            double hi = lo + (double)g->voxel * (double)(n[a] - 1);
            if (dir64[a] != 0.0) {
                double t1 = (lo - o64[a]) / dir64[a];
                double t2 = (hi - o64[a]) / dir64[a];
                double tmn = t1 < t2 ? t1 : t2;
                if (tmn > l0) l0 = tmn;
            }
        }
        double la = l0 + (double)(hit - 1) * (double)h;
        double lb = l0 + (double)hit * (double)h;
        double pa[3], pb[3];
        for (int a = 0; a < 3; ++a) {
            pa[a] = o64[a] + la * dir64[a];
            pb[a] = o64[a] + lb * dir64[a];
        }
        double Fa = prev_inside ? trilinear64(g, tsdf, pa) : 1.0;
        double Fb = trilinear64(g, tsdf, pb);
        double lam_star = la + (double)h * Fa / (Fa - Fb);
        double V[3], Vc[3];
        for (int a = 0; a < 3; ++a) V[a] = o64[a] + lam_star * dir64[a];
        cam_apply64(cam, V, Vc);
        out_depth[k] = Vc[2];
        for (int c = 0; c < 3; ++c) out_rgb[(size_t)c * npix + k] = trilinear64(g, rgb + (size_t)c * N, V);
        if (out_hit_k) out_hit_k[k] = hit;
    }
}

/* ========================================================================= */
/* O3 -- EWA projection of one Gaussian (Sec. 3.1, Eq. 3; "following 3DGS"). */
/*                                                                            */
/* q^ = q/|q|, R_q its rotation, s = exp(log_scale), sigma = sigmoid(logit),  */
/* Sigma_3D = R_q diag(s^2) R_q^T, p_c = R mu + t,                            */
/* J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]],                          */
/* Sigma_2D = (J R) Sigma_3D (J R)^T + dilation I, conic = Sigma_2D^-1,        */
/* centre m = (fx x/z + cx, fy y/z + cy), depth d = z.                         */
/* Culled when z < z_near (binary32 decision), when det Sigma_2D <= 0, or      */
/* when 255 sigma <= 1 (then no pixel can reach alpha >= 1/255).              */
/* The support is the ellipse where sigma exp(-q/2) >= 1/255, i.e.             */
/* q <= kappa = 2 ln(255 sigma); box = m +- sqrt(kappa Sigma_xx, kappa Sigma_yy).*/
/* ========================================================================= */
static void quat_to_rot(const double q[4], double Rm[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    Rm[0] = 1.0 - 2.0 * (y * y + z * z);
    Rm[1] = 2.0 * (x * y - w * z);
    Rm[2] = 2.0 * (x * z + w * y);
    Rm[3] = 2.0 * (x * y + w * z);
    Rm[4] = 1.0 - 2.0 * (x * x + z * z);
    Rm[5] = 2.0 * (y * z - w * x);
    Rm[6] = 2.0 * (x * z - w * y);
    Rm[7] = 2.0 * (y * z + w * x);
    Rm[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* ------------------------------------------------------------------------- */
/* View-dependent colour (Sec. 3.1: SH coefficients per Gaussian, following   */
/* 3DGS).  c(d) = rgb + sum_{l=1..L} sum_m sh_{l,m} Y_{l,m}(d) for the unit   */
/* direction d from the camera centre to the Gaussian, with the real          */
/* spherical harmonics in the basis and order 3DGS uses (the degree-0 term is */
/* stored directly as the colour, so its constant and offset are absorbed;    */
/* the colour is not clamped).  Y[k] for k = 0 .. K-1 (bands 1..L in order)   */
/* and, when dY is given, dY[3k + a] = dY_k / dd_a with d's components taken  */
/* as independent (the normalisation is applied by the caller).               */
/* ------------------------------------------------------------------------- */
static void sh_basis(int L, const double d[3], double* Y, double* dY)
{
    const double x = d[0], y = d[1], z = d[2];
    const double c1 = 0.4886025119029199;
    const double c2[5] = {1.0925484305920792, -1.0925484305920792, 0.31539156525252005, -1.0925484305920792,
                          0.5462742152960396};
    const double c3[7] = {-0.5900435899266435, 2.890611442640554, -0.4570457994644658, 0.3731763325901154,
                          -0.4570457994644658, 1.445305721320277, -0.5900435899266435};
    double v[15], g[45];
    memset(g, 0, sizeof(g));
    /* band 1 */
    v[0] = -c1 * y;  g[0 * 3 + 1] = -c1;
    v[1] = c1 * z;   g[1 * 3 + 2] = c1;
    v[2] = -c1 * x;  g[2 * 3 + 0] = -c1;
    /* band 2 */
    v[3] = c2[0] * x * y;                    g[3 * 3 + 0] = c2[0] * y; g[3 * 3 + 1] = c2[0] * x;
    v[4] = c2[1] * y * z;                    g[4 * 3 + 1] = c2[1] * z; g[4 * 3 + 2] = c2[1] * y;
    v[5] = c2[2] * (2 * z * z - x * x - y * y);
    g[5 * 3 + 0] = -2 * c2[2] * x; g[5 * 3 + 1] = -2 * c2[2] * y; g[5 * 3 + 2] = 4 * c2[2] * z;
    v[6] = c2[3] * x * z;                    g[6 * 3 + 0] = c2[3] * z; g[6 * 3 + 2] = c2[3] * x;
    v[7] = c2[4] * (x * x - y * y);          g[7 * 3 + 0] = 2 * c2[4] * x; g[7 * 3 + 1] = -2 * c2[4] * y;
    /* band 3 */
    v[8] = c3[0] * y * (3 * x * x - y * y);
    g[8 * 3 + 0] = 6 * c3[0] * x * y; g[8 * 3 + 1] = c3[0] * (3 * x * x - 3 * y * y);
    v[9] = c3[1] * x * y * z;
    g[9 * 3 + 0] = c3[1] * y * z; g[9 * 3 + 1] = c3[1] * x * z; g[9 * 3 + 2] = c3[1] * x * y;
    v[10] = c3[2] * y * (4 * z * z - x * x - y * y);
    g[10 * 3 + 0] = -2 * c3[2] * x * y; g[10 * 3 + 1] = c3[2] * (4 * z * z - x * x - 3 * y * y);
    g[10 * 3 + 2] = 8 * c3[2] * y * z;
    v[11] = c3[3] * z * (2 * z * z - 3 * x * x - 3 * y * y);
    g[11 * 3 + 0] = -6 * c3[3] * x * z; g[11 * 3 + 1] = -6 * c3[3] * y * z;
    g[11 * 3 + 2] = c3[3] * (6 * z * z - 3 * x * x - 3 * y * y);
    v[12] = c3[4] * x * (4 * z * z - x * x - y * y);
    g[12 * 3 + 0] = c3[4] * (4 * z * z - 3 * x * x - y * y); g[12 * 3 + 1] = -2 * c3[4] * x * y;
    g[12 * 3 + 2] = 8 * c3[4] * x * z;
    v[13] = c3[5] * z * (x * x - y * y);
    g[13 * 3 + 0] = 2 * c3[5] * x * z; g[13 * 3 + 1] = -2 * c3[5] * y * z; g[13 * 3 + 2] = c3[5] * (x * x - y * y);
    v[14] = c3[6] * x * (x * x - 3 * y * y);
    g[14 * 3 + 0] = c3[6] * (3 * x * x - 3 * y * y); g[14 * 3 + 1] = -6 * c3[6] * x * y;
    const int K = (L + 1) * (L + 1) - 1;
    for (int k = 0; k < K; ++k) Y[k] = v[k];
    if (dY)
        for (int k = 0; k < 3 * K; ++k) dY[k] = g[k];
}

/* Exposed for the library pin (scipy's spherical harmonics). */
void orc_sh_basis(int32_t L, const double* d, double* Y, double* dY) { sh_basis(L, d, Y, dY); }

static void project_one(const orc_cfg* cfg, const orc_gauss* G, const orc_cam* cam, int i, orc_proj* P)
{
    const int M = G->count;
    memset(P, 0, sizeof(*P));
    /* binary32 decision: depth key and near cull */
    float mu0 = G->mean[i], mu1 = G->mean[M + i], mu2 = G->mean[2 * M + i];
    float z32 = d32_row(cam->R, cam->t, 2, mu0, mu1, mu2);
    P->depth32 = z32;
    if (!(z32 >= cfg->z_near)) return;

    double mu[3] = {mu0, mu1, mu2};
    cam_apply64(cam, mu, P->pc);
    double x = P->pc[0], y = P->pc[1], z = P->pc[2];
    /* colour from this camera: d = (mu - o) / |mu - o|, camera centre o = -R^T t */
    {
        double v[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double o = -((double)cam->R[0 * 3 + a] * cam->t[0] + (double)cam->R[1 * 3 + a] * cam->t[1] +
                               (double)cam->R[2 * 3 + a] * cam->t[2]);
            v[a] = mu[a] - o;
            r2 += v[a] * v[a];
        }
        P->dist = sqrt(r2);
        for (int a = 0; a < 3; ++a) P->dir[a] = v[a] / P->dist;
        for (int c = 0; c < 3; ++c) P->col[c] = (double)G->rgb[c * M + i];
        if (G->sh_degree > 0) {
            const int K = (G->sh_degree + 1) * (G->sh_degree + 1) - 1;
            double Y[15];
            sh_basis(G->sh_degree, P->dir, Y, NULL);
            for (int c = 0; c < 3; ++c)
                for (int k = 0; k < K; ++k) P->col[c] += (double)G->sh[((size_t)c * K + k) * M + i] * Y[k];
        }
    }
    double q[4] = {G->quat[i], G->quat[M + i], G->quat[2 * M + i], G->quat[3 * M + i]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    P->qnorm = qn;
    for (int a = 0; a < 4; ++a) P->qn[a] = q[a] / qn;
    quat_to_rot(P->qn, P->Rq);
    for (int a = 0; a < 3; ++a) P->s[a] = exp((double)G->log_scale[a * M + i]);
    /* Sigma_3D = Rq diag(s^2) Rq^T */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->Rq[3 * r + k] * P->s[k] * P->s[k] * P->Rq[3 * c + k];
            P->S3[3 * r + c] = acc;
        }
    double fx = cam->fx, fy = cam->fy;
    P->J[0] = fx / z;
    P->J[1] = 0.0;
    P->J[2] = -fx * x / (z * z);
    P->J[3] = 0.0;
    P->J[4] = fy / z;
    P->J[5] = -fy * y / (z * z);
    /* W = J R (2x3) */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->J[3 * r + k] * (double)cam->R[3 * k + c];
            P->W[3 * r + c] = acc;
        }
    /* Sigma_2D = W S3 W^T + dilation I */
    double T[6]; /* W S3 */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->W[3 * r + k] * P->S3[3 * k + c];
            T[3 * r + c] = acc;
        }
    double S2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += T[3 * r + k] * P->W[3 * c + k];
            S2[2 * r + c] = acc;
        }
    double A = S2[0] + (double)cfg->dilation, B = 0.5 * (S2[1] + S2[2]), C = S2[3] + (double)cfg->dilation;
    P->cov[0] = A;
    P->cov[1] = B;
    P->cov[2] = C;
    double det = A * C - B * B;
    if (!(det > 0.0)) return;
    P->conic[0] = C / det;
    P->conic[1] = -B / det;
    P->conic[2] = A / det;
    P->m[0] = fx * x / z + (double)cam->cx;
    P->m[1] = fy * y / z + (double)cam->cy;
    P->depth = z;
    P->sigma = sigmoid64((double)G->opacity_logit[i]);
    if (!(255.0 * P->sigma > 1.0)) return;
    double kappa = 2.0 * log(255.0 * P->sigma);
    double rx = sqrt(kappa * A), ry = sqrt(kappa * C);
    P->box[0] = P->m[0] - rx;
    P->box[1] = P->m[0] + rx;
    P->box[2] = P->m[1] - ry;
    P->box[3] = P->m[1] + ry;
    P->valid = 1;
}

/* Flat export of the projection for tests: per Gaussian i
   out[i*16 + ...] = valid, m(2), cov(3), conic(3), sigma, depth, depth32, box(4). */
void orc_project(const orc_cfg* cfg, const orc_gauss* G, const orc_cam* cam, double* out)
{
    for (int i = 0; i < G->count; ++i) {
        orc_proj P;
        project_one(cfg, G, cam, i, &P);
        double* o = out + (size_t)i * 16;
        o[0] = P.valid;
        o[1] = P.m[0];
        o[2] = P.m[1];
        o[3] = P.cov[0];
        o[4] = P.cov[1];
        o[5] = P.cov[2];
        o[6] = P.conic[0];
        o[7] = P.conic[1];
        o[8] = P.conic[2];
        o[9] = P.sigma;
        o[10] = P.depth;
        o[11] = (double)P.depth32;
        o[12] = P.box[0];
        o[13] = P.box[1];
        o[14] = P.box[2];
        o[15] = P.box[3];
    }
}

/* ========================================================================= */
/* O4/O5 -- per-pixel compositing over the SDF base (second pass, Sec. 3.1).  */
/* ========================================================================= */

typedef struct {
    int32_t g;       /* Gaussian index                 */
    float key;       /* binary32 depth, the sort key   */
    double alpha;    /* after the cap (sorted mode)    */
    double raw;      /* sigma exp(power), before cap   */
    int32_t capped;  /* raw > alpha_max                */
} orc_cand;

static int cand_cmp(const void* pa, const void* pb)
{
    const orc_cand* a = (const orc_cand*)pa;
    const orc_cand* b = (const orc_cand*)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->g > b->g) - (a->g < b->g);
}

#define ORC_FLAG_ALPHA_MIN 1
#define ORC_FLAG_ALPHA_MAX 2
#define ORC_FLAG_T_MIN 4
#define ORC_REL_MARGIN_ALPHA 2e-5
#define ORC_REL_MARGIN_T 1e-3

/*
 * Candidates of one pixel: every projected Gaussian that passes the depth test
 * d_i < D_t + eps of Eq. 1-2 (the test in binary32, D_t = +inf when the SDF
 * ray missed) and whose opacity at the pixel, sigma exp(-q/2) of Eq. 3, is at
 * least 1/255.  Every Gaussian is evaluated; nothing is skipped by its box.
 * Sorted by (binary32 depth, index) for the over-operator.
 */
static int gather_candidates(const orc_cfg* cfg, const orc_proj* P, int M, double px, double py,
                             float dcull32, orc_cand* out, int32_t* flag)
{
    int n = 0;
    float thr = dcull32 + cfg->eps_cull;
    const double amin = cfg->alpha_min, amax = cfg->alpha_max;
    for (int i = 0; i < M; ++i) {
        const orc_proj* p = &P[i];
        if (!p->valid) continue;
        if (!(p->depth32 < thr)) continue;
        double dx = px - p->m[0], dy = py - p->m[1];
        double power = -0.5 * (p->conic[0] * dx * dx + 2.0 * p->conic[1] * dx * dy + p->conic[2] * dy * dy);
        double raw = p->sigma * exp(power);
        if (fabs(raw - amin) <= ORC_REL_MARGIN_ALPHA * amin) *flag |= ORC_FLAG_ALPHA_MIN;
        if (raw < amin) continue;
        if (cfg->mode == 0 && fabs(raw - amax) <= ORC_REL_MARGIN_ALPHA * amax) *flag |= ORC_FLAG_ALPHA_MAX;
        out[n].g = i;
        out[n].key = p->depth32;
        out[n].raw = raw;
        out[n].capped = (cfg->mode == 0) && (raw > amax);
        out[n].alpha = out[n].capped ? amax : raw;
        ++n;
    }
    if (cfg->mode == 0) qsort(out, (size_t)n, sizeof(orc_cand), cand_cmp);
    return n;
}

/* Result of the forward pass at one pixel. */
typedef struct {
    double C[3], D, T;
    int32_t n_used;  /* contributors composited (sorted) / blended (sort-free) */
    double W;        /* sort-free: total Gaussian weight W_G                     */
    uint64_t order;  /* sorted: signature of the composited sequence (position  */
                     /* k, Gaussian g) -> sum (k+1)(g+1) * odd constant mod 2^64 */
} orc_pix;

/*
 * Sorted mode (the contract): front-to-back over the candidates.
 *   T_0 = 1; alpha_i capped at alpha_max; stop before the Gaussian that would
 *   take T below T_min; w_i = alpha_i T_i; C* = sum w_i c_i + T_final C_t,
 *   D* = sum w_i d_i + T_final D_t (D* = 0 where D_t is invalid).
 * Sort-free mode (Eq. 1, 2, 4): C_G = sum alpha_i c_i, W_G = sum alpha_i,
 *   C* = (C_t W_t + C_G) / (W_t + W_G) with W_t = 1; the depth is blended the
 *   same way.
 */
static void composite_pixel(const orc_cfg* cfg, const orc_proj* P, const orc_gauss* G,
                            const orc_cand* cand, int n, const double Ct[3], double Dt, int dvalid,
                            orc_pix* out, int32_t* flag)
{
    const int M = G->count;
    if (cfg->mode == 0) {
        double T = 1.0, AC[3] = {0, 0, 0}, AD = 0.0;
        uint64_t order = 0;
        int used = 0;
        for (int k = 0; k < n; ++k) {
            double a = cand[k].alpha;
            double Tn = T * (1.0 - a);
            if (cfg->T_min > 0.0f && fabs(Tn - cfg->T_min) <= ORC_REL_MARGIN_T * cfg->T_min)
                *flag |= ORC_FLAG_T_MIN;
            if (Tn < (double)cfg->T_min) break;
            double w = a * T;
            int g = cand[k].g;
            for (int c = 0; c < 3; ++c) AC[c] += w * P[g].col[c];
            AD += w * P[g].depth;
            T = Tn;
            order += (uint64_t)(used + 1) * (uint64_t)(g + 1) * 0x9E3779B97F4A7C15ull;
            ++used;
        }
        for (int c = 0; c < 3; ++c) out->C[c] = AC[c] + T * Ct[c];
        out->D = dvalid ? AD + T * Dt : 0.0;
        out->T = T;
        out->n_used = used;
        out->W = 0.0;
        out->order = order;
    } else {
        double Wg = 0.0, CG[3] = {0, 0, 0}, ZG = 0.0;
        for (int k = 0; k < n; ++k) {
            double a = cand[k].alpha;
            int g = cand[k].g;
            Wg += a;
            for (int c = 0; c < 3; ++c) CG[c] += a * P[g].col[c];
            ZG += a * P[g].depth;
        }
        for (int c = 0; c < 3; ++c) out->C[c] = (Ct[c] + CG[c]) / (1.0 + Wg);
        out->D = dvalid ? (Dt + ZG) / (1.0 + Wg) : 0.0;
        out->T = 1.0 / (1.0 + Wg);
        out->n_used = n;
        out->W = Wg;
        out->order = 0;
    }
}

static orc_proj* project_all(const orc_cfg* cfg, const orc_gauss* G, const orc_cam* cam)
{
    orc_proj* P = (orc_proj*)malloc(sizeof(orc_proj) * (size_t)(G->count > 0 ? G->count : 1));
    for (int i = 0; i < G->count; ++i) project_one(cfg, G, cam, i, &P[i]);
    return P;
}

/*
 * Render a list of pixels of one view.
 * base_rgb [3][H][W], base_depth [H][W] (0 = SDF ray missed).
 * out_rgb [3][npix], out_depth [npix], out_T [npix] (optional), out_flag [npix]
 * (optional), out_n [npix] (optional), out_W [npix] (optional, sort-free W_G).
 */
void orc_render(const orc_cfg* cfg, const orc_gauss* G, const orc_cam* cam, const float* base_rgb,
                const float* base_depth, int32_t npix, const int32_t* pix, double* out_rgb,
                double* out_depth, double* out_T, int32_t* out_flag, int32_t* out_n, double* out_W,
                uint64_t* out_order)
{
    const int W = cam->width, H = cam->height;
    const size_t HW = (size_t)W * H;
    orc_proj* P = project_all(cfg, G, cam);
#pragma omp parallel
    {
        orc_cand* cand = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(G->count > 0 ? G->count : 1));
#pragma omp for schedule(dynamic, 16)
        for (int32_t k = 0; k < npix; ++k) {
            int32_t p = pix ? pix[k] : k;
            int col = p % W, row = p / W;
            float dt32 = base_depth[p];
            int dvalid = dt32 > 0.0f;
            float dcull32 = dvalid ? dt32 : INFINITY;
            double Ct[3] = {base_rgb[p], base_rgb[HW + p], base_rgb[2 * HW + p]};
            int32_t flag = 0;
            int n = gather_candidates(cfg, P, G->count, (double)col, (double)row, dcull32, cand, &flag);
            orc_pix r;
            composite_pixel(cfg, P, G, cand, n, Ct, (double)dt32, dvalid, &r, &flag);
            for (int c = 0; c < 3; ++c) out_rgb[(size_t)c * npix + k] = r.C[c];
            out_depth[k] = r.D;
            if (out_T) out_T[k] = r.T;
            if (out_flag) out_flag[k] = flag;
            if (out_n) out_n[k] = r.n_used;
            if (out_W) out_W[k] = r.W;
            if (out_order) out_order[k] = r.order;
        }
        free(cand);
    }
    free(P);
}

/* ========================================================================= */
/* O6 -- loss: L1 colour (Eq. 7) + lambda_depth * L1 depth.                   */
/*   L = 1/(3HW) sum |C* - C_obs| + lambda/|Omega| sum_Omega |D* - D_obs|,     */
/*   Omega = { D_obs > 0 and D_t > 0 }; the depth term is 0 if Omega is empty. */
/* Writes dL/dC* and dL/dD* (times `scale`) when the pointers are non-NULL;   */
/* d|x|/dx is taken as 0 at x = 0.                                            */
/* ========================================================================= */
static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

double orc_loss(const orc_cfg* cfg, int32_t W, int32_t H, const double* rgb, const double* depth,
                const float* target_rgb, const float* target_depth, const float* base_depth,
                double scale, double* g_rgb, double* g_depth, int64_t* out_omega)
{
    const size_t HW = (size_t)W * H;
    double sc = 0.0, sd = 0.0;
    int64_t nom = 0;
    for (size_t p = 0; p < HW; ++p) {
        for (int c = 0; c < 3; ++c) sc += fabs(rgb[c * HW + p] - (double)target_rgb[c * HW + p]);
        if (target_depth[p] > 0.0f && base_depth[p] > 0.0f) {
            sd += fabs(depth[p] - (double)target_depth[p]);
            ++nom;
        }
    }
    double L = sc / (3.0 * (double)HW) + (nom > 0 ? (double)cfg->lambda_depth * sd / (double)nom : 0.0);
    if (g_rgb) {
        for (size_t p = 0; p < HW; ++p)
            for (int c = 0; c < 3; ++c)
                g_rgb[c * HW + p] = scale * sgn(rgb[c * HW + p] - (double)target_rgb[c * HW + p]) / (3.0 * (double)HW);
    }
    if (g_depth) {
        for (size_t p = 0; p < HW; ++p) {
            int in = target_depth[p] > 0.0f && base_depth[p] > 0.0f;
            g_depth[p] = (in && nom > 0)
                             ? scale * (double)cfg->lambda_depth * sgn(depth[p] - (double)target_depth[p]) / (double)nom
                             : 0.0;
        }
    }
    if (out_omega) *out_omega = nom;
    return L;
}

/* ========================================================================= */
/* O7 -- gradients.                                                           */
/* Per pixel, the derivative of the composite with respect to each            */
/* contributor's colour c_i, depth d_i and opacity alpha_i; then alpha through */
/* Eq. 3 to sigma, the 2D centre and the conic; then the EWA chain back to     */
/* the parameters.  Thresholds (cull, 1/255, cap, stop, order) are piecewise   */
/* constant and contribute nothing.                                            */
/* The pose enters as T_cw <- Exp(xi) T_cw with xi = (rho, phi) at 0, so       */
/* p_c moves by rho + phi x p_c and the camera-frame covariance by             */
/* [phi]x Sigma_c - Sigma_c [phi]x.  The SDF maps C_t, D_t are held constant   */
/* (they are cached per optimisation window, Sec. 3.2.2).                     */
/* ========================================================================= */

/* 10 per-Gaussian screen-space adjoints */
enum { A_MX = 0, A_MY, A_CA, A_CB, A_CC, A_SIG, A_R, A_G, A_B, A_D, A_N };

static void pixel_adjoint(const orc_cfg* cfg, const orc_proj* P, const orc_gauss* G, const orc_cand* cand,
                          int n, const orc_pix* fw, double px, double py, const double gC[3], double gD,
                          double* acc /*[M][A_N]*/)
{
    const int M = G->count;
    if (cfg->mode == 0) {
        double T = 1.0, PC[3] = {0, 0, 0}, PD = 0.0;
        for (int k = 0; k < fw->n_used; ++k) {
            const orc_cand* cd = &cand[k];
            int g = cd->g;
            const orc_proj* p = &P[g];
            double a = cd->alpha, w = a * T;
            double c[3] = {p->col[0], p->col[1], p->col[2]};
            double d = p->depth;
            for (int ch = 0; ch < 3; ++ch) PC[ch] += w * c[ch];
            PD += w * d;
            double* A = acc + (size_t)g * A_N;
            A[A_R] += w * gC[0];
            A[A_G] += w * gC[1];
            A[A_B] += w * gC[2];
            A[A_D] += w * gD;
            if (!cd->capped) {
                double dal = T * (gC[0] * c[0] + gC[1] * c[1] + gC[2] * c[2] + gD * d) -
                             (gC[0] * (fw->C[0] - PC[0]) + gC[1] * (fw->C[1] - PC[1]) +
                              gC[2] * (fw->C[2] - PC[2]) + gD * (fw->D - PD)) /
                                 (1.0 - a);
                double dx = px - p->m[0], dy = py - p->m[1];
                double dp = dal * a;       /* d alpha / d power = alpha */
                A[A_SIG] += dal * a / p->sigma; /* d alpha / d sigma = exp(power) */
                A[A_MX] += dp * (p->conic[0] * dx + p->conic[1] * dy);
                A[A_MY] += dp * (p->conic[1] * dx + p->conic[2] * dy);
                A[A_CA] += dp * (-0.5 * dx * dx);
                A[A_CB] += dp * (-dx * dy);
                A[A_CC] += dp * (-0.5 * dy * dy);
            }
            T *= (1.0 - a);
        }
    } else {
        double inv = 1.0 / (1.0 + fw->W);
        for (int k = 0; k < n; ++k) {
            const orc_cand* cd = &cand[k];
            int g = cd->g;
            const orc_proj* p = &P[g];
            double a = cd->alpha;
            double c[3] = {p->col[0], p->col[1], p->col[2]};
            double d = p->depth;
            double* A = acc + (size_t)g * A_N;
            A[A_R] += a * inv * gC[0];
            A[A_G] += a * inv * gC[1];
            A[A_B] += a * inv * gC[2];
            A[A_D] += a * inv * gD;
            double dal = inv * (gC[0] * (c[0] - fw->C[0]) + gC[1] * (c[1] - fw->C[1]) +
                                gC[2] * (c[2] - fw->C[2]) + gD * (d - fw->D));
            double dx = px - p->m[0], dy = py - p->m[1];
            double dp = dal * a;
            A[A_SIG] += dal * a / p->sigma;
            A[A_MX] += dp * (p->conic[0] * dx + p->conic[1] * dy);
            A[A_MY] += dp * (p->conic[1] * dx + p->conic[2] * dy);
            A[A_CA] += dp * (-0.5 * dx * dx);
            A[A_CB] += dp * (-dx * dy);
            A[A_CC] += dp * (-0.5 * dy * dy);
        }
    }
}

/* EWA chain rule for one Gaussian: screen-space adjoints -> parameters + pose. */
static void projection_adjoint(const orc_proj* p, const orc_cam* cam, const orc_gauss* G, const double* A, int M,
                               int i, double* g_mean, double* g_log_scale, double* g_quat, double* g_opacity,
                               double* g_rgb, double* g_sh, double* g_pose)
{
    const double x = p->pc[0], y = p->pc[1], z = p->pc[2];
    const double fx = cam->fx, fy = cam->fy;
    double R[9];
    for (int k = 0; k < 9; ++k) R[k] = cam->R[k];

    g_rgb[i] += A[A_R];
    g_rgb[M + i] += A[A_G];
    g_rgb[2 * M + i] += A[A_B];
    /* SH bands: the coefficients, then the view direction d = (mu - o) / |mu - o|.
       Its adjoint moves the centre by (I - d d^T) / |mu - o| times it; the camera
       centre moves by -R^T rho under the left perturbation (not with phi), so rho
       takes R times the same vector. */
    if (G->sh_degree > 0) {
        const int K = (G->sh_degree + 1) * (G->sh_degree + 1) - 1;
        double Y[15], dY[45], gd[3] = {0, 0, 0};
        sh_basis(G->sh_degree, p->dir, Y, dY);
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < K; ++k) {
                const double coef = (double)G->sh[((size_t)c * K + k) * M + i];
                if (g_sh) g_sh[((size_t)c * K + k) * M + i] += A[A_R + c] * Y[k];
                for (int a = 0; a < 3; ++a) gd[a] += A[A_R + c] * coef * dY[3 * k + a];
            }
        const double dd = p->dir[0] * gd[0] + p->dir[1] * gd[1] + p->dir[2] * gd[2];
        double u[3];
        for (int a = 0; a < 3; ++a) u[a] = (gd[a] - p->dir[a] * dd) / p->dist;
        for (int a = 0; a < 3; ++a) g_mean[a * M + i] += u[a];
        if (g_pose)
            for (int r = 0; r < 3; ++r) g_pose[r] += R[3 * r + 0] * u[0] + R[3 * r + 1] * u[1] + R[3 * r + 2] * u[2];
    }
    g_opacity[i] += A[A_SIG] * p->sigma * (1.0 - p->sigma);

    /* conic -> Sigma_2D:  G2 = -Q Gq Q, Gq the symmetric full-matrix adjoint */
    double Q[4] = {p->conic[0], p->conic[1], p->conic[1], p->conic[2]};
    double Gq[4] = {A[A_CA], 0.5 * A[A_CB], 0.5 * A[A_CB], A[A_CC]};
    double T1[4], G2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) T1[2 * r + c] = Q[2 * r + 0] * Gq[0 * 2 + c] + Q[2 * r + 1] * Gq[1 * 2 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) G2[2 * r + c] = -(T1[2 * r + 0] * Q[0 * 2 + c] + T1[2 * r + 1] * Q[1 * 2 + c]);

    /* Sigma_2D = W S3 W^T:  G3 = W^T G2 W,  G_W = 2 G2 W S3 */
    const double* Wm = p->W;
    double G3[9], GW[6], G2W[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) G2W[3 * r + c] = G2[2 * r + 0] * Wm[0 * 3 + c] + G2[2 * r + 1] * Wm[1 * 3 + c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G3[3 * r + c] = Wm[0 * 3 + r] * G2W[0 * 3 + c] + Wm[1 * 3 + r] * G2W[1 * 3 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += G2W[3 * r + k] * p->S3[3 * k + c];
            GW[3 * r + c] = 2.0 * acc;
        }
    /* W = J R:  G_J = G_W R^T */
    double GJ[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += GW[3 * r + k] * R[3 * c + k];
            GJ[3 * r + c] = acc;
        }
    /* camera-frame centre adjoint g_p */
    double gp[3] = {0, 0, 0};
    double z2 = z * z, z3 = z2 * z;
    gp[0] += GJ[2] * (-fx / z2);
    gp[1] += GJ[5] * (-fy / z2);
    gp[2] += GJ[0] * (-fx / z2) + GJ[2] * (2.0 * fx * x / z3) + GJ[4] * (-fy / z2) + GJ[5] * (2.0 * fy * y / z3);
    gp[0] += A[A_MX] * fx / z;
    gp[2] += -A[A_MX] * fx * x / z2;
    gp[1] += A[A_MY] * fy / z;
    gp[2] += -A[A_MY] * fy * y / z2;
    gp[2] += A[A_D];
    /* mean: p_c = R mu + t */
    for (int c = 0; c < 3; ++c) g_mean[c * M + i] += R[0 * 3 + c] * gp[0] + R[1 * 3 + c] * gp[1] + R[2 * 3 + c] * gp[2];

    /* Sigma_3D = Mm Mm^T with Mm = Rq diag(s) */
    double Mm[9], GM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Mm[3 * r + c] = p->Rq[3 * r + c] * p->s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += G3[3 * r + k] * Mm[3 * k + c];
            GM[3 * r + c] = 2.0 * acc;
        }
    for (int k = 0; k < 3; ++k) {
        double gs = 0.0;
        for (int r = 0; r < 3; ++r) gs += p->Rq[3 * r + k] * GM[3 * r + k];
        g_log_scale[k * M + i] += gs * p->s[k];
    }
    double GR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GR[3 * r + c] = GM[3 * r + c] * p->s[c];
    const double w = p->qn[0], qx = p->qn[1], qy = p->qn[2], qz = p->qn[3];
    double gq[4];
    gq[0] = 2.0 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
    gq[1] = 2.0 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.0 * qx * GR[4] - w * GR[5] + qz * GR[6] + w * GR[7] -
                   2.0 * qx * GR[8]);
    gq[2] = 2.0 * (-2.0 * qy * GR[0] + qx * GR[1] + w * GR[2] + qx * GR[3] + qz * GR[5] - w * GR[6] + qz * GR[7] -
                   2.0 * qy * GR[8]);
    gq[3] = 2.0 * (-2.0 * qz * GR[0] - w * GR[1] + qx * GR[2] + w * GR[3] - 2.0 * qz * GR[4] + qy * GR[5] +
                   qx * GR[6] + qy * GR[7]);
    double dot = p->qn[0] * gq[0] + p->qn[1] * gq[1] + p->qn[2] * gq[2] + p->qn[3] * gq[3];
    for (int k = 0; k < 4; ++k) g_quat[k * M + i] += (gq[k] - p->qn[k] * dot) / p->qnorm;

    /* pose: rho gets g_p; phi gets p_c x g_p + 2 vee(G_c S_c - S_c G_c) */
    if (g_pose) {
        double Sc[9], tmp[9], Gc[9], tmp2[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * r + k] * p->S3[3 * k + c];
                tmp[3 * r + c] = acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += tmp[3 * r + k] * R[3 * c + k];
                Sc[3 * r + c] = acc;
            }
        /* G_c = J^T G2 J */
        double G2J[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) G2J[3 * r + c] = G2[2 * r + 0] * p->J[0 * 3 + c] + G2[2 * r + 1] * p->J[1 * 3 + c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Gc[3 * r + c] = p->J[0 * 3 + r] * G2J[0 * 3 + c] + p->J[1 * 3 + r] * G2J[1 * 3 + c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Gc[3 * r + k] * Sc[3 * k + c] - Sc[3 * r + k] * Gc[3 * k + c];
                tmp2[3 * r + c] = acc;
            }
        g_pose[0] += gp[0];
        g_pose[1] += gp[1];
        g_pose[2] += gp[2];
        g_pose[3] += y * gp[2] - z * gp[1] + 2.0 * tmp2[7];
        g_pose[4] += z * gp[0] - x * gp[2] + 2.0 * tmp2[2];
        g_pose[5] += x * gp[1] - y * gp[0] + 2.0 * tmp2[3];
    }
}

/*
 * Backward of orc_render for one view, given dL/dC* (g_pix_rgb [3][npix]) and
 * dL/dD* (g_pix_depth [npix]) at the listed pixels.  Gradients are ADDED into
 * g_mean [3][M], g_log_scale [3][M], g_quat [4][M], g_opacity [M], g_rgb [3][M]
 * and g_pose [6] (rho, phi).  Optionally the 10 screen-space adjoints per
 * Gaussian are added into g_screen [M][10].
 */
void orc_render_bwd(const orc_cfg* cfg, const orc_gauss* G, const orc_cam* cam, const float* base_rgb,
                    const float* base_depth, int32_t npix, const int32_t* pix, const double* g_pix_rgb,
                    const double* g_pix_depth, double* g_mean, double* g_log_scale, double* g_quat,
                    double* g_opacity, double* g_rgb, double* g_sh, double* g_pose, double* g_screen)
{
    const int W = cam->width, H = cam->height;
    const size_t HW = (size_t)W * H;
    const int M = G->count;
    orc_proj* P = project_all(cfg, G, cam);
    double* acc = (double*)calloc((size_t)(M > 0 ? M : 1) * A_N, sizeof(double));
    /* the pixels' contributors and forward values (in parallel), kept per pixel */
    orc_cand** lists = (orc_cand**)calloc((size_t)(npix > 0 ? npix : 1), sizeof(orc_cand*));
    int* counts = (int*)malloc(sizeof(int) * (size_t)(npix > 0 ? npix : 1));
    orc_pix* fws = (orc_pix*)malloc(sizeof(orc_pix) * (size_t)(npix > 0 ? npix : 1));
#pragma omp parallel
    {
        orc_cand* cand = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(M > 0 ? M : 1));
#pragma omp for schedule(dynamic, 16)
        for (int32_t k = 0; k < npix; ++k) {
            int32_t p = pix ? pix[k] : k;
            int col = p % W, row = p / W;
            float dt32 = base_depth[p];
            int dvalid = dt32 > 0.0f;
            float dcull32 = dvalid ? dt32 : INFINITY;
            double Ct[3] = {base_rgb[p], base_rgb[HW + p], base_rgb[2 * HW + p]};
            double gD = dvalid ? g_pix_depth[k] : 0.0;
            counts[k] = -1;
            if (g_pix_rgb[k] == 0.0 && g_pix_rgb[(size_t)npix + k] == 0.0 && g_pix_rgb[2 * (size_t)npix + k] == 0.0 &&
                gD == 0.0)
                continue;
            int32_t flag = 0;
            int n = gather_candidates(cfg, P, M, (double)col, (double)row, dcull32, cand, &flag);
            composite_pixel(cfg, P, G, cand, n, Ct, (double)dt32, dvalid, &fws[k], &flag);
            lists[k] = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(n > 0 ? n : 1));
            memcpy(lists[k], cand, sizeof(orc_cand) * (size_t)n);
            counts[k] = n;
        }
        free(cand);
    }
    /* the adjoints, added in pixel order */
    for (int32_t k = 0; k < npix; ++k) {
        if (counts[k] < 0) continue;
        int32_t p = pix ? pix[k] : k;
        int col = p % W, row = p / W;
        int dvalid = base_depth[p] > 0.0f;
        double gC[3] = {g_pix_rgb[k], g_pix_rgb[(size_t)npix + k], g_pix_rgb[2 * (size_t)npix + k]};
        double gD = dvalid ? g_pix_depth[k] : 0.0;
        pixel_adjoint(cfg, P, G, lists[k], counts[k], &fws[k], (double)col, (double)row, gC, gD, acc);
        free(lists[k]);
    }
    free(lists);
    free(counts);
    free(fws);
    for (int i = 0; i < M; ++i) {
        if (!P[i].valid) continue;
        const double* A = acc + (size_t)i * A_N;
        if (g_screen)
            for (int a = 0; a < A_N; ++a) g_screen[(size_t)i * A_N + a] += A[a];
        projection_adjoint(&P[i], cam, G, A, M, i, g_mean, g_log_scale, g_quat, g_opacity, g_rgb, g_sh, g_pose);
    }
    free(acc);
    free(P);
}

/* ========================================================================= */
/* O8 -- Adam on one parameter array, step t >= 1:                            */
/*   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;                            */
/*   theta <- theta - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).           */
/* The learning rates per attribute come from Appendix C.                     */
/* ========================================================================= */
void orc_adam(int64_t n, double* param, const double* grad, double* m, double* v, double lr, double b1,
              double b2, double eps, int32_t t)
{
    double bc1 = 1.0 - pow(b1, (double)t);
    double bc2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * grad[k];
        v[k] = b2 * v[k] + (1.0 - b2) * grad[k] * grad[k];
        double mh = m[k] / bc1, vh = v[k] / bc2;
        param[k] -= lr * mh / (sqrt(vh) + eps);
    }
}
