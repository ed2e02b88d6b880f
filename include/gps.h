/*
 * gps.h -- C ABI of the MI355X (gfx950) implementation of the per-frame mapping
 * path of Gaussian-plus-SDF SLAM (Peng, Zhou, Shao, arXiv 2509.11574):
 * colourised-TSDF fusion, SDF raycast, the differentiable 3D-Gaussian overlay
 * composited over the SDF base image, its photometric + depth loss, the
 * analytic backward pass (Gaussian parameters and 6-DoF camera pose) and Adam;
 * around it, Gaussian removal and insertion and point-to-plane ICP tracking.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers unless the comment says "host".  Arrays are
 *    float32 unless stated otherwise, planar (structure of arrays), C order.  Images are [H][W]
 *    (depth) and [3][H][W] (colour); lattices are indexed
 *    x + nx*(y + ny*z); Gaussian attributes are [k][M] (one plane per
 *    component).
 *  - Cameras map world to camera: p_c = R p_w + t, R row-major, OpenCV axes
 *    (x right, y down, z forward).  Pixel (col, row) is sampled at (col, row);
 *    projection is u = fx x/z + cx, v = fy y/z + cy.
 *  - The caller owns every buffer.  The library allocates no device memory and
 *    keeps no state between calls other than cached device attributes and the
 *    fixed scratch array of gps_icp_reduce_noalloc.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work and returns without synchronising, except gps_device_status
 *    and gps_read_stats, which synchronise the stream they are given.
 *  - Argument errors are returned synchronously and nothing is launched.
 *    Failures discovered on the device (too many tile instances for the
 *    workspace) set a sticky status word inside the workspace; read it with
 *    gps_device_status.  Launch failures return GPS_ERR_HIP.
 *  - A sequence of calls with unchanged arguments launches an identical
 *    sequence of kernels with identical arguments and never reads device data
 *    on the host, so it may be captured in a HIP graph and replayed.
 *  - Every entry point is deterministic: the same inputs give bitwise the same
 *    outputs (no floating-point atomics anywhere), except a render with
 *    GPS_RENDER_NO_SORT, whose summation order follows the binning's atomics.
 *  - Calls that share a workspace must not run concurrently.
 */
#ifndef GPS_H_
#define GPS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPS_ABI_VERSION 5

/* Size in floats of gps_volume.brick_min for an nx x ny x nz lattice. */
#define GPS_BRICKS_(n) (((n) + 7) / 8)
#define GPS_SUPERBRICKS_(n) ((GPS_BRICKS_(n) + 3) / 4)
#define GPS_BRICK_MIN_FLOATS(nx, ny, nz)                                                  \
    ((size_t)GPS_BRICKS_(nx) * GPS_BRICKS_(ny) * GPS_BRICKS_(nz) +                        \
     (size_t)GPS_SUPERBRICKS_(nx) * GPS_SUPERBRICKS_(ny) * GPS_SUPERBRICKS_(nz))
#define GPS_MAX_VIEWS 16 /* views per render call */

typedef int32_t gps_status;
#define GPS_OK 0
#define GPS_ERR_INVALID_ARG (-1)
#define GPS_ERR_WORKSPACE_TOO_SMALL (-2)
#define GPS_ERR_CAPACITY (-3)           /* device: more tile instances than the workspace holds */
#define GPS_ERR_HIP (-4)                /* a HIP runtime call or launch failed                 */
#define GPS_ERR_UNSUPPORTED_DEVICE (-5) /* the current device is not gfx950                    */
#define GPS_ERR_UNSUPPORTED_CONFIG (-6) /* tile / batch / pixels-per-thread not compiled in    */

typedef struct gps_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9]; /* world -> camera rotation, row-major */
    float t[3]; /* world -> camera translation         */
} gps_camera;

/* Colourised TSDF volume S: every lattice point stores a truncated signed
 * distance and an RGB colour (Sec. 3.1 "Gaussian-plus-SDF"), here as a dense
 * lattice.  Point (x,y,z) sits at origin + voxel*(x,y,z). */
typedef struct gps_volume {
    int32_t nx, ny, nz;
    float origin[3];
    float voxel;      /* lattice spacing (m)                                   */
    float trunc;      /* truncation distance mu (m)                            */
    float max_weight; /* fusion weights saturate here                          */
    float* tsdf;       /* [N] truncated SDF in units of mu, initialise to 1     */
    float* weight;     /* [N] fusion weight, initialise to 0                    */
    float* rgb;        /* [3][N] colour, initialise to 0                        */
    float* rgb_weight; /* [N] colour weight, initialise to 0                    */
    float* brick_min;  /* optional GPS_BRICK_MIN_FLOATS(nx, ny, nz) floats of
                          scratch for empty-space skipping in gps_raycast (minima
                          of 8^3-voxel bricks, then of 4^3-brick superbricks);
                          NULL disables */
} gps_volume;

/* The Gaussian set G = {p_i, sigma_i, r_i, s_i, SH_i} (Sec. 3.1; SH following
 * 3DGS).  The colour seen from a camera whose centre is o is
 *   c_i(d) = rgb_i + sum_{l=1..L} sum_{m=-l..l} sh_i[l,m] Y_lm(d),
 *   d = (p_i - o) / |p_i - o|,
 * with the real spherical harmonics of 3DGS (Condon-Shortley phase, sine terms
 * for m < 0); the degree-0 coefficient is stored directly as the linear colour
 * rgb_i (its constant and offset absorbed) and the colour is not clamped.  The
 * same struct carries gradients and Adam moments. */
typedef struct gps_gaussians {
    int32_t count;        /* M                                              */
    float* mean;          /* [3][M] centre p_i (world, m)                   */
    float* log_scale;     /* [3][M] log of the axis scales s_i              */
    float* quat;          /* [4][M] rotation r_i as (w, x, y, z), any norm  */
    float* opacity_logit; /* [M]    sigma_i = 1/(1+exp(-logit))             */
    float* rgb;           /* [3][M] degree-0 colour rgb_i                   */
    int32_t sh_degree;    /* L in 0..3 (0: view-independent colour)         */
    float* sh;            /* [3][K][M], K = (L+1)^2 - 1 coefficients per
                             channel (bands 1..L, m = -l..l); NULL when L = 0 */
} gps_gaussians;

/* One view of a render call. */
typedef struct gps_view {
    gps_camera cam;
    const float* base_rgb;     /* [3][H][W] SDF colour C_t  (from gps_raycast)     */
    const float* base_depth;   /* [H][W]    SDF depth D_t, 0 = ray missed          */
    const float* target_rgb;   /* [3][H][W] observed colour C_k, NULL = no loss    */
    const float* target_depth; /* [H][W]    observed depth D_k (0 = invalid)       */
    float* out_rgb;            /* [3][H][W] rendered C* (written by render_fwd)    */
    float* out_depth;          /* [H][W]    rendered D* (0 where D_t is invalid)   */
    const float* pose_xi;      /* [6] or NULL: xi = (rho, phi); the view is rendered
                                  from Exp(xi) T_cw instead of the camera's T_cw
                                  (read on the device when the view table is
                                  written: by render_fwd / render_bwd, or by
                                  gps_views_upload for GPS_RENDER_VIEWS_PRESET)  */
    float* out_aux;            /* [H][W] or NULL: written by render_fwd with the
                                  final transmittance T_final (mode 0) or the
                                  Gaussian weight W_G of Eq. 2 (mode 1)          */
} gps_view;

/* Renderer constants (each is a reading of the paper where it is silent). */
typedef struct gps_render_cfg {
    int32_t tile_w, tile_h;  /* screen tile: 8x8, 16x16, 16x32 or 32x16            */
    int32_t batch;           /* Gaussians staged in LDS per step: 128, 256 or 512  */
    int32_t pix_per_thread;  /* pixels per lane: 1, 2 or 4                         */
    int32_t mode;            /* 0 sorted over-compositing (the default); 1 the
                                sort-free blend of Eq. 1, 2, 4                     */
    float eps_cull;          /* epsilon of the depth test of Eq. 1-2 (m)           */
    float lambda_depth;      /* weight of the L1 depth term                        */
    float dilation;          /* px^2 added to the diagonal of Sigma_2D (0.3)       */
    float alpha_min;         /* 1/255 (Sec. 3.1, after Eq. 3)                      */
    float alpha_max;         /* opacity cap of sorted mode (0.99)                  */
    float T_min;             /* transmittance stop of sorted mode (1e-4, 0 = off)   */
    float z_near;            /* centres nearer than this are culled (0.2 m)        */
    int64_t max_instances;   /* capacity for (view, tile, Gaussian) slots;
                                0 = 32 per view-Gaussian, at least 2^20            */
    int32_t flags;           /* GPS_RENDER_VIEWS_PRESET, GPS_RENDER_BWD_PER_GAUSSIAN,
                                GPS_RENDER_NO_SORT (or-ed), or 0                   */
} gps_render_cfg;

/* The render kernels read the view table (cameras and image pointers) from the
 * workspace, with the per-tile maxima of the views' base depths that drive the
 * tile-level depth cull.  By default gps_render_fwd writes the table of its
 * `views` argument there and takes those maxima (gps_render_bwd writes the
 * table only).  With this flag both launch no such upload and use the table
 * and maxima written by the last gps_views_upload on the workspace; the
 * `views` argument must then describe views of the same sizes (it still sizes
 * the launches), and the base images must not have changed since that upload.
 * This lets one captured forward + backward + Adam iteration be replayed for
 * new camera poses or new base images: upload, then replay. */
#define GPS_RENDER_VIEWS_PRESET 1

/* Sort-free mode (mode 1) only: gps_render_bwd forms each view-Gaussian's
 * screen-space adjoints the way Sec. 3.1 and Appendix B organise the backward of
 * the sort-free blend: per Gaussian, summed in-thread over the pixels of its
 * support box (one block per screen tile holds the tile's per-pixel adjoint state
 * in LDS; its wavefronts take the tile's Gaussians one at a time, their lanes
 * sweeping the Gaussian's box 64 pixels at a time; one wave reduction per
 * Gaussian and tile), with no ordering and no atomics; instead of the tile
 * backward's per-pixel-group reductions.  Same results up to rounding;
 * GPS_ERR_UNSUPPORTED_CONFIG in mode 0 or for tiles other than 8x8, 16x16, 16x32
 * and 32x16. */
#define GPS_RENDER_BWD_PER_GAUSSIAN 2

/* Sort-free mode (mode 1) only: no per-tile depth sort at all (Sec. 3.1: the
 * blend of Eq. 1, 2, 4 is independent of order).  Each tile's list is taken in
 * the order the binning emitted it, every record of the list is visited (no list
 * is cut short by the depth order), and the long-list sort is not launched.  The
 * emission order comes from atomic counters, so the order of the floating-point
 * sums -- and the last bits of C*, D* and W_G -- may differ between calls (the
 * only exception to the determinism of the other entry points); the gradients
 * differ from call to call only through those bits.  GPS_ERR_UNSUPPORTED_CONFIG
 * in mode 0. */
#define GPS_RENDER_NO_SORT 4

/* One Adam parameter group. */
typedef struct gps_adam_group {
    float* param;
    const float* grad;
    float* m; /* first moment, initialise to 0  */
    float* v; /* second moment, initialise to 0 */
    int64_t n;
    float lr;
} gps_adam_group;

/* Counters of the last render call in a workspace (read with gps_read_stats). */
typedef struct gps_stats {
    int32_t status;            /* sticky status word                              */
    int32_t n_views;
    int64_t n_instances;       /* tile slots of the last forward: the screen tiles
                                  covered by the support boxes (before the depth
                                  cull); the capacity bounds this number          */
    int64_t capacity;          /* instances the workspace holds                   */
    int64_t sort_fallback;     /* tiles longer than the LDS sort holds            */
    int64_t n_tiles;
    int64_t pairs_eval;        /* (pixel, instance) opacity evaluations, summed over
                                  every forward since gps_workspace_reset          */
    int64_t pairs_contrib;     /* of those, pairs composited into the pixel        */
    float loss;                /* last forward's loss                             */
    float view_omega[GPS_MAX_VIEWS]; /* |Omega_v|: pixels in each view's depth term */
} gps_stats;

int32_t gps_abi_version(void);
const char* gps_status_string(gps_status s);

/* Fills `cfg` (host) with the defaults: 16x16 tiles, batch 256, 1 pixel per
 * lane, sorted mode, eps 0.01, lambda 1, dilation 0.3, alpha 1/255..0.99,
 * T_min 1e-4, z_near 0.2, automatic capacity. */
void gps_render_cfg_default(gps_render_cfg* cfg);

/* Bytes of workspace a render call with these arguments needs (host call,
 * nothing launched).  cams: host array of n_views cameras. */
gps_status gps_workspace_size(const gps_render_cfg* cfg, int32_t n_gaussians, const gps_camera* cams,
                              int32_t n_views, size_t* out_bytes);

/* Clears the workspace header (sticky status, counters, Adam step counter).
 * Call once after allocating a workspace, and after a capacity error before
 * replaying with a larger workspace. */
gps_status gps_workspace_reset(void* ws, size_t ws_bytes, void* stream);

/* TSDF + colour fusion of one RGB-D frame (Sec. 3.2.1, "SDF fusion", the
 * projective update of KinectFusion/InfiniTAM).  For every lattice point in
 * front of the camera whose nearest pixel has depth d > 0: eta = d - z; points
 * with eta < -mu are left alone; otherwise tsdf <- (w tsdf + min(1, eta/mu))
 * / (w + 1) and w <- min(w + 1, max_weight); inside |eta| <= mu the colour is
 * averaged the same way with its own weight.
 * depth [H][W] (m, 0 = invalid), rgb [3][H][W].  Updates vol in place. */
gps_status gps_fuse(const gps_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                    void* stream);

/* SDF raycast (Sec. 3.1 first pass; Sec. 3.2.1): each pixel's ray marches with
 * step `step` (0 = voxel/2) from depth z_near until the trilinear signed
 * distance turns from positive to non-positive; the crossing is refined by the
 * secant; D_t is the camera depth of the surface point V and C_t the trilinear
 * colour of the eight voxels around V.  Misses give D_t = 0, C_t = 0.
 * cams: host array of n_views (<= GPS_MAX_VIEWS) cameras; out_depth, out_rgb:
 * host arrays of n_views device pointers ([H][W] and [3][H][W] of each view).
 * If vol->brick_min is set it is rebuilt from vol->tsdf first and used to skip
 * samples whose 2x2x2 stencil is known positive (the result is unchanged). */
gps_status gps_raycast(const gps_volume* vol, const gps_camera* cams, int32_t n_views, float* const* out_depth,
                       float* const* out_rgb, float z_near, float step, void* stream);

/* ---- Voxel-block hash of the colourised TSDF (Sec. 3.2.1, "SDF fusion": the SDF
 * and colour live in a global hash table of voxel blocks, following InfiniTAM).
 * The lattice of a region (points origin + voxel * (x, y, z), 0 <= x < nx, ...) is
 * split into blocks of 8^3 points; only allocated blocks hold values, in planar
 * pools (24 B per point; point (lx, ly, lz) of pool block b at b*512 + lx + 8 (ly +
 * 8 lz)); every other point reads tsdf 1, weight 0, colour 0.  Memory grows with
 * the allocated blocks, not with nx*ny*nz.  Block (bx, by, bz) has the key
 * bx | by << 21 | bz << 42 (at most 2^21 blocks per axis); the table is open-
 * addressing with linear probing.  All arrays are caller-owned device memory. */
#define GPS_HASH_BLOCK 8
#define GPS_HASH_EMPTY 0xffffffffffffffffull
typedef struct gps_hash_volume {
    int32_t nx, ny, nz;     /* region, lattice points per axis (the raycast's box)    */
    float origin[3];
    float voxel, trunc, max_weight;
    int32_t n_buckets;      /* power of two; at least twice the capacity is advised   */
    int32_t capacity;       /* pool blocks                                            */
    uint64_t* keys;         /* [n_buckets] block keys, GPS_HASH_EMPTY = free          */
    int32_t* slots;         /* [n_buckets] pool block of each key (-1: no room)       */
    uint64_t* block_key;    /* [capacity] key of each pool block, allocation order    */
    int32_t* state;         /* [4]: blocks allocated (may exceed capacity after an
                               overflow), allocated before the last fusion, blocks
                               visible in the last fusion, status bits (1: the pool
                               overflowed, 2: the table filled up)                     */
    int32_t* visible;       /* [capacity] scratch: pool blocks seen by the last fusion */
    float* block_min;       /* [capacity] scratch for the raycast's skipping of
                               positive blocks, or NULL                                */
    float* tsdf;            /* [capacity * 512]                                       */
    float* weight;          /* [capacity * 512]                                       */
    float* rgb;             /* [3][capacity * 512]                                    */
    float* rgb_weight;      /* [capacity * 512]                                       */
} gps_hash_volume;

/* Empties the table and the counters (fills keys with GPS_HASH_EMPTY; pools are
 * initialised block by block as blocks are allocated).  Two kernels. */
gps_status gps_hash_reset(const gps_hash_volume* vol, void* stream);

/* Fuses one RGB-D frame: (1) allocation -- for every pixel with depth d > 0 the
 * blocks holding its ray's points at camera depths d + k voxel, |k| <=
 * ceil(trunc / voxel), inside the region, decided in binary32 (the block
 * coordinate of a point is floor(((R^T (x - t))_a - origin_a) / (8 voxel)) with
 * the camera-frame point x = (z (i - cx) / fx, z (j - cy) / fy, z)); new blocks
 * start at tsdf 1, weights 0, colour 0; (2) the visible list -- allocated blocks
 * whose lattice box projects into the image (conservative); (3) the update of
 * gps_fuse applied to every point of the visible blocks.  The result equals
 * gps_fuse on a dense lattice whose points outside the allocated blocks are left
 * alone.  A full pool or table sets a status bit in state[3] (sticky until
 * gps_hash_reset); blocks without room are then read as unallocated.
 * depth [H][W], rgb [3][H][W].  Five kernels, nothing read back. */
gps_status gps_hash_fuse(const gps_hash_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                         void* stream);

/* The raycast of gps_raycast over the hashed volume (same march, decisions and
 * values; the march runs inside the region's box): samples whose 2x2x2 stencil
 * lies in one block that is unallocated, or whose points are all positive
 * (vol->block_min), are skipped, which does not change the crossing found.
 * cams, out_depth, out_rgb as in gps_raycast.
 * range (optional, device scratch of range_floats floats, at least
 * GPS_HASH_RANGE_FLOATS summed over the views): the camera-depth interval that
 * the allocated blocks, grown by one voxel, cover in each 16x16-pixel tile of each
 * view is formed first, and the rays of a tile march only over their samples in
 * that interval (every sample outside it has a stencil of unallocated points, so
 * it reads positive and the crossing is the same); the free space in front of the
 * first block costs nothing.  NULL: the rays march the whole region.  Two kernels,
 * four with range.  GPS_ERR_INVALID_ARG for a range shorter than needed. */
#define GPS_HASH_TILE 16
#define GPS_HASH_RANGE_FLOATS(width, height) \
    (2 * (((width) + GPS_HASH_TILE - 1) / GPS_HASH_TILE) * (((height) + GPS_HASH_TILE - 1) / GPS_HASH_TILE))
gps_status gps_hash_raycast(const gps_hash_volume* vol, const gps_camera* cams, int32_t n_views,
                            float* const* out_depth, float* const* out_rgb, float z_near, float step, float* range,
                            size_t range_floats, void* stream);

/* Forward render of n_views (<= GPS_MAX_VIEWS) views (views: host array) and,
 * when every view has target_rgb, the loss
 *   L = (1/V) sum_v [ mean_{pixels,channels} |C* - C_k| (Eq. 7)
 *                    + lambda_depth * mean_{Omega_v} |D* - D_k| ],
 *   Omega_v = { D_k > 0 and D_t > 0 },
 * written to out_loss (device float, may be NULL).
 * Per view: EWA projection of every Gaussian (Eq. 3, following 3DGS), binning
 * into screen tiles with an exact tile-level depth cull, a per-tile depth sort,
 * and compositing over the SDF base:
 *   mode 0: front to back, alpha_i = min(alpha_max, sigma_i exp(-q/2)),
 *           skipping alpha < alpha_min, stopping at the first Gaussian with
 *           d_i >= D_t + eps (the depth test of Eq. 1-2) or when the
 *           transmittance would fall below T_min;
 *           C* = sum alpha_i T_i c_i + T_final C_t, D* likewise with d_i, D_t;
 *   mode 1: C* = (C_t + sum alpha_i c_i) / (1 + sum alpha_i) (Eq. 1, 2, 4).
 * The workspace keeps what gps_render_bwd needs; render_bwd must follow on
 * the same workspace with unchanged inputs. */
gps_status gps_render_fwd(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views, int32_t n_views,
                          void* ws, size_t ws_bytes, float* out_loss, void* stream);

/* Backward of gps_render_fwd: the analytic gradient of the loss (Eq. 7 plus the
 * depth term) through the blend (Eq. 1, 2, 4 in mode 1, front-to-back over the
 * SDF image in mode 0) and the opacity of Eq. 3, to the Gaussian parameters and
 * the camera pose (Sec. 3.1; the paper's backward for its blend is described
 * after Eq. 4 and in Appendix B).  The upstream adjoint is either
 *   - the fused loss (dL_drgb == NULL): dL/dC*, dL/dD* of the loss above,
 *     scaled by *loss_scale (device float; NULL = 1), or
 *   - explicit per-view images (dL_drgb, dL_ddepth: host arrays of n_views
 *     device pointers to [3][H][W] and [H][W]; dL_ddepth may be NULL).
 * Per pixel the transmittance and prefix colour are recomputed front to back
 * (nothing per pixel is stored by the forward); each (tile, Gaussian) instance
 * gets one partial reduced across its tile's pixels with wavefront DPP
 * reductions, and each Gaussian sums its instances in a fixed order, so no
 * floating-point atomics are used.
 * grads: gradients with respect to every attribute of g (overwritten).
 * dpose: [n_views][6] gradient with respect to xi = (rho, phi) of the left
 * perturbation T_cw <- Exp(xi) T_cw (may be NULL): at xi = 0, or at the view's
 * pose_xi when it is set (the gradient at the perturbed pose times the
 * transposed left Jacobian of SE(3) at xi).
 * After a capacity overflow of the forward (sticky GPS_ERR_CAPACITY) no slot is
 * read: every gradient and dpose is zero (and gps_render_bwd_adam leaves the
 * parameters, moments and step counter unchanged). */
gps_status gps_render_bwd(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views, int32_t n_views,
                          const float* const* dL_drgb, const float* const* dL_ddepth, const float* loss_scale,
                          gps_gaussians* grads, float* dpose, void* ws, size_t ws_bytes, void* stream);

/* Writes the view table of `views` (and, for an explicit-adjoint backward,
 * the per-view dL_drgb / dL_ddepth device pointers; both may be NULL) into the
 * workspace, and the per-tile maxima of the views' base depths (read now: call
 * again after a base image changes), for calls made with
 * GPS_RENDER_VIEWS_PRESET.  Same argument checks as gps_render_fwd; two
 * kernels are launched on `stream`. */
gps_status gps_views_upload(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views,
                            int32_t n_views, const float* const* dL_drgb, const float* const* dL_ddepth, void* ws,
                            size_t ws_bytes, void* stream);

/* Adam over n_groups (<= 8) parameter groups in one launch (groups: host
 * array), with the per-attribute learning rates of Appendix C supplied by the
 * caller:  m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * p <- p - lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 * The step t is `step` (>= 1) when step_counter is NULL; otherwise
 * t = *step_counter + 1 is read on the device and the counter is incremented
 * once the update is done (for graph replay). */
gps_status gps_adam_step(const gps_adam_group* groups, int32_t n_groups, int32_t step, int32_t* step_counter,
                         float beta1, float beta2, float eps, void* stream);

/* ---- Backward with the Adam step in its epilogue (one optimisation iteration's
 * backward + Adam without the separate Adam launch).  The same as gps_render_bwd
 * followed by gps_adam_step over the attribute groups (five, six with SH) with the learning
 * rates below, and bitwise the same parameters, moments and counter; `g` is
 * updated in place after its gradient is formed.  grads may be NULL (the
 * gradients are then not stored). */
typedef struct gps_adam_fused {
    gps_gaussians m, v;   /* first and second moments (device), same layout and count as g */
    float lr_mean, lr_log_scale, lr_quat, lr_opacity, lr_rgb;
    float lr_sh;          /* the SH bands above 0 (0.0005 in Appendix C)    */
    float beta1, beta2, eps;
    int32_t step;         /* 1-based step, used when step_counter is NULL */
    int32_t* step_counter;/* device int32 or NULL: t = *step_counter + 1, incremented afterwards */
} gps_adam_fused;

gps_status gps_render_bwd_adam(const gps_render_cfg* cfg, gps_gaussians* g, const gps_view* views, int32_t n_views,
                               const float* const* dL_drgb, const float* const* dL_ddepth, const float* loss_scale,
                               gps_gaussians* grads, float* dpose, const gps_adam_fused* adam, void* ws,
                               size_t ws_bytes, void* stream);

/* ---- Gaussian removal (Sec. 3.2.2, Eq. 8) ---------------------------------
 * A Gaussian is removed when its opacity sigmoid(o) is below min_opacity, or its
 * largest scale exp(l) is above max_scale or below min_scale (0.005, 0.1 and
 * 0.003 in the paper).  The tests are taken on the stored parameters in
 * binary32: o < logit(min_opacity), max(l) > ln(max_scale), max(l) <
 * ln(min_scale), each threshold computed in binary64 and rounded once. */
typedef struct gps_removal_cfg {
    float min_opacity;
    float max_scale;
    float min_scale;
} gps_removal_cfg;

/* Fills `cfg` (host) with the paper's thresholds. */
void gps_removal_cfg_default(gps_removal_cfg* cfg);

/* Scratch bytes that gps_remove_gaussians needs for n_gaussians. */
gps_status gps_removal_workspace_size(int32_t n_gaussians, size_t* out_bytes);

/* Stable compaction.  sets_in[0] decides (n = sets_in[0].count); the kept
 * Gaussians of every set sets_in[0 .. n_sets) (for example the parameters and
 * their two Adam moments; every set has count n) are written in their original
 * order to sets_out[k] as planar [rows][n_kept] arrays (row stride n_kept; each
 * output array has room for rows * n floats), and n_kept to *out_count (a
 * device int32).  Inputs and outputs must not overlap.  n_sets: 1 .. 4.
 * ws: gps_removal_workspace_size bytes of device memory, 256-byte aligned.
 * Three kernels on `stream`; nothing is read back on the host. */
gps_status gps_remove_gaussians(const gps_removal_cfg* cfg, const gps_gaussians* sets_in, gps_gaussians* sets_out,
                                int32_t n_sets, int32_t* out_count, void* ws, size_t ws_bytes, void* stream);

/* ---- Gaussian insertion (Sec. 3.2.2, Eq. 6 and the paragraph after it; App. A)
 * Mask: pixels with an SDF surface (D_t > 0) whose colour error is above delta_c
 * and whose Gaussian weight W_G is below delta_W; the colour error is the mean
 * of the three absolute channel differences, tested in binary32 as
 * (|e0| + |e1|) + |e2| > 3 delta_c.  A mask pixel is taken when the caller's
 * uniform number for it is below `fraction` (the 25 % sample).  Each taken
 * pixel u gets a Gaussian at the SDF surface point V*(u) (its depth D_t
 * back-projected), coloured C_k(u), opacity `opacity`, shaped as a disc whose
 * short axis is the vertex-map normal N*(u) (normalised cross product of the
 * central differences of V*, turned to face the camera; the direction to the
 * camera where a neighbour has no surface): scales (s1, s1, flat_ratio s1),
 * s1 = min(scale_cap, root mean square distance to the three mask vertices
 * nearest to V*(u)), searched over the whole mask (u itself excluded; with
 * fewer than three other mask vertices the mean runs over those there are,
 * with none s1 = scale_cap).  App. A prints the square root of the mean
 * distance; the root mean square distance is the reading used here. */
typedef struct gps_insert_cfg {
    float delta_c;     /* 0.05 */
    float delta_w;     /* 4 */
    float fraction;    /* 0.25 */
    float scale_cap;   /* 0.1 */
    float flat_ratio;  /* 0.1 */
    float opacity;     /* 0.5 */
} gps_insert_cfg;

/* Fills `cfg` (host) with the paper's constants. */
void gps_insert_cfg_default(gps_insert_cfg* cfg);

/* Scratch bytes that gps_insert_gaussians needs for a width x height frame. */
gps_status gps_insertion_workspace_size(int32_t width, int32_t height, size_t* out_bytes);

/* New Gaussians for one frame.  Images (device, planar): render_rgb C* [3][H][W]
 * and weight W_G [H][W] of the current Gaussians over the SDF image (sort-free
 * forward), frame_rgb C_k [3][H][W], sdf_depth D_t [H][W] (0 = miss), rand
 * [H][W] uniform numbers in [0, 1).  out: out->count = capacity, planar
 * [rows][capacity] arrays; the taken pixels fill positions 0 .. in row-major
 * pixel order, those past the capacity are dropped; out_pixel (optional,
 * [capacity]) receives their pixel indices; *out_count (device int32) the
 * number of taken pixels (possibly above the capacity).  ws:
 * gps_insertion_workspace_size bytes, 256-byte aligned.  Five kernels. */
gps_status gps_insert_gaussians(const gps_insert_cfg* cfg, const gps_camera* cam, const float* render_rgb,
                                const float* frame_rgb, const float* weight, const float* sdf_depth, const float* rand,
                                gps_gaussians* out, int32_t* out_pixel, int32_t* out_count, void* ws, size_t ws_bytes,
                                void* stream);

/* ---- Camera tracking (Sec. 3.2.1, "Camera tracking", Eq. 5): point-to-plane ICP.
 * The pose being tracked is a device array `pose` [12] = R (row-major), t of the
 * current camera, world to camera like gps_camera; the model is the previous
 * frame's SDF raycast depth D_t (full resolution, 0 = miss) seen from `prev_cam`.
 * A step: gps_icp_reduce on one level of the current depth hierarchy, then
 * gps_icp_solve; every call only enqueues work and reads the pose from device
 * memory, so a whole coarse-to-fine loop can be captured as a graph. */

/* One level of the depth hierarchy: out [height/2][width/2] (integer division)
 * holds the mean of the valid (> 0) depths of each 2x2 block, 0 when none is
 * valid (sum and division in binary64, rounded once).  The level's intrinsics
 * are f/2 and (c - 1/2)/2.  width, height >= 2. */
gps_status gps_depth_downsample(const float* depth, int32_t width, int32_t height, float* out, void* stream);

/* Host call: the camera of level `level` (0 = full resolution) of the depth
 * hierarchy of `cam`: each level halves the size (integer division), the focal
 * lengths, and maps the principal point to (c - 1/2) / 2 (the centre of a
 * coarse pixel is the mean of its 2x2 block's centres); computed in binary64,
 * rounded once.  R and t are copied.  GPS_ERR_INVALID_ARG for level outside
 * 0..16 or a level smaller than one pixel. */
gps_status gps_level_camera(const gps_camera* cam, int32_t level, gps_camera* out);

/* Scratch bytes for gps_icp_reduce on a level of width x height pixels. */
gps_status gps_icp_workspace_size(int32_t width, int32_t height, size_t* out_bytes);

/* The Gauss-Newton system of Eq. 5 at the device pose, for one level.
 * level_cam: the level's size and intrinsics (its R and t are not read);
 * level_depth [height][width] (device).  For every pixel with depth d > 0: the
 * vertex V = ((i - cx) d / fx, (j - cy) d / fy, d), its world point p, the
 * nearest pixel u^ of its projection into prev_cam, which must lie in the image
 * with its four neighbours, all with a raycast surface; V*, the back-projection
 * of D_t(u^), and N*, the normalised cross product of the central differences
 * of the back-projected D_t; pairs farther apart than dist_thresh (m) are
 * dropped.  r = (p - V*) . N*, J = (N*, p x N*) for the left perturbation
 * T_{g,k} <- Exp(xi) T_{g,k} of the camera-to-world pose, xi = (rho, phi).
 * out_sys (device, binary64 [29]): the upper triangle of H = sum J J^T
 * (row-major, 21), g = sum J r (6), sum r^2, the pair count.  Sums in a fixed
 * order (no atomics).  ws: gps_icp_workspace_size bytes, 256-byte aligned. */
gps_status gps_icp_reduce(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                          const float* level_depth, const float* pose, float dist_thresh, double* out_sys, void* ws,
                          size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight tracking loops, harnesses that forbid hipMalloc): gps_icp_reduce without
 * the workspace.  Same arguments, checks, kernels and bitwise the same out_sys.
 * The block sums go to a scratch array inside the library, GPS_ICP_SCRATCH_BYTES
 * bytes per GPU, held from the first call on that GPU until the process ends; it
 * holds the sums of the widest grid the reduce launches, so every level size that
 * gps_icp_reduce accepts fits (a larger need returns
 * GPS_ERR_WORKSPACE_TOO_SMALL).  Nothing is allocated and nothing is cleared:
 * each call overwrites the sums it reads.  All calls on one GPU share that array,
 * so calls that overlap on one GPU (on different streams or threads) race; the
 * caller serialises them. */
#define GPS_ICP_SCRATCH_BYTES (29 * 1024 * 4)
gps_status gps_icp_reduce_noalloc(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                                  const float* level_depth, const float* pose, float dist_thresh, double* out_sys,
                                  void* stream);

/* One Gauss-Newton step of Eq. 5: gps_icp_reduce followed by gps_icp_solve on its
 * system, with the system's sum and the solve in one launch (two kernels instead of
 * three).  out_sys receives the system as gps_icp_reduce writes it, pose is updated
 * in place and out_xi (optional) receives xi, bitwise as the two calls give them.
 * Arguments and checks as gps_icp_reduce; pose is read and written. */
gps_status gps_icp_step(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                        const float* level_depth, float* pose, float dist_thresh, double* out_sys, float* out_xi,
                        void* ws, size_t ws_bytes, void* stream);

/* Solves H xi = -g (Cholesky, binary64) and applies T_{g,k} <- Exp(xi) T_{g,k}
 * to the device pose in place; out_xi (optional, device [6]) receives xi.  With
 * fewer than 6 pairs or H not positive definite the pose is kept and xi = 0. */
gps_status gps_icp_solve(const double* sys, float* pose, float* out_xi, void* stream);

/* Reads the sticky status word of a workspace (synchronises `stream`). */
gps_status gps_device_status(const void* ws, size_t ws_bytes, int32_t* out_status, void* stream);

/* Reads the counters of the last render call (synchronises `stream`). */
gps_status gps_read_stats(const void* ws, size_t ws_bytes, gps_stats* out, void* stream);

/* ---- Optional per-kernel timing (not part of the mapping path) ----------
 * While profiling is on for the calling thread, every kernel the library
 * launches from that thread is bracketed by two HIP events recorded on its
 * launch stream.  gps_profile_read synchronises those events and returns, per
 * kernel name, the number of launches and the summed event time since the last
 * gps_profile_start.  State is thread-local; events are created on first use
 * and kept until the thread exits. */
typedef struct gps_kernel_time {
    char name[32];
    int64_t launches;
    double total_ms;
} gps_kernel_time;

gps_status gps_profile_start(void);
gps_status gps_profile_stop(void);
gps_status gps_profile_read(gps_kernel_time* out, int32_t max_kernels, int32_t* n_out);

/* ---- Streaming kernels of known traffic (not part of the mapping path) ----
 * For scaling the hardware's memory counters (FETCH_SIZE, WRITE_SIZE) to bytes:
 * gps_stream_read reads the n floats of device array x once and writes one
 * float per block (gps_stream_blocks() floats) to device array out;
 * gps_stream_write writes v to the n floats of device array y once and reads
 * nothing.  16-byte accesses when the array is 16-byte aligned.  Null pointers
 * or n = 0 return GPS_ERR_INVALID_ARG; nothing is launched then. */
int32_t gps_stream_blocks(void);
gps_status gps_stream_read(const float* x, size_t n, float* out, void* stream);
gps_status gps_stream_write(float* y, size_t n, float v, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GPS_H_ */
