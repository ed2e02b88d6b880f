// C ABI of libgps (declared in include/gps.h): argument validation, the
// workspace map, view tables and kernel launches.  No entry point allocates
// device memory; every argument error is reported before anything is launched.
#include <atomic>
#include <cmath>
#include <cstring>

#include "gps_internal.h"
#include "binning.h"
#include "launch.h"
#include "prof.h"

namespace gps {
bool tile_config_supported(const gps_render_cfg* cfg);

static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

static bool cam_ok(const gps_camera& c)
{
    if (c.width <= 0 || c.height <= 0 || c.width > (1 << 18) || c.height > (1 << 18)) return false;
    const float vals[4] = {c.fx, c.fy, c.cx, c.cy};
    for (float v : vals)
        if (!std::isfinite(v)) return false;
    if (c.fx == 0.0f || c.fy == 0.0f) return false;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(c.R[k])) return false;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c.t[k])) return false;
    return true;
}

static gps_status check_device()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GPS_ERR_HIP;
    if (dev < 0 || dev >= 64) return GPS_ERR_UNSUPPORTED_DEVICE;
    int st = cache[dev].load(std::memory_order_relaxed);
    if (st == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return GPS_ERR_HIP;
        st = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        cache[dev].store(st, std::memory_order_relaxed);
    }
    return st == 1 ? GPS_OK : GPS_ERR_UNSUPPORTED_DEVICE;
}

static gps_status compute_layout(const gps_render_cfg* cfg, int M, const gps_camera* cams, int V, WsLayout* L)
{
    if (!cfg || !cams || !L || M < 0 || V < 1 || V > GPS_MAX_VIEWS) return GPS_ERR_INVALID_ARG;
    if (cfg->mode != 0 && cfg->mode != 1) return GPS_ERR_INVALID_ARG;
    if (!tile_config_supported(cfg)) return GPS_ERR_UNSUPPORTED_CONFIG;
    if (cfg->max_instances < 0) return GPS_ERR_INVALID_ARG;
    if (cfg->flags & ~(GPS_RENDER_VIEWS_PRESET | GPS_RENDER_BWD_PER_GAUSSIAN | GPS_RENDER_NO_SORT))
        return GPS_ERR_INVALID_ARG;
    if ((cfg->flags & GPS_RENDER_NO_SORT) && cfg->mode != 1) return GPS_ERR_UNSUPPORTED_CONFIG;
    const float consts[7] = {cfg->eps_cull, cfg->lambda_depth, cfg->dilation, cfg->alpha_min,
                             cfg->alpha_max, cfg->T_min, cfg->z_near};
    for (float c : consts)
        if (!std::isfinite(c) || c < 0.0f) return GPS_ERR_INVALID_ARG;
    if (!(cfg->alpha_min > 0.0f) || !(cfg->alpha_max > cfg->alpha_min) || !(cfg->alpha_max < 1.0f) ||
        !(cfg->z_near > 0.0f) || !(cfg->dilation > 0.0f))
        return GPS_ERR_INVALID_ARG;
    long long n_tiles = 0, npix = 0;
    for (int v = 0; v < V; ++v) {
        if (!cam_ok(cams[v])) return GPS_ERR_INVALID_ARG;
        const long long tx = (cams[v].width + cfg->tile_w - 1) / cfg->tile_w;
        const long long ty = (cams[v].height + cfg->tile_h - 1) / cfg->tile_h;
        if (tx > 65534 || ty > 65534) return GPS_ERR_INVALID_ARG;
        n_tiles += tx * ty;
        npix += (long long)cams[v].width * cams[v].height;
    }
    const long long nvg = (long long)V * M;
    if (nvg >= (1ll << 31) || n_tiles >= (1ll << 31) || npix >= (1ll << 31)) return GPS_ERR_INVALID_ARG;
    unsigned long long cap = cfg->max_instances > 0 ? (unsigned long long)cfg->max_instances
                                                    : (unsigned long long)std::max<long long>(1ll << 20, 32 * nvg);
    if (cap >= 0xffffffffull) return GPS_ERR_INVALID_ARG;
    L->n_tiles = (int)n_tiles;
    L->nvg = (int)nvg;
    L->nblk_vg = (int)((nvg + kBlk - 1) / kBlk);
    L->nblk_g = (M + kBlk - 1) / kBlk;
    L->cap = cap;
    size_t o = 0;
    L->hdr = o;
    o = align_up(o + 1024);
    L->vtab = o;
    o = align_up(o + sizeof(ViewTable));
    L->tilemax = o;
    o = align_up(o + 4 * (size_t)n_tiles);
    L->tile_cnt = o;
    o = align_up(o + 4 * (size_t)kCntSplit * n_tiles);
    L->tile_start = o;
    o = align_up(o + 4 * (size_t)(n_tiles + 1));
    L->tile_queue = o;
    o = align_up(o + 4 * (size_t)n_tiles);
    L->tile_loss = o;
    o = align_up(o + 16 * (size_t)n_tiles);
    L->tile_pairs = o;
    o = align_up(o + 8 * (size_t)n_tiles);
    L->pix_aux = o;
    o = align_up(o + 4 * (size_t)npix);
    L->rec = o;
    o = align_up(o + 4 * kRecFloats * (size_t)nvg);
    L->cnt = o;
    o = align_up(o + 4 * (size_t)nvg);
    L->off = o;
    o = align_up(o + 4 * (size_t)nvg);
    L->blk_sum = o;
    o = align_up(o + 4 * (size_t)L->nblk_vg);
    L->blk_off = o;
    o = align_up(o + 4 * (size_t)L->nblk_vg);
    L->keys = o;
    o = align_up(o + 8 * (size_t)cap);
    L->inst_vg = o;
    o = align_up(o + 4 * (size_t)cap);
    L->partial = o;
    o = align_up(o + 4 * (size_t)kAdj * cap);
    L->pose_part = o;
    o = align_up(o + 4 * 6 * (size_t)V * (size_t)(L->nblk_g > 0 ? L->nblk_g : 1));
    L->total = o;
    static_assert(sizeof(WsHeader) <= 1024, "workspace header");
    return GPS_OK;
}

// The SH bands of a Gaussian set (or of its gradients or moments): degree 0..3 equal
// to `degree`, coefficients present when there are any.
static bool sh_ok(const gps_gaussians* x, int degree, int count)
{
    if (x->sh_degree < 0 || x->sh_degree > 3 || x->sh_degree != degree) return false;
    return degree == 0 || count == 0 || x->sh != nullptr;
}

static gps_status build_tables(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views, int V,
                               ViewTable* vt, RParams* rp, WsLayout* L)
{
    if (!g || !views) return GPS_ERR_INVALID_ARG;
    if (g->count < 0) return GPS_ERR_INVALID_ARG;
    if (g->count > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity_logit || !g->rgb))
        return GPS_ERR_INVALID_ARG;
    if (!sh_ok(g, g->sh_degree, g->count)) return GPS_ERR_INVALID_ARG;
    gps_camera cams[GPS_MAX_VIEWS];
    if (V < 1 || V > GPS_MAX_VIEWS) return GPS_ERR_INVALID_ARG;
    for (int v = 0; v < V; ++v) cams[v] = views[v].cam;
    gps_status st = compute_layout(cfg, g->count, cams, V, L);
    if (st != GPS_OK) return st;
    std::memset(vt, 0, sizeof(*vt));
    vt->n = V;
    int tb = 0, pb = 0;
    for (int v = 0; v < V; ++v) {
        const gps_view& s = views[v];
        if (!s.base_rgb || !s.base_depth || !s.out_rgb || !s.out_depth) return GPS_ERR_INVALID_ARG;
        DevView& d = vt->v[v];
        d.cam.fx = s.cam.fx;
        d.cam.fy = s.cam.fy;
        d.cam.cx = s.cam.cx;
        d.cam.cy = s.cam.cy;
        for (int k = 0; k < 9; ++k) d.cam.R[k] = s.cam.R[k];
        for (int k = 0; k < 3; ++k) d.cam.t[k] = s.cam.t[k];
        d.cam.W = s.cam.width;
        d.cam.H = s.cam.height;
        d.tiles_x = (s.cam.width + cfg->tile_w - 1) / cfg->tile_w;
        d.tiles_y = (s.cam.height + cfg->tile_h - 1) / cfg->tile_h;
        d.tile_base = tb;
        d.pix_base = pb;
        tb += d.tiles_x * d.tiles_y;
        pb += s.cam.width * s.cam.height;
        d.base_rgb = s.base_rgb;
        d.base_depth = s.base_depth;
        d.target_rgb = s.target_rgb;
        d.target_depth = s.target_depth;
        d.out_rgb = s.out_rgb;
        d.out_depth = s.out_depth;
        d.pose_xi = s.pose_xi;
        d.out_aux = s.out_aux;
    }
    vt->n_tiles = tb;
    rp->eps = cfg->eps_cull;
    rp->lambda = cfg->lambda_depth;
    rp->dil = cfg->dilation;
    rp->amin = cfg->alpha_min;
    rp->amax = cfg->alpha_max;
    rp->Tmin = cfg->T_min;
    rp->znear = cfg->z_near;
    rp->mode = (cfg->mode == 1 && (cfg->flags & GPS_RENDER_NO_SORT)) ? 2 : cfg->mode;  // 2: sort-free, unsorted
    rp->M = g->count;
    rp->V = V;
    rp->nvg = L->nvg;
    rp->tile_w = cfg->tile_w;
    rp->tile_h = cfg->tile_h;
    rp->cap = L->cap;
    return GPS_OK;
}

__global__ void __launch_bounds__(256) k_ws_reset(char* ws)
{
    unsigned int* p = reinterpret_cast<unsigned int*>(ws);
    p[threadIdx.x] = 0u;  // 256 lanes x 4 bytes = the 1 KiB header
}

gps_status launch_ws_reset(char* ws, hipStream_t s)
{
    GPS_LAUNCH(K_WS_RESET, s, k_ws_reset, dim3(1), dim3(256), 0, s, ws);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps

using namespace gps;

extern "C" {

int32_t gps_abi_version(void) { return GPS_ABI_VERSION; }

const char* gps_status_string(gps_status s)
{
    switch (s) {
    case GPS_OK: return "ok";
    case GPS_ERR_INVALID_ARG: return "invalid argument";
    case GPS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case GPS_ERR_CAPACITY: return "tile-instance capacity exceeded (device)";
    case GPS_ERR_HIP: return "HIP runtime error";
    case GPS_ERR_UNSUPPORTED_DEVICE: return "unsupported device (gfx950 required)";
    case GPS_ERR_UNSUPPORTED_CONFIG: return "unsupported tile/batch/pixels-per-thread combination";
    default: return "unknown status";
    }
}

void gps_render_cfg_default(gps_render_cfg* c)
{
    if (!c) return;
    c->tile_w = 16;
    c->tile_h = 16;
    c->batch = 256;
    c->pix_per_thread = 1;
    c->mode = 0;
    c->eps_cull = 0.01f;
    c->lambda_depth = 1.0f;
    c->dilation = 0.3f;
    c->alpha_min = 1.0f / 255.0f;
    c->alpha_max = 0.99f;
    c->T_min = 1e-4f;
    c->z_near = 0.2f;
    c->max_instances = 0;
    c->flags = 0;
}

gps_status gps_workspace_size(const gps_render_cfg* cfg, int32_t n_gaussians, const gps_camera* cams,
                              int32_t n_views, size_t* out_bytes)
{
    if (!out_bytes) return GPS_ERR_INVALID_ARG;
    WsLayout L;
    gps_status st = compute_layout(cfg, n_gaussians, cams, n_views, &L);
    if (st != GPS_OK) return st;
    *out_bytes = L.total;
    return GPS_OK;
}

gps_status gps_workspace_reset(void* ws, size_t ws_bytes, void* stream)
{
    if (!ws || ws_bytes < 1024 || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_ws_reset(static_cast<char*>(ws), (hipStream_t)stream);
}

gps_status gps_fuse(const gps_volume* vol, const gps_camera* cam, const float* depth, const float* rgb, void* stream)
{
    if (!vol || !cam || !depth || !rgb) return GPS_ERR_INVALID_ARG;
    if (vol->nx < 2 || vol->ny < 2 || vol->nz < 2) return GPS_ERR_INVALID_ARG;
    if ((unsigned long long)vol->nx * vol->ny * vol->nz >= (1ull << 32)) return GPS_ERR_INVALID_ARG;
    if (!vol->tsdf || !vol->weight || !vol->rgb || !vol->rgb_weight) return GPS_ERR_INVALID_ARG;
    if (!(vol->voxel > 0.0f) || !(vol->trunc > 0.0f) || !(vol->max_weight >= 1.0f)) return GPS_ERR_INVALID_ARG;
    if (!cam_ok(*cam)) return GPS_ERR_INVALID_ARG;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_fuse(vol, cam, depth, rgb, (hipStream_t)stream);
}

gps_status gps_raycast(const gps_volume* vol, const gps_camera* cams, int32_t n_views, float* const* out_depth,
                       float* const* out_rgb, float z_near, float step, void* stream)
{
    if (!vol || !cams || !out_depth || !out_rgb) return GPS_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > GPS_MAX_VIEWS) return GPS_ERR_INVALID_ARG;
    if (vol->nx < 2 || vol->ny < 2 || vol->nz < 2) return GPS_ERR_INVALID_ARG;
    if ((unsigned long long)vol->nx * vol->ny * vol->nz >= (1ull << 32)) return GPS_ERR_INVALID_ARG;
    if (!vol->tsdf || !vol->rgb || !(vol->voxel > 0.0f)) return GPS_ERR_INVALID_ARG;
    if (!(z_near >= 0.0f) || !std::isfinite(z_near) || !(step >= 0.0f) || !std::isfinite(step))
        return GPS_ERR_INVALID_ARG;
    if (step != 0.0f && step < 1e-3f * vol->voxel) return GPS_ERR_INVALID_ARG;
    for (int v = 0; v < n_views; ++v)
        if (!cam_ok(cams[v]) || !out_depth[v] || !out_rgb[v]) return GPS_ERR_INVALID_ARG;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_raycast(vol, cams, n_views, out_depth, out_rgb, z_near, step, (hipStream_t)stream);
}

static gps_status hash_vol_ok(const gps_hash_volume* v)
{
    if (!v) return GPS_ERR_INVALID_ARG;
    if (v->nx < 2 || v->ny < 2 || v->nz < 2) return GPS_ERR_INVALID_ARG;
    const int lim = (1 << 21) * GPS_HASH_BLOCK;  // block coordinates take 21 bits
    if (v->nx > lim || v->ny > lim || v->nz > lim) return GPS_ERR_INVALID_ARG;
    if (!(v->voxel > 0.0f) || !std::isfinite(v->voxel) || !(v->trunc > 0.0f) || !std::isfinite(v->trunc) ||
        !(v->max_weight >= 1.0f))
        return GPS_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(v->origin[k])) return GPS_ERR_INVALID_ARG;
    if (v->n_buckets < 2 || v->n_buckets > (1 << 30) || (v->n_buckets & (v->n_buckets - 1))) return GPS_ERR_INVALID_ARG;
    if (v->capacity < 1 || (int64_t)v->capacity * GPS_HASH_BLOCK * GPS_HASH_BLOCK * GPS_HASH_BLOCK > (int64_t(1) << 40))
        return GPS_ERR_INVALID_ARG;
    if (!v->keys || !v->slots || !v->block_key || !v->state || !v->visible || !v->tsdf || !v->weight || !v->rgb ||
        !v->rgb_weight)
        return GPS_ERR_INVALID_ARG;
    if ((double)v->trunc / (double)v->voxel > 1024.0) return GPS_ERR_INVALID_ARG;  // band points per ray
    return GPS_OK;
}

gps_status gps_hash_reset(const gps_hash_volume* vol, void* stream)
{
    gps_status st = hash_vol_ok(vol);
    if (st != GPS_OK) return st;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_hash_reset(vol, (hipStream_t)stream);
}

gps_status gps_hash_fuse(const gps_hash_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                         void* stream)
{
    gps_status st = hash_vol_ok(vol);
    if (st != GPS_OK) return st;
    if (!cam || !depth || !rgb || !cam_ok(*cam)) return GPS_ERR_INVALID_ARG;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_hash_fuse(vol, cam, depth, rgb, (hipStream_t)stream);
}

gps_status gps_hash_raycast(const gps_hash_volume* vol, const gps_camera* cams, int32_t n_views,
                            float* const* out_depth, float* const* out_rgb, float z_near, float step, float* range,
                            size_t range_floats, void* stream)
{
    gps_status st = hash_vol_ok(vol);
    if (st != GPS_OK) return st;
    if (!cams || !out_depth || !out_rgb || n_views < 1 || n_views > GPS_MAX_VIEWS) return GPS_ERR_INVALID_ARG;
    if (!(z_near >= 0.0f) || !std::isfinite(z_near) || !(step >= 0.0f) || !std::isfinite(step))
        return GPS_ERR_INVALID_ARG;
    if (step != 0.0f && step < 1e-3f * vol->voxel) return GPS_ERR_INVALID_ARG;
    for (int v = 0; v < n_views; ++v)
        if (!cam_ok(cams[v]) || !out_depth[v] || !out_rgb[v]) return GPS_ERR_INVALID_ARG;
    if (range && (((uintptr_t)range & 7) || range_floats < hash_range_floats(cams, n_views)))
        return GPS_ERR_INVALID_ARG;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_hash_raycast(vol, cams, n_views, out_depth, out_rgb, z_near, step, range, (hipStream_t)stream);
}

gps_status gps_render_fwd(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views, int32_t n_views,
                          void* ws, size_t ws_bytes, float* out_loss, void* stream)
{
    ViewTable vt;
    RParams rp;
    WsLayout L;
    gps_status st = build_tables(cfg, g, views, n_views, &vt, &rp, &L);
    if (st != GPS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < L.total) return GPS_ERR_WORKSPACE_TOO_SMALL;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_render_fwd(cfg, rp, g, vt, L, static_cast<char*>(ws), out_loss, (hipStream_t)stream);
}

static gps_status render_bwd_common(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views,
                                    int32_t n_views, const float* const* dL_drgb, const float* const* dL_ddepth,
                                    const float* loss_scale, gps_gaussians* grads, float* dpose,
                                    const gps_adam_fused* adam, void* ws, size_t ws_bytes, void* stream)
{
    ViewTable vt;
    RParams rp;
    WsLayout L;
    gps_status st = build_tables(cfg, g, views, n_views, &vt, &rp, &L);
    if (st != GPS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < L.total) return GPS_ERR_WORKSPACE_TOO_SMALL;
    if (!grads && !adam) return GPS_ERR_INVALID_ARG;
    if (grads && (grads->count != g->count ||
                  (g->count > 0 && (!grads->mean || !grads->log_scale || !grads->quat || !grads->opacity_logit ||
                                    !grads->rgb)) ||
                  !sh_ok(grads, g->sh_degree, g->count)))
        return GPS_ERR_INVALID_ARG;
    if (adam) {
        const gps_gaussians* mv[2] = {&adam->m, &adam->v};
        for (const gps_gaussians* x : mv)
            if (x->count != g->count ||
                (g->count > 0 && (!x->mean || !x->log_scale || !x->quat || !x->opacity_logit || !x->rgb)) ||
                !sh_ok(x, g->sh_degree, g->count))
                return GPS_ERR_INVALID_ARG;
        const float lr[6] = {adam->lr_mean, adam->lr_log_scale, adam->lr_quat, adam->lr_opacity, adam->lr_rgb,
                             adam->lr_sh};
        for (float x : lr)
            if (!std::isfinite(x)) return GPS_ERR_INVALID_ARG;
        if (!(adam->beta1 >= 0.0f && adam->beta1 < 1.0f) || !(adam->beta2 >= 0.0f && adam->beta2 < 1.0f) ||
            !(adam->eps > 0.0f) || (!adam->step_counter && adam->step < 1))
            return GPS_ERR_INVALID_ARG;
    }
    const int explicit_up = dL_drgb != nullptr;
    for (int v = 0; v < n_views; ++v) {
        if (explicit_up) {
            if (!dL_drgb[v]) return GPS_ERR_INVALID_ARG;
            vt.v[v].g_rgb = dL_drgb[v];
            vt.v[v].g_depth = dL_ddepth ? dL_ddepth[v] : nullptr;
        } else if (!views[v].target_rgb) {
            return GPS_ERR_INVALID_ARG;  // the fused-loss adjoint needs targets
        }
    }
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_render_bwd(cfg, rp, g, vt, L, static_cast<char*>(ws), explicit_up, loss_scale, grads, dpose, adam,
                             (hipStream_t)stream);
}

gps_status gps_render_bwd(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views, int32_t n_views,
                          const float* const* dL_drgb, const float* const* dL_ddepth, const float* loss_scale,
                          gps_gaussians* grads, float* dpose, void* ws, size_t ws_bytes, void* stream)
{
    if (!grads) return GPS_ERR_INVALID_ARG;
    return render_bwd_common(cfg, g, views, n_views, dL_drgb, dL_ddepth, loss_scale, grads, dpose, nullptr, ws,
                             ws_bytes, stream);
}

gps_status gps_render_bwd_adam(const gps_render_cfg* cfg, gps_gaussians* g, const gps_view* views, int32_t n_views,
                               const float* const* dL_drgb, const float* const* dL_ddepth, const float* loss_scale,
                               gps_gaussians* grads, float* dpose, const gps_adam_fused* adam, void* ws,
                               size_t ws_bytes, void* stream)
{
    if (!adam) return GPS_ERR_INVALID_ARG;
    return render_bwd_common(cfg, g, views, n_views, dL_drgb, dL_ddepth, loss_scale, grads, dpose, adam, ws,
                             ws_bytes, stream);
}

gps_status gps_views_upload(const gps_render_cfg* cfg, const gps_gaussians* g, const gps_view* views,
                            int32_t n_views, const float* const* dL_drgb, const float* const* dL_ddepth, void* ws,
                            size_t ws_bytes, void* stream)
{
    ViewTable vt;
    RParams rp;
    WsLayout L;
    gps_status st = build_tables(cfg, g, views, n_views, &vt, &rp, &L);
    if (st != GPS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < L.total) return GPS_ERR_WORKSPACE_TOO_SMALL;
    for (int v = 0; v < n_views; ++v) {
        if (dL_drgb) {
            if (!dL_drgb[v]) return GPS_ERR_INVALID_ARG;
            vt.v[v].g_rgb = dL_drgb[v];
            vt.v[v].g_depth = dL_ddepth ? dL_ddepth[v] : nullptr;
        }
    }
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_views_upload(vt, rp, L, static_cast<char*>(ws), 1, (hipStream_t)stream);
}

gps_status gps_adam_step(const gps_adam_group* groups, int32_t n_groups, int32_t step, int32_t* step_counter,
                         float beta1, float beta2, float eps, void* stream)
{
    if (!groups || n_groups < 1 || n_groups > 8) return GPS_ERR_INVALID_ARG;
    if (!step_counter && step < 1) return GPS_ERR_INVALID_ARG;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !std::isfinite(eps))
        return GPS_ERR_INVALID_ARG;
    for (int k = 0; k < n_groups; ++k) {
        const gps_adam_group& gr = groups[k];
        if (gr.n < 0 || !std::isfinite(gr.lr)) return GPS_ERR_INVALID_ARG;
        if (gr.n > 0 && (!gr.param || !gr.grad || !gr.m || !gr.v)) return GPS_ERR_INVALID_ARG;
    }
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_adam(groups, n_groups, step, step_counter, beta1, beta2, eps, (hipStream_t)stream);
}

static gps_status check_removal_args(const gps_removal_cfg* cfg, const gps_gaussians* sets_in,
                                     const gps_gaussians* sets_out, int32_t n_sets)
{
    if (!cfg || !sets_in || !sets_out || n_sets < 1 || n_sets > 4) return GPS_ERR_INVALID_ARG;
    if (!(cfg->min_opacity > 0.0f && cfg->min_opacity < 1.0f) || !(cfg->max_scale > 0.0f) ||
        !(cfg->min_scale > 0.0f) || !(cfg->min_scale <= cfg->max_scale))
        return GPS_ERR_INVALID_ARG;
    const int M = sets_in[0].count;
    if (M < 0) return GPS_ERR_INVALID_ARG;
    for (int k = 0; k < n_sets; ++k) {
        const gps_gaussians& gi = sets_in[k];
        const gps_gaussians& go = sets_out[k];
        if (gi.count != M) return GPS_ERR_INVALID_ARG;
        if (M > 0 && (!gi.mean || !gi.log_scale || !gi.quat || !gi.opacity_logit || !gi.rgb || !go.mean ||
                      !go.log_scale || !go.quat || !go.opacity_logit || !go.rgb))
            return GPS_ERR_INVALID_ARG;
        // every set carries the SH bands of the first (and its output too)
        if (!sh_ok(&gi, sets_in[0].sh_degree, M) || !sh_ok(&go, sets_in[0].sh_degree, M)) return GPS_ERR_INVALID_ARG;
    }
    return GPS_OK;
}

void gps_removal_cfg_default(gps_removal_cfg* cfg)
{
    if (!cfg) return;
    cfg->min_opacity = 0.005f;
    cfg->max_scale = 0.1f;
    cfg->min_scale = 0.003f;
}

gps_status gps_removal_workspace_size(int32_t n_gaussians, size_t* out_bytes)
{
    if (n_gaussians < 0 || !out_bytes) return GPS_ERR_INVALID_ARG;
    *out_bytes = removal_workspace_bytes(n_gaussians);
    return GPS_OK;
}

gps_status gps_remove_gaussians(const gps_removal_cfg* cfg, const gps_gaussians* sets_in, gps_gaussians* sets_out,
                                int32_t n_sets, int32_t* out_count, void* ws, size_t ws_bytes, void* stream)
{
    gps_status st0 = check_removal_args(cfg, sets_in, sets_out, n_sets);
    if (st0 != GPS_OK) return st0;
    const int M = sets_in[0].count;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < removal_workspace_bytes(M)) return GPS_ERR_WORKSPACE_TOO_SMALL;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_remove_gaussians(cfg, sets_in, sets_out, n_sets, out_count, static_cast<char*>(ws),
                                   (hipStream_t)stream);
}

void gps_insert_cfg_default(gps_insert_cfg* cfg)
{
    if (!cfg) return;
    cfg->delta_c = 0.05f;
    cfg->delta_w = 4.0f;
    cfg->fraction = 0.25f;
    cfg->scale_cap = 0.1f;
    cfg->flat_ratio = 0.1f;
    cfg->opacity = 0.5f;
}

static bool insert_frame_ok(int32_t W, int32_t H)
{
    return W > 0 && H > 0 && (int64_t)W * H <= (int64_t(1) << 30);
}

gps_status gps_insertion_workspace_size(int32_t width, int32_t height, size_t* out_bytes)
{
    if (!out_bytes || !insert_frame_ok(width, height)) return GPS_ERR_INVALID_ARG;
    *out_bytes = insertion_workspace_bytes(width, height);
    return GPS_OK;
}

gps_status gps_insert_gaussians(const gps_insert_cfg* cfg, const gps_camera* cam, const float* render_rgb,
                                const float* frame_rgb, const float* weight, const float* sdf_depth, const float* rand,
                                gps_gaussians* out, int32_t* out_pixel, int32_t* out_count, void* ws, size_t ws_bytes,
                                void* stream)
{
    if (!cfg || !cam || !out || !cam_ok(*cam) || !insert_frame_ok(cam->width, cam->height)) return GPS_ERR_INVALID_ARG;
    if (!(cfg->delta_c >= 0.0f) || !std::isfinite(cfg->delta_c) || !(cfg->delta_w > 0.0f) ||
        !(cfg->fraction >= 0.0f && cfg->fraction <= 1.0f) ||
        !(cfg->scale_cap > 0.0f) || !std::isfinite(cfg->scale_cap) || !(cfg->flat_ratio > 0.0f) ||
        !(cfg->flat_ratio <= 1.0f) || !(cfg->opacity > 0.0f && cfg->opacity < 1.0f))
        return GPS_ERR_INVALID_ARG;
    if (!render_rgb || !frame_rgb || !weight || !sdf_depth || !rand || !out_count) return GPS_ERR_INVALID_ARG;
    if (out->count < 0) return GPS_ERR_INVALID_ARG;
    if (out->count > 0 && (!out->mean || !out->log_scale || !out->quat || !out->opacity_logit || !out->rgb))
        return GPS_ERR_INVALID_ARG;
    if (!sh_ok(out, out->sh_degree, out->count)) return GPS_ERR_INVALID_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < insertion_workspace_bytes(cam->width, cam->height)) return GPS_ERR_WORKSPACE_TOO_SMALL;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_insert_gaussians(cfg, dev_cam(*cam), render_rgb, frame_rgb, weight, sdf_depth, rand, out, out_pixel,
                                   out_count, static_cast<char*>(ws), (hipStream_t)stream);
}

gps_status gps_depth_downsample(const float* depth, int32_t width, int32_t height, float* out, void* stream)
{
    if (!depth || !out || width < 2 || height < 2 || (int64_t)width * height > (int64_t(1) << 30))
        return GPS_ERR_INVALID_ARG;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_depth_downsample(depth, width, height, out, (hipStream_t)stream);
}

gps_status gps_level_camera(const gps_camera* cam, int32_t level, gps_camera* out)
{
    if (!cam || !out || level < 0 || level > 16) return GPS_ERR_INVALID_ARG;
    int32_t W = cam->width, H = cam->height;
    double fx = cam->fx, fy = cam->fy, cx = cam->cx, cy = cam->cy;
    for (int k = 0; k < level; ++k) {
        if (W < 2 || H < 2) return GPS_ERR_INVALID_ARG;
        W /= 2;  // a level holds the 2x2 blocks that fit
        H /= 2;
        fx *= 0.5;
        fy *= 0.5;
        cx = (cx - 0.5) * 0.5;  // pixel centres: coarse (i, j) is the mean of 2i, 2i + 1
        cy = (cy - 0.5) * 0.5;
    }
    gps_camera c = *cam;
    c.width = W;
    c.height = H;
    c.fx = (float)fx;
    c.fy = (float)fy;
    c.cx = (float)cx;
    c.cy = (float)cy;
    *out = c;
    return GPS_OK;
}

gps_status gps_icp_workspace_size(int32_t width, int32_t height, size_t* out_bytes)
{
    if (!out_bytes || width <= 0 || height <= 0 || (int64_t)width * height > (int64_t(1) << 30))
        return GPS_ERR_INVALID_ARG;
    *out_bytes = icp_workspace_bytes(width, height);
    return GPS_OK;
}

static gps_status icp_reduce_args_ok(const gps_camera* prev_cam, const float* prev_depth,
                                     const gps_camera* level_cam, const float* level_depth, const float* pose,
                                     float dist_thresh, const double* out_sys)
{
    if (!prev_cam || !level_cam || !prev_depth || !level_depth || !pose || !out_sys) return GPS_ERR_INVALID_ARG;
    if (!cam_ok(*prev_cam) || !(level_cam->width > 0 && level_cam->height > 0) ||
        !std::isfinite(level_cam->fx) || !std::isfinite(level_cam->fy) || !std::isfinite(level_cam->cx) ||
        !std::isfinite(level_cam->cy) || level_cam->fx == 0.0f || level_cam->fy == 0.0f)
        return GPS_ERR_INVALID_ARG;
    if ((int64_t)level_cam->width * level_cam->height > (int64_t(1) << 30) ||
        (int64_t)prev_cam->width * prev_cam->height > (int64_t(1) << 30))
        return GPS_ERR_INVALID_ARG;
    if (!(dist_thresh > 0.0f) || !std::isfinite(dist_thresh)) return GPS_ERR_INVALID_ARG;
    return GPS_OK;
}

gps_status gps_icp_reduce(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                          const float* level_depth, const float* pose, float dist_thresh, double* out_sys, void* ws,
                          size_t ws_bytes, void* stream)
{
    gps_status st = icp_reduce_args_ok(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, out_sys);
    if (st != GPS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < icp_workspace_bytes(level_cam->width, level_cam->height)) return GPS_ERR_WORKSPACE_TOO_SMALL;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_icp_reduce(*prev_cam, prev_depth, *level_cam, level_depth, pose, dist_thresh, out_sys,
                             static_cast<char*>(ws), (hipStream_t)stream);
}

gps_status gps_icp_reduce_noalloc(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                                  const float* level_depth, const float* pose, float dist_thresh, double* out_sys,
                                  void* stream)
{
    gps_status st = icp_reduce_args_ok(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, out_sys);
    if (st != GPS_OK) return st;
    st = check_device();
    if (st != GPS_OK) return st;
    char* scr = nullptr;
    size_t scr_bytes = 0;
    st = icp_scratch(&scr, &scr_bytes);
    if (st != GPS_OK) return st;
    if (icp_partial_bytes(level_cam->width, level_cam->height) > scr_bytes) return GPS_ERR_WORKSPACE_TOO_SMALL;
    return launch_icp_reduce(*prev_cam, prev_depth, *level_cam, level_depth, pose, dist_thresh, out_sys, scr,
                             (hipStream_t)stream);
}

gps_status gps_icp_step(const gps_camera* prev_cam, const float* prev_depth, const gps_camera* level_cam,
                        const float* level_depth, float* pose, float dist_thresh, double* out_sys, float* out_xi,
                        void* ws, size_t ws_bytes, void* stream)
{
    gps_status st = icp_reduce_args_ok(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, out_sys);
    if (st != GPS_OK) return st;
    if (!ws || ((uintptr_t)ws & 255)) return GPS_ERR_INVALID_ARG;
    if (ws_bytes < icp_workspace_bytes(level_cam->width, level_cam->height)) return GPS_ERR_WORKSPACE_TOO_SMALL;
    st = check_device();
    if (st != GPS_OK) return st;
    return launch_icp_reduce(*prev_cam, prev_depth, *level_cam, level_depth, pose, dist_thresh, out_sys,
                             static_cast<char*>(ws), (hipStream_t)stream, pose, out_xi);
}

gps_status gps_icp_solve(const double* sys, float* pose, float* out_xi, void* stream)
{
    if (!sys || !pose) return GPS_ERR_INVALID_ARG;
    gps_status st = check_device();
    if (st != GPS_OK) return st;
    return launch_icp_solve(sys, pose, out_xi, (hipStream_t)stream);
}

gps_status gps_device_status(const void* ws, size_t ws_bytes, int32_t* out_status, void* stream)
{
    if (!ws || ws_bytes < 1024 || !out_status) return GPS_ERR_INVALID_ARG;
    WsHeader h;
    if (hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess) return GPS_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GPS_ERR_HIP;
    *out_status = h.status;
    return GPS_OK;
}

gps_status gps_read_stats(const void* ws, size_t ws_bytes, gps_stats* out, void* stream)
{
    if (!ws || ws_bytes < 1024 || !out) return GPS_ERR_INVALID_ARG;
    WsHeader h;
    if (hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess) return GPS_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GPS_ERR_HIP;
    std::memset(out, 0, sizeof(*out));
    out->status = h.status;
    out->n_views = h.n_views;
    out->n_instances = (int64_t)h.n_inst;
    out->sort_fallback = (int64_t)h.n_fallback;
    out->capacity = (int64_t)h.cap;
    out->pairs_eval = (int64_t)h.pairs_eval;
    out->pairs_contrib = (int64_t)h.pairs_contrib;
    out->n_tiles = h.n_tiles;
    out->loss = h.loss;
    for (int v = 0; v < GPS_MAX_VIEWS; ++v) out->view_omega[v] = h.view_stats[v][2];
    return GPS_OK;
}

}  // extern "C"
