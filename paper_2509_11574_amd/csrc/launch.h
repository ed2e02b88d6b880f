// Host-side launch functions shared between the sources of the library (each
// defined in one .hip file, called from the C ABI in api.hip or from another
// launch function).  Host code only: no kernel depends on this header.
#pragma once

#include "gps_internal.h"

namespace gps {

// ---------------------------------------------------------------------------
// Host-side launch entry points (defined in the .hip files).
// ---------------------------------------------------------------------------
gps_status launch_fuse(const gps_volume* vol, const gps_camera* cam, const float* depth, const float* rgb,
                       hipStream_t s);
gps_status launch_raycast(const gps_volume* vol, const gps_camera* cams, int n_views, float* const* out_depth,
                          float* const* out_rgb, float z_near, float step, hipStream_t s);
gps_status launch_render_fwd(const gps_render_cfg* cfg, const RParams& rp, const gps_gaussians* g,
                             const ViewTable& vt, const WsLayout& L, char* ws, float* out_loss, hipStream_t s);
gps_status launch_render_bwd(const gps_render_cfg* cfg, const RParams& rp, const gps_gaussians* g,
                             const ViewTable& vt, const WsLayout& L, char* ws, int explicit_upstream,
                             const float* loss_scale, gps_gaussians* grads, float* dpose, const gps_adam_fused* adam,
                             hipStream_t s);
bool dispatch_cfwd(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                   hipStream_t s);
bool dispatch_cbwd(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                   int explicit_up, const float* loss_scale, hipStream_t s);
bool dispatch_cbwd_pg(const gps_render_cfg* cfg, const ViewTable* vt, const RParams& rp, const WsPtrs& w, int n_tiles,
                      int explicit_up, const float* loss_scale, hipStream_t s);
gps_status launch_views_upload(const ViewTable& vt, const RParams& rp, const WsLayout& L, char* ws, int with_tilemax,
                               hipStream_t s);
gps_status launch_adam(const gps_adam_group* groups, int n_groups, int step, int* step_counter, float b1, float b2,
                       float eps, hipStream_t s);
gps_status launch_ws_reset(char* ws, hipStream_t s);
size_t removal_workspace_bytes(int M);
gps_status launch_remove_gaussians(const gps_removal_cfg* cfg, const gps_gaussians* sets_in, gps_gaussians* sets_out,
                                   int n_sets, int* out_count, char* ws, hipStream_t s);
size_t insertion_workspace_bytes(int W, int H);
gps_status launch_insert_gaussians(const gps_insert_cfg* cfg, const DevCam& cam, const float* render_rgb,
                                   const float* frame_rgb, const float* weight, const float* sdf_depth,
                                   const float* rnd, gps_gaussians* out, int* out_pixel, int* out_count, char* ws,
                                   hipStream_t s);
size_t icp_workspace_bytes(int W, int H);
size_t icp_partial_bytes(int W, int H);
gps_status icp_scratch(char** out, size_t* bytes);
gps_status launch_depth_downsample(const float* in, int W, int H, float* out, hipStream_t s);
gps_status launch_icp_reduce(const gps_camera& prev, const float* prev_depth, const gps_camera& lvl,
                             const float* depth, const float* pose, float dist_thresh, double* sys, char* ws,
                             hipStream_t s, float* step_pose = nullptr, float* step_xi = nullptr);
gps_status launch_icp_solve(const double* sys, float* pose, float* out_xi, hipStream_t s);
gps_status launch_hash_reset(const gps_hash_volume* v, hipStream_t s);
gps_status launch_hash_fuse(const gps_hash_volume* v, const gps_camera* cam, const float* depth, const float* rgb,
                            hipStream_t s);
size_t hash_range_floats(const gps_camera* cams, int n_views);
gps_status launch_hash_raycast(const gps_hash_volume* v, const gps_camera* cams, int n_views, float* const* out_depth,
                               float* const* out_rgb, float z_near, float step, float* range, hipStream_t s);

}  // namespace gps
