"""MI355X (gfx950) implementation of the Gaussian-plus-SDF mapping path.

The compute lives in libgps.so (hand-written HIP kernels behind the C ABI of
include/gps.h); ``gps`` is its thin ctypes binding with torch.autograd wrappers.
"""
from . import gps
from .gps import (Adam, Camera, GpsError, HashVolume, Render, RenderCfg, RenderLoss, Session, View, Volume, Workspace,
                  adam_step, camera, depth_downsample, fuse, gaussians_to_device, icp_reduce, icp_reduce_noalloc,
                  icp_solve, icp_step, icp_track, hash_fuse, hash_raycast, insert_gaussians, lib, pose_tensor, raycast, remove_gaussians,
                  render_bwd, render_bwd_adam, render_fwd, workspace_size, zeros_like_gaussians, PAPER_LR, TILE_CONFIGS)

__all__ = ["gps", "Adam", "Camera", "GpsError", "HashVolume", "Render", "RenderCfg", "RenderLoss", "Session", "View", "Volume",
           "Workspace", "adam_step", "camera", "depth_downsample", "fuse", "gaussians_to_device", "icp_reduce",
           "icp_reduce_noalloc", "icp_solve", "icp_step", "icp_track", "hash_fuse", "hash_raycast", "insert_gaussians", "lib", "pose_tensor", "raycast",
           "remove_gaussians", "render_bwd", "render_bwd_adam", "render_fwd", "workspace_size", "zeros_like_gaussians", "PAPER_LR", "TILE_CONFIGS"]
