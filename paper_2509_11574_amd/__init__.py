"""MI355X (gfx950) implementation of the Gaussian-plus-SDF mapping path.

The compute lives in libgps.so (hand-written HIP kernels behind the C ABI of
include/gps.h); ``gps`` is its thin ctypes binding with torch.autograd wrappers.
"""
from . import gps
from .gps import (Adam, Camera, GpsError, Render, RenderCfg, RenderLoss, Session, View, Volume, Workspace,
                  adam_step, camera, fuse, gaussians_to_device, insert_gaussians, lib, raycast, remove_gaussians,
                  render_bwd, render_fwd, workspace_size, zeros_like_gaussians, PAPER_LR, TILE_CONFIGS)

__all__ = ["gps", "Adam", "Camera", "GpsError", "Render", "RenderCfg", "RenderLoss", "Session", "View", "Volume",
           "Workspace", "adam_step", "camera", "fuse", "gaussians_to_device", "insert_gaussians", "lib", "raycast",
           "remove_gaussians", "render_bwd", "render_fwd", "workspace_size", "zeros_like_gaussians", "PAPER_LR", "TILE_CONFIGS"]
