"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only produces inputs: analytic scenes (spheres, boxes and an
inward-facing room box with procedural stripe/checker albedo), pinhole camera
poses, RGB-D frames obtained by exact ray/primitive intersection, and seeded
initial Gaussians.  It holds none of the mapping method's own arithmetic (no
TSDF fusion, no voxel raycast, no splatting, no loss or optimiser), and it
imports neither the product package nor the reference implementation.

Seeds (NumPy PCG64): 0 geometry, 1 albedo, 2 trajectory, 3 depth noise,
4 Gaussians.
"""
from .scene import (Camera, Scene, look_at, intrinsics_for, scene_small, scene_room, orbit_cameras,
                    render_frame, seed_gaussians, surface_points, workload_small, workload_room_frames,
                    insertion_inputs, STANDARD_VIEWS)

__all__ = ["Camera", "Scene", "look_at", "intrinsics_for", "scene_small", "scene_room", "orbit_cameras",
           "render_frame", "seed_gaussians", "surface_points", "workload_small", "workload_room_frames",
           "insertion_inputs", "STANDARD_VIEWS"]
