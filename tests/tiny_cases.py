"""Small seeded inputs for the CPU pins (shared by oracle and GPU parity tests;
no arithmetic of the method lives here)."""
from __future__ import annotations

import math

import numpy as np


def rot_xyz(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rz = np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


class RCfg:
    """Plain renderer constants (mirrors oracle.RenderCfg without importing it)."""

    def __init__(self, mode=0, eps_cull=0.02, lambda_depth=1.0, dilation=0.3, alpha_min=1 / 255,
                 alpha_max=0.99, T_min=1e-4, z_near=0.2):
        r32 = lambda v: float(np.float32(v))  # the values a float32 configuration field holds
        self.mode = mode
        self.eps_cull, self.lambda_depth, self.dilation = r32(eps_cull), r32(lambda_depth), r32(dilation)
        self.alpha_min, self.alpha_max, self.T_min, self.z_near = r32(alpha_min), r32(alpha_max), r32(T_min), r32(z_near)


def tiny_case(seed=0, M=30, W=40, H=30, f=40.0, log_scale=-2.6, invalid_frac=0.1, rotate=True):
    """A non-trivial camera (rotated, translated), random base colour/depth (some invalid),
    and M Gaussians in front of it spread over the view at depths 1.0-2.4 m."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    R = rot_xyz(*(rng.uniform(-0.4, 0.4, 3))) if rotate else np.eye(3)
    t = rng.uniform(-0.3, 0.3, 3) if rotate else np.zeros(3)
    r32 = lambda v: float(np.float32(v))  # intrinsics exactly as a float32 camera holds them
    cam = {"width": W, "height": H, "fx": r32(f), "fy": r32(f * 1.05), "cx": r32(W / 2 - 0.3),
           "cy": r32(H / 2 + 0.2), "R": R.astype(np.float32), "t": t.astype(np.float32)}
    # camera-frame positions -> world
    z = rng.uniform(1.0, 2.4, M)
    u = rng.uniform(-2, W + 2, M)
    v = rng.uniform(-2, H + 2, M)
    pc = np.stack([(u - cam["cx"]) / cam["fx"] * z, (v - cam["cy"]) / cam["fy"] * z, z])
    Rd = cam["R"].astype(np.float64)
    mean = Rd.T @ (pc - cam["t"].astype(np.float64)[:, None])
    q = rng.normal(size=(4, M))
    q /= np.linalg.norm(q, axis=0)
    q *= rng.uniform(0.7, 1.4, M)  # not unit: exercises the normalisation
    g = {"mean": mean.astype(np.float32),
         "log_scale": (log_scale + 0.3 * rng.normal(size=(3, M))).astype(np.float32),
         "quat": q.astype(np.float32),
         "opacity_logit": rng.normal(0.0, 1.0, M).astype(np.float32),
         "rgb": rng.uniform(0, 1, (3, M)).astype(np.float32)}
    base_rgb = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    base_depth = rng.uniform(1.2, 2.6, (H, W)).astype(np.float32)
    base_depth[rng.uniform(size=(H, W)) < invalid_frac] = 0.0
    target_rgb = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    target_depth = rng.uniform(1.0, 2.6, (H, W)).astype(np.float32)
    target_depth[rng.uniform(size=(H, W)) < invalid_frac] = 0.0
    return {"cam": cam, "gauss": g, "base_rgb": base_rgb, "base_depth": base_depth,
            "target_rgb": target_rgb, "target_depth": target_depth}
