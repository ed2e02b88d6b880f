"""Analytic scenes, camera trajectories, RGB-D frames and initial Gaussians.

Everything is computed in float64 with torch (CPU or GPU) and returned as
float32 NumPy arrays (or float32 torch tensors on the requested device) in the
planar layouts the rest of the project uses: depth [H][W] (metres, 0 = no
surface), rgb [3][H][W] in [0,1], Gaussians as [3][M] / [4][M] / [M] arrays.

Camera convention: world -> camera rigid transform p_c = R p_w + t, with the
camera looking along +z, x to the right and y down; pinhole projection
u = fx x/z + cx, v = fy y/z + cy with pixel (col, row) sampled at (col, row).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


# --------------------------------------------------------------------------- #
# Cameras                                                                      #
# --------------------------------------------------------------------------- #
@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3,3) float32, world -> camera
    t: np.ndarray  # (3,) float32

    def as_dict(self):
        return {"width": self.width, "height": self.height, "fx": self.fx, "fy": self.fy, "cx": self.cx,
                "cy": self.cy, "R": self.R.copy(), "t": self.t.copy()}

    @property
    def center(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for a camera at `eye` looking at `target` (x right, y down, z forward)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def intrinsics_for(width: int, height: int):
    """Intrinsics for the larger frames: fx = fy = 0.9375 W, principal point at the image centre
    (this keeps the 56-degree horizontal field of view of the 160x120, f=150 frame)."""
    f = 0.9375 * width
    return f, f, width / 2.0, height / 2.0


# --------------------------------------------------------------------------- #
# Scenes                                                                       #
# --------------------------------------------------------------------------- #
@dataclass
class Scene:
    sph_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    sph_r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    box_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    box_h: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    room_lo: np.ndarray | None = None
    room_hi: np.ndarray | None = None
    # albedo per primitive, in the order spheres, boxes, room:
    pat_kind: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))  # 0 stripes, 1 checker
    pat_period: np.ndarray = field(default_factory=lambda: np.zeros(0))
    pat_axis: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    col_a: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    col_b: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    # the volume the scene is meant to be fused into
    dims: tuple = (64, 64, 64)
    origin: tuple = (0.0, 0.0, 0.0)
    voxel: float = 0.02
    trunc: float = 0.08

    @property
    def n_prims(self):
        return len(self.sph_r) + len(self.box_h) + (1 if self.room_lo is not None else 0)


def _albedo_params(rng, n, period_lo, period_hi):
    kind = rng.integers(0, 2, size=n)
    period = rng.uniform(period_lo, period_hi, size=n)
    axis = rng.integers(0, 3, size=n)
    ca = rng.uniform(0.05, 0.95, size=(n, 3))
    cb = rng.uniform(0.05, 0.95, size=(n, 3))
    return kind, period, axis, ca, cb


def scene_small(seed_geom: int = 0, seed_albedo: int = 1) -> Scene:
    """64^3 lattice at 2 cm over a 1.26 m cube: 6 spheres (r ~ U[0.08, 0.2] m) and 4 axis-aligned
    boxes (half-extents ~ U[0.05, 0.15] m) at seeded positions inside; union of the primitives.
    Stripe or checker albedo with periods ~ U[3, 10] cm and two colours per primitive."""
    rng = np.random.Generator(np.random.PCG64(seed_geom))
    ext = 0.02 * 63
    sph_r = rng.uniform(0.08, 0.2, size=6)
    sph_c = np.stack([rng.uniform(0.25 + r, ext - 0.25 - r, size=3) for r in sph_r])
    box_h = rng.uniform(0.05, 0.15, size=(4, 3))
    box_c = np.stack([rng.uniform(0.25 + h, ext - 0.25 - h) for h in box_h])
    rng_a = np.random.Generator(np.random.PCG64(seed_albedo))
    kind, period, axis, ca, cb = _albedo_params(rng_a, 10, 0.03, 0.10)
    return Scene(sph_c=sph_c, sph_r=sph_r, box_c=box_c, box_h=box_h, pat_kind=kind, pat_period=period,
                 pat_axis=axis, col_a=ca, col_b=cb, dims=(64, 64, 64), origin=(0.0, 0.0, 0.0), voxel=0.02,
                 trunc=0.08)


def scene_room(n: int = 256, seed_geom: int = 0, seed_albedo: int = 1) -> Scene:
    """A 2.56 m room fused into an n^3 lattice (256 -> 1 cm voxels, 512 -> 5 mm): floor, ceiling and
    four walls inset 5 cm from the lattice boundary, plus 20 seeded spheres and boxes placed between
    the camera orbit and the walls; textured (stripe/checker) albedo everywhere."""
    rng = np.random.Generator(np.random.PCG64(seed_geom))
    side = 2.56
    voxel = side / n
    centre = np.array([side / 2, side / 2, side / 2])
    n_sph, n_box = 10, 10

    def place(k, size):
        ang = rng.uniform(0, 2 * math.pi, size=k)
        rad = rng.uniform(0.78, 1.02, size=k)
        zz = rng.uniform(0.25, 2.25, size=k)
        zz = np.maximum(zz, 0.05 + size)  # stand on or above the floor
        return np.stack([centre[0] + rad * np.cos(ang), centre[1] + rad * np.sin(ang), zz], axis=1)

    sph_r = rng.uniform(0.08, 0.2, size=n_sph)
    sph_c = place(n_sph, sph_r)
    box_h = rng.uniform(0.05, 0.15, size=(n_box, 3))
    box_c = place(n_box, box_h[:, 2])
    rng_a = np.random.Generator(np.random.PCG64(seed_albedo))
    kind, period, axis, ca, cb = _albedo_params(rng_a, n_sph + n_box + 1, 0.03, 0.12)
    kind[-1], period[-1] = 1, 0.25  # the room: a 25 cm checker
    return Scene(sph_c=sph_c, sph_r=sph_r, box_c=box_c, box_h=box_h, room_lo=np.full(3, 0.05),
                 room_hi=np.full(3, side - 0.05), pat_kind=kind, pat_period=period, pat_axis=axis, col_a=ca,
                 col_b=cb, dims=(n, n, n), origin=(0.0, 0.0, 0.0), voxel=voxel, trunc=4 * voxel)


# --------------------------------------------------------------------------- #
# Exact ray casting of the analytic primitives                                 #
# --------------------------------------------------------------------------- #
def _cast(scene: Scene, o, d):
    """o (3,) and d [N,3] unit (float64 torch).  Returns t [N] (inf = miss), prim id [N], normal [N,3]."""
    N = d.shape[0]
    dev = d.device
    best = torch.full((N,), math.inf, dtype=torch.float64, device=dev)
    pid = torch.full((N,), -1, dtype=torch.int64, device=dev)
    nrm = torch.zeros((N, 3), dtype=torch.float64, device=dev)
    tmin = 1e-6
    k = 0
    for c, r in zip(scene.sph_c, scene.sph_r):
        c = torch.as_tensor(c, dtype=torch.float64, device=dev)
        oc = o - c
        b = d @ oc
        cc = float(oc @ oc) - float(r) ** 2
        disc = b * b - cc
        ok = disc >= 0
        sq = torch.sqrt(torch.clamp(disc, min=0))
        t0 = -b - sq
        t1 = -b + sq
        t = torch.where(t0 > tmin, t0, t1)
        hit = ok & (t > tmin) & (t < best)
        best = torch.where(hit, t, best)
        pid = torch.where(hit, torch.full_like(pid, k), pid)
        p = o + t[:, None] * d
        nrm = torch.where(hit[:, None], (p - c) / float(r), nrm)
        k += 1
    for c, h in zip(scene.box_c, scene.box_h):
        c = torch.as_tensor(c, dtype=torch.float64, device=dev)
        h = torch.as_tensor(h, dtype=torch.float64, device=dev)
        with torch.no_grad():
            inv = 1.0 / torch.where(d.abs() < 1e-300, torch.full_like(d, 1e-300), d)
            t1 = (c - h - o) * inv
            t2 = (c + h - o) * inv
            tn = torch.minimum(t1, t2).max(dim=1).values
            tf = torch.maximum(t1, t2).min(dim=1).values
        hit = (tn <= tf) & (tn > tmin) & (tn < best)
        best = torch.where(hit, tn, best)
        pid = torch.where(hit, torch.full_like(pid, k), pid)
        p = o + tn[:, None] * d
        q = (p - c) / h
        ax = q.abs().argmax(dim=1)
        n = torch.zeros_like(d)
        n.scatter_(1, ax[:, None], torch.sign(q.gather(1, ax[:, None])))
        nrm = torch.where(hit[:, None], n, nrm)
        k += 1
    if scene.room_lo is not None:
        lo = torch.as_tensor(scene.room_lo, dtype=torch.float64, device=dev)
        hi = torch.as_tensor(scene.room_hi, dtype=torch.float64, device=dev)
        inv = 1.0 / torch.where(d.abs() < 1e-300, torch.full_like(d, 1e-300), d)
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        tf_ax = torch.maximum(t1, t2)
        tf, ax = tf_ax.min(dim=1)
        hit = (tf > tmin) & (tf < best)
        best = torch.where(hit, tf, best)
        pid = torch.where(hit, torch.full_like(pid, k), pid)
        n = torch.zeros_like(d)
        n.scatter_(1, ax[:, None], -torch.sign(d.gather(1, ax[:, None])))
        nrm = torch.where(hit[:, None], n, nrm)
    return best, pid, nrm


def _albedo(scene: Scene, p, pid):
    dev = p.device
    kind = torch.as_tensor(scene.pat_kind, device=dev)
    per = torch.as_tensor(scene.pat_period, dtype=torch.float64, device=dev)
    axis = torch.as_tensor(scene.pat_axis, device=dev)
    ca = torch.as_tensor(scene.col_a, dtype=torch.float64, device=dev)
    cb = torch.as_tensor(scene.col_b, dtype=torch.float64, device=dev)
    ok = pid >= 0
    q = torch.clamp(pid, min=0)
    cell = torch.floor(p / per[q][:, None]).to(torch.int64)
    stripe = cell.gather(1, axis[q][:, None])[:, 0]
    checker = cell.sum(dim=1)
    sel = torch.where(kind[q] == 0, stripe, checker) % 2 == 0
    col = torch.where(sel[:, None], ca[q], cb[q])
    return torch.where(ok[:, None], col, torch.zeros_like(col))


def _rays(cam: Camera, dev):
    H, W = cam.height, cam.width
    jj, ii = torch.meshgrid(torch.arange(H, dtype=torch.float64, device=dev),
                            torch.arange(W, dtype=torch.float64, device=dev), indexing="ij")
    r = torch.stack([(ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy, torch.ones_like(ii)], dim=-1).reshape(-1, 3)
    rn = r.norm(dim=1)
    R = torch.as_tensor(cam.R.astype(np.float64), device=dev)
    d = (r / rn[:, None]) @ R  # R^T r / |r|
    o = torch.as_tensor(cam.center, dtype=torch.float64, device=dev)
    return o, d, rn


def render_frame(scene: Scene, cam: Camera, noise_sigma_per_m2: float = 0.0, seed_noise: int = 3,
                 frame_index: int = 0, device="cpu", as_torch: bool = False):
    """Exact RGB-D frame of the analytic scene: depth = camera z of the first surface (0 = miss),
    rgb = albedo there.  Optional depth noise N(0, (noise_sigma_per_m2 * z^2)^2)."""
    dev = torch.device(device)
    o, d, rn = _rays(cam, dev)
    t, pid, _ = _cast(scene, o, d)
    hit = torch.isfinite(t)
    z = torch.where(hit, t / rn, torch.zeros_like(t))
    p = o + torch.where(hit, t, torch.zeros_like(t))[:, None] * d
    col = _albedo(scene, p, pid)
    if noise_sigma_per_m2 > 0:
        rng = np.random.Generator(np.random.PCG64([seed_noise, frame_index]))
        eps = torch.as_tensor(rng.standard_normal(z.shape[0]), device=dev)
        z = torch.where(hit, z + noise_sigma_per_m2 * z * z * eps, z)
        z = torch.clamp(z, min=0)
    H, W = cam.height, cam.width
    depth = z.reshape(H, W).to(torch.float32)
    rgb = col.T.reshape(3, H, W).to(torch.float32)
    if as_torch:
        return depth.contiguous(), rgb.contiguous()
    return np.ascontiguousarray(depth.cpu().numpy()), np.ascontiguousarray(rgb.cpu().numpy())


def surface_points(scene: Scene, cam: Camera, pix: np.ndarray, device="cpu"):
    """World points and unit normals of the first surface seen through the listed pixels (float64)."""
    dev = torch.device(device)
    o, d, _ = _rays(cam, dev)
    sel = torch.as_tensor(pix, device=dev)
    t, pid, n = _cast(scene, o, d[sel])
    p = o + t[:, None] * d[sel]
    return p.cpu().numpy(), n.cpu().numpy(), np.isfinite(t.cpu().numpy())


# --------------------------------------------------------------------------- #
# Trajectories                                                                 #
# --------------------------------------------------------------------------- #
def orbit_cameras(n_frames: int, width: int, height: int, side: float = 2.56, seed_traj: int = 2,
                  frames=None):
    """Smooth seeded orbit: radius 0.5 m about the room centre, height bob +-0.1 m, each camera
    looking across the room through a point 1 m beyond the centre."""
    rng = np.random.Generator(np.random.PCG64(seed_traj))
    th0 = rng.uniform(0, 2 * math.pi)
    yaw_off = rng.uniform(-0.3, 0.3)
    c = np.full(3, side / 2)
    fx, fy, cx, cy = intrinsics_for(width, height)
    cams = []
    idx = range(n_frames) if frames is None else frames
    for k in idx:
        th = th0 + 2 * math.pi * k / 100.0
        eye = c + np.array([0.5 * math.cos(th), 0.5 * math.sin(th), 0.1 * math.sin(2 * th)])
        tgt = c + np.array([math.cos(th + math.pi + yaw_off), math.sin(th + math.pi + yaw_off), -0.1])
        R, t = look_at(eye, tgt)
        cams.append(Camera(width, height, fx, fy, cx, cy, R, t))
    return cams


def small_camera() -> Camera:
    """160x120, f = 150, principal point (80, 60), about 1.6 m from the cube centre looking at it."""
    c = np.full(3, 0.02 * 63 / 2)
    eye = c + 1.6 * np.array([math.cos(0.6) * math.cos(0.35), math.sin(0.6) * math.cos(0.35), math.sin(0.35)])
    R, t = look_at(eye, c)
    return Camera(160, 120, 150.0, 150.0, 80.0, 60.0, R, t)


# --------------------------------------------------------------------------- #
# Gaussians                                                                    #
# --------------------------------------------------------------------------- #
def seed_gaussians(scene: Scene, cams, depth_frames, M: int, seed: int = 4, normal_sigma=None,
                   log_scale_mean=-4.5, log_scale_std=0.3):
    """M Gaussians at seeded surface points seen by the given frames, offset along the surface
    normal by N(0, (0.5 voxel)^2); log-scales ~ N(-4.5, 0.3) per axis, opacity logits ~ N(0, 1),
    rgb ~ U[0, 1], quaternion = normalise(N(0, I_4))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if normal_sigma is None:
        normal_sigma = 0.5 * scene.voxel
    nf = len(cams)
    means = np.zeros((M, 3))
    filled = 0
    while filled < M:
        need = M - filled
        fi = rng.integers(0, nf, size=need)
        out = []
        for f in range(nf):
            k = np.nonzero(fi == f)[0]
            if k.size == 0:
                continue
            dep = np.asarray(depth_frames[f]).reshape(-1)
            valid = np.nonzero(dep > 0)[0]
            pix = valid[rng.integers(0, valid.size, size=k.size)]
            p, n, ok = surface_points(scene, cams[f], pix)
            off = rng.normal(0.0, normal_sigma, size=k.size)
            out.append((p + off[:, None] * n)[ok])
        got = np.concatenate(out, axis=0)[:need]
        means[filled:filled + got.shape[0]] = got
        filled += got.shape[0]
    log_scale = rng.normal(log_scale_mean, log_scale_std, size=(3, M))
    opacity_logit = rng.normal(0.0, 1.0, size=M)
    rgb = rng.uniform(0.0, 1.0, size=(3, M))
    q = rng.normal(0.0, 1.0, size=(4, M))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {"mean": f32(means.T), "log_scale": f32(log_scale), "quat": f32(q),
            "opacity_logit": f32(opacity_logit), "rgb": f32(rgb)}


# --------------------------------------------------------------------------- #
# Standard workloads                                                           #
# --------------------------------------------------------------------------- #
def workload_small(M: int = 2000):
    """64^3 at 2 cm, one noise-free 160x120 frame, truncation 8 cm, M Gaussians near the surface."""
    scene = scene_small()
    cam = small_camera()
    depth, rgb = render_frame(scene, cam)
    g = seed_gaussians(scene, [cam], [depth], M)
    return {"scene": scene, "cam": cam, "depth": depth, "rgb": rgb, "gauss": g}


def workload_room_frames(n: int = 256, width: int = 1280, height: int = 720, frames=range(1),
                         noise: float = 1e-3, device="cpu", as_torch=False):
    """Frames of the room orbit (depth noise sigma = noise * z^2, i.e. 1 mm at 1 m)."""
    scene = scene_room(n)
    cams = orbit_cameras(0, width, height, frames=list(frames))
    out = []
    for k, cam in zip(frames, cams):
        d, c = render_frame(scene, cam, noise_sigma_per_m2=noise, frame_index=k, device=device,
                            as_torch=as_torch)
        out.append((cam, d, c))
    return scene, out


# Views of the mixed-resolution keyframe batch: frame index and resolution.
STANDARD_VIEWS = [(0, 1280, 720), (12, 1280, 720), (25, 1280, 720), (37, 640, 480), (50, 640, 480),
                  (62, 640, 480), (75, 320, 240), (87, 320, 240)]


def insertion_inputs(scene: Scene, cam: Camera, seed: int = 5, hole_fraction: float = 0.02,
                     noise_sigma_per_m2: float = 0.002, device="cpu"):
    """Inputs of one Gaussian-insertion call for a frame of `scene` seen from `cam`: the
    frame's depth (with noise and seeded holes, 0 = no surface) and colour, a stand-in for
    the current map's rendering (the frame colour plus seeded per-pixel noise of sigma 0.05
    and, on a quarter of 8x8 blocks, an offset of 0.15), a Gaussian weight uniform in
    [0, 8) and the uniform draw in [0, 1).  All float32 numpy arrays, planar."""
    depth, rgb = render_frame(scene, cam, noise_sigma_per_m2=noise_sigma_per_m2, device=device)
    H, W = depth.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    depth = np.where(rng.uniform(size=(H, W)) < hole_fraction, 0.0, depth).astype(np.float32)
    blocks = rng.uniform(size=((H + 7) // 8, (W + 7) // 8)) < 0.25
    offset = np.kron(blocks, np.ones((8, 8)))[:H, :W] * 0.15
    render = (rgb + rng.normal(0.0, 0.05, size=rgb.shape) + offset[None]).astype(np.float32)
    weight = rng.uniform(0.0, 8.0, size=(H, W)).astype(np.float32)
    draw = rng.uniform(size=(H, W)).astype(np.float32)
    return tuple(np.ascontiguousarray(a, np.float32) for a in (render, rgb, weight, depth, draw))
