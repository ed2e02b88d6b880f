"""Thin Python binding of libgps (include/gps.h): ctypes argument marshalling only.

Every step of the mapping path runs in the HIP kernels of libgps.so; this
module converts torch tensors to device pointers, forwards the current HIP
stream and raises on any non-OK status.  There is no fallback: importing it
without the built library raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgps.so")
MAX_VIEWS = 16

OK = 0
STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "capacity exceeded",
                -4: "HIP error", -5: "unsupported device", -6: "unsupported config"}


class GpsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({status})")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3)]


class VolumeS(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("voxel", ctypes.c_float), ("trunc", ctypes.c_float),
                ("max_weight", ctypes.c_float), ("tsdf", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("rgb_weight", ctypes.c_void_p), ("brick_min", ctypes.c_void_p)]


class HashVolumeS(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("voxel", ctypes.c_float), ("trunc", ctypes.c_float),
                ("max_weight", ctypes.c_float), ("n_buckets", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("keys", ctypes.c_void_p), ("slots", ctypes.c_void_p), ("block_key", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("visible", ctypes.c_void_p), ("block_min", ctypes.c_void_p),
                ("tsdf", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("rgb_weight", ctypes.c_void_p)]


class GaussiansS(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("sh_degree", ctypes.c_int32), ("sh", ctypes.c_void_p)]


class ViewS(ctypes.Structure):
    _fields_ = [("cam", Camera), ("base_rgb", ctypes.c_void_p), ("base_depth", ctypes.c_void_p),
                ("target_rgb", ctypes.c_void_p), ("target_depth", ctypes.c_void_p),
                ("out_rgb", ctypes.c_void_p), ("out_depth", ctypes.c_void_p), ("pose_xi", ctypes.c_void_p),
                ("out_aux", ctypes.c_void_p)]


class RenderCfgS(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("pix_per_thread", ctypes.c_int32), ("mode", ctypes.c_int32), ("eps_cull", ctypes.c_float),
                ("lambda_depth", ctypes.c_float), ("dilation", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float), ("z_near", ctypes.c_float),
                ("max_instances", ctypes.c_int64), ("flags", ctypes.c_int32)]


class RemovalCfgS(ctypes.Structure):
    _fields_ = [("min_opacity", ctypes.c_float), ("max_scale", ctypes.c_float), ("min_scale", ctypes.c_float)]


class InsertCfgS(ctypes.Structure):
    _fields_ = [("delta_c", ctypes.c_float), ("delta_w", ctypes.c_float), ("fraction", ctypes.c_float),
                ("scale_cap", ctypes.c_float), ("flat_ratio", ctypes.c_float),
                ("opacity", ctypes.c_float)]


class AdamGroupS(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("n", ctypes.c_int64), ("lr", ctypes.c_float)]


class StatsS(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_views", ctypes.c_int32), ("n_instances", ctypes.c_int64),
                ("capacity", ctypes.c_int64), ("sort_fallback", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("pairs_eval", ctypes.c_int64), ("pairs_contrib", ctypes.c_int64),
                ("loss", ctypes.c_float), ("view_omega", ctypes.c_float * MAX_VIEWS)]


class KernelTimeS(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


ABI_VERSION = 5  # include/gps.h GPS_ABI_VERSION

EXPORTS = ["gps_abi_version", "gps_status_string", "gps_render_cfg_default", "gps_workspace_size",
           "gps_workspace_reset", "gps_fuse", "gps_raycast", "gps_render_fwd", "gps_render_bwd",
           "gps_adam_step", "gps_device_status", "gps_read_stats", "gps_profile_start", "gps_profile_stop",
           "gps_profile_read", "gps_views_upload", "gps_removal_cfg_default", "gps_removal_workspace_size",
           "gps_remove_gaussians", "gps_insert_cfg_default", "gps_insertion_workspace_size",
           "gps_insert_gaussians", "gps_depth_downsample", "gps_icp_workspace_size", "gps_icp_reduce",
           "gps_icp_solve", "gps_render_bwd_adam", "gps_level_camera", "gps_icp_reduce_noalloc",
           "gps_hash_reset", "gps_hash_fuse", "gps_hash_raycast", "gps_stream_blocks", "gps_stream_read",
           "gps_stream_write", "gps_icp_step"]

_lib = None


def lib():
    """Load libgps.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_11574_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        L.gps_abi_version.restype = ctypes.c_int32
        if L.gps_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI {L.gps_abi_version()}, this binding needs {ABI_VERSION}: rebuild it")
        P, I32, I64, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        L.gps_abi_version.restype = I32
        L.gps_status_string.argtypes = [I32]
        L.gps_status_string.restype = ctypes.c_char_p
        L.gps_render_cfg_default.argtypes = [P]
        L.gps_render_cfg_default.restype = None
        L.gps_workspace_size.argtypes = [P, I32, P, I32, ctypes.POINTER(ctypes.c_size_t)]
        L.gps_workspace_reset.argtypes = [P, ctypes.c_size_t, P]
        L.gps_fuse.argtypes = [P, P, P, P, P]
        L.gps_raycast.argtypes = [P, P, I32, P, P, F, F, P]
        L.gps_render_fwd.argtypes = [P, P, P, I32, P, ctypes.c_size_t, P, P]
        L.gps_render_bwd.argtypes = [P, P, P, I32, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.gps_adam_step.argtypes = [P, I32, I32, P, F, F, F, P]
        L.gps_device_status.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(I32), P]
        L.gps_read_stats.argtypes = [P, ctypes.c_size_t, P, P]
        L.gps_views_upload.argtypes = [P, P, P, I32, P, P, P, ctypes.c_size_t, P]
        L.gps_profile_start.argtypes = []
        L.gps_profile_stop.argtypes = []
        L.gps_profile_read.argtypes = [P, I32, ctypes.POINTER(I32)]
        L.gps_removal_cfg_default.argtypes = [P]
        L.gps_removal_cfg_default.restype = None
        L.gps_removal_workspace_size.argtypes = [I32, ctypes.POINTER(ctypes.c_size_t)]
        L.gps_remove_gaussians.argtypes = [P, P, P, I32, P, P, ctypes.c_size_t, P]
        L.gps_insert_cfg_default.argtypes = [P]
        L.gps_insert_cfg_default.restype = None
        L.gps_insertion_workspace_size.argtypes = [I32, I32, ctypes.POINTER(ctypes.c_size_t)]
        L.gps_insert_gaussians.argtypes = [P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.gps_depth_downsample.argtypes = [P, I32, I32, P, P]
        L.gps_icp_workspace_size.argtypes = [I32, I32, ctypes.POINTER(ctypes.c_size_t)]
        L.gps_icp_reduce.argtypes = [P, P, P, P, P, F, P, P, ctypes.c_size_t, P]
        L.gps_icp_reduce_noalloc.argtypes = [P, P, P, P, P, F, P, P]
        L.gps_icp_step.argtypes = [P, P, P, P, P, F, P, P, P, ctypes.c_size_t, P]
        L.gps_hash_reset.argtypes = [P, P]
        L.gps_stream_blocks.restype = I32
        L.gps_stream_read.argtypes = [P, ctypes.c_size_t, P, P]
        L.gps_stream_write.argtypes = [P, ctypes.c_size_t, F, P]
        L.gps_hash_fuse.argtypes = [P, P, P, P, P]
        L.gps_hash_raycast.argtypes = [P, P, I32, P, P, F, F, P, ctypes.c_size_t, P]
        L.gps_icp_solve.argtypes = [P, P, P, P]
        L.gps_render_bwd_adam.argtypes = [P, P, P, I32, P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.gps_level_camera.argtypes = [P, I32, P]
        for n in EXPORTS:
            if n not in ("gps_render_cfg_default", "gps_status_string", "gps_abi_version", "gps_removal_cfg_default",
                         "gps_insert_cfg_default"):
                getattr(L, n).restype = I32
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != OK:
        raise GpsError(st, what)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, name="tensor", numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype not in (torch.float32, torch.int32, torch.int64, torch.uint8):
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------- #
# Cameras, volumes, Gaussians                                                  #
# --------------------------------------------------------------------------- #
def camera(c) -> Camera:
    """From a dict or object with width, height, fx, fy, cx, cy, R (3x3), t (3)."""
    if isinstance(c, Camera):
        return c
    g = (lambda k: c[k]) if isinstance(c, dict) else (lambda k: getattr(c, k))
    out = Camera()
    out.width, out.height = int(g("width")), int(g("height"))
    out.fx, out.fy, out.cx, out.cy = (float(g(k)) for k in ("fx", "fy", "cx", "cy"))
    R = np.asarray(g("R"), np.float32).reshape(9)
    t = np.asarray(g("t"), np.float32).reshape(3)
    for k in range(9):
        out.R[k] = float(R[k])
    for k in range(3):
        out.t[k] = float(t[k])
    return out


@dataclass
class Volume:
    """Dense colourised TSDF lattice on the GPU (planar float32 arrays)."""
    dims: tuple
    origin: tuple
    voxel: float
    trunc: float
    max_weight: float = 100.0
    device: str = "cuda"
    skip_bricks: bool = True
    tsdf: torch.Tensor = field(init=False)
    weight: torch.Tensor = field(init=False)
    rgb: torch.Tensor = field(init=False)
    rgb_weight: torch.Tensor = field(init=False)
    brick_min: torch.Tensor | None = field(init=False)

    def __post_init__(self):
        nx, ny, nz = (int(d) for d in self.dims)
        N = nx * ny * nz
        self.tsdf = torch.ones(N, dtype=torch.float32, device=self.device)
        self.weight = torch.zeros(N, dtype=torch.float32, device=self.device)
        self.rgb = torch.zeros(3, N, dtype=torch.float32, device=self.device)
        self.rgb_weight = torch.zeros(N, dtype=torch.float32, device=self.device)
        bx, by, bz = (math.ceil(d / 8) for d in (nx, ny, nz))
        nb = bx * by * bz + math.ceil(bx / 4) * math.ceil(by / 4) * math.ceil(bz / 4)  # GPS_BRICK_MIN_FLOATS
        self.brick_min = torch.zeros(nb, dtype=torch.float32, device=self.device) if self.skip_bricks else None

    def struct(self) -> VolumeS:
        s = VolumeS()
        s.nx, s.ny, s.nz = (int(d) for d in self.dims)
        for k in range(3):
            s.origin[k] = float(self.origin[k])
        s.voxel, s.trunc, s.max_weight = float(self.voxel), float(self.trunc), float(self.max_weight)
        N = s.nx * s.ny * s.nz
        s.tsdf = _ptr(self.tsdf, "tsdf", N)
        s.weight = _ptr(self.weight, "weight", N)
        s.rgb = _ptr(self.rgb, "rgb", 3 * N)
        s.rgb_weight = _ptr(self.rgb_weight, "rgb_weight", N)
        s.brick_min = _ptr(self.brick_min, "brick_min") if self.brick_min is not None else None
        return s


GAUSS_KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
GAUSS_ROWS = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "rgb": 3}


# SH bands above degree 0 (optional key "sh", [3][K][M]): coefficients per channel for
# degree 1, 2, 3, and back
SH_COEFFS = {0: 0, 1: 3, 2: 8, 3: 15}
SH_DEGREE_OF = {v: k for k, v in SH_COEFFS.items()}


def gauss_keys(g: dict) -> tuple:
    """The attribute keys of a Gaussian dict: the five, plus "sh" when it carries SH bands."""
    return GAUSS_KEYS + (("sh",) if g.get("sh") is not None else ())


def sh_degree(g: dict) -> int:
    sh = g.get("sh")
    if sh is None:
        return 0
    if sh.dim() != 3 or sh.shape[0] != 3 or sh.shape[1] not in SH_DEGREE_OF:
        raise ValueError("sh must have shape [3, K, M] with K = 3, 8 or 15")
    return SH_DEGREE_OF[int(sh.shape[1])]


def gaussians_struct(g: dict) -> GaussiansS:
    M = int(g["opacity_logit"].numel())
    s = GaussiansS()
    s.count = M
    for k in GAUSS_KEYS:
        setattr(s, k, _ptr(g[k], k, GAUSS_ROWS[k] * M))
    L = sh_degree(g)
    s.sh_degree = L
    s.sh = _ptr(g["sh"], "sh", 3 * SH_COEFFS[L] * M) if L > 0 else None
    return s


def gaussians_to_device(g: dict, device="cuda") -> dict:
    keys = GAUSS_KEYS + (("sh",) if g.get("sh") is not None else ())
    return {k: torch.as_tensor(np.ascontiguousarray(g[k], np.float32)).to(device) for k in keys}


def zeros_like_gaussians(g: dict) -> dict:
    return {k: torch.zeros_like(g[k]) for k in gauss_keys(g)}


@dataclass
class RenderCfg:
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 256
    pix_per_thread: int = 1
    mode: int = 0
    eps_cull: float = 0.01
    lambda_depth: float = 1.0
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    z_near: float = 0.2
    max_instances: int = 0
    views_preset: bool = False  # read the view table uploaded by views_upload (for graph replay)
    bwd_per_gaussian: bool = False  # sort-free mode: per-Gaussian backward over pixel chunks (Appendix B)
    no_sort: bool = False  # sort-free mode: no per-tile depth sort (lists in emission order)

    def struct(self) -> RenderCfgS:
        return RenderCfgS(self.tile_w, self.tile_h, self.batch, self.pix_per_thread, self.mode, self.eps_cull,
                          self.lambda_depth, self.dilation, self.alpha_min, self.alpha_max, self.T_min,
                          self.z_near, int(self.max_instances),
                          (1 if self.views_preset else 0) | (2 if self.bwd_per_gaussian else 0) |
                          (4 if self.no_sort else 0))


# Tile / batch / pixels-per-lane combinations compiled into libgps.
TILE_CONFIGS = [(8, 8, 128, 1), (8, 8, 256, 1), (8, 8, 512, 1), (16, 16, 128, 1), (16, 16, 256, 1),
                (16, 16, 128, 2), (16, 16, 256, 2), (16, 16, 512, 2), (16, 16, 128, 4), (16, 16, 256, 4),
                (16, 16, 512, 4), (16, 32, 128, 1), (16, 32, 128, 2), (16, 32, 256, 2), (16, 32, 128, 4),
                (16, 32, 256, 4), (16, 32, 512, 4), (32, 16, 128, 2), (32, 16, 256, 2)]


# --------------------------------------------------------------------------- #
# SDF side                                                                     #
# --------------------------------------------------------------------------- #
def fuse(vol: Volume, cam, depth: torch.Tensor, rgb: torch.Tensor, stream=None):
    c = camera(cam)
    s = vol.struct()
    _check(lib().gps_fuse(ctypes.byref(s), ctypes.byref(c), _ptr(depth, "depth", c.width * c.height),
                          _ptr(rgb, "rgb", 3 * c.width * c.height), _stream(stream)), "gps_fuse")


def raycast(vol: Volume, cams, z_near=0.2, step=0.0, out=None, stream=None):
    """Returns a list of (depth [H,W], rgb [3,H,W]) per camera (allocated unless `out` is given)."""
    cams = [camera(c) for c in cams]
    V = len(cams)
    if out is None:
        out = [(torch.empty(c.height, c.width, dtype=torch.float32, device=vol.tsdf.device),
                torch.empty(3, c.height, c.width, dtype=torch.float32, device=vol.tsdf.device)) for c in cams]
    carr = (Camera * V)(*cams)
    dptr = (ctypes.c_void_p * V)(*[_ptr(d, "out_depth", c.width * c.height).value for (d, _), c in zip(out, cams)])
    cptr = (ctypes.c_void_p * V)(*[_ptr(r, "out_rgb", 3 * c.width * c.height).value for (_, r), c in zip(out, cams)])
    s = vol.struct()
    _check(lib().gps_raycast(ctypes.byref(s), carr, V, dptr, cptr, float(z_near), float(step), _stream(stream)),
           "gps_raycast")
    return out


# --------------------------------------------------------------------------- #
# Voxel-block hash of the TSDF (Sec. 3.2.1)                                    #
# --------------------------------------------------------------------------- #
HASH_BLOCK = 8
HASH_TILE = 16  # include/gps.h GPS_HASH_TILE


@dataclass
class HashVolume:
    """Colourised TSDF in a voxel-block hash (gps_hash_volume): a region of dims lattice
    points, blocks of 8^3 points allocated from the depth frames, `capacity` pool
    blocks, `n_buckets` table buckets (default: the power of two >= 2 * capacity)."""
    dims: tuple
    origin: tuple
    voxel: float
    trunc: float
    capacity: int
    n_buckets: int = 0
    max_weight: float = 100.0
    device: str = "cuda"
    skip_blocks: bool = True

    def __post_init__(self):
        cap = int(self.capacity)
        if self.n_buckets <= 0:
            self.n_buckets = 1 << max(1, (2 * cap - 1).bit_length())
        nb, dev = int(self.n_buckets), self.device
        self.keys = torch.empty(nb, dtype=torch.int64, device=dev)
        self.slots = torch.empty(nb, dtype=torch.int32, device=dev)
        self.block_key = torch.empty(cap, dtype=torch.int64, device=dev)
        self.state_t = torch.zeros(4, dtype=torch.int32, device=dev)
        self.visible = torch.empty(cap, dtype=torch.int32, device=dev)
        self.block_min = torch.empty(cap, dtype=torch.float32, device=dev) if self.skip_blocks else None
        n = cap * HASH_BLOCK ** 3
        self.tsdf = torch.empty(n, dtype=torch.float32, device=dev)
        self.weight = torch.empty(n, dtype=torch.float32, device=dev)
        self.rgb = torch.empty(3, n, dtype=torch.float32, device=dev)
        self.rgb_weight = torch.empty(n, dtype=torch.float32, device=dev)
        self.reset()

    def struct(self) -> HashVolumeS:
        s = HashVolumeS()
        s.nx, s.ny, s.nz = (int(d) for d in self.dims)
        for k in range(3):
            s.origin[k] = float(self.origin[k])
        s.voxel, s.trunc, s.max_weight = float(self.voxel), float(self.trunc), float(self.max_weight)
        s.n_buckets, s.capacity = int(self.n_buckets), int(self.capacity)
        for name in ("keys", "slots", "block_key", "visible", "tsdf", "weight", "rgb", "rgb_weight"):
            setattr(s, name, _ptr(getattr(self, name), name))
        s.state = _ptr(self.state_t, "state", 4)
        s.block_min = _ptr(self.block_min, "block_min") if self.block_min is not None else None
        return s

    def reset(self, stream=None):
        s = self.struct()
        _check(lib().gps_hash_reset(ctypes.byref(s), _stream(stream)), "gps_hash_reset")

    def state(self) -> dict:
        """Counters (reads them back: synchronises)."""
        a = self.state_t.cpu().tolist()
        return {"allocated": a[0], "allocated_before": a[1], "visible": a[2], "status": a[3]}


def hash_fuse(vol: HashVolume, cam, depth: torch.Tensor, rgb: torch.Tensor, stream=None):
    c = camera(cam)
    s = vol.struct()
    _check(lib().gps_hash_fuse(ctypes.byref(s), ctypes.byref(c), _ptr(depth, "depth", c.width * c.height),
                               _ptr(rgb, "rgb", 3 * c.width * c.height), _stream(stream)), "gps_hash_fuse")


def hash_range_floats(cams) -> int:
    """Floats of the depth-range scratch of hash_raycast for these cameras."""
    t = HASH_TILE
    return sum(2 * ((c.width + t - 1) // t) * ((c.height + t - 1) // t) for c in (camera(c) for c in cams))


def hash_raycast(vol: HashVolume, cams, z_near=0.2, step=0.0, out=None, stream=None, range_scratch=True):
    """As raycast, over the hashed volume.  range_scratch: True (a scratch tensor is
    allocated here), a float32 device tensor of at least hash_range_floats(cams)
    elements, or None/False (the rays march the whole region)."""
    cams = [camera(c) for c in cams]
    V = len(cams)
    if out is None:
        out = [(torch.empty(c.height, c.width, dtype=torch.float32, device=vol.tsdf.device),
                torch.empty(3, c.height, c.width, dtype=torch.float32, device=vol.tsdf.device)) for c in cams]
    carr = (Camera * V)(*cams)
    dptr = (ctypes.c_void_p * V)(*[_ptr(d, "out_depth", c.width * c.height).value for (d, _), c in zip(out, cams)])
    cptr = (ctypes.c_void_p * V)(*[_ptr(r, "out_rgb", 3 * c.width * c.height).value for (_, r), c in zip(out, cams)])
    s = vol.struct()
    rng = None
    if range_scratch is True:
        rng = torch.empty(hash_range_floats(cams), dtype=torch.float32, device=vol.tsdf.device)
    elif range_scratch is not None and range_scratch is not False:
        rng = range_scratch
    _check(lib().gps_hash_raycast(ctypes.byref(s), carr, V, dptr, cptr, float(z_near), float(step),
                                  _ptr(rng, "range_scratch"), rng.numel() if rng is not None else 0,
                                  _stream(stream)), "gps_hash_raycast")
    return out


# --------------------------------------------------------------------------- #
# Per-kernel timing (HIP events on the launch stream, thread-local)            #
# --------------------------------------------------------------------------- #
def stream_read(x, out):
    """Reads every element of the float32 device tensor x once (measurement support: a
    kernel of known read traffic); out receives one float per block (stream_blocks())."""
    if x.dtype != torch.float32 or out.dtype != torch.float32:
        raise TypeError("x and out must be float32")
    if out.numel() < stream_blocks():
        raise ValueError(f"out holds {out.numel()} floats, the read writes {stream_blocks()}")
    _check(lib().gps_stream_read(_ptr(x, "x"), x.numel(), _ptr(out, "out"), _stream()), "gps_stream_read")


def stream_write(y, v: float):
    """Writes v to every element of the float32 device tensor y once (measurement support:
    a kernel of known write traffic)."""
    if y.dtype != torch.float32:
        raise TypeError("y must be float32")
    _check(lib().gps_stream_write(_ptr(y, "y"), y.numel(), float(v), _stream()), "gps_stream_write")


def stream_blocks() -> int:
    return int(lib().gps_stream_blocks())


def profile_start():
    _check(lib().gps_profile_start(), "gps_profile_start")


def profile_stop():
    _check(lib().gps_profile_stop(), "gps_profile_stop")


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since profile_start (synchronises the recorded events)."""
    arr = (KernelTimeS * 32)()
    n = ctypes.c_int32(0)
    _check(lib().gps_profile_read(arr, 32, ctypes.byref(n)), "gps_profile_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


# --------------------------------------------------------------------------- #
# Render                                                                       #
# --------------------------------------------------------------------------- #
@dataclass
class View:
    cam: object
    base_rgb: torch.Tensor
    base_depth: torch.Tensor
    target_rgb: torch.Tensor | None = None
    target_depth: torch.Tensor | None = None
    out_rgb: torch.Tensor | None = None
    out_depth: torch.Tensor | None = None
    out_aux: torch.Tensor | None = None  # [H,W]: T_final (sorted) or W_G (sort-free), written by render_fwd

    def __post_init__(self):
        c = camera(self.cam)
        dev = self.base_rgb.device
        if self.out_rgb is None:
            self.out_rgb = torch.empty(3, c.height, c.width, dtype=torch.float32, device=dev)
        if self.out_depth is None:
            self.out_depth = torch.empty(c.height, c.width, dtype=torch.float32, device=dev)

    def struct(self, pose_xi: torch.Tensor | None = None) -> ViewS:
        """pose_xi: optional [6] device tensor, the left perturbation the view is rendered at."""
        c = camera(self.cam)
        HW = c.width * c.height
        return ViewS(c, _ptr(self.base_rgb, "base_rgb", 3 * HW), _ptr(self.base_depth, "base_depth", HW),
                     _ptr(self.target_rgb, "target_rgb", 3 * HW), _ptr(self.target_depth, "target_depth", HW),
                     _ptr(self.out_rgb, "out_rgb", 3 * HW), _ptr(self.out_depth, "out_depth", HW),
                     _ptr(pose_xi, "pose_xi", 6), _ptr(self.out_aux, "out_aux", HW))


def workspace_size(cfg: RenderCfg, n_gaussians: int, cams) -> int:
    cams = [camera(c) for c in cams]
    carr = (Camera * len(cams))(*cams)
    out = ctypes.c_size_t(0)
    cs = cfg.struct()
    _check(lib().gps_workspace_size(ctypes.byref(cs), int(n_gaussians), carr, len(cams), ctypes.byref(out)),
           "gps_workspace_size")
    return out.value


class Workspace:
    """Caller-owned device workspace for render_fwd / render_bwd (sized for cfg, M and the cameras)."""

    def __init__(self, cfg: RenderCfg, n_gaussians: int, cams, device="cuda", stream=None):
        self.nbytes = workspace_size(cfg, n_gaussians, cams)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.reset(stream)

    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())

    def reset(self, stream=None):
        _check(lib().gps_workspace_reset(self.ptr(), self.nbytes, _stream(stream)), "gps_workspace_reset")

    def status(self, stream=None) -> int:
        st = ctypes.c_int32(0)
        _check(lib().gps_device_status(self.ptr(), self.nbytes, ctypes.byref(st), _stream(stream)),
               "gps_device_status")
        return st.value

    def stats(self, stream=None) -> dict:
        s = StatsS()
        _check(lib().gps_read_stats(self.ptr(), self.nbytes, ctypes.byref(s), _stream(stream)), "gps_read_stats")
        return {"status": s.status, "n_views": s.n_views, "n_instances": s.n_instances, "capacity": s.capacity,
                "sort_fallback": s.sort_fallback, "n_tiles": s.n_tiles, "loss": s.loss,
                "pairs_eval": s.pairs_eval, "pairs_contrib": s.pairs_contrib,
                "view_omega": list(s.view_omega)[:max(s.n_views, 0)]}


def _views_array(views, pose_xi=None):
    V = len(views)
    if not 1 <= V <= MAX_VIEWS:
        raise ValueError(f"1..{MAX_VIEWS} views per call")
    if pose_xi is not None:
        if pose_xi.dtype != torch.float32 or tuple(pose_xi.shape) != (V, 6) or not pose_xi.is_contiguous():
            raise ValueError("pose_xi must be a contiguous float32 [n_views, 6] tensor")
        return (ViewS * V)(*[v.struct(pose_xi[i]) for i, v in enumerate(views)])
    return (ViewS * V)(*[v.struct() for v in views])


def render_fwd(cfg: RenderCfg, gauss: dict, views, ws: Workspace, out_loss: torch.Tensor | None = None,
               stream=None, pose_xi: torch.Tensor | None = None):
    """pose_xi: optional [V, 6] device tensor; view v is rendered from Exp(pose_xi[v]) T_cw."""
    cs = cfg.struct()
    gs = gaussians_struct(gauss)
    va = _views_array(views, pose_xi)
    _check(lib().gps_render_fwd(ctypes.byref(cs), ctypes.byref(gs), va, len(views), ws.ptr(), ws.nbytes,
                                _ptr(out_loss, "out_loss", 1) if out_loss is not None else None, _stream(stream)),
           "gps_render_fwd")


def views_upload(cfg: RenderCfg, gauss: dict, views, ws: Workspace, dL_drgb=None, dL_ddepth=None, stream=None,
                 pose_xi: torch.Tensor | None = None):
    """Write the view table into the workspace for calls made with cfg.views_preset."""
    cs = cfg.struct()
    gs = gaussians_struct(gauss)
    va = _views_array(views, pose_xi)
    V = len(views)
    rgb_arr = dep_arr = None
    if dL_drgb is not None:
        rgb_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_drgb").value for t in dL_drgb])
        if dL_ddepth is not None:
            dep_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_ddepth").value if t is not None else None
                                             for t in dL_ddepth])
    _check(lib().gps_views_upload(ctypes.byref(cs), ctypes.byref(gs), va, V, rgb_arr, dep_arr, ws.ptr(), ws.nbytes,
                                  _stream(stream)), "gps_views_upload")


def render_bwd(cfg: RenderCfg, gauss: dict, views, ws: Workspace, grads: dict, dpose: torch.Tensor | None = None,
               dL_drgb=None, dL_ddepth=None, loss_scale: torch.Tensor | None = None, stream=None,
               pose_xi: torch.Tensor | None = None):
    """pose_xi must be the tensor the matching render_fwd was given (dpose is then dL/dpose_xi)."""
    cs = cfg.struct()
    gs = gaussians_struct(gauss)
    gg = gaussians_struct(grads)
    va = _views_array(views, pose_xi)
    V = len(views)
    rgb_arr = dep_arr = None
    if dL_drgb is not None:
        rgb_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_drgb").value for t in dL_drgb])
        if dL_ddepth is not None:
            dep_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_ddepth").value if t is not None else None
                                             for t in dL_ddepth])
    _check(lib().gps_render_bwd(ctypes.byref(cs), ctypes.byref(gs), va, V, rgb_arr, dep_arr,
                                _ptr(loss_scale, "loss_scale", 1) if loss_scale is not None else None,
                                ctypes.byref(gg), _ptr(dpose, "dpose", 6 * V) if dpose is not None else None,
                                ws.ptr(), ws.nbytes, _stream(stream)), "gps_render_bwd")


class AdamFusedS(ctypes.Structure):
    _fields_ = [("m", GaussiansS), ("v", GaussiansS), ("lr_mean", ctypes.c_float), ("lr_log_scale", ctypes.c_float),
                ("lr_quat", ctypes.c_float), ("lr_opacity", ctypes.c_float), ("lr_rgb", ctypes.c_float),
                ("lr_sh", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_int32), ("step_counter", ctypes.c_void_p)]


def render_bwd_adam(cfg: RenderCfg, gauss: dict, views, ws: Workspace, opt: "Adam", grads: dict | None = None,
                    dpose: torch.Tensor | None = None, dL_drgb=None, dL_ddepth=None,
                    loss_scale: torch.Tensor | None = None, stream=None):
    """Backward with the Adam step of `opt` applied in its epilogue (gps_render_bwd_adam):
    the same parameters, moments and step counter as render_bwd followed by opt.step."""
    cs = cfg.struct()
    gs = gaussians_struct(gauss)
    gg = gaussians_struct(grads) if grads is not None else None
    va = _views_array(views)
    V = len(views)
    rgb_arr = dep_arr = None
    if dL_drgb is not None:
        rgb_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_drgb").value for t in dL_drgb])
        if dL_ddepth is not None:
            dep_arr = (ctypes.c_void_p * V)(*[_ptr(t, "dL_ddepth").value if t is not None else None
                                             for t in dL_ddepth])
    opt.t += 1
    af = AdamFusedS(gaussians_struct(opt.m), gaussians_struct(opt.v), float(opt.lr["mean"]),
                    float(opt.lr["log_scale"]), float(opt.lr["quat"]), float(opt.lr["opacity_logit"]),
                    float(opt.lr["rgb"]), float(opt.lr["sh"]), opt.b1, opt.b2, opt.eps, opt.t,
                    ctypes.c_void_p(opt.counter.data_ptr()) if opt.counter is not None else None)
    _check(lib().gps_render_bwd_adam(ctypes.byref(cs), ctypes.byref(gs), va, V, rgb_arr, dep_arr,
                                     _ptr(loss_scale, "loss_scale", 1) if loss_scale is not None else None,
                                     ctypes.byref(gg) if gg is not None else None,
                                     _ptr(dpose, "dpose", 6 * V) if dpose is not None else None,
                                     ctypes.byref(af), ws.ptr(), ws.nbytes, _stream(stream)), "gps_render_bwd_adam")


# Learning rates per attribute (Appendix C): position, SH0 (applied to rgb),
# alpha (applied to the opacity logit), scale (log-scale), rotation (quaternion),
# the SH bands above 0.
PAPER_LR = {"mean": 1.6e-4, "rgb": 2.5e-3, "opacity_logit": 0.05, "log_scale": 5e-3, "quat": 1e-3, "sh": 5e-4}


class Adam:
    """Adam state for a Gaussian set; one fused launch per step (gps_adam_step)."""

    def __init__(self, params: dict, lr: dict | None = None, betas=(0.9, 0.999), eps=1e-15,
                 device_counter: bool = True):
        self.params = params
        self.lr = dict(PAPER_LR if lr is None else lr)
        self.b1, self.b2 = betas
        self.eps = eps
        self.m = {k: torch.zeros_like(params[k]) for k in gauss_keys(params)}
        self.v = {k: torch.zeros_like(params[k]) for k in gauss_keys(params)}
        self.t = 0
        self.counter = torch.zeros(1, dtype=torch.int32, device=params["mean"].device) if device_counter else None

    def step(self, grads: dict, stream=None):
        keys = gauss_keys(self.params)
        groups = (AdamGroupS * len(keys))()
        for i, k in enumerate(keys):
            p = self.params[k]
            groups[i] = AdamGroupS(_ptr(p, k), _ptr(grads[k], "grad " + k, p.numel()), _ptr(self.m[k]),
                                   _ptr(self.v[k]), p.numel(), float(self.lr[k]))
        self.t += 1
        ctr = ctypes.c_void_p(self.counter.data_ptr()) if self.counter is not None else None
        _check(lib().gps_adam_step(groups, len(keys), self.t, ctr, self.b1, self.b2, self.eps,
                                   _stream(stream)), "gps_adam_step")


def adam_step(groups, step, b1=0.9, b2=0.999, eps=1e-15, step_counter=None, stream=None):
    """groups: list of (param, grad, m, v, lr) tensors."""
    arr = (AdamGroupS * len(groups))()
    for i, (p, g, m, v, lr) in enumerate(groups):
        arr[i] = AdamGroupS(_ptr(p), _ptr(g, "grad", p.numel()), _ptr(m, "m", p.numel()), _ptr(v, "v", p.numel()),
                            p.numel(), float(lr))
    ctr = _ptr(step_counter, "step_counter", 1) if step_counter is not None else None
    _check(lib().gps_adam_step(arr, len(groups), int(step), ctr, float(b1), float(b2), float(eps),
                               _stream(stream)), "gps_adam_step")


# --------------------------------------------------------------------------- #
# autograd                                                                     #
# --------------------------------------------------------------------------- #
class Session:
    """Everything a differentiable render needs besides the parameters: config, views, workspace."""

    def __init__(self, cfg: RenderCfg, views, n_gaussians: int, device="cuda"):
        self.cfg = cfg
        self.views = list(views)
        self.ws = Workspace(cfg, n_gaussians, [v.cam for v in self.views], device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)


def _pose_arg(pose_xi, n_views):
    """The [V, 6] float32 device tensor the library reads, or None."""
    if pose_xi is None:
        return None
    xi = pose_xi.detach()
    if tuple(xi.shape) != (n_views, 6):
        raise ValueError(f"pose_xi must have shape ({n_views}, 6)")
    return xi.to(torch.float32).contiguous()


class RenderLoss(torch.autograd.Function):
    """loss = RenderLoss.apply(mean, log_scale, quat, opacity_logit, rgb, pose_xi, session[, sh]).
    pose_xi [V,6] (or None): view v is rendered from Exp(pose_xi[v]) T_cw, the left perturbation of its
    camera, translation first; its gradient is dL/dpose_xi at the given value.  sh (optional,
    [3,K,M]): the SH bands above degree 0 (view-dependent colour)."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, rgb, pose_xi, session: Session, sh=None):
        g = {"mean": mean, "log_scale": log_scale, "quat": quat, "opacity_logit": opacity_logit, "rgb": rgb, "sh": sh}
        xi = _pose_arg(pose_xi, len(session.views))
        render_fwd(session.cfg, g, session.views, session.ws, out_loss=session.loss, pose_xi=xi)
        ctx.session = session
        ctx.pose_given = pose_xi is not None
        ctx.has_sh = sh is not None
        ctx.save_for_backward(mean, log_scale, quat, opacity_logit, rgb, xi, sh)
        return session.loss.clone().reshape(())

    @staticmethod
    def backward(ctx, gloss):
        s = ctx.session
        mean, log_scale, quat, opacity_logit, rgb, xi, sh = ctx.saved_tensors
        g = {"mean": mean, "log_scale": log_scale, "quat": quat, "opacity_logit": opacity_logit, "rgb": rgb, "sh": sh}
        grads = zeros_like_gaussians(g)
        dpose = torch.zeros(len(s.views), 6, dtype=torch.float32, device=mean.device)
        scale = gloss.detach().to(torch.float32).reshape(1).contiguous()
        render_bwd(s.cfg, g, s.views, s.ws, grads, dpose, loss_scale=scale, pose_xi=xi)
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity_logit"], grads["rgb"],
                dpose if ctx.pose_given else None, None, grads["sh"] if ctx.has_sh else None)


class Render(torch.autograd.Function):
    """rgb_0, depth_0, rgb_1, depth_1, ... = Render.apply(mean, log_scale, quat, opacity_logit, rgb, pose_xi,
    session[, sh]) for arbitrary downstream losses (pose_xi and sh as in RenderLoss)."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, rgb, pose_xi, session: Session, sh=None):
        g = {"mean": mean, "log_scale": log_scale, "quat": quat, "opacity_logit": opacity_logit, "rgb": rgb, "sh": sh}
        xi = _pose_arg(pose_xi, len(session.views))
        render_fwd(session.cfg, g, session.views, session.ws, pose_xi=xi)
        ctx.session = session
        ctx.pose_given = pose_xi is not None
        ctx.has_sh = sh is not None
        ctx.save_for_backward(mean, log_scale, quat, opacity_logit, rgb, xi, sh)
        outs = []
        for v in session.views:
            outs += [v.out_rgb.clone(), v.out_depth.clone()]
        return tuple(outs)

    @staticmethod
    def backward(ctx, *gouts):
        s = ctx.session
        mean, log_scale, quat, opacity_logit, rgb, xi, sh = ctx.saved_tensors
        g = {"mean": mean, "log_scale": log_scale, "quat": quat, "opacity_logit": opacity_logit, "rgb": rgb, "sh": sh}
        grads = zeros_like_gaussians(g)
        dpose = torch.zeros(len(s.views), 6, dtype=torch.float32, device=mean.device)
        drgb, ddep = [], []
        for i, v in enumerate(s.views):
            gr, gd = gouts[2 * i], gouts[2 * i + 1]
            drgb.append((gr if gr is not None else torch.zeros_like(v.out_rgb)).contiguous())
            ddep.append((gd if gd is not None else torch.zeros_like(v.out_depth)).contiguous())
        render_bwd(s.cfg, g, s.views, s.ws, grads, dpose, dL_drgb=drgb, dL_ddepth=ddep, pose_xi=xi)
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity_logit"], grads["rgb"],
                dpose if ctx.pose_given else None, None, grads["sh"] if ctx.has_sh else None)


def remove_gaussians(params: dict, companions=(), min_opacity=0.005, max_scale=0.1, min_scale=0.003, stream=None):
    """Gaussian removal of Eq. 8 (gps_remove_gaussians): returns the kept Gaussians of
    `params` in their original order, the same rows of every companion set (for
    example Adam moments), and the kept count.  Reads the count back (synchronises)."""
    M = int(params["opacity_logit"].numel())
    dev = params["opacity_logit"].device
    sets = [params] + list(companions)
    L = sh_degree(params)
    K = SH_COEFFS[L]
    outs = [{k: torch.empty(GAUSS_ROWS[k], max(M, 1), dtype=torch.float32, device=dev) for k in GAUSS_KEYS}
            for _ in sets]
    if L > 0:
        for o in outs:
            o["sh"] = torch.empty(3 * K, max(M, 1), dtype=torch.float32, device=dev)
    arr_in = (GaussiansS * len(sets))(*[gaussians_struct(s) for s in sets])
    arr_out = (GaussiansS * len(sets))()
    for i, o in enumerate(outs):
        arr_out[i].count = M
        for k in GAUSS_KEYS:
            setattr(arr_out[i], k, ctypes.c_void_p(o[k].data_ptr()))
        arr_out[i].sh_degree = L
        arr_out[i].sh = ctypes.c_void_p(o["sh"].data_ptr()) if L > 0 else None
    nbytes = ctypes.c_size_t(0)
    _check(lib().gps_removal_workspace_size(M, ctypes.byref(nbytes)), "gps_removal_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    cfg = RemovalCfgS(min_opacity, max_scale, min_scale)
    _check(lib().gps_remove_gaussians(ctypes.byref(cfg), arr_in, arr_out, len(sets),
                                      ctypes.c_void_p(count.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      nbytes.value, _stream(stream)), "gps_remove_gaussians")
    n = int(count.item())
    shaped = [{k: o[k].reshape(-1)[:GAUSS_ROWS[k] * n].view(GAUSS_ROWS[k], n) if GAUSS_ROWS[k] > 1
               else o[k].reshape(-1)[:n] for k in GAUSS_KEYS} for o in outs]
    if L > 0:
        for sh_, o in zip(shaped, outs):
            sh_["sh"] = o["sh"].reshape(-1)[:3 * K * n].view(3, K, n)
    return shaped[0], shaped[1:], n


def insert_gaussians(cam, render_rgb, frame_rgb, weight, sdf_depth, rand, capacity=None, delta_c=0.05, delta_w=4.0,
                     fraction=0.25, scale_cap=0.1, flat_ratio=0.1, opacity=0.5, sh_degree=0, stream=None):
    """Gaussian insertion of Eq. 6 and App. A (gps_insert_gaussians): the new Gaussians
    (planar [rows][n] tensors, row-major pixel order), their pixel indices and the
    number of sampled pixels n_taken (the output keeps min(n_taken, capacity));
    `capacity` defaults to every pixel.  Reads the count back (synchronises)."""
    c = camera(cam)
    W, H = c.width, c.height
    dev = frame_rgb.device
    cap = W * H if capacity is None else int(capacity)
    out = {k: torch.empty(GAUSS_ROWS[k], max(cap, 1), dtype=torch.float32, device=dev) for k in GAUSS_KEYS}
    K = SH_COEFFS[int(sh_degree)]
    if K:
        out["sh"] = torch.empty(3 * K, max(cap, 1), dtype=torch.float32, device=dev)
    pix = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    g = GaussiansS()
    g.count = cap
    for k in GAUSS_KEYS:
        setattr(g, k, ctypes.c_void_p(out[k].data_ptr()))
    g.sh_degree = int(sh_degree)
    g.sh = ctypes.c_void_p(out["sh"].data_ptr()) if K else None
    nbytes = ctypes.c_size_t(0)
    _check(lib().gps_insertion_workspace_size(W, H, ctypes.byref(nbytes)), "gps_insertion_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    cfg = InsertCfgS(delta_c, delta_w, fraction, scale_cap, flat_ratio, opacity)
    _check(lib().gps_insert_gaussians(ctypes.byref(cfg), ctypes.byref(c), _ptr(render_rgb, "render_rgb", 3 * W * H),
                                      _ptr(frame_rgb, "frame_rgb", 3 * W * H), _ptr(weight, "weight", W * H),
                                      _ptr(sdf_depth, "sdf_depth", W * H), _ptr(rand, "rand", W * H),
                                      ctypes.byref(g), ctypes.c_void_p(pix.data_ptr()),
                                      ctypes.c_void_p(count.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      nbytes.value, _stream(stream)), "gps_insert_gaussians")
    n_taken = int(count.item())
    n = min(n_taken, cap)
    res = {k: out[k][:, :n] if GAUSS_ROWS[k] > 1 else out[k].reshape(-1)[:n] for k in GAUSS_KEYS}
    if K:
        res["sh"] = out["sh"][:, :n].reshape(3, K, n).contiguous()
    return res, pix[:n], n_taken


# --------------------------------------------------------------------------- #
# Camera tracking (Eq. 5)                                                      #
# --------------------------------------------------------------------------- #
def level_camera(cam, level: int) -> dict:
    """Size and intrinsics of a level of the depth hierarchy (gps_level_camera)."""
    src = camera({**cam, "R": cam.get("R", np.eye(3)), "t": cam.get("t", np.zeros(3))})
    out = Camera()
    _check(lib().gps_level_camera(ctypes.byref(src), int(level), ctypes.byref(out)), "gps_level_camera")
    c = dict(cam)
    c.update(width=out.width, height=out.height, fx=out.fx, fy=out.fy, cx=out.cx, cy=out.cy)
    return c


def depth_downsample(depth: torch.Tensor, stream=None) -> torch.Tensor:
    """One level of the depth hierarchy (gps_depth_downsample)."""
    H, W = depth.shape
    out = torch.empty(H // 2, W // 2, dtype=torch.float32, device=depth.device)
    _check(lib().gps_depth_downsample(_ptr(depth, "depth", W * H), W, H, ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream)), "gps_depth_downsample")
    return out


def pose_tensor(cam, device="cuda") -> torch.Tensor:
    """The [12] device pose (R row-major, t; world to camera) of a camera dict."""
    R = np.asarray(cam["R"], np.float32).reshape(9)
    t = np.asarray(cam["t"], np.float32).reshape(3)
    return torch.as_tensor(np.concatenate([R, t])).to(device)


class IcpWorkspace:
    def __init__(self, width: int, height: int, device="cuda"):
        n = ctypes.c_size_t(0)
        _check(lib().gps_icp_workspace_size(width, height, ctypes.byref(n)), "gps_icp_workspace_size")
        self.nbytes = n.value
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.sys = torch.zeros(29, dtype=torch.float64, device=device)
        self.xi = torch.zeros(6, dtype=torch.float32, device=device)


def icp_reduce(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, ws: IcpWorkspace, stream=None):
    """Gauss-Newton system of Eq. 5 at the device pose (gps_icp_reduce) into ws.sys."""
    pc, lc = camera(prev_cam), camera({**level_cam, "R": np.eye(3), "t": np.zeros(3)})
    _check(lib().gps_icp_reduce(ctypes.byref(pc), _ptr(prev_depth, "prev_depth", pc.width * pc.height),
                                ctypes.byref(lc), _ptr(level_depth, "level_depth", lc.width * lc.height),
                                _ptr(pose, "pose", 12), float(dist_thresh), ctypes.c_void_p(ws.sys.data_ptr()),
                                ctypes.c_void_p(ws.buf.data_ptr()), ws.nbytes, _stream(stream)), "gps_icp_reduce")
    return ws.sys


def icp_reduce_noalloc(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, out_sys: torch.Tensor,
                       stream=None):
    """gps_icp_reduce_noalloc: the system of Eq. 5 into out_sys (device float64 [29]) with the
    library's fixed scratch instead of a workspace (nothing is allocated)."""
    pc, lc = camera(prev_cam), camera({**level_cam, "R": np.eye(3), "t": np.zeros(3)})
    if not (out_sys.is_cuda and out_sys.dtype == torch.float64 and out_sys.is_contiguous() and out_sys.numel() >= 29):
        raise ValueError("out_sys must be a contiguous device float64 tensor of at least 29 elements")
    _check(lib().gps_icp_reduce_noalloc(ctypes.byref(pc), _ptr(prev_depth, "prev_depth", pc.width * pc.height),
                                        ctypes.byref(lc), _ptr(level_depth, "level_depth", lc.width * lc.height),
                                        _ptr(pose, "pose", 12), float(dist_thresh),
                                        ctypes.c_void_p(out_sys.data_ptr()), _stream(stream)),
           "gps_icp_reduce_noalloc")
    return out_sys


def icp_step(prev_cam, prev_depth, level_cam, level_depth, pose, dist_thresh, ws: IcpWorkspace, stream=None):
    """One Gauss-Newton step (gps_icp_step): the system into ws.sys, the pose updated in
    place, xi into ws.xi -- icp_reduce then icp_solve with one launch fewer."""
    pc, lc = camera(prev_cam), camera({**level_cam, "R": np.eye(3), "t": np.zeros(3)})
    _check(lib().gps_icp_step(ctypes.byref(pc), _ptr(prev_depth, "prev_depth", pc.width * pc.height),
                              ctypes.byref(lc), _ptr(level_depth, "level_depth", lc.width * lc.height),
                              _ptr(pose, "pose", 12), float(dist_thresh), ctypes.c_void_p(ws.sys.data_ptr()),
                              ctypes.c_void_p(ws.xi.data_ptr()), ctypes.c_void_p(ws.buf.data_ptr()), ws.nbytes,
                              _stream(stream)), "gps_icp_step")
    return ws.sys


def icp_solve(sys: torch.Tensor, pose: torch.Tensor, xi: torch.Tensor | None = None, stream=None):
    """Solve and apply one Gauss-Newton step to the device pose (gps_icp_solve)."""
    _check(lib().gps_icp_solve(ctypes.c_void_p(sys.data_ptr()), _ptr(pose, "pose", 12),
                               ctypes.c_void_p(xi.data_ptr()) if xi is not None else None, _stream(stream)),
           "gps_icp_solve")


def icp_track(prev_cam, prev_depth, cur_cam, cur_depth, pose: torch.Tensor, iters=(4, 4, 6),
              dist_thresh=(0.1, 0.05, 0.02), ws: IcpWorkspace | None = None, pyramid=None, stream=None):
    """Coarse-to-fine tracking of the current frame against the previous frame's raycast
    depth; `pose` (device [12], world to camera) is refined in place.  iters and
    dist_thresh list the levels from the coarsest to the finest.  Nothing is read
    back to the host."""
    L = len(iters)
    if pyramid is None:
        pyramid = [cur_depth]
        for _ in range(L - 1):
            pyramid.append(depth_downsample(pyramid[-1], stream))
    if ws is None:
        ws = IcpWorkspace(cur_cam["width"], cur_cam["height"], device=cur_depth.device)
    for k in range(L):
        lvl = L - 1 - k
        lc = level_camera(cur_cam, lvl)
        for _ in range(iters[k]):
            icp_step(prev_cam, prev_depth, lc, pyramid[lvl], pose, dist_thresh[k], ws, stream)
    return pose
