"""ctypes front end of the FP64 reference implementation in ``gps_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
this module, and this module never imports the product package.

All array arguments are NumPy arrays; float32 inputs are passed exactly as the
GPU kernels receive them, outputs come back as float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gps_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: every binary32 statement of the decision arithmetic rounds once.
# -fopenmp: independent pixels and lattice points on threads (results do not depend on the count).
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile gps_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("voxel", ctypes.c_float),
                ("trunc", ctypes.c_float), ("max_weight", ctypes.c_float)]


class Gauss(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("sh_degree", ctypes.c_int32), ("sh", ctypes.c_void_p)]


class Cfg(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("eps_cull", ctypes.c_float),
                ("lambda_depth", ctypes.c_float), ("dilation", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("z_near", ctypes.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_fuse.argtypes = [P, P, P, P, P, P, P, P, P, ctypes.c_int32]
        L.orc_fuse_points.argtypes = [P, P, ctypes.c_int64, P, P, P, P, P, P, P]
        L.orc_fuse_points.restype = None
        L.orc_alloc_blocks.argtypes = [P, P, P, ctypes.c_int32, P]
        L.orc_alloc_blocks.restype = None
        L.orc_fuse.restype = None
        L.orc_raycast.argtypes = [P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_int32, P, P, P, P]
        L.orc_raycast.restype = None
        L.orc_trilinear.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_trilinear.restype = ctypes.c_double
        L.orc_project.argtypes = [P, P, P, P]
        L.orc_project.restype = None
        L.orc_render.argtypes = [P, P, P, P, P, ctypes.c_int32, P, P, P, P, P, P, P, P]
        L.orc_render.restype = None
        L.orc_loss.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, ctypes.c_double, P, P, P]
        L.orc_loss.restype = ctypes.c_double
        L.orc_render_bwd.argtypes = [P, P, P, P, P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_sh_basis.argtypes = [ctypes.c_int32, P, P, P]
        L.orc_sh_basis.restype = None
        L.orc_render_bwd.restype = None
        L.orc_adam.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int32]
        L.orc_adam.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_set_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """OpenMP threads of the reference (n <= 0 keeps the current count); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- #
# Plain-data descriptions used by the wrapper (no product types).              #
# --------------------------------------------------------------------------- #
@dataclass
class RenderCfg:
    """Renderer constants (see the reading of each in gps_oracle.c)."""
    mode: int = 0
    eps_cull: float = 0.01
    lambda_depth: float = 1.0
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    z_near: float = 0.2

    def c(self) -> Cfg:
        return Cfg(self.mode, self.eps_cull, self.lambda_depth, self.dilation,
                   self.alpha_min, self.alpha_max, self.T_min, self.z_near)


def make_cam(width, height, fx, fy, cx, cy, R, t) -> Cam:
    c = Cam()
    c.width, c.height = int(width), int(height)
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    R = np.asarray(R, dtype=np.float32).reshape(9)
    t = np.asarray(t, dtype=np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    return c


def cam_from(camd) -> Cam:
    """Accept a Cam, or any object/dict with width, height, fx, fy, cx, cy, R, t."""
    if isinstance(camd, Cam):
        return camd
    g = (lambda k: camd[k]) if isinstance(camd, dict) else (lambda k: getattr(camd, k))
    return make_cam(g("width"), g("height"), g("fx"), g("fy"), g("cx"), g("cy"), g("R"), g("t"))


def make_grid(dims, origin, voxel, trunc, max_weight=100.0) -> Grid:
    g = Grid()
    g.nx, g.ny, g.nz = (int(d) for d in dims)
    for k in range(3):
        g.origin[k] = float(origin[k])
    g.voxel, g.trunc, g.max_weight = float(voxel), float(trunc), float(max_weight)
    return g


class _GaussKeep:
    """Keeps the float32 copies alive for as long as the ctypes struct is used."""

    def __init__(self, mean, log_scale, quat, opacity_logit, rgb, sh=None):
        self.arrs = [_f32(mean), _f32(log_scale), _f32(quat), _f32(opacity_logit).reshape(-1), _f32(rgb)]
        M = self.arrs[3].shape[0]
        assert self.arrs[0].shape == (3, M) and self.arrs[1].shape == (3, M)
        assert self.arrs[2].shape == (4, M) and self.arrs[4].shape == (3, M)
        self.L = 0
        self.sh = None
        if sh is not None:
            self.sh = _f32(sh)
            K = self.sh.shape[1]
            self.L = SH_DEGREE_OF[K]
            assert self.sh.shape == (3, K, M)
        self.s = Gauss(M, *[_ptr(a) for a in self.arrs], self.L, _ptr(self.sh))
        self.M = M


# coefficients per channel of the view-dependent bands for each SH degree, and back
SH_COEFFS = {0: 0, 1: 3, 2: 8, 3: 15}
SH_DEGREE_OF = {v: k for k, v in SH_COEFFS.items()}


def gauss(g) -> _GaussKeep:
    """g: dict with mean [3,M], log_scale [3,M], quat [4,M], opacity_logit [M], rgb [3,M] and
    optionally sh [3,K,M] (K = 3, 8 or 15: the bands 1..L of degree L = 1, 2, 3)."""
    return _GaussKeep(g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], g["rgb"], g.get("sh"))


def sh_basis(L: int, d):
    """The real SH of bands 1..L at unit direction d (Y [K]) and their partial
    derivatives with respect to d's components taken as independent (dY [K,3])."""
    K = SH_COEFFS[L]
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(max(K, 1))
    dY = np.zeros((max(K, 1), 3))
    lib().orc_sh_basis(int(L), _ptr(d), _ptr(Y), _ptr(dY))
    return Y[:K], dY[:K]


# --------------------------------------------------------------------------- #
# Wrapped entry points                                                         #
# --------------------------------------------------------------------------- #
def new_volume(grid: Grid):
    N = grid.nx * grid.ny * grid.nz
    return {"tsdf": np.ones(N), "weight": np.zeros(N), "rgb": np.zeros((3, N)), "rgb_weight": np.zeros(N)}


def fuse(grid: Grid, vol: dict, cam, depth, rgb, block_mask=None, block=8):
    """In-place FP64 fusion of one frame into ``vol`` (dict of float64 arrays).  With
    ``block_mask`` (uint8 [nbz][nby][nbx], blocks of ``block``^3 lattice points) only the
    points of allocated blocks are updated: fusion into a voxel-block hash."""
    cam = cam_from(cam)
    depth = _f32(depth)
    rgb = _f32(rgb)
    assert depth.shape == (cam.height, cam.width) and rgb.shape == (3, cam.height, cam.width)
    for k in ("tsdf", "weight", "rgb", "rgb_weight"):
        assert vol[k].dtype == np.float64 and vol[k].flags.c_contiguous
    if block_mask is not None:
        assert block_mask.dtype == np.uint8 and block_mask.size == np.prod(block_grid(grid, block))
        block_mask = np.ascontiguousarray(block_mask)
    lib().orc_fuse(ctypes.byref(grid), _ptr(vol["tsdf"]), _ptr(vol["weight"]), _ptr(vol["rgb"]),
                   _ptr(vol["rgb_weight"]), ctypes.byref(cam), _ptr(depth), _ptr(rgb), _ptr(block_mask),
                   int(block))
    return vol


def new_points(n: int) -> dict:
    """Initial values of n lattice points (tsdf 1, weights 0, colour 0), stored compactly."""
    return {"tsdf": np.ones(n), "weight": np.zeros(n), "rgb": np.zeros((3, n)), "rgb_weight": np.zeros(n)}


def fuse_points(grid: Grid, idx, pts: dict, cam, depth, rgb):
    """The fusion of one frame at the lattice points idx (x + nx (y + ny z)) only, their
    values in ``pts`` (from new_points), updated in place: the same update as ``fuse``."""
    cam = cam_from(cam)
    depth = _f32(depth)
    rgb = _f32(rgb)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = idx.size
    assert depth.shape == (cam.height, cam.width) and rgb.shape == (3, cam.height, cam.width)
    for k in ("tsdf", "weight", "rgb", "rgb_weight"):
        assert pts[k].dtype == np.float64 and pts[k].flags.c_contiguous and pts[k].size == (3 if k == "rgb" else 1) * n
    lib().orc_fuse_points(ctypes.byref(grid), _ptr(idx), n, _ptr(pts["tsdf"]), _ptr(pts["weight"]), _ptr(pts["rgb"]),
                          _ptr(pts["rgb_weight"]), ctypes.byref(cam), _ptr(depth), _ptr(rgb))
    return pts


def block_grid(grid: Grid, block=8):
    """Blocks per axis (x, y, z) of the lattice split into ``block``^3 blocks."""
    return tuple((n + block - 1) // block for n in (grid.nx, grid.ny, grid.nz))


def alloc_blocks(grid: Grid, cam, depth, mask=None, block=8):
    """Voxel blocks a frame allocates (orc_alloc_blocks): uint8 mask [nbz][nby][nbx], updated
    in place when given (allocation accumulates over frames)."""
    cam = cam_from(cam)
    depth = _f32(depth)
    assert depth.shape == (cam.height, cam.width)
    nbx, nby, nbz = block_grid(grid, block)
    if mask is None:
        mask = np.zeros((nbz, nby, nbx), np.uint8)
    assert mask.dtype == np.uint8 and mask.shape == (nbz, nby, nbx) and mask.flags.c_contiguous
    lib().orc_alloc_blocks(ctypes.byref(grid), ctypes.byref(cam), _ptr(depth), int(block), _ptr(mask))
    return mask


def raycast(grid: Grid, tsdf32, rgb32, cam, z_near=0.2, step=0.0, pix=None):
    """Returns depth [npix], rgb [3,npix], hit sample index [npix] (-1 = miss)."""
    cam = cam_from(cam)
    tsdf32 = _f32(tsdf32).reshape(-1)
    rgb32 = _f32(rgb32).reshape(3, -1)
    if pix is None:
        npix, pixp = cam.width * cam.height, None
    else:
        pix = np.ascontiguousarray(pix, dtype=np.int32)
        npix, pixp = pix.shape[0], pix
    d = np.zeros(npix)
    c = np.zeros((3, npix))
    k = np.zeros(npix, dtype=np.int32)
    lib().orc_raycast(ctypes.byref(grid), _ptr(tsdf32), _ptr(rgb32), ctypes.byref(cam), z_near, step,
                      npix, _ptr(pixp), _ptr(d), _ptr(c), _ptr(k))
    return d, c, k


def trilinear(grid: Grid, field32, p):
    f = _f32(field32).reshape(-1)
    return lib().orc_trilinear(ctypes.byref(grid), _ptr(f), float(p[0]), float(p[1]), float(p[2]))


def project(cfg: RenderCfg, g, cam):
    """Per-Gaussian projection, a dict of arrays (see orc_project)."""
    cam = cam_from(cam)
    G = gauss(g)
    out = np.zeros((G.M, 16))
    c = cfg.c()
    lib().orc_project(ctypes.byref(c), ctypes.byref(G.s), ctypes.byref(cam), _ptr(out))
    return {"valid": out[:, 0] > 0.5, "m": out[:, 1:3], "cov": out[:, 3:6], "conic": out[:, 6:9],
            "sigma": out[:, 9], "depth": out[:, 10], "depth32": out[:, 11].astype(np.float32),
            "box": out[:, 12:16]}


def render(cfg: RenderCfg, g, cam, base_rgb, base_depth, pix=None):
    """Returns dict rgb [3,npix], depth, T, flag, n, W (float64 / int32) and order (uint64: a
    signature of each pixel's composited sequence in sorted mode, 0 in sort-free mode)."""
    cam = cam_from(cam)
    G = gauss(g)
    base_rgb = _f32(base_rgb).reshape(3, -1)
    base_depth = _f32(base_depth).reshape(-1)
    assert base_depth.shape[0] == cam.width * cam.height
    if pix is None:
        npix, pixp = cam.width * cam.height, None
    else:
        pixp = np.ascontiguousarray(pix, dtype=np.int32)
        npix = pixp.shape[0]
    rgb = np.zeros((3, npix))
    depth = np.zeros(npix)
    T = np.zeros(npix)
    flag = np.zeros(npix, dtype=np.int32)
    n = np.zeros(npix, dtype=np.int32)
    W = np.zeros(npix)
    order = np.zeros(npix, dtype=np.uint64)
    c = cfg.c()
    lib().orc_render(ctypes.byref(c), ctypes.byref(G.s), ctypes.byref(cam), _ptr(base_rgb), _ptr(base_depth),
                     npix, _ptr(pixp), _ptr(rgb), _ptr(depth), _ptr(T), _ptr(flag), _ptr(n), _ptr(W), _ptr(order))
    return {"rgb": rgb, "depth": depth, "T": T, "flag": flag, "n": n, "W": W, "order": order}


def loss(cfg: RenderCfg, W: int, H: int, rgb, depth, target_rgb, target_depth, base_depth, scale=1.0,
         want_grad=True):
    """Per-view loss; returns (L, g_rgb [3,HW] or None, g_depth [HW] or None, |Omega|)."""
    rgb = _f64(rgb).reshape(3, -1)
    depth = _f64(depth).reshape(-1)
    trgb = _f32(target_rgb).reshape(3, -1)
    tdep = _f32(target_depth).reshape(-1)
    bdep = _f32(base_depth).reshape(-1)
    g_rgb = np.zeros_like(rgb) if want_grad else None
    g_dep = np.zeros_like(depth) if want_grad else None
    om = ctypes.c_int64(0)
    c = cfg.c()
    L = lib().orc_loss(ctypes.byref(c), W, H, _ptr(rgb), _ptr(depth), _ptr(trgb), _ptr(tdep), _ptr(bdep),
                       float(scale), _ptr(g_rgb), _ptr(g_dep), ctypes.byref(om))
    return L, g_rgb, g_dep, om.value


def render_bwd(cfg: RenderCfg, g, cam, base_rgb, base_depth, g_pix_rgb, g_pix_depth, pix=None,
               want_screen=False):
    """Gradients (float64) for the listed pixels' upstream adjoints."""
    cam = cam_from(cam)
    G = gauss(g)
    M = G.M
    base_rgb = _f32(base_rgb).reshape(3, -1)
    base_depth = _f32(base_depth).reshape(-1)
    if pix is None:
        npix, pixp = cam.width * cam.height, None
    else:
        pixp = np.ascontiguousarray(pix, dtype=np.int32)
        npix = pixp.shape[0]
    gpr = _f64(g_pix_rgb).reshape(3, npix)
    gpd = _f64(g_pix_depth).reshape(npix)
    out = {"mean": np.zeros((3, M)), "log_scale": np.zeros((3, M)), "quat": np.zeros((4, M)),
           "opacity_logit": np.zeros(M), "rgb": np.zeros((3, M)), "pose": np.zeros(6)}
    if G.L > 0:
        out["sh"] = np.zeros((3, SH_COEFFS[G.L], M))
    scr = np.zeros((M, 10)) if want_screen else None
    c = cfg.c()
    lib().orc_render_bwd(ctypes.byref(c), ctypes.byref(G.s), ctypes.byref(cam), _ptr(base_rgb),
                         _ptr(base_depth), npix, _ptr(pixp), _ptr(gpr), _ptr(gpd), _ptr(out["mean"]),
                         _ptr(out["log_scale"]), _ptr(out["quat"]), _ptr(out["opacity_logit"]),
                         _ptr(out["rgb"]), _ptr(out.get("sh")), _ptr(out["pose"]), _ptr(scr))
    if want_screen:
        out["screen"] = scr
    return out


def adam(param, grad, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-15):
    """In-place FP64 Adam step on float64 arrays."""
    for a in (param, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(param.size, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), lr, b1, b2, eps, int(t))


# Learning rates per attribute, Appendix C (position, SH0 -> rgb, alpha -> opacity
# logit, scale -> log-scale, rotation -> quaternion).
PAPER_LR = {"mean": 1.6e-4, "rgb": 2.5e-3, "opacity_logit": 0.05, "log_scale": 5e-3, "quat": 1e-3, "sh": 5e-4}


# --------------------------------------------------------------------------- #
# Gaussian removal (Sec. 3.2.2, Eq. 8).                                        #
# --------------------------------------------------------------------------- #
# A Gaussian is deleted when its opacity sigma = sigmoid(o) is below
# delta_sigma, or its largest scale s = exp(l) is above delta_s_max, or its
# largest scale is below delta_s_min.  Reading: sigmoid and exp are increasing,
# so the tests are taken on the stored parameters, o < logit(delta_sigma) and
# max(l) > ln(delta_s_max), max(l) < ln(delta_s_min), each in binary32 against
# the threshold computed in binary64 and rounded to binary32 once -- the
# precision in which the parameters are stored, so that the keep/delete
# decision is a plain comparison of stored values.
REMOVAL_DEFAULTS = {"min_opacity": 0.005, "max_scale": 0.1, "min_scale": 0.003}


def removal_thresholds(min_opacity=0.005, max_scale=0.1, min_scale=0.003):
    """(logit threshold, ln max scale, ln min scale), binary32."""
    return (np.float32(np.log(min_opacity / (1.0 - min_opacity))), np.float32(np.log(max_scale)),
            np.float32(np.log(min_scale)))


def removal_keep(g, min_opacity=0.005, max_scale=0.1, min_scale=0.003):
    """Boolean mask of the Gaussians Eq. 8 keeps (plain loop over Gaussians)."""
    t_o, t_hi, t_lo = removal_thresholds(min_opacity, max_scale, min_scale)
    o = np.asarray(g["opacity_logit"], np.float32).reshape(-1)
    ls = np.asarray(g["log_scale"], np.float32).reshape(3, -1)
    keep = np.zeros(o.size, bool)
    for i in range(o.size):
        lmax = max(ls[0, i], ls[1, i], ls[2, i])
        delete = (o[i] < t_o) or (lmax > t_hi) or (lmax < t_lo)
        keep[i] = not delete
    return keep


def remove_gaussians(g, companions=(), **thresholds):
    """The kept Gaussians of `g`, in their original order, and the same rows of
    every companion set (e.g. Adam moments); each a dict of [rows][n_kept] arrays."""
    keep = removal_keep(g, **thresholds)
    idx = np.nonzero(keep)[0]
    rows = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "rgb": 3}
    pick = lambda s: {k: np.asarray(v).reshape(rows[k], keep.size)[:, idx] for k, v in s.items()}
    return pick(g), [pick(c) for c in companions], idx


# --------------------------------------------------------------------------- #
# Gaussian insertion (Sec. 3.2.2, Eq. 6 and the paragraph after it; App. A).  #
# --------------------------------------------------------------------------- #
# Readings (the paper is silent on these):
#  * colour error |C*(u) - C_k(u)|: the mean over the three channels of the
#    absolute difference (the per-pixel L1 of the loss), tested as the binary32
#    sum (|e0| + |e1|) + |e2| > 3 delta_c (threshold computed in binary64,
#    rounded once); W_G(u) < delta_W in binary32; pixels where the SDF ray
#    missed (D_t = 0) have no surface point and are left out of the mask;
#  * the 25 % uniform sample: a pixel of the mask is taken when the caller's
#    uniform number for it is below the fraction (binary32);
#  * V*(u): the camera-frame point (u - c_x) d / f_x, (v - c_y) d / f_y, d of the
#    SDF depth d = D_t(u), taken to the world frame; N*(u): the normalised cross
#    product of the central differences of V* along x and along y, turned to
#    face the camera; where a neighbour is missing, the direction to the camera;
#  * App. A: the three mask vertices nearest to V*(u) are searched among the mask
#    pixels of the (2R + 1)^2 window around u (R = 4; the whole mask would be a
#    quadratic search), nearest first, ties by pixel index; s1 = min(0.1,
#    sqrt(mean of their distances)), s2 = s1, s3 = 0.1 s1 (a disc whose short
#    axis is the normal); with no such vertex, s1 = 0.1;
#  * rotation: the quaternion (w, x, y, z) that turns the local z axis onto the
#    normal, (1 + n_z, -n_y, n_x, 0) normalised, (0, 1, 0, 0) when n = -z;
#  * opacity 0.5 (logit 0), colour C_k(u); new Gaussians in row-major pixel order.
INSERT_DEFAULTS = {"delta_c": 0.05, "delta_w": 4.0, "fraction": 0.25, "scale_cap": 0.1,
                   "flat_ratio": 0.1, "opacity": 0.5}


def insertion_mask(render_rgb, frame_rgb, weight, sdf_depth, delta_c=0.05, delta_w=4.0):
    """Eq. 6 mask (binary32 decisions), [H][W] bool: an SDF surface, colour error (the
    mean of the three absolute channel differences, as (|e0| + |e1|) + |e2| > 3 delta_c)
    and Gaussian weight below delta_W.  Elementwise binary32 array arithmetic rounds
    every operation once, as a scalar loop would."""
    C = np.asarray(render_rgb, np.float32)
    K = np.asarray(frame_rgb, np.float32)
    t_c, t_w = np.float32(3.0 * delta_c), np.float32(delta_w)
    Wg = np.asarray(weight, np.float32)
    D = np.asarray(sdf_depth, np.float32)
    e = (np.abs(C[0] - K[0]) + np.abs(C[1] - K[1])) + np.abs(C[2] - K[2])
    assert e.dtype == np.float32
    return (D > 0) & (e > t_c) & (Wg < t_w)


def _vertex_map(cam, D):
    """World points V*(u) of every pixel with depth D (binary64), [H][W][3]; 0 where D = 0."""
    H, W = D.shape
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64).reshape(3)
    jj, ii = np.mgrid[0:H, 0:W]
    d = D.astype(np.float64)
    xc = np.stack([(ii - float(cam["cx"])) / float(cam["fx"]) * d, (jj - float(cam["cy"])) / float(cam["fy"]) * d, d],
                  axis=-1)
    V = (xc - t) @ R  # rows of R^T (x - t)
    V[D <= 0] = 0.0
    return V


def insert_gaussians(cam, render_rgb, frame_rgb, weight, sdf_depth, rand, delta_c=0.05, delta_w=4.0,
                     fraction=0.25, scale_cap=0.1, flat_ratio=0.1, opacity=0.5):
    """New Gaussians for the sampled mask pixels (dict of [rows][n] float64 arrays) and
    their pixel indices (row-major).

    Appendix A: the scale comes from the three mask vertices V*(u_1..3), u_k in the
    whole mask M (not only the sample), closest to V*(u); u itself is not its own
    neighbour.  The formula prints the square root of the mean distance; it is read
    as the root mean square of the three distances (the 3DGS / RTG-SLAM
    initialisation it follows): s1 = min(scale_cap, sqrt(mean of d_k^2)), s2 = s1,
    s3 = flat_ratio * s1.  With fewer than three other mask vertices the mean runs
    over those there are; with none, s1 = scale_cap.  The neighbours are found by
    brute force over every mask vertex (binary64 distances)."""
    D = np.asarray(sdf_depth, np.float32)
    H, W = D.shape
    K = np.asarray(frame_rgb, np.float32)
    mask = insertion_mask(render_rgb, frame_rgb, weight, sdf_depth, delta_c, delta_w)
    take = mask & (np.asarray(rand, np.float32) < np.float32(fraction))
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    center = -R.T @ np.asarray(cam["t"], np.float64).reshape(3)
    V = _vertex_map(cam, D)
    valid = D > 0
    mask_idx = np.nonzero(mask.reshape(-1))[0]
    mask_V = V.reshape(-1, 3)[mask_idx]
    pix = [(j, i) for j in range(H) for i in range(W) if take[j, i]]
    out = {"mean": [], "log_scale": [], "quat": [], "opacity_logit": [], "rgb": []}
    for (j, i) in pix:
        p = V[j, i]
        if 0 < i < W - 1 and 0 < j < H - 1 and valid[j, i - 1] and valid[j, i + 1] and valid[j - 1, i] and valid[j + 1, i]:
            n = np.cross(V[j, i + 1] - V[j, i - 1], V[j + 1, i] - V[j - 1, i])
            nn = np.linalg.norm(n)
            n = n / nn if nn > 0 else center - p
        else:
            n = center - p
        n = n / np.linalg.norm(n)
        if np.dot(n, center - p) < 0:
            n = -n
        # the three nearest other mask vertices: squared distances to every mask vertex
        d2 = ((mask_V - p) ** 2).sum(axis=1)
        others = mask_idx != j * W + i
        d2 = np.sort(d2[others])[:3]
        s1 = scale_cap if d2.size == 0 else min(scale_cap, float(np.sqrt(d2.mean())))
        q = np.array([1.0 + n[2], -n[1], n[0], 0.0])
        q = q / np.linalg.norm(q) if np.linalg.norm(q) > 1e-12 else np.array([0.0, 1.0, 0.0, 0.0])
        out["mean"].append(p)
        out["log_scale"].append(np.log([s1, s1, flat_ratio * s1]))
        out["quat"].append(q)
        out["opacity_logit"].append([np.log(opacity / (1.0 - opacity))])
        out["rgb"].append(K[:, j, i].astype(np.float64))
    rows = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "rgb": 3}
    res = {k: np.array(v, np.float64).T.reshape(rows[k], len(pix)) if pix else np.zeros((rows[k], 0))
           for k, v in out.items()}
    return res, np.array([j * W + i for (j, i) in pix], np.int64)
