"""Pins of the reference's binary32 decisions against the definitions evaluated in binary64.

Where floating point decides an integer, the reference takes the decision in binary32 with
a fixed order of operations (the precision the GPU kernels decide in).  Each decision
below is checked against the same definition evaluated in binary64: they must agree
wherever the binary64 value is farther from the decision's threshold than binary32
rounding can reach, and the disagreements (counted and printed) may only sit within
that reach.

* Fusion (Sec. 3.2.1): which lattice points a frame updates, the pixel each one reads
  (the nearest pixel of its projection) and the truncation test eta >= -mu; observed
  through the reference's fused values on a frame whose depth differs at every pixel.
* Raycast (Sec. 3.1 first pass): the sample at which the march finds the first
  positive-to-non-positive change of the trilinear signed distance, against a binary64
  march whose trilinear interpolation is scipy's (map_coordinates, order 1).
* Depth key and depth test (Eq. 1-2): the binary32 camera depth that orders the
  Gaussians and is compared with D_t + eps, against the binary64 depth of the centre.
"""
import numpy as np
import scipy.ndimage as ndi

import synth
from oracle import oracle as O


def _frame(W=160, H=120, frame=5):
    scene = synth.scene_room(128)
    cam = synth.orbit_cameras(0, W, H, frames=[frame])[0]
    d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=2e-3, frame_index=frame)
    return scene, cam.as_dict(), d, c


def test_fusion_decisions():
    scene, cam, d, c = _frame()
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    vol = O.fuse(grid, O.new_volume(grid), cam, d, c)
    nx, ny, nz = scene.dims
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    org = np.array([grid.origin[k] for k in range(3)], np.float64)
    vox = float(np.float32(grid.voxel))
    p = np.stack([org[0] + vox * xx.reshape(-1), org[1] + vox * yy.reshape(-1), org[2] + vox * zz.reshape(-1)])
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    pc = R @ p + t[:, None]
    fx, fy, cx, cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    H, W = d.shape
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * pc[0] / pc[2] + cx
        v = fy * pc[1] / pc[2] + cy
    iu, iv = np.floor(u + 0.5), np.floor(v + 0.5)
    inside = (pc[2] > 0) & (iu >= 0) & (iu < W) & (iv >= 0) & (iv < H)
    dpx = np.zeros(pc.shape[1])
    dpx[inside] = d[iv[inside].astype(int), iu[inside].astype(int)]
    mu = float(np.float32(grid.trunc))
    eta = dpx - pc[2]
    upd64 = inside & (dpx > 0) & (eta >= -mu)
    # decisions within binary32 reach: a projection near a pixel edge, eta near -mu, z near 0
    near = inside & ((np.abs(u + 0.5 - np.round(u + 0.5)) < 1e-4) | (np.abs(v + 0.5 - np.round(v + 0.5)) < 1e-4) |
                     (np.abs(eta + mu) < 1e-5))
    upd = vol["weight"] > 0
    flips = upd != upd64
    assert upd64.sum() > 100_000
    assert not (flips & ~near).any(), int((flips & ~near).sum())
    # the pixel read: the fused value is min(1, eta / mu) of that pixel's depth
    both = upd & upd64 & ~near
    want = np.minimum(1.0, eta[both] / mu)
    assert np.abs(vol["tsdf"][both] - want).max() < 1e-6
    print(f"fusion: {int(upd64.sum())} points updated, {int(near.sum())} within binary32 reach of a pixel edge "
          f"or the truncation, {int(flips.sum())} decisions differ")


def test_raycast_crossing_sample():
    scene, cam, d, c = _frame()
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    vol = O.fuse(grid, O.new_volume(grid), cam, d, c)
    t32 = vol["tsdf"].astype(np.float32)
    nx, ny, nz = scene.dims
    F = t32.reshape(nz, ny, nx).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(2))
    H, W = d.shape
    pix = np.sort(rng.choice(W * H, 400, replace=False)).astype(np.int32)
    _, _, rk = O.raycast(grid, t32, vol["rgb"].astype(np.float32), cam, z_near=0.2, pix=pix)
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    o = -R.T @ t
    fx, fy, cx, cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    org = np.array([grid.origin[k] for k in range(3)], np.float64)
    vox = float(np.float32(grid.voxel))
    h = vox / 2
    n = np.array([nx, ny, nz])
    agree = near = 0
    for k, p in enumerate(pix):
        col, row = p % W, p // W
        r = np.array([(col - cx) / fx, (row - cy) / fy, 1.0])
        dirw = R.T @ r / np.linalg.norm(r)
        lam0, lam1 = 0.2 * np.linalg.norm(r), np.inf
        for a in range(3):
            lo, hi = org[a], org[a] + vox * (n[a] - 1)
            t1, t2 = (lo - o[a]) / dirw[a], (hi - o[a]) / dirw[a]
            lam0, lam1 = max(lam0, min(t1, t2)), min(lam1, max(t1, t2))
        ns = int(np.floor((lam1 - lam0) / h))
        lam = lam0 + h * np.arange(ns + 1)
        g = (o[:, None] + lam[None] * dirw[:, None] - org[:, None]) / vox  # lattice coordinates
        ins = ((np.floor(g) >= 0) & (np.floor(g) <= (n[:, None] - 2))).all(axis=0)
        Fv = np.where(ins, ndi.map_coordinates(F, g[::-1], order=1, mode="nearest"), 1.0)
        cross = np.flatnonzero((Fv[:-1] > 0) & (Fv[1:] <= 0))
        hit64 = int(cross[0]) + 1 if cross.size else -1
        if hit64 == rk[k]:
            agree += 1
            continue
        # a difference is allowed only where a deciding value is within binary32 reach of 0
        s = [x for x in (hit64, rk[k]) if x >= 0]
        amb = any(abs(Fv[x]) < 1e-5 or abs(Fv[x - 1]) < 1e-5 for x in s)
        assert amb, (int(p), hit64, int(rk[k]))
        near += 1
    assert (rk >= 0).sum() > 300
    print(f"raycast: {agree} of {pix.size} crossing samples equal, {near} differ within binary32 reach of 0")


def test_depth_key_and_depth_test():
    scene = synth.scene_room()
    cams = synth.orbit_cameras(0, 320, 240, frames=list(range(0, 100, 10)))
    depths = [synth.render_frame(scene, c)[0] for c in cams]
    g = synth.seed_gaussians(scene, cams, depths, 20_000)
    cam = cams[3].as_dict()
    pr = O.project(O.RenderCfg(eps_cull=scene.voxel), g, cam)
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    z64 = R[2] @ g["mean"].astype(np.float64) + t[2]
    z32 = pr["depth32"].astype(np.float64)
    # the binary32 depth is within a few roundings of the binary64 one
    assert np.abs(z32 - z64).max() <= 4 * 2.0 ** -24 * (np.abs(R[2]) @ np.abs(g["mean"]) + abs(t[2])).max()
    # the order of the keys (ties by index) is the binary64 order except for near ties
    o32 = np.lexsort((np.arange(z32.size), z32))
    o64 = np.argsort(z64, kind="stable")
    pos64 = np.empty_like(o64)
    pos64[o64] = np.arange(o64.size)
    inv = np.flatnonzero(np.diff(pos64[o32]) < 0)
    for i in inv:
        a, b = o32[i], o32[i + 1]
        assert abs(z64[a] - z64[b]) < 1e-6 * abs(z64[a]), (a, b, z64[a], z64[b])
    # the depth test of Eq. 1-2 (binary32: z32 < D_t + eps) against binary64, on random D_t
    rng = np.random.Generator(np.random.PCG64(3))
    Dt = (z64 + rng.normal(0.0, 0.02, z64.size)).astype(np.float32)
    eps = np.float32(scene.voxel)
    dec32 = pr["depth32"] < (Dt + eps).astype(np.float32)
    dec64 = z64 < Dt.astype(np.float64) + float(eps)
    near = np.abs(z64 - (Dt.astype(np.float64) + float(eps))) < 1e-6 * np.abs(z64)
    assert not ((dec32 != dec64) & ~near).any()
    print(f"depth key: {inv.size} adjacent near-ties ordered differently; depth test: "
          f"{int((dec32 != dec64).sum())} of {z64.size} decisions differ, all within binary32 reach")
