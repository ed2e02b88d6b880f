"""Pins of the oracle's TSDF fusion and SDF raycast, its loss and its Adam step (CPU only)."""
import math

import numpy as np
import pytest
import torch


def _plane_setup(oracle, Z=1.41, col=(0.2, 0.6, 0.9), n=16, voxel=0.05, mu=0.1, wmax=100.0):
    W = H = 64
    cam = {"width": W, "height": H, "fx": 40.0, "fy": 40.0, "cx": 32.0, "cy": 32.0,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    origin = (-0.375, -0.375, 1.0)
    grid = oracle.make_grid((n, n, n), origin, voxel, mu, wmax)
    depth = np.full((H, W), Z, np.float32)
    rgb = np.broadcast_to(np.asarray(col, np.float32)[:, None, None], (3, H, W)).copy()
    return cam, grid, depth, rgb


def test_fusion_plane_closed_form(oracle):
    """A fronto-parallel plane at depth Z seen by a camera whose frustum holds the whole lattice:
    tsdf(v) = min(1, (Z - z_v)/mu) where Z - z_v >= -mu, untouched (1, weight 0) behind that, and the
    colour equals the plane colour inside the band |Z - z_v| <= mu."""
    cam, grid, depth, rgb = _plane_setup(oracle)
    vol = oracle.new_volume(grid)
    oracle.fuse(grid, vol, cam, depth, rgb)
    n = grid.nx
    k = np.arange(n)
    zv = float(np.float32(1.0)) + float(np.float32(0.05)) * k  # lattice z as the grid's float32 fields give it
    eta = float(np.float32(1.41)) - zv
    mu = float(np.float32(0.1))
    exp_t = np.where(eta >= -mu, np.minimum(1.0, eta / mu), 1.0)
    exp_w = np.where(eta >= -mu, 1.0, 0.0)
    band = np.abs(eta) <= mu
    tsdf = vol["tsdf"].reshape(n, n, n)  # [z][y][x]
    np.testing.assert_allclose(tsdf, np.broadcast_to(exp_t[:, None, None], tsdf.shape), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(vol["weight"].reshape(n, n, n), np.broadcast_to(exp_w[:, None, None], (n, n, n)))
    col = vol["rgb"].reshape(3, n, n, n)
    for c in range(3):
        expect = np.where(band, float(np.float32((0.2, 0.6, 0.9)[c])), 0.0)
        np.testing.assert_allclose(col[c], np.broadcast_to(expect[:, None, None], (n, n, n)), atol=1e-15)


def test_fusion_repeat_invariants(oracle):
    """Fusing the same frame again leaves every value unchanged and adds one to each weight, which
    saturates at max_weight."""
    cam, grid, depth, rgb = _plane_setup(oracle, wmax=3.0)
    vol = oracle.new_volume(grid)
    oracle.fuse(grid, vol, cam, depth, rgb)
    first = {k: v.copy() for k, v in vol.items()}
    for rep in range(2, 6):
        oracle.fuse(grid, vol, cam, depth, rgb)
        np.testing.assert_allclose(vol["tsdf"], first["tsdf"], atol=1e-14)
        np.testing.assert_allclose(vol["rgb"], first["rgb"], atol=1e-14)
        np.testing.assert_array_equal(vol["weight"], np.minimum(first["weight"] * rep, 3.0))
        assert vol["weight"].max() <= 3.0 and vol["rgb_weight"].max() <= 3.0


def test_raycast_plane_closed_form(oracle):
    """Within the band the fused field is linear along z, and both the trilinear interpolation and
    the secant step are exact on linear fields, so the raycast returns D_t = Z and C_t = the plane
    colour; rays that leave the lattice without a crossing return D_t = 0."""
    cam, grid, depth, rgb = _plane_setup(oracle)
    vol = oracle.new_volume(grid)
    oracle.fuse(grid, vol, cam, depth, rgb)
    d, c, k = oracle.raycast(grid, vol["tsdf"].astype(np.float32), vol["rgb"].astype(np.float32), cam)
    W = cam["width"]
    jj, ii = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    central = ((ii >= 24) & (ii <= 40) & (jj >= 24) & (jj <= 40)).reshape(-1)
    assert (k[central] > 0).all()
    np.testing.assert_allclose(d[central], float(np.float32(1.41)), atol=2e-6)
    for ch, val in enumerate((0.2, 0.6, 0.9)):
        np.testing.assert_allclose(c[ch, central], float(np.float32(val)), atol=1e-6)
    corner = ((ii < 8) & (jj < 8)).reshape(-1)
    assert (d[corner] == 0).all() and (k[corner] == -1).all()


def test_trilinear_matches_grid_sample(oracle):
    """The binary64 trilinear interpolation equals torch.nn.functional.grid_sample(align_corners=True)."""
    rng = np.random.Generator(np.random.PCG64(3))
    nx, ny, nz = 5, 6, 7
    grid = oracle.make_grid((nx, ny, nz), (0.1, -0.2, 0.3), 0.25, 0.5)
    f = rng.normal(size=nx * ny * nz).astype(np.float32)
    vox = np.float32(0.25)
    o = np.float32([0.1, -0.2, 0.3]).astype(np.float64)
    gpts = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(50, 3))
    pts = o + gpts * float(vox)
    vals = np.array([oracle.trilinear(grid, f, p) for p in pts])
    inp = torch.as_tensor(f.astype(np.float64).reshape(1, 1, nz, ny, nx))
    gn = (pts - o) / float(vox) / np.array([nx - 1, ny - 1, nz - 1]) * 2 - 1
    ref = torch.nn.functional.grid_sample(inp, torch.as_tensor(gn).reshape(1, 1, 1, 50, 3), mode="bilinear",
                                          align_corners=True).reshape(-1).numpy()
    np.testing.assert_allclose(vals, ref, rtol=1e-12, atol=1e-12)


def _sphere_depth(cam, c, r):
    W, H = cam["width"], cam["height"]
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d = np.stack([(ii - cam["cx"]) / cam["fx"], (jj - cam["cy"]) / cam["fy"], np.ones_like(ii, float)], -1)
    rn = np.linalg.norm(d, axis=-1)
    u = d / rn[..., None]
    b = u @ (-c)
    disc = b * b - (c @ c - r * r)
    t = -b - np.sqrt(np.maximum(disc, 0))
    return np.where(disc > 0, t / rn, 0.0).astype(np.float32)


def test_sphere_fuse_and_raycast_bound(oracle):
    """A sphere fused from one viewpoint and raycast from it: away from the silhouette the depth is
    within one voxel of the analytic depth, and the fused signed distance has the sign of the true
    signed distance for voxels in the band more than two voxels from the surface."""
    W, H, f = 96, 72, 80.0
    cam = {"width": W, "height": H, "fx": f, "fy": f, "cx": 48.0, "cy": 36.0,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    c, r = np.array([0.02, -0.03, 1.6]), 0.3
    n, voxel = 48, 0.02
    origin = (-0.47, -0.47, 1.1)
    grid = oracle.make_grid((n, n, n), origin, voxel, 4 * voxel)
    depth = _sphere_depth(cam, c, r)
    rgb = np.full((3, H, W), 0.5, np.float32)
    vol = oracle.new_volume(grid)
    oracle.fuse(grid, vol, cam, depth, rgb)
    d, _, _ = oracle.raycast(grid, vol["tsdf"].astype(np.float32), vol["rgb"].astype(np.float32), cam)
    d = d.reshape(H, W)
    inner = np.zeros((H, W), bool)
    inner[2:-2, 2:-2] = True
    for dy in (-2, -1, 0, 1, 2):
        for dx in (-2, -1, 0, 1, 2):
            inner &= np.roll(np.roll(depth > 0, dy, 0), dx, 1)
    assert inner.sum() > 500
    assert np.abs(d[inner] - depth[inner]).max() <= voxel
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    P = np.stack([origin[0] + voxel * xx, origin[1] + voxel * yy, origin[2] + voxel * zz], -1).reshape(-1, 3)
    sdf = np.linalg.norm(P - c, axis=1) - r
    band = (vol["weight"] > 0) & (np.abs(vol["tsdf"]) < 1) & (np.abs(sdf) > 2 * voxel)
    agree = np.sign(vol["tsdf"][band]) == np.sign(sdf[band])
    assert band.sum() > 1000 and agree.mean() > 0.99


def test_loss_matches_torch_l1(oracle):
    """L = l1(C*, C_obs) + lambda l1(D*, D_obs over Omega) with torch's mean-reduced L1, and its
    gradient equals autograd of that expression."""
    rng = np.random.Generator(np.random.PCG64(9))
    W, H = 20, 15
    rgb = rng.uniform(size=(3, H * W))
    depth = rng.uniform(1, 2, size=H * W)
    trgb = rng.uniform(size=(3, H, W)).astype(np.float32)
    tdep = rng.uniform(1, 2, size=(H, W)).astype(np.float32)
    tdep[rng.uniform(size=(H, W)) < 0.2] = 0
    bdep = rng.uniform(1, 2, size=(H, W)).astype(np.float32)
    bdep[rng.uniform(size=(H, W)) < 0.2] = 0
    cfg = oracle.RenderCfg(lambda_depth=0.7)
    L, gr, gd, om = oracle.loss(cfg, W, H, rgb, depth, trgb, tdep, bdep, scale=2.0)
    C = torch.tensor(rgb, requires_grad=True)
    D = torch.tensor(depth, requires_grad=True)
    mask = torch.as_tensor((tdep.reshape(-1) > 0) & (bdep.reshape(-1) > 0))
    lam = float(np.float32(0.7))
    ref = torch.nn.functional.l1_loss(C, torch.as_tensor(trgb.reshape(3, -1).astype(np.float64))) + \
        lam * torch.nn.functional.l1_loss(D[mask], torch.as_tensor(tdep.reshape(-1).astype(np.float64))[mask])
    (2.0 * ref).backward()
    assert om == int(mask.sum())
    assert L == pytest.approx(float(ref.detach()), rel=1e-13)
    np.testing.assert_allclose(gr, C.grad.numpy(), rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(gd, D.grad.numpy(), rtol=1e-13, atol=1e-18)


def test_adam_matches_torch(oracle):
    """Three Adam steps (beta1 0.9, beta2 0.999, eps 1e-15, lr of the position group) equal
    torch.optim.Adam in float64."""
    rng = np.random.Generator(np.random.PCG64(10))
    p0 = rng.normal(size=1000)
    grads = [rng.normal(size=1000) * 10 ** rng.uniform(-6, 1, 1000) for _ in range(3)]
    grads[1][:10] = 0.0
    lr = oracle.PAPER_LR["mean"]
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lr, betas=(0.9, 0.999), eps=1e-15)
    for t, g in enumerate(grads, start=1):
        oracle.adam(p, g, m, v, lr, t)
        tp.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_paper_learning_rates(oracle):
    """The per-attribute learning rates are the ones printed in Appendix C (golden fixture)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    lr = gold["learning_rates"]["values"]
    assert oracle.PAPER_LR == {"mean": lr["position"], "rgb": lr["SH0"], "opacity_logit": lr["alpha"],
                               "log_scale": lr["scale"], "quat": lr["rotation"], "sh": lr["SH_rest"]}
    assert oracle.RenderCfg().alpha_min == gold["alpha_threshold"]["value"]
