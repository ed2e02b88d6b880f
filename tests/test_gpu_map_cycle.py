"""Map maintenance driven by the renderer (Sec. 3.2.2): insertion (Eq. 6, App. A) from
the colour C* and the Gaussian weight W_G (Eq. 2) of a real sort-free render over the
SDF image, then optimisation, then removal (Eq. 8).

* Parity: the GPU renders and inserts; the reference renders the same Gaussians over
  the same SDF images (its own binary64 C* and W_G) and inserts from those.  The taken
  pixels agree except where the reference's colour error or weight lies within
  rounding reach of delta_c or delta_W (both sides decide in binary32 from their own
  render); at the common pixels the new Gaussians agree to the insertion tolerances,
  the log-scale only where no flipped mask vertex can be among the three nearest.
* A GPU-only keyframe loop on the room (fusion, raycast, sort-free render, insertion,
  ten optimisation iterations with Adam in the backward's epilogue, removal), checked
  by properties that hold at any size: the map grows by exactly the taken pixels, new
  Gaussians sit on the SDF surface at their pixel with opacity 0.5 and the frame's
  colour, the loss falls, and removal keeps exactly the Gaussians that pass Eq. 8
  (decided in binary64 here, away from the thresholds' rounding), in order, with their
  moments.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, cfg_pair, h, say, t

pytestmark = pytest.mark.gpu
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
ROWS = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "rgb": 3}


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    P.lib()
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.lib()
    return O


def _seed(scene, W, H, M, frames=range(0, 100, 10)):
    cams = synth.orbit_cameras(0, W, H, frames=list(frames))
    depths = [synth.render_frame(scene, c)[0] for c in cams]
    return synth.seed_gaussians(scene, cams, depths, M)


def test_insertion_from_sort_free_render(P, O):
    say("map cycle: insertion from a sort-free render, 320x240, 20k Gaussians")
    W, H, M = 320, 240, 20_000
    scene = synth.scene_room()
    cam = synth.orbit_cameras(0, W, H, frames=[7])[0]
    camd = cam.as_dict()
    d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=7)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    ref = O.fuse(grid, O.new_volume(grid), camd, d, c)
    rd, rc, _ = O.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), camd)
    base_rgb = rc.reshape(3, H, W).astype(np.float32)
    base_depth = rd.reshape(H, W).astype(np.float32)
    gauss = _seed(scene, W, H, M)
    rand = np.random.Generator(np.random.PCG64(17)).uniform(size=(H, W)).astype(np.float32)
    # GPU: sort-free render (C*, W_G), then insertion from those images
    gc, oc = cfg_pair(P, O, mode=1, eps=scene.voxel)
    view = P.View(camd, t(base_rgb), t(base_depth), t(c), t(d), out_aux=torch.empty(H, W, device=DEV))
    ws = P.Workspace(gc, M, [camd], device=DEV)
    P.render_fwd(gc, {k: t(v) for k, v in gauss.items()}, [view], ws)
    out, pix, n_taken = P.insert_gaussians(camd, view.out_rgb, t(c), view.out_aux, t(base_depth), t(rand))
    torch.cuda.synchronize()
    gpix = h(pix).astype(np.int64) if pix.numel() else np.zeros(0, np.int64)
    got = {k: h(out[k]).astype(np.float64).reshape(ROWS[k], -1) for k in KEYS}
    # reference: its own render, its own insertion
    r = O.render(oc, gauss, camd, base_rgb, base_depth)
    C_ref, W_ref = r["rgb"].reshape(3, H, W), r["W"].reshape(H, W)
    # pixels where a 1/255 test or the depth test is within rounding reach (flagged by the
    # reference) may count a Gaussian on one side only: W_G then differs by about 1/255
    flagged = (r["flag"] != 0).reshape(H, W)
    assert flagged.mean() < 0.02
    assert np.abs(h(view.out_aux) - W_ref)[~flagged].max() <= 1e-4 * max(1.0, W_ref.max())
    want, wpix = O.insert_gaussians(camd, C_ref, c, W_ref, base_depth, rand)
    wpix = np.asarray(wpix, np.int64)
    # decisions within rounding reach of a threshold (the reference's binary64 values)
    e = np.abs(C_ref - c.astype(np.float64)).sum(axis=0)
    near = (np.abs(e - 0.15) <= 1e-4) | (np.abs(W_ref - 4.0) <= 1e-4 * 4.0) | flagged
    near_flat = near.reshape(-1)
    flips = np.setxor1d(gpix, wpix)
    say(f"  taken: GPU {gpix.size}, reference {wpix.size}, flipped {flips.size}, "
        f"near-threshold pixels {int(near.sum())}")
    assert wpix.size > 200 and n_taken == gpix.size
    assert near_flat[flips].all(), flips[~near_flat[flips]]
    # mask pixels that differ (not only taken ones): their vertices may change neighbours
    m_gpu = O.insertion_mask(h(view.out_rgb), c, h(view.out_aux), base_depth)
    m_ref = O.insertion_mask(C_ref, c, W_ref, base_depth)
    mflip = np.flatnonzero((m_gpu != m_ref).reshape(-1))
    assert near_flat[mflip].all()
    common, gi, wi = np.intersect1d(gpix, wpix, return_indices=True)
    g = {k: got[k][:, gi] for k in KEYS}
    w = {k: want[k][:, wi] for k in KEYS}
    np.testing.assert_array_equal(g["rgb"], w["rgb"])
    np.testing.assert_allclose(g["opacity_logit"], w["opacity_logit"], rtol=0, atol=1e-7)
    np.testing.assert_allclose(g["mean"], w["mean"], rtol=0, atol=4e-6)
    s1 = np.exp(w["log_scale"][0])
    if mflip.size:
        # vertex of each flipped mask pixel (back-projected SDF depth, world frame)
        R = np.asarray(camd["R"], np.float64).reshape(3, 3)
        tv = np.asarray(camd["t"], np.float64)
        jj, ii = np.divmod(mflip, W)
        dd = base_depth.reshape(-1)[mflip].astype(np.float64)
        xc = np.stack([(ii - camd["cx"]) / camd["fx"] * dd, (jj - camd["cy"]) / camd["fy"] * dd, dd])
        vf = R.T @ (xc - tv[:, None])
        dist = np.linalg.norm(w["mean"][:, :, None] - vf[:, None, :], axis=0).min(axis=1)
        safe = dist > np.sqrt(3.0) * s1 * 1.01
    else:
        safe = np.ones(common.size, bool)
    assert safe.mean() > 0.9
    np.testing.assert_allclose(g["log_scale"][:, safe], w["log_scale"][:, safe], rtol=0, atol=1e-4)


def _removal_keep64(p):
    """Eq. 8 in binary64 on the stored values, and the decisions within rounding reach."""
    o = p["opacity_logit"].astype(np.float64).reshape(-1)
    sig = 1.0 / (1.0 + np.exp(-o))
    smax = np.exp(p["log_scale"].astype(np.float64).max(axis=0))
    keep = (sig >= 0.005) & (smax <= 0.1) & (smax >= 0.003)
    near = (np.abs(sig - 0.005) <= 1e-6 * 0.005) | (np.abs(smax - 0.1) <= 1e-6 * 0.1) | \
        (np.abs(smax - 0.003) <= 1e-6 * 0.003)
    return keep, near


def test_keyframe_loop_properties(P):
    say("map cycle: three keyframes of the room at 320x240 (insert, optimise, remove)")
    from paper_2509_11574_amd.mapping import GaussianMap, insert_from_render
    W, H = 320, 240
    scene = synth.scene_room()
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=DEV)
    gmap = GaussianMap(P.gaussians_to_device(_seed(scene, W, H, 5_000), DEV))
    cfg = P.RenderCfg(eps_cull=scene.voxel)
    rng = np.random.Generator(np.random.PCG64(23))
    for f in (0, 10, 20):
        cam = synth.orbit_cameras(0, W, H, frames=[f])[0]
        camd = cam.as_dict()
        d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=f, device=DEV, as_torch=True)
        P.fuse(vol, camd, d, c)
        (bd, bc), = P.raycast(vol, [camd], z_near=cfg.z_near)
        view = P.View(camd, bc, bd, c, d)
        n0 = gmap.count
        rand = t(rng.uniform(size=(H, W)))
        new, pix, n_taken = insert_from_render(gmap, cfg, view, rand)
        torch.cuda.synchronize()
        assert gmap.count == n0 + n_taken and n_taken == pix.numel() > 50, (n0, n_taken, gmap.count)
        # new Gaussians: on the SDF surface at their pixel, opacity 0.5, the frame's colour
        pp = h(pix).astype(np.int64)
        mu = h(new["mean"]).astype(np.float64)
        R = np.asarray(camd["R"], np.float64).reshape(3, 3)
        pc = R @ mu + np.asarray(camd["t"], np.float64)[:, None]
        zt = h(bd).reshape(-1)[pp]
        assert np.abs(pc[2] - zt).max() <= 1e-5 * zt.max()
        u = camd["fx"] * pc[0] / pc[2] + camd["cx"]
        v = camd["fy"] * pc[1] / pc[2] + camd["cy"]
        assert np.abs(u - pp % W).max() < 1e-3 and np.abs(v - pp // W).max() < 1e-3
        assert (h(new["opacity_logit"]) == 0.0).all()
        np.testing.assert_array_equal(h(new["rgb"]), h(c).reshape(3, -1)[:, pp])
        # ten iterations of optimisation on the grown map
        ws = P.Workspace(cfg, gmap.count, [camd], device=DEV)
        loss = torch.zeros(1, device=DEV)
        losses = []
        for _ in range(10):
            P.render_fwd(cfg, gmap.params, [view], ws, out_loss=loss)
            losses.append(float(loss.item()))
            P.render_bwd_adam(cfg, gmap.params, [view], ws, gmap.opt)
        torch.cuda.synchronize()
        assert ws.status() == 0
        assert losses[-1] < losses[0], losses
        # removal with both moments: exactly the Gaussians that pass Eq. 8, in order
        before = {k: h(v).reshape(ROWS[k], -1) for k, v in gmap.params.items()}
        mb = {k: h(v).reshape(ROWS[k], -1) for k, v in gmap.opt.m.items()}
        keep, near = _removal_keep64(before)
        n_kept = gmap.prune()
        torch.cuda.synchronize()
        assert not near.any()
        assert n_kept == int(keep.sum()) and gmap.count == n_kept
        for k in KEYS:
            np.testing.assert_array_equal(h(gmap.params[k]).reshape(ROWS[k], -1), before[k][:, keep])
            np.testing.assert_array_equal(h(gmap.opt.m[k]).reshape(ROWS[k], -1), mb[k][:, keep])
        say(f"  frame {f}: +{n_taken} Gaussians, loss {losses[0]:.5f} -> {losses[-1]:.5f}, "
            f"kept {n_kept} of {keep.size}")
