"""GPU parity at the benchmark's full sizes, on outputs the reference computes one by one.

* room at 1 cm: 256^3 lattice, two 1280x720 frames, 100,000 Gaussians -- fusion compared on
  every lattice point, raycast on every pixel, render forward on 2,000 sampled pixels,
  backward with the upstream adjoint placed on those pixels, the fused loss against the L1 of
  the output images, Adam on every parameter;
* batch of 8 keyframes of mixed resolution (3x1280x720, 3x640x480, 2x320x240) sharing
  300,000 Gaussians in one call -- 150 sampled pixels per view, forward and backward;
* room at 5 mm: 512^3 fusion of one 1280x720 frame, every lattice point.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, cfg_pair, gauss_dev, h, normwise, report_flags, say, t

pytestmark = pytest.mark.gpu
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.lib()
    return O


def _seed_gaussians(scene, W, H, M):
    cams = synth.orbit_cameras(0, W, H, frames=list(range(0, 100, 10)))
    depths = [synth.render_frame(scene, c)[0] for c in cams]
    return synth.seed_gaussians(scene, cams, depths, M)


@pytest.fixture(scope="module")
def room(O):
    say("full-size room: building inputs and the reference fusion/raycast")
    scene, fr = synth.workload_room_frames(frames=[0, 1])
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    ref = O.new_volume(grid)
    for cam, d, c in fr:
        O.fuse(grid, ref, cam.as_dict(), d, c)
    t32, c32 = ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32)
    cam1 = fr[1][0]
    rd, rc, rk = O.raycast(grid, t32, c32, cam1.as_dict(), z_near=0.2)
    gauss = _seed_gaussians(scene, 1280, 720, 100_000)
    rng = np.random.Generator(np.random.PCG64(77))
    pix = np.sort(rng.choice(1280 * 720, 2000, replace=False)).astype(np.int32)
    return {"scene": scene, "frames": fr, "grid": grid, "ref": ref, "t32": t32, "c32": c32, "rd": rd, "rc": rc,
            "rk": rk, "gauss": gauss, "pix": pix}


def test_room_fusion_every_point(P, O, room):
    sc = room["scene"]
    vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, device=DEV)
    for cam, d, c in room["frames"]:
        P.fuse(vol, cam.as_dict(), t(d), t(c))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h(vol.weight), room["ref"]["weight"].astype(np.float32))
    np.testing.assert_array_equal(h(vol.rgb_weight), room["ref"]["rgb_weight"].astype(np.float32))
    assert np.abs(h(vol.tsdf) - room["ref"]["tsdf"]).max() < 2e-5
    assert np.abs(h(vol.rgb) - room["ref"]["rgb"]).max() < 2e-5


def test_room_raycast_every_pixel(P, O, room):
    sc = room["scene"]
    vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, device=DEV)
    vol.tsdf.copy_(t(room["t32"]))
    vol.rgb.copy_(t(room["c32"]))
    (gd, gc), = P.raycast(vol, [room["frames"][1][0].as_dict()], z_near=0.2)
    torch.cuda.synchronize()
    gd, gc = h(gd).reshape(-1), h(gc).reshape(3, -1)
    np.testing.assert_array_equal(gd > 0, room["rk"] >= 0)
    hit = room["rk"] >= 0
    assert hit.mean() > 0.9
    assert np.abs(gd[hit] - room["rd"][hit]).max() <= 1e-4 * room["rd"][hit].max()
    assert normwise(gc, room["rc"]) < 1e-4


@pytest.mark.parametrize("tile", [(16, 16, 256, 1), (16, 32, 128, 2), (16, 32, 256, 2), (16, 16, 128, 4),
                                  (32, 16, 256, 2)])
def test_room_render_sampled(P, O, room, tile):
    say(f"full-size render: 1280x720, 100k Gaussians, tile {tile}")
    cam = room["frames"][1][0].as_dict()
    d1, c1 = room["frames"][1][1], room["frames"][1][2]
    base_rgb = room["rc"].reshape(3, 720, 1280).astype(np.float32)
    base_depth = room["rd"].reshape(720, 1280).astype(np.float32)
    gc, oc = cfg_pair(P, O, eps=room["scene"].voxel, tile=tile)
    view = P.View(cam, t(base_rgb), t(base_depth), t(c1), t(d1))
    ws = P.Workspace(gc, 100_000, [cam], device=DEV)
    gd = gauss_dev(room["gauss"])
    loss = torch.zeros(1, device=DEV)
    P.render_fwd(gc, gd, [view], ws, out_loss=loss)
    torch.cuda.synchronize()
    assert ws.status() == 0
    pix = room["pix"]
    r = O.render(oc, room["gauss"], cam, base_rgb, base_depth, pix=pix)
    keep = r["flag"] == 0
    assert keep.mean() > 0.97
    C = h(view.out_rgb).reshape(3, -1)
    D = h(view.out_depth).reshape(-1)
    assert normwise(C[:, pix], r["rgb"], keep) < 1e-4
    assert normwise(D[pix], r["depth"], keep) < 1e-4
    report_flags("room 1280x720 sampled pixels", keep, C[:, pix], r["rgb"])
    # the fused loss equals the L1 of the output images (a property at any size)
    om = (d1.reshape(-1) > 0) & (base_depth.reshape(-1) > 0)
    L = np.abs(C.astype(np.float64) - c1.reshape(3, -1)).mean() + \
        np.abs(D.astype(np.float64)[om] - d1.reshape(-1)[om]).mean()
    assert abs(loss.item() - L) <= 1e-4 * L
    # backward with the upstream adjoint on the sampled (unflagged) pixels only
    rng = np.random.Generator(np.random.PCG64(78))
    gC = np.zeros((3, 720 * 1280), np.float32)
    gD = np.zeros(720 * 1280, np.float32)
    ps = pix[keep]
    gC[:, ps] = rng.normal(size=(3, ps.size))
    gD[ps] = rng.normal(size=ps.size)
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(1, 6, device=DEV)
    P.render_bwd(gc, gd, [view], ws, grads, dpose, dL_drgb=[t(gC).reshape(3, 720, 1280)],
                 dL_ddepth=[t(gD).reshape(720, 1280)])
    torch.cuda.synchronize()
    ref = O.render_bwd(oc, room["gauss"], cam, base_rgb, base_depth, gC[:, ps], gD[ps], pix=ps)
    for k in KEYS:
        assert normwise(h(grads[k]), ref[k]) < 1e-3, (k, normwise(h(grads[k]), ref[k]))
    assert normwise(h(dpose)[0], ref["pose"]) < 1e-3


def test_room_adam_every_parameter(P, O, room):
    rng = np.random.Generator(np.random.PCG64(79))
    gd = gauss_dev(room["gauss"])
    opt = P.Adam(gd)
    g = {k: (rng.normal(size=v.shape) * 1e-3).astype(np.float32) for k, v in room["gauss"].items()}
    opt.step({k: t(v) for k, v in g.items()})
    torch.cuda.synchronize()
    for k in KEYS:
        p = room["gauss"][k].astype(np.float64).reshape(-1).copy()
        O.adam(p, g[k].astype(np.float64).reshape(-1), np.zeros_like(p), np.zeros_like(p), O.PAPER_LR[k], 1)
        assert np.abs(h(gd[k]).reshape(-1) - p).max() <= 1e-6 * np.abs(p).max() + 1e-7, k


def test_keyframe_batch_sampled(P, O):
    """8 keyframes of mixed resolution and 300k Gaussians in one forward/backward call."""
    say("keyframe batch: 8 views, 300k Gaussians")
    scene = synth.scene_room(256)
    views_np = []
    for (k, W, H) in synth.STANDARD_VIEWS:
        cam = synth.orbit_cameras(0, W, H, frames=[k])[0]
        d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=k)
        # analytic frame (noise free) as the SDF base, the noisy frame as the target
        bd, bc = synth.render_frame(scene, cam)
        views_np.append({"cam": cam.as_dict(), "base_rgb": bc, "base_depth": bd, "target_rgb": c, "target_depth": d})
    gauss = _seed_gaussians(scene, 1280, 720, 300_000)
    gc, oc = cfg_pair(P, O, eps=scene.voxel)
    views = [P.View(v["cam"], t(v["base_rgb"]), t(v["base_depth"]), t(v["target_rgb"]), t(v["target_depth"]))
             for v in views_np]
    ws = P.Workspace(gc, 300_000, [v.cam for v in views], device=DEV)
    gd = gauss_dev(gauss)
    P.render_fwd(gc, gd, views, ws)
    torch.cuda.synchronize()
    assert ws.status() == 0
    rng = np.random.Generator(np.random.PCG64(80))
    ups_rgb, ups_dep, refs = [], [], None
    for v, vn in zip(views, views_np):
        W, H = vn["cam"]["width"], vn["cam"]["height"]
        pix = np.sort(rng.choice(W * H, 150, replace=False)).astype(np.int32)
        r = O.render(oc, gauss, vn["cam"], vn["base_rgb"], vn["base_depth"], pix=pix)
        keep = r["flag"] == 0
        C = h(v.out_rgb).reshape(3, -1)
        assert normwise(C[:, pix], r["rgb"], keep) < 1e-4
        gC = np.zeros((3, W * H), np.float32)
        gD = np.zeros(W * H, np.float32)
        ps = pix[keep]
        gC[:, ps] = rng.normal(size=(3, ps.size))
        gD[ps] = rng.normal(size=ps.size)
        ups_rgb.append(t(gC).reshape(3, H, W))
        ups_dep.append(t(gD).reshape(H, W))
        rg = O.render_bwd(oc, gauss, vn["cam"], vn["base_rgb"], vn["base_depth"], gC[:, ps], gD[ps], pix=ps)
        refs = rg if refs is None else {k: refs[k] + rg[k] if k != "pose" else np.vstack([refs[k], rg[k]])
                                        for k in refs}
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(8, 6, device=DEV)
    P.render_bwd(gc, gd, views, ws, grads, dpose, dL_drgb=ups_rgb, dL_ddepth=ups_dep)
    torch.cuda.synchronize()
    for k in KEYS:
        assert normwise(h(grads[k]), refs[k]) < 1e-3, k
    assert normwise(h(dpose), refs["pose"]) < 1e-3
    # The backward is bitwise reproducible: no floating-point atomics, fixed
    # reduction orders, and no data race between the wavefronts of a block.
    for _ in range(3):
        g2 = P.zeros_like_gaussians(gd)
        dp2 = torch.zeros(8, 6, device=DEV)
        P.render_bwd(gc, gd, views, ws, g2, dp2, dL_drgb=ups_rgb, dL_ddepth=ups_dep)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(g2[k], grads[k]), k
        assert torch.equal(dp2, dpose)


def test_room_5mm_fusion_every_point(P, O):
    say("512^3 fusion")
    scene, fr = synth.workload_room_frames(n=512, frames=[3])
    cam, d, c = fr[0]
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    ref = O.new_volume(grid)
    O.fuse(grid, ref, cam.as_dict(), d, c)
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=DEV)
    P.fuse(vol, cam.as_dict(), t(d), t(c))
    torch.cuda.synchronize()
    w = h(vol.weight)
    np.testing.assert_array_equal(w, ref["weight"].astype(np.float32))
    upd = ref["weight"] > 0
    assert upd.sum() > 1_000_000
    assert np.abs(h(vol.tsdf)[upd] - ref["tsdf"][upd]).max() < 2e-5
