"""The backward with the Adam step in its epilogue (gps_render_bwd_adam) against the
separate backward and Adam launches (gps_render_bwd + gps_adam_step): over three
optimisation iterations, bitwise the same parameters, Adam moments, step counter,
gradients and pose gradient, in both compositing modes, with and without the pose
output (the counter is then advanced by its own launch) and without stored gradients.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, say, t

pytestmark = pytest.mark.gpu
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    P.lib()
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def room_view():
    scene = synth.scene_room()
    cam = synth.orbit_cameras(0, 320, 240, frames=[0])[0]
    depth, rgb = synth.render_frame(scene, cam)
    seed_cams = synth.orbit_cameras(0, 320, 240, frames=list(range(0, 100, 10)))
    seed_depths = [synth.render_frame(scene, c)[0] for c in seed_cams]
    gauss = synth.seed_gaussians(scene, seed_cams, seed_depths, 20000)
    return scene, cam, depth, rgb, gauss


def _setup(P, room_view, mode):
    scene, cam, depth, rgb, gauss = room_view
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=DEV)
    P.fuse(vol, cam.as_dict(), t(depth), t(rgb))
    (bd, brgb), = P.raycast(vol, [cam.as_dict()], z_near=0.2)
    view = P.View(cam.as_dict(), brgb, bd, t(rgb), t(depth))
    cfg = P.RenderCfg(mode=mode, eps_cull=scene.voxel)
    return cfg, view, P.gaussians_to_device(gauss, DEV)


@pytest.mark.parametrize("mode,with_pose,with_grads", [(0, True, True), (1, True, True), (0, False, True),
                                                       (0, True, False)])
def test_fused_adam_matches_separate_launches(P, room_view, mode, with_pose, with_grads):
    say(f"fused backward + Adam: mode {mode}, pose {with_pose}, grads {with_grads}")
    cfg, view, g0 = _setup(P, room_view, mode)
    M = g0["opacity_logit"].numel()
    pa = {k: v.clone() for k, v in g0.items()}
    pb = {k: v.clone() for k, v in g0.items()}
    oa, ob = P.Adam(pa), P.Adam(pb)
    ws_a = P.Workspace(cfg, M, [view.cam], device=DEV)
    ws_b = P.Workspace(cfg, M, [view.cam], device=DEV)
    ga, gb = P.zeros_like_gaussians(pa), P.zeros_like_gaussians(pb)
    da, db = torch.zeros(1, 6, device=DEV), torch.zeros(1, 6, device=DEV)
    la, lb = torch.zeros(1, device=DEV), torch.zeros(1, device=DEV)
    for it in range(3):
        P.render_fwd(cfg, pa, [view], ws_a, out_loss=la)
        P.render_bwd(cfg, pa, [view], ws_a, ga, da if with_pose else None)
        oa.step(ga)
        P.render_fwd(cfg, pb, [view], ws_b, out_loss=lb)
        P.render_bwd_adam(cfg, pb, [view], ws_b, ob, grads=gb if with_grads else None,
                          dpose=db if with_pose else None)
        torch.cuda.synchronize()
        assert torch.equal(la, lb), it
        for k in KEYS:
            assert torch.equal(pa[k], pb[k]), (it, k)
            assert torch.equal(oa.m[k], ob.m[k]) and torch.equal(oa.v[k], ob.v[k]), (it, k)
            if with_grads:
                assert torch.equal(ga[k], gb[k]), (it, k)
        if with_pose:
            assert torch.equal(da, db), it
        assert int(oa.counter.item()) == int(ob.counter.item()) == it + 1
    assert not torch.equal(pa["mean"], g0["mean"])  # the steps moved the Gaussians
