"""The large streaming configuration over a long sequence: a 512^3 lattice at 5 mm
(3.2 GB) fused with 1000 orbit frames of 1280x720 (ten turns of the orbit, new depth
noise every frame) while 1,000,000 Gaussians are optimised -- 10 batched iterations per
frame over the latest 4 keyframes, a new keyframe every 10 frames (Sec. 3.2.1 fusion,
Sec. 3.1 mapping over a window of target views).

Spot checks every 100 frames:
* Fusion, at 20,000 lattice points (half uniform over the lattice, half within 4 voxels of
  the scene's surfaces, chosen from the synthetic scene's own geometry): the reference's
  update of those points alone over every frame so far (orc_fuse_points).  Weights are
  bit-exact, including the cap of 100 that the points seen in 100 frames reach; tsdf and
  colour are within 1e-4, the binary32 bound of the 512^3 fusion test (after the cap the
  update is a running average that keeps 100/101 of the old value, so rounding does not
  build up).
* Mapping: the device status is 0, every loss is finite, and each window of keyframes ends
  its 100 iterations (10 frames) at a lower loss than it started.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, h, say

pytestmark = pytest.mark.gpu
N_FRAMES, CHECK_EVERY, N_POINTS = 1000, 100, 20_000


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


def _sample_points(scene, cam0, rng):
    nx, ny, nz = scene.dims
    N = nx * ny * nz
    uni = rng.choice(N, N_POINTS // 2, replace=False)
    pix = rng.choice(cam0.width * cam0.height, N_POINTS // 2, replace=False)
    p, _, ok = synth.surface_points(scene, cam0, pix)
    p = p[ok]
    g = np.rint((p - np.asarray(scene.origin)) / scene.voxel).astype(np.int64)
    g += rng.integers(-4, 5, size=g.shape)
    g = np.clip(g, 0, np.array([nx, ny, nz]) - 1)
    near = g[:, 0] + nx * (g[:, 1] + ny * g[:, 2])
    return np.unique(np.concatenate([uni, near]))


def test_large_stream_spot_checks(P, O):
    from paper_2509_11574_amd.graph import IterationGraph
    say(f"large stream: 512^3 at 5 mm, 1M Gaussians, {N_FRAMES} frames of 1280x720")
    scene = synth.scene_room(512)
    W, H = 1280, 720
    cams = synth.orbit_cameras(0, W, H, frames=list(range(N_FRAMES)))
    seed_cams = synth.orbit_cameras(0, W, H, frames=list(range(0, 100, 10)))
    seed_depths = [synth.render_frame(scene, c, device=DEV, as_torch=True)[0].cpu().numpy() for c in seed_cams]
    params = P.gaussians_to_device(synth.seed_gaussians(scene, seed_cams, seed_depths, 1_000_000), DEV)
    cfg = P.RenderCfg(eps_cull=scene.voxel)
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=DEV)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    rng = np.random.Generator(np.random.PCG64(17))
    idx = _sample_points(scene, cams[0], rng)
    pts = O.new_points(idx.size)
    idx_dev = torch.as_tensor(idx, device=DEV)

    def frame(k):
        return synth.render_frame(scene, cams[k], noise_sigma_per_m2=1e-3, frame_index=k, device=DEV, as_torch=True)

    # the first window: keyframes 0, 10, 20, 30 fused in order, then their bases raycast
    ring, views = [], []
    for k in range(0, 40):
        d, c = frame(k)
        P.fuse(vol, cams[k].as_dict(), d, c)
        O.fuse_points(grid, idx, pts, cams[k].as_dict(), h(d), h(c))
        if k % 10 == 0:
            bd, bc = torch.empty(H, W, device=DEV), torch.empty(3, H, W, device=DEV)
            ring.append((bd, bc))
            views.append((k, d, c))
    views = [P.View(cams[k].as_dict(), bc, bd, c, d) for (k, d, c), (bd, bc) in zip(views, ring)]
    for v, (bd, bc) in zip(views, ring):
        P.raycast(vol, [v.cam], z_near=cfg.z_near, out=[(bd, bc)])
    grads = P.zeros_like_gaussians(params)
    opt = P.Adam(params)
    ws = P.Workspace(cfg, 1_000_000, [v.cam for v in views], device=DEV)
    loss = torch.zeros(1, device=DEV)
    g = IterationGraph(cfg, params, views, ws, grads, opt, loss, torch.zeros(len(views), 6, device=DEV))
    first_loss, window_drop = None, []
    for k in range(40, N_FRAMES):
        d, c = frame(k)
        cam = cams[k].as_dict()
        P.fuse(vol, cam, d, c)
        O.fuse_points(grid, idx, pts, cam, h(d), h(c))
        if k % 10 == 0:  # a new keyframe replaces the oldest of the window
            if first_loss is not None:  # the window's loss at its end against its start
                window_drop.append((first_loss, float(loss)))
            first_loss = None
            slot = (k // 10) % 4
            bd, bc = ring[slot]
            P.raycast(vol, [cam], z_near=cfg.z_near, out=[(bd, bc)])
            views[slot] = P.View(cam, bc, bd, c, d)
            g.set_views(views)
        for it in range(10):
            g.replay()
            if first_loss is None:
                first_loss = float(loss)
        if (k + 1) % CHECK_EVERY == 0:
            torch.cuda.synchronize()
            st = ws.stats()
            assert st["status"] == 0, st
            w_gpu = h(vol.weight[idx_dev])
            np.testing.assert_array_equal(w_gpu, pts["weight"].astype(np.float32))
            dt = np.abs(h(vol.tsdf[idx_dev]) - pts["tsdf"]).max()
            dc = np.abs(h(vol.rgb[:, idx_dev]) - pts["rgb"]).max()
            capped = int((pts["weight"] == 100.0).sum())
            say(f"  frame {k + 1}: {idx.size} points, {capped} at the weight cap, max |tsdf| diff {dt:.2e}, "
                f"max |rgb| diff {dc:.2e}, window loss {float(loss):.5f}")
            assert dt <= 1e-4 and dc <= 1e-4
    window_drop.append((first_loss, float(loss)))
    L = np.array(window_drop)
    assert np.isfinite(L).all()
    assert (L[:, 1] < L[:, 0]).all(), L  # every window's 100 iterations lower its loss
    assert (pts["weight"] == 100.0).sum() >= 100  # the cap is exercised
    say(f"  {len(L)} windows, loss {L[0, 0]:.5f} -> {L[0, 1]:.5f} in the first, {L[-1, 0]:.5f} -> {L[-1, 1]:.5f} "
        f"in the last")
