"""The allocation-free ICP reduce (gps_icp_reduce_noalloc, fixed library scratch)
against gps_icp_reduce with its workspace: bitwise the same system (same kernels,
same fixed summation order), on two calls in a row, the second on a smaller level
(fewer block sums than the first call left in the scratch), then the larger level
again."""
import numpy as np
import pytest
import torch

import synth
from oracle import icp as OI
from tests.gpu_util import DEV, say, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    P.lib()
    assert torch.cuda.is_available()
    return P


def _pair(W, H, xi=(0.012, -0.008, 0.014, 0.012, -0.015, 0.02)):
    scene = synth.scene_room()
    camA = synth.orbit_cameras(0, W, H, frames=[0])[0]
    RA, tA = camA.R.astype(np.float64), camA.t.astype(np.float64)
    Rx, tx = OI.se3_exp(np.asarray(xi))
    Rg2, tg2 = Rx @ RA.T, Rx @ (-RA.T @ tA) + tx
    camB = synth.Camera(W, H, camA.fx, camA.fy, camA.cx, camA.cy, Rg2.T.astype(np.float32),
                        (-Rg2.T @ tg2).astype(np.float32))
    DA, _ = synth.render_frame(scene, camA, device=DEV)
    DB, _ = synth.render_frame(scene, camB, device=DEV)
    return camA.as_dict(), DA, camB.as_dict(), DB


def test_noalloc_reduce_matches_the_workspace_reduce(P):
    say("no-alloc ICP reduce: 1280x720 level 0, then level 2, then level 0")
    camA, DA, camB, DB = _pair(1280, 720)
    pyramid = [t(DB)]
    for _ in range(2):
        pyramid.append(P.depth_downsample(pyramid[-1]))
    pose = P.pose_tensor(camA)
    ws = P.gps.IcpWorkspace(1280, 720)
    out = torch.zeros(29, dtype=torch.float64, device=DEV)
    for lvl, dist in ((0, 0.02), (2, 0.1), (0, 0.05)):
        lc = P.gps.level_camera(camB, lvl)
        want = P.icp_reduce(camA, t(DA), lc, pyramid[lvl], pose, dist, ws).cpu().numpy().copy()
        out.fill_(np.nan)
        got = P.icp_reduce_noalloc(camA, t(DA), lc, pyramid[lvl], pose, dist, out).cpu().numpy().copy()
        assert want[28] > (1000 if lvl == 2 else 100_000), want[28]     # pairs found
        np.testing.assert_array_equal(got, want)


def test_noalloc_reduce_in_a_tracking_loop(P):
    """The whole coarse-to-fine loop with the allocation-free reduce gives bitwise the
    pose of the loop with the workspace."""
    say("no-alloc ICP reduce: coarse-to-fine tracking at 640x480")
    camA, DA, camB, DB = _pair(640, 480)
    pyramid = [t(DB)]
    for _ in range(2):
        pyramid.append(P.depth_downsample(pyramid[-1]))
    poses = []
    for noalloc in (False, True):
        pose = P.pose_tensor(camA)
        ws = P.gps.IcpWorkspace(640, 480)
        for k, (iters, dist) in enumerate(((4, 0.1), (4, 0.05), (6, 0.02))):
            lvl = 2 - k
            lc = P.gps.level_camera(camB, lvl)
            for _ in range(iters):
                if noalloc:
                    P.icp_reduce_noalloc(camA, t(DA), lc, pyramid[lvl], pose, dist, ws.sys)
                else:
                    P.icp_reduce(camA, t(DA), lc, pyramid[lvl], pose, dist, ws)
                P.icp_solve(ws.sys, pose, ws.xi)
        poses.append(pose.cpu().numpy().copy())
    np.testing.assert_array_equal(poses[0], poses[1])
    Rt = np.asarray(camB["R"], np.float64)
    assert np.abs(poses[1][:9].reshape(3, 3) - Rt).max() < 1e-3
