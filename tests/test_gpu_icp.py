"""GPU parity of ICP camera tracking (Sec. 3.2.1, Eq. 5) against the reference.

* depth hierarchy: bit-exact (binary64 sum and division on both sides, one rounding);
* the Gauss-Newton system at one level: H, g, sum r^2 and the pair count against the
  reference, whose per-pair record flags the decisions within rounding reach of a
  pixel boundary or of the distance threshold; the tolerance is a binary32 bound
  (H 1e-5 relative, g 1e-4 relative plus 1e-6 per pair) plus what the flagged pairs
  can contribute, and the count may differ by at most the flagged pairs;
* the solve and pose update on the same system (binary64 on both sides);
* the system is bitwise reproducible;
* tracking: the room at 160x120 against the reference's own tracking, and at the
  full 1280x720 against the true camera motion (from 2 cm and 1.6 degrees off).
"""
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


def _room_pair(W, H, xi=(0.012, -0.008, 0.014, 0.012, -0.015, 0.02)):
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


def _sys_np(A, g, E, n):
    iu = np.triu_indices(6)
    return np.concatenate([A[iu], g, [E, n]])


def _unpack(s):
    s = np.asarray(s, np.float64)
    A = np.zeros((6, 6))
    A[np.triu_indices(6)] = s[:21]
    A = A + np.triu(A, 1).T
    return A, s[21:27], s[27], s[28]


@pytest.mark.parametrize("W,H", [(160, 120), (33, 17), (2, 2), (1280, 720)])
def test_depth_downsample_bitexact(P, W, H):
    say(f"icp: depth hierarchy {W}x{H}")
    rng = np.random.default_rng(W + H)
    D = rng.uniform(0.3, 3.0, (H, W)).astype(np.float32)
    D[rng.uniform(size=(H, W)) < 0.3] = 0.0
    got = P.depth_downsample(t(D)).cpu().numpy()
    want = OI.downsample_depth(D)
    assert got.shape == want.shape and np.array_equal(got, want)


def _check_system(P, camA, DA, lcam, Dl, R, tvec, dist):
    pose = torch.as_tensor(np.concatenate([np.asarray(R, np.float32).reshape(9),
                                           np.asarray(tvec, np.float32).reshape(3)])).to(DEV)
    ws = P.gps.IcpWorkspace(lcam["width"], lcam["height"])
    sys = P.icp_reduce(camA, t(DA), lcam, t(Dl), pose, dist, ws).cpu().numpy().copy()
    A, g, E, n, recs = OI.icp_system(camA, DA, lcam, Dl, np.asarray(R, np.float32), np.asarray(tvec, np.float32),
                                     dist, margins=True)
    Ag, gg, Eg, ng = _unpack(sys)
    fl = [(r, J) for r, J, f in recs if f]
    fl_A = sum((np.linalg.norm(np.outer(J, J)) for _, J in fl), 0.0)
    fl_g = sum((np.linalg.norm(J * r) for r, J in fl), 0.0)
    fl_E = sum((r * r for r, _ in fl), 0.0)
    assert n > 500
    assert abs(ng - n) <= len(fl), (ng, n, len(fl))
    assert np.linalg.norm(Ag - A) <= 1e-5 * np.linalg.norm(A) + 2 * fl_A
    assert np.linalg.norm(gg - g) <= 1e-4 * np.linalg.norm(g) + 1e-6 * n + 2 * fl_g
    assert abs(Eg - E) <= 1e-3 * E + 1e-10 * n + 2 * fl_E
    return pose, sys, ws


@pytest.mark.parametrize("W,H,level", [(160, 120, 0), (320, 240, 0), (320, 240, 1), (320, 240, 2)])
def test_icp_system_parity(P, W, H, level):
    say(f"icp: system {W}x{H} level {level}")
    camA, DA, camB, DB = _room_pair(W, H)
    lcam = OI.level_camera(camB, level)
    Dl = DB
    for _ in range(level):
        Dl = OI.downsample_depth(Dl)
    # at the start pose (frame A's) and at the true pose
    _check_system(P, camA, DA, lcam, Dl, camA["R"], camA["t"], 0.1)
    _check_system(P, camA, DA, lcam, Dl, camB["R"], camB["t"], 0.05)


def test_icp_system_is_reproducible(P):
    say("icp: reproducibility")
    camA, DA, camB, DB = _room_pair(320, 240)
    pose = P.pose_tensor(camA)
    ws = P.gps.IcpWorkspace(320, 240)
    a = P.icp_reduce(camA, t(DA), camB, t(DB), pose, 0.1, ws).cpu().numpy().copy()
    b = P.icp_reduce(camA, t(DA), camB, t(DB), pose, 0.1, ws).cpu().numpy().copy()
    assert np.array_equal(a, b)


def test_icp_solve_parity(P):
    say("icp: solve and update")
    camA, DA, camB, DB = _room_pair(160, 120)
    R0, t0 = np.asarray(camA["R"], np.float32), np.asarray(camA["t"], np.float32)
    A, g, E, n = OI.icp_system(camA, DA, camB, DB, R0, t0, 0.1)
    sys = torch.as_tensor(_sys_np(A, g, E, n)).to(DEV)
    pose = P.pose_tensor(camA)
    xi = torch.zeros(6, device=DEV)
    P.icp_solve(sys, pose, xi)
    R1, t1, xi_ref = OI.gn_step(A, g, n, R0, t0)
    np.testing.assert_allclose(xi.cpu().numpy(), xi_ref, rtol=1e-6, atol=1e-9)
    pr = pose.cpu().numpy()
    np.testing.assert_allclose(pr[:9].reshape(3, 3), R1, atol=2e-7)
    np.testing.assert_allclose(pr[9:], t1, atol=5e-7)
    # fewer than 6 pairs, or an H that is not positive definite: the pose is kept
    for bad in (_sys_np(A, g, E, 5), _sys_np(-A, g, E, n)):
        pose2 = P.pose_tensor(camA)
        xi2 = torch.ones(6, device=DEV)
        P.icp_solve(torch.as_tensor(bad).to(DEV), pose2, xi2)
        assert np.array_equal(pose2.cpu().numpy(), P.pose_tensor(camA).cpu().numpy())
        assert np.array_equal(xi2.cpu().numpy(), np.zeros(6, np.float32))


def test_icp_step_is_reduce_then_solve(P):
    """gps_icp_step (the system's sum and the solve in one launch) against gps_icp_reduce
    followed by gps_icp_solve: system, pose and xi bitwise equal over four steps on two
    levels."""
    say("icp: fused step against reduce + solve")
    camA, DA, camB, DB = _room_pair(320, 240)
    ws1, ws2 = P.gps.IcpWorkspace(320, 240), P.gps.IcpWorkspace(320, 240)
    pose1, pose2 = P.pose_tensor(camA), P.pose_tensor(camA)
    D1 = t(DB)
    D2 = P.depth_downsample(D1)
    for lvl, D in ((1, D2), (1, D2), (0, D1), (0, D1)):
        lc = P.gps.level_camera(camB, lvl)
        P.icp_reduce(camA, t(DA), lc, D, pose1, 0.1, ws1)
        P.icp_solve(ws1.sys, pose1, ws1.xi)
        P.icp_step(camA, t(DA), lc, D, pose2, 0.1, ws2)
        torch.cuda.synchronize()
        assert torch.equal(ws1.sys, ws2.sys) and torch.equal(pose1, pose2) and torch.equal(ws1.xi, ws2.xi)
    assert not torch.equal(pose1, P.pose_tensor(camA))  # the steps moved the pose


def _angle(R, RB):
    """Rotation angle of R RB^T from both its symmetric and skew parts (arccos of the
    trace alone loses half the digits near 0)."""
    M = R @ RB.T
    s = 0.5 * np.linalg.norm([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.arctan2(s, 0.5 * (np.trace(M) - 1)))


def _pose_err(pose, cam):
    p = pose.cpu().numpy().astype(np.float64)
    R, tv = p[:9].reshape(3, 3), p[9:]
    RB, tB = np.asarray(cam["R"], np.float64), np.asarray(cam["t"], np.float64)
    dc = np.linalg.norm(-R.T @ tv + RB.T @ tB)
    return dc, _angle(R, RB)


def test_icp_track_matches_the_reference(P):
    say("icp: tracking 160x120 against the reference")
    camA, DA, camB, DB = _room_pair(160, 120)
    pose = P.pose_tensor(camA)
    P.icp_track(camA, t(DA), camB, t(DB), pose)
    R, tv = OI.track(camA, DA, camB, DB, np.asarray(camA["R"], np.float64), np.asarray(camA["t"], np.float64))
    ref = {"R": R, "t": tv}
    dc, ang = _pose_err(pose, ref)
    assert dc < 5e-5 and ang < 5e-5, (dc, ang)


def test_icp_track_full_size(P):
    say("icp: tracking 1280x720 against the true motion")
    camA, DA, camB, DB = _room_pair(1280, 720)
    pose = P.pose_tensor(camA)
    d0, a0 = _pose_err(pose, camB)
    P.icp_track(camA, t(DA), camB, t(DB), pose)
    dc, ang = _pose_err(pose, camB)
    assert d0 > 0.015 and a0 > 0.02
    assert dc < 1e-3 and ang < 1e-3, (dc, ang)


def test_icp_track_graph_replay(P):
    """A whole coarse-to-fine tracking loop captured as one HIP graph: every replay (with
    eager tracking runs and synchronisations between them) gives the eager pose bitwise."""
    say("icp: tracking loop as a graph")
    camA, DA, camB, DB = _room_pair(320, 240)
    dA, dB = t(DA), t(DB)
    pose0 = P.pose_tensor(camA)
    ws = P.gps.IcpWorkspace(320, 240)
    pyr = [dB]
    for _ in range(2):
        pyr.append(P.depth_downsample(pyr[-1]))
    pose_e = pose0.clone()
    P.icp_track(camA, dA, camB, dB, pose_e, ws=ws, pyramid=pyr)
    torch.cuda.synchronize()
    pose_g = pose0.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.icp_track(camA, dA, camB, dB, pose_g, ws=ws, pyramid=pyr)
    for _ in range(3):
        pose_g.copy_(pose0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(pose_g, pose_e)
        pose_x = pose0.clone()
        P.icp_track(camA, dA, camB, dB, pose_x, ws=ws, pyramid=pyr)
        torch.cuda.synchronize()
        assert torch.equal(pose_x, pose_e)
    assert _pose_err(pose_g, camB)[0] < 1e-3
