"""Pins of the reference implementation of ICP tracking (Sec. 3.2.1, Eq. 5).

* Exp of SE(3) against the matrix exponential of the twist (scipy, a library routine);
* the resolution hierarchy: constant, holes, an empty block, and the level intrinsics
  (a coarse pixel of a fronto-parallel plane back-projects to the centroid of its block);
* the system at the true pose of an identical frame: every residual and g vanish;
* g = (1/2) dE/dxi by central differences of E = sum r^2 over Exp perturbations of the
  pose (on a plane model, where association changes do not move the residual);
* H = sum J J^T is symmetric positive semi-definite, rank 3 on a plane;
* end to end: from a pose off by 2 cm and 1.6 degrees, coarse-to-fine tracking of the
  room at 160x120 recovers the true pose of the current frame to the discretisation
  bias of nearest-pixel association on curved surfaces (under 1 mm and 2 mrad; a sign
  or transpose mistake in J or in the update diverges instead).
"""
import math

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import icp as I


def _twist(xi):
    rho, phi = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    M[:3, 3] = rho
    return M


@pytest.mark.parametrize("scale", [1e-14, 1e-6, 0.1, 1.0, 3.0])
def test_se3_exp_is_the_matrix_exponential(scale):
    rng = np.random.default_rng(int(-math.log10(scale) * 10) + 50)
    xi = rng.normal(size=6) * scale
    R, t = I.se3_exp(xi)
    E = scipy.linalg.expm(_twist(xi))
    np.testing.assert_allclose(R, E[:3, :3], atol=1e-12)
    np.testing.assert_allclose(t, E[:3, 3], atol=1e-12)


def test_downsample_depth():
    D = np.full((6, 8), 1.5, np.float32)
    assert np.array_equal(I.downsample_depth(D), np.full((3, 4), 1.5, np.float32))
    D = np.zeros((5, 7), np.float32)       # odd sizes: the last row and column are dropped
    D[0, 0], D[0, 1], D[1, 1] = 1.0, 2.0, 4.0   # three valid of one block
    D[2, 2] = 3.0                               # one valid
    D[4, 6] = 9.0                               # outside every block
    out = I.downsample_depth(D)
    assert out.shape == (2, 3)
    assert out[0, 0] == np.float32(7.0 / 3.0) and out[1, 1] == 3.0
    assert np.count_nonzero(out) == 2


def test_level_intrinsics_put_the_coarse_centre_at_the_block_centre():
    cam = {"width": 64, "height": 48, "fx": 60.0, "fy": 55.0, "cx": 31.7, "cy": 23.2,
           "R": np.eye(3), "t": np.zeros(3)}
    d = 1.25
    for lvl in (1, 2):
        c = I.level_camera(cam, lvl)
        s = 2 ** lvl
        assert (c["width"], c["height"]) == (64 // s, 48 // s)
        for (i, j) in ((0, 0), (3, 5), (c["width"] - 1, c["height"] - 1)):
            coarse = I._backproject_cam(c, i, j, d)
            fine = np.mean([I._backproject_cam(cam, s * i + a, s * j + b, d) for a in range(s) for b in range(s)],
                           axis=0)
            np.testing.assert_allclose(coarse, fine, atol=1e-12)


def _room_pair(W=160, H=120, xi=(0.012, -0.008, 0.014, 0.012, -0.015, 0.02)):
    scene = synth.scene_room()
    camA = synth.orbit_cameras(0, W, H, frames=[0])[0]
    RA, tA = camA.R.astype(np.float64), camA.t.astype(np.float64)
    Rx, tx = I.se3_exp(np.asarray(xi))
    Rg, tg = RA.T, -RA.T @ tA                  # camera to world of A, moved by Exp(xi)
    Rg2, tg2 = Rx @ Rg, Rx @ tg + tx
    camB = synth.Camera(W, H, camA.fx, camA.fy, camA.cx, camA.cy, Rg2.T.astype(np.float32),
                        (-Rg2.T @ tg2).astype(np.float32))
    DA, _ = synth.render_frame(scene, camA)
    DB, _ = synth.render_frame(scene, camB)
    return camA.as_dict(), DA, camB.as_dict(), DB


def test_identical_frame_at_its_own_pose_has_zero_residuals():
    camA, DA, _, _ = _room_pair()
    A, g, E, n, recs = I.icp_system(camA, DA, camA, DA, camA["R"], camA["t"], 0.05, margins=True)
    assert n > 0.8 * np.count_nonzero(DA)
    assert max(abs(r) for r, _, _ in recs) < 1e-9 and E < 1e-15
    np.testing.assert_allclose(g, 0.0, atol=1e-9)
    np.testing.assert_allclose(A, A.T, atol=0)
    assert np.linalg.eigvalsh(A).min() > 0


def _plane_model(W=48, H=40):
    """A tilted plane seen by the previous camera, and a bumpy surface near it for the current one."""
    cam = {"width": W, "height": H, "fx": 50.0, "fy": 50.0, "cx": W / 2 - 0.3, "cy": H / 2 + 0.2,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    jj, ii = np.mgrid[0:H, 0:W]
    xn, yn = (ii - cam["cx"]) / 50.0, (jj - cam["cy"]) / 50.0
    a, b, z0 = 0.3, -0.2, 1.5                  # plane z = z0 + a x + b y
    Dp = (z0 / (1 - a * xn - b * yn)).astype(np.float32)
    Dc = (Dp * (1 + 0.01 * np.sin(ii / 3.0) * np.cos(jj / 4.0))).astype(np.float32)
    return cam, Dp, Dc


def test_g_is_half_the_gradient_of_the_squared_residuals():
    cam, Dp, Dc = _plane_model()
    R0, t0 = np.eye(3), np.array([0.004, -0.003, 0.01])
    A, g, E, n = I.icp_system(cam, Dp, cam, Dc, R0, t0, 1.0)
    assert n > 1000
    R_g, t_g = R0.T, -R0.T @ t0
    h = 1e-6
    for k in range(6):
        Es = []
        for s in (1, -1):
            e = np.zeros(6)
            e[k] = s * h
            Rx, tx = I.se3_exp(e)
            R2, t2 = Rx @ R_g, Rx @ t_g + tx
            Es.append(I.icp_system(cam, Dp, cam, Dc, R2.T, -R2.T @ t2, 1.0)[2])
        np.testing.assert_allclose((Es[0] - Es[1]) / (2 * h), 2 * g[k], rtol=1e-5, atol=1e-9)
    w = np.linalg.eigvalsh(A)
    assert w.min() > -1e-9 * w.max()
    assert np.sum(w > 1e-6 * w.max()) == 3    # a plane fixes three of the six degrees of freedom


def test_tracking_recovers_the_true_pose():
    camA, DA, camB, DB = _room_pair()
    R0, t0 = np.asarray(camA["R"], np.float64), np.asarray(camA["t"], np.float64)
    RB, tB = np.asarray(camB["R"], np.float64), np.asarray(camB["t"], np.float64)
    c0 = -R0.T @ t0
    cB = -RB.T @ tB
    assert np.linalg.norm(c0 - cB) > 0.015
    R, t = I.track(camA, DA, camB, DB, R0, t0)
    c = -R.T @ t
    M = R @ RB.T
    ang = np.arctan2(0.5 * np.linalg.norm([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]]),
                     0.5 * (np.trace(M) - 1))
    assert np.linalg.norm(c - cB) < 1e-3 and ang < 2e-3, (np.linalg.norm(c - cB), ang)
