"""Reference implementation of point-to-plane ICP camera tracking (Sec. 3.2.1,
"Camera tracking", Eq. 5) in binary64.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the CPU-baseline leg of
``bench.py``.  The product package never imports this module, and this module
never imports the product package.

Conventions: a camera maps world to camera coordinates, x_c = R x_w + t;
pixel (i, j) has its centre at the continuous coordinate (i, j);
pi(x, y, z) = (f_x x / z + c_x, f_y y / z + c_y); the nearest pixel of (u, v)
is (floor(u + 1/2), floor(v + 1/2)).

Readings (the paper defers to KinectFusion and InfiniTAM and is silent on these):
  * Eq. 5 is minimised over the camera-to-world pose T_{g,k} of the current
    frame; xi = (rho, phi) is a left perturbation, T_{g,k} <- Exp(xi) T_{g,k},
    and each Gauss-Newton step solves H xi = -g for the system of Eq. 5
    linearised at xi = 0 (H = sum J J^T, g = sum J r, J = (N, p x N));
  * V^l_k(u): the current depth back-projected with the intrinsics of the
    level; p = T_{g,k} V^l_k(u);
  * projective association: u^ = the nearest pixel of the projection of p into
    the previous camera; the model maps V^{*,g}_{k-1} and N^{*,g}_{k-1} come from
    the previous frame's SDF raycast depth at full resolution: V* its
    back-projection, N* the normalised cross product of the central
    differences of V* along x and along y (a pixel needs its four neighbours
    with a surface), turned to face the previous camera;
  * a pair is kept when d > 0 at u, u^ lies in the image with its four
    neighbours, D_{t,k-1}(u^) > 0, and |p - V*| <= the caller's distance
    threshold (no normal-angle test: Eq. 5 has none);
  * resolution hierarchy: each level halves the previous one (floor of
    width / 2 and height / 2); a coarse pixel holds the mean of the valid
    (> 0) depths of its 2x2 block, 0 when none is valid; its intrinsics are
    f / 2 and (c - 1/2) / 2, so that its centre is the centre of the block;
  * a step is skipped (pose unchanged) when fewer than 6 pairs remain or H is
    not positive definite.
"""
from __future__ import annotations

import numpy as np


def _K(cam):
    return float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])


def _pose(cam):
    return (np.asarray(cam["R"], np.float64).reshape(3, 3), np.asarray(cam["t"], np.float64).reshape(3))


def downsample_depth(depth):
    """One level of the resolution hierarchy: [H][W] -> [H // 2][W // 2], float32
    (the mean of the valid depths of each 2x2 block in binary64, rounded once)."""
    D = np.asarray(depth, np.float32)
    H, W = D.shape
    out = np.zeros((H // 2, W // 2), np.float32)
    for j in range(H // 2):
        for i in range(W // 2):
            vals = [float(D[2 * j + b, 2 * i + a]) for b in (0, 1) for a in (0, 1) if D[2 * j + b, 2 * i + a] > 0]
            if vals:
                s = 0.0
                for v in vals:
                    s += v
                out[j, i] = np.float32(s / len(vals))
    return out


def level_camera(cam, level):
    """Intrinsics and size of a pyramid level (the pose is copied unchanged)."""
    c = dict(cam)
    for _ in range(level):
        c["width"], c["height"] = c["width"] // 2, c["height"] // 2
        c["fx"], c["fy"] = c["fx"] / 2.0, c["fy"] / 2.0
        c["cx"], c["cy"] = (c["cx"] - 0.5) / 2.0, (c["cy"] - 0.5) / 2.0
    return c


def _backproject_cam(cam, i, j, d):
    fx, fy, cx, cy = _K(cam)
    return np.array([(i - cx) / fx * d, (j - cy) / fy * d, d])


def model_maps(prev_cam, prev_depth):
    """V*, N* of the previous frame in world coordinates ([H][W][3]) and a validity mask."""
    D = np.asarray(prev_depth, np.float32)
    H, W = D.shape
    R, t = _pose(prev_cam)
    X = np.zeros((H, W, 3))
    for j in range(H):
        for i in range(W):
            if D[j, i] > 0:
                X[j, i] = _backproject_cam(prev_cam, i, j, float(D[j, i]))
    V = (X - t) @ R            # R^T (x_c - t), row vectors
    N = np.zeros((H, W, 3))
    ok = np.zeros((H, W), bool)
    for j in range(1, H - 1):
        for i in range(1, W - 1):
            if D[j, i] > 0 and D[j, i - 1] > 0 and D[j, i + 1] > 0 and D[j - 1, i] > 0 and D[j + 1, i] > 0:
                n = np.cross(X[j, i + 1] - X[j, i - 1], X[j + 1, i] - X[j - 1, i])
                nn = np.linalg.norm(n)
                if nn > 0:
                    n = n / nn
                    if np.dot(n, X[j, i]) > 0:     # face the camera (at the origin of its frame)
                        n = -n
                    N[j, i] = R.T @ n
                    ok[j, i] = True
    return V, N, ok


def icp_system(prev_cam, prev_depth, cur_cam, cur_depth, R_c, t_c, dist_thresh, margins=False):
    """The Gauss-Newton system of Eq. 5 at the pose (R_c, t_c) (world to camera) of the
    current frame, for one level (cur_cam: that level's intrinsics, cur_depth its depth).
    Returns (H 6x6, g 6, sum r^2, pair count) and, with margins=True, also a per-pair
    record (residual, J, flagged) where `flagged` marks decisions within rounding reach:
    an association coordinate within 2e-3 px of a pixel boundary or a distance within
    1e-5 relative of the threshold."""
    V, N, ok = model_maps(prev_cam, prev_depth)
    Dp = np.asarray(prev_depth, np.float32)
    Hp, Wp = Dp.shape
    Rp, tp = _pose(prev_cam)
    fx, fy, cx, cy = _K(prev_cam)
    R_c = np.asarray(R_c, np.float64).reshape(3, 3)
    t_c = np.asarray(t_c, np.float64).reshape(3)
    D = np.asarray(cur_depth, np.float32)
    H, W = D.shape
    A = np.zeros((6, 6))
    g = np.zeros(6)
    E, n = 0.0, 0
    recs = []
    for j in range(H):
        for i in range(W):
            d = float(D[j, i])
            if not d > 0:
                continue
            X = _backproject_cam(cur_cam, i, j, d)
            p = R_c.T @ (X - t_c)
            q = Rp @ p + tp
            if not q[2] > 0:
                continue
            u = fx * q[0] / q[2] + cx
            v = fy * q[1] / q[2] + cy
            a, b = int(np.floor(u + 0.5)), int(np.floor(v + 0.5))
            near = min(abs((u + 0.5) - np.round(u + 0.5)), abs((v + 0.5) - np.round(v + 0.5))) < 2e-3
            if not (1 <= a <= Wp - 2 and 1 <= b <= Hp - 2) or not ok[b, a]:
                if margins and near:
                    recs.append((0.0, np.zeros(6), True))
                continue
            diff = p - V[b, a]
            dist = np.linalg.norm(diff)
            near = near or abs(dist / dist_thresh - 1.0) < 1e-5
            if dist > dist_thresh:
                if margins and near:
                    recs.append((0.0, np.zeros(6), True))
                continue
            nrm = N[b, a]
            r = float(np.dot(diff, nrm))
            J = np.concatenate([nrm, np.cross(p, nrm)])
            A += np.outer(J, J)
            g += J * r
            E += r * r
            n += 1
            if margins:
                recs.append((r, J, near))
    if margins:
        return A, g, E, n, recs
    return A, g, E, n


def se3_exp(xi):
    """Exp of xi = (rho, phi) in SE(3): (R, t) of the 4x4 matrix exponential of the twist."""
    rho = np.asarray(xi[:3], np.float64)
    phi = np.asarray(xi[3:], np.float64)
    th = np.linalg.norm(phi)
    Wx = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + Wx, rho + 0.5 * Wx @ rho
    a = np.sin(th) / th
    b = (1.0 - np.cos(th)) / th ** 2
    c = (th - np.sin(th)) / th ** 3
    R = np.eye(3) + a * Wx + b * Wx @ Wx
    Vm = np.eye(3) + b * Wx + c * Wx @ Wx
    return R, Vm @ rho


def gn_step(A, g, n, R_c, t_c):
    """Solve A xi = -g and apply T_{g,k} <- Exp(xi) T_{g,k}; returns (R_c, t_c, xi)
    of the camera (world to camera); unchanged when n < 6 or A is not positive definite."""
    R_c = np.asarray(R_c, np.float64).reshape(3, 3)
    t_c = np.asarray(t_c, np.float64).reshape(3)
    if n < 6:
        return R_c, t_c, np.zeros(6)
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return R_c, t_c, np.zeros(6)
    xi = -np.linalg.solve(L.T, np.linalg.solve(L, g))
    Rx, tx = se3_exp(xi)
    R_g, t_g = R_c.T, -R_c.T @ t_c          # camera to world
    R_g2, t_g2 = Rx @ R_g, Rx @ t_g + tx
    return R_g2.T, -R_g2.T @ t_g2, xi


def track(prev_cam, prev_depth, cur_cam, cur_depth, R0, t0, iters=(4, 4, 6), dist_thresh=(0.1, 0.05, 0.02)):
    """Coarse-to-fine tracking: iters[l] Gauss-Newton steps at level l, coarsest first
    (iters and dist_thresh are listed from the coarsest level to the finest)."""
    L = len(iters)
    pyr = [np.asarray(cur_depth, np.float32)]
    for _ in range(L - 1):
        pyr.append(downsample_depth(pyr[-1]))
    R, t = np.asarray(R0, np.float64), np.asarray(t0, np.float64)
    for k in range(L):
        lvl = L - 1 - k
        cam_l = level_camera(cur_cam, lvl)
        for _ in range(iters[k]):
            A, g, E, n = icp_system(prev_cam, prev_depth, cam_l, pyr[lvl], R, t, dist_thresh[k])
            R, t, _ = gn_step(A, g, n, R, t)
    return R, t
