"""Pins of the reference implementation of Gaussian insertion (Sec. 3.2.2,
Eq. 6 and the paragraph after it; Appendix A).

The mask, the sample, and the initial position, orientation, scale, opacity
and colour are checked on hand-built pixels and on planes whose vertex maps,
normals and neighbour distances have closed forms.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _cam(W, H, f):
    return {"width": W, "height": H, "fx": f, "fy": f, "cx": (W - 1) / 2, "cy": (H - 1) / 2,
            "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}


def _quat_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_defaults_are_the_paper_constants():
    ins = GOLD["insertion"]
    assert O.INSERT_DEFAULTS["delta_c"] == ins["delta_c"] and O.INSERT_DEFAULTS["delta_w"] == ins["delta_W"]
    assert O.INSERT_DEFAULTS["fraction"] == ins["sample_fraction"]
    assert O.INSERT_DEFAULTS["opacity"] == ins["initial_opacity"]
    assert O.INSERT_DEFAULTS["scale_cap"] == GOLD["init_scale_cap"]["value"]
    assert O.INSERT_DEFAULTS["flat_ratio"] == GOLD["init_scale_cap"]["flat_ratio"]


def test_mask_criteria():
    H, W = 1, 6
    K = np.full((3, H, W), 0.5, np.float32)
    C = K.copy()
    C[:, 0, 1] += 0.06    # mean error 0.06 > 0.05
    C[:, 0, 2] += 0.04    # 0.04: below
    C[0, 0, 3] += 0.18    # one channel 0.18: mean 0.06
    C[:, 0, 4] += 0.06    # error, but W_G >= 4
    C[:, 0, 5] += 0.06    # error, but no SDF surface
    Wg = np.zeros((H, W), np.float32)
    Wg[0, 4] = 4.0
    D = np.ones((H, W), np.float32)
    D[0, 5] = 0.0
    assert O.insertion_mask(C, K, Wg, D).tolist() == [[False, True, False, True, False, False]]


def test_fronto_parallel_plane():
    W, H, f, d = 12, 10, 200.0, 0.5
    cam = _cam(W, H, f)
    D = np.full((H, W), d, np.float32)
    K = np.random.default_rng(1).uniform(size=(3, H, W)).astype(np.float32)
    C = K + 0.1
    out, pix = O.insert_gaussians(cam, C, K, np.zeros((H, W), np.float32), D, np.zeros((H, W), np.float32))
    assert pix.size == H * W  # everything is in the mask and, with zeros for the draw, in the sample
    jj, ii = pix // W, pix % W
    np.testing.assert_allclose(out["mean"][0], (ii - cam["cx"]) * d / f, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["mean"][1], (jj - cam["cy"]) * d / f, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["mean"][2], d, rtol=0, atol=1e-12)
    # three neighbours at d / f: s1 = d / f (the root mean square, below the cap), the short
    # axis a tenth of it; a corner has two at d / f and the diagonal one at sqrt(2) d / f
    corner = ((ii == 0) | (ii == W - 1)) & ((jj == 0) | (jj == H - 1))
    s1 = np.where(corner, d / f * np.sqrt((1 + 1 + 2) / 3), d / f)
    np.testing.assert_allclose(np.exp(out["log_scale"]), np.vstack([s1, s1, 0.1 * s1]), rtol=1e-12)
    # inside the image the normal is the plane's, facing the camera (-z); on the border
    # (a neighbour missing) it is the direction to the camera; the rotation takes z onto it
    border = (ii == 0) | (ii == W - 1) | (jj == 0) | (jj == H - 1)
    for k, q in enumerate(out["quat"].T):
        p = out["mean"][:, k]
        want = -p / np.linalg.norm(p) if border[k] else np.array([0.0, 0.0, -1.0])
        np.testing.assert_allclose(_quat_rot(q) @ [0, 0, 1], want, atol=1e-12)
    np.testing.assert_allclose(out["opacity_logit"], 0.0)
    np.testing.assert_allclose(out["rgb"], K.reshape(3, -1)[:, pix])


def test_scale_cap_and_tilted_plane():
    W, H, f = 14, 12, 15.0
    cam = _cam(W, H, f)
    a, z0 = 0.4, 2.0  # plane z = z0 + a x in the camera frame
    jj, ii = np.mgrid[0:H, 0:W]
    xn = (ii - cam["cx"]) / f
    D = (z0 / (1 - a * xn)).astype(np.float32)  # depth of the ray through each pixel
    K = np.zeros((3, H, W), np.float32)
    out, pix = O.insert_gaussians(cam, K + 1.0, K, np.zeros((H, W), np.float32), D, np.zeros((H, W), np.float32))
    n_ref = np.array([a, 0.0, -1.0]) / np.hypot(a, 1.0)  # plane normal, facing the camera at the origin
    interior = [(p // W, p % W) for p in pix]
    for k, (j, i) in enumerate(interior):
        R = _quat_rot(out["quat"][:, k])
        if 0 < i < W - 1 and 0 < j < H - 1:
            np.testing.assert_allclose(R @ [0, 0, 1], n_ref, atol=1e-5)  # D is stored in binary32
    # neighbours about z / f >= 0.13 apart: above the 0.1 cap, so every s1 is capped
    np.testing.assert_allclose(np.exp(out["log_scale"][0]), 0.1, rtol=1e-12)


def test_nearest_vertices_over_the_whole_mask():
    """A sparse mask over a rough surface: the three nearest mask vertices of every new
    Gaussian come from the whole mask, wherever they are in the image, and s1 is their root
    mean square distance, against a k-d tree over the mask's vertices (scipy)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(7)
    W, H, f = 48, 36, 40.0
    cam = _cam(W, H, f)
    D = (1.2 + 0.3 * rng.uniform(size=(H, W))).astype(np.float32)  # rough: neighbours in depth, not pixels
    D[rng.uniform(size=(H, W)) < 0.05] = 0.0
    K = rng.uniform(size=(3, H, W)).astype(np.float32)
    C = K.copy()
    err = rng.uniform(size=(H, W)) < 0.08  # a sparse mask: about 8 % of the pixels
    C[:, err] += 0.2
    u = rng.uniform(size=(H, W)).astype(np.float32)
    out, pix = O.insert_gaussians(cam, C, K, np.zeros((H, W), np.float32), D, u)
    mask = O.insertion_mask(C, K, np.zeros((H, W), np.float32), D)
    jj, ii = np.nonzero(mask)
    d = D[jj, ii].astype(np.float64)
    Vm = np.stack([(ii - cam["cx"]) / f * d, (jj - cam["cy"]) / f * d, d], axis=1)
    tree = cKDTree(Vm)
    assert pix.size > 10
    far = 0
    for k, p in enumerate(pix):
        q = np.array([(p % W - cam["cx"]) / f * D[p // W, p % W], (p // W - cam["cy"]) / f * D[p // W, p % W],
                      D[p // W, p % W]], np.float64)
        dist, idx = tree.query(q, k=4)  # itself first
        assert dist[0] == 0.0
        rms = np.sqrt(np.mean(dist[1:] ** 2))
        np.testing.assert_allclose(np.exp(out["log_scale"][0, k]), min(0.1, rms), rtol=1e-12)
        # how often a neighbour lies outside a 9 x 9 pixel window (what a window search would miss)
        pj, pi = jj[idx[1:]], ii[idx[1:]]
        far += int((np.abs(pj - p // W) > 4).any() or (np.abs(pi - p % W) > 4).any())
    assert far > 0  # the case the whole-mask search exists for occurs in this input


def test_fewer_than_three_other_mask_vertices():
    """Two mask pixels: each one's only neighbour is the other (mean over one); one mask
    pixel: no neighbour, s1 = the cap."""
    W, H, f = 20, 10, 100.0
    cam = _cam(W, H, f)
    D = np.full((H, W), 1.0, np.float32)
    K = np.zeros((3, H, W), np.float32)
    C = K.copy()
    C[:, 2, 3] = 0.5
    C[:, 4, 6] = 0.5
    out, pix = O.insert_gaussians(cam, C, K, np.zeros((H, W), np.float32), D, np.zeros((H, W), np.float32))
    assert pix.tolist() == [2 * W + 3, 4 * W + 6]
    gap = np.hypot(3, 2) / f  # both at depth 1: the pixel offset scaled by d / f (below the cap)
    np.testing.assert_allclose(np.exp(out["log_scale"][0]), [gap] * 2, rtol=1e-12)
    C[:, 4, 6] = 0.0
    out, pix = O.insert_gaussians(cam, C, K, np.zeros((H, W), np.float32), D, np.zeros((H, W), np.float32))
    assert pix.tolist() == [2 * W + 3]
    np.testing.assert_allclose(np.exp(out["log_scale"][0]), [0.1], rtol=1e-12)


def test_sample_is_the_uniform_draw_below_the_fraction():
    rng = np.random.default_rng(3)
    W, H = 40, 30
    cam = _cam(W, H, 60.0)
    D = np.full((H, W), 1.0, np.float32)
    K = rng.uniform(size=(3, H, W)).astype(np.float32)
    C = K + rng.choice([0.0, 0.2], size=(1, H, W)).astype(np.float32)
    u = rng.uniform(size=(H, W)).astype(np.float32)
    mask = O.insertion_mask(C, K, np.zeros((H, W), np.float32), D)
    _, pix = O.insert_gaussians(cam, C, K, np.zeros((H, W), np.float32), D, u)
    assert np.array_equal(pix, np.nonzero((mask & (u < np.float32(0.25))).reshape(-1))[0])
    assert abs(pix.size / mask.sum() - 0.25) < 0.06
