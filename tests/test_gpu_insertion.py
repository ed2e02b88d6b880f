"""GPU parity of Gaussian insertion (Sec. 3.2.2, Eq. 6; Appendix A) against the reference.

Bit-exact: the mask and sample decisions (binary32 on both sides), the number of
sampled pixels, their row-major order and pixel indices, the colours and the
opacity.  Within binary32 tolerances derived from the arithmetic: the surface
point, the log-scales (distances of neighbouring vertices, a few millimetres,
formed from camera-frame coordinates of up to a few metres: relative error
about 1e-4 at worst), and the disc axis, which is what the covariance depends
on (its sign is the camera-facing choice; it is compared exactly away from
grazing surfaces).  The quaternion itself is compared where the shortest-arc
rotation is well conditioned (axis not near -z).

The three nearest mask vertices of App. A are searched over the whole mask on
both sides (the reference by brute force over every mask vertex).

Inputs: the small analytic scene at 160x120 and the room at 320x240, whole
frames; sparse masks whose nearest vertices lie far away in the image, isolated
mask pixels (capped scales) and masks of one and two pixels; the room at
1280x720 on 300 sampled Gaussians (the reference samples only those, over the
same whole-frame mask); plus capacity limits, empty samples and odd frame sizes.
"""
import numpy as np
import pytest
import torch

import synth
from synth.scene import small_camera
from tests.gpu_util import DEV, say, t

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
    return O


def _rot_z(q):
    """Third column of the rotation of each quaternion (w, x, y, z), columns of q."""
    q = q / np.linalg.norm(q, axis=0)
    w, x, y, z = q
    return np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])


def _gpu(P, cam, inputs, **kw):
    C, K, Wg, D, r = inputs
    out, pix, n_taken = P.insert_gaussians(cam, t(C), t(K), t(Wg), t(D), t(r), **kw)
    torch.cuda.synchronize()
    n = pix.numel()
    res = {k: out[k].cpu().numpy().astype(np.float64).reshape(ROWS[k], n) for k in KEYS}
    return res, pix.cpu().numpy().astype(np.int64), n_taken


def _compare(got, want, cam, mean_atol=4e-6, ls_atol=1e-4, axis_atol=5e-4):
    np.testing.assert_array_equal(got["rgb"], want["rgb"])
    np.testing.assert_allclose(got["opacity_logit"], want["opacity_logit"], rtol=0, atol=1e-7)
    np.testing.assert_allclose(got["mean"], want["mean"], rtol=0, atol=mean_atol)
    np.testing.assert_allclose(got["log_scale"], want["log_scale"], rtol=0, atol=ls_atol)
    qn = np.linalg.norm(got["quat"], axis=0)
    np.testing.assert_allclose(qn, 1.0, atol=1e-6)
    az, bz = _rot_z(got["quat"]), _rot_z(want["quat"])
    # the disc axis up to sign (the covariance), then its sign away from grazing views
    dot = np.sum(az * bz, axis=0)
    assert np.all(np.abs(dot) > 1 - axis_atol ** 2 / 2 - 1e-7), np.min(np.abs(dot))
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    centre = -R.T @ np.asarray(cam["t"], np.float64)
    view = centre[:, None] - want["mean"]
    view /= np.linalg.norm(view, axis=0)
    facing = np.abs(np.sum(bz * view, axis=0)) > 1e-3
    assert np.all(dot[facing] > 0)
    np.testing.assert_allclose(az[:, facing], bz[:, facing], rtol=0, atol=axis_atol)
    good = (1 + bz[2]) > 0.05
    np.testing.assert_allclose(got["quat"][:, good], want["quat"][:, good], rtol=0, atol=2 * axis_atol)


def _room_cam(W, H, frame=0):
    return synth.orbit_cameras(0, W, H, frames=[frame])[0]


@pytest.mark.parametrize("which", ["small160x120", "room320x240"])
def test_insertion_parity_whole_frame(P, O, which):
    say(f"insertion parity: {which}")
    if which == "small160x120":
        scene, cam = synth.scene_small(), small_camera()
    else:
        scene, cam = synth.scene_room(), _room_cam(320, 240)
    inputs = synth.insertion_inputs(scene, cam, device=DEV)
    want, wpix = O.insert_gaussians(cam.as_dict(), *inputs)
    got, pix, n_taken = _gpu(P, cam.as_dict(), inputs)
    assert n_taken == wpix.size > 100
    np.testing.assert_array_equal(pix, wpix)
    _compare(got, want, cam.as_dict())


@pytest.mark.parametrize("density", [0.002, 0.02, 0.2])
def test_insertion_sparse_masks(P, O, density):
    """Masks of a given density over the room at 160x120: at low density the three nearest
    mask vertices are many blocks away in the image or beyond the cap distance."""
    say(f"insertion parity: sparse mask, density {density}")
    scene, cam = synth.scene_room(), _room_cam(160, 120, frame=7)
    C, K, Wg, D, r = synth.insertion_inputs(scene, cam, seed=11, device=DEV)
    rng = np.random.default_rng(int(density * 1e4))
    err = rng.uniform(size=D.shape) < density
    C = K.copy()
    C[:, err] += 0.3
    Wg = np.zeros_like(Wg)
    r = np.where(rng.uniform(size=D.shape) < 0.5, 0.0, 1.0).astype(np.float32)
    inputs = (C, K, Wg, D, r)
    want, wpix = O.insert_gaussians(cam.as_dict(), *inputs)
    got, pix, n_taken = _gpu(P, cam.as_dict(), inputs)
    assert n_taken == wpix.size > 0
    np.testing.assert_array_equal(pix, wpix)
    _compare(got, want, cam.as_dict())
    if density < 0.01:
        assert (np.exp(want["log_scale"][0]) >= 0.1 - 1e-12).any()   # isolated: capped
    else:
        assert (np.exp(want["log_scale"][0]) < 0.1).any()            # neighbours within reach


@pytest.mark.parametrize("n_mask", [1, 2, 3, 4])
def test_insertion_tiny_masks(P, O, n_mask):
    """One to four mask pixels far apart in the image: the mean runs over the other mask
    vertices there are (none: the cap), found wherever they are in the frame."""
    say(f"insertion parity: {n_mask} mask pixels")
    W, H = 96, 64
    cam = {"width": W, "height": H, "fx": 300.0, "fy": 300.0, "cx": W / 2, "cy": H / 2,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    D = np.full((H, W), 1.5, np.float32)
    K = np.zeros((3, H, W), np.float32)
    C = K.copy()
    # the first two are 0.083 m apart (below the cap), the others half a metre away
    for (j, i) in [(3, 5), (10, 20), (60, 90), (40, 7)][:n_mask]:
        C[:, j, i] = 0.5
    z = np.zeros((H, W), np.float32)
    want, wpix = O.insert_gaussians(cam, C, K, z, D, z)
    got, pix, n_taken = _gpu(P, cam, (C, K, z, D, z))
    assert n_taken == wpix.size == n_mask
    np.testing.assert_array_equal(pix, wpix)
    _compare(got, want, cam)
    if n_mask == 2:
        assert (np.exp(want["log_scale"][0]) < 0.09).all()


def test_insertion_capacity_and_empty(P, O):
    say("insertion: capacity limits, empty sample")
    scene, cam = synth.scene_room(), _room_cam(160, 120, frame=3)
    inputs = synth.insertion_inputs(scene, cam, seed=12, device=DEV)
    want, wpix = O.insert_gaussians(cam.as_dict(), *inputs)
    for cap in (0, 1, 57, wpix.size, wpix.size + 5):
        got, pix, n_taken = _gpu(P, cam.as_dict(), inputs, capacity=cap)
        assert n_taken == wpix.size
        k = min(cap, wpix.size)
        np.testing.assert_array_equal(pix, wpix[:k])
        _compare(got, {kk: v[:, :k] for kk, v in want.items()}, cam.as_dict())
    got, pix, n_taken = _gpu(P, cam.as_dict(), inputs, fraction=0.0)
    assert n_taken == 0 and pix.size == 0
    C, K, Wg, D, r = inputs
    got, pix, n_taken = _gpu(P, cam.as_dict(), (C, K, Wg, np.zeros_like(D), r), fraction=1.0)
    assert n_taken == 0


@pytest.mark.parametrize("W,H", [(1, 1), (3, 2), (17, 1), (257, 3), (33, 29)])
def test_insertion_odd_sizes(P, O, W, H):
    say(f"insertion: frame {W}x{H}")
    rng = np.random.default_rng(W * 1000 + H)
    cam = {"width": W, "height": H, "fx": 40.0, "fy": 42.0, "cx": W / 2, "cy": H / 2,
           "R": synth.look_at((0.3, -0.2, 0.1), (0.5, 1.5, 0.4))[0], "t": np.array([0.1, -0.3, 1.2], np.float32)}
    D = rng.uniform(0.5, 2.0, (H, W)).astype(np.float32)
    D[rng.uniform(size=(H, W)) < 0.1] = 0.0
    K = rng.uniform(size=(3, H, W)).astype(np.float32)
    C = (K + rng.normal(0, 0.1, (3, H, W))).astype(np.float32)
    Wg = rng.uniform(0, 8, (H, W)).astype(np.float32)
    r = rng.uniform(size=(H, W)).astype(np.float32)
    want, wpix = O.insert_gaussians(cam, C, K, Wg, D, r, fraction=0.8)
    got, pix, n_taken = _gpu(P, cam, (C, K, Wg, D, r), fraction=0.8)
    assert n_taken == wpix.size
    np.testing.assert_array_equal(pix, wpix)
    _compare(got, want, cam)


def test_insertion_plane_closed_form(P):
    """A fronto-parallel plane at depth d: every pixel is sampled, the means are the
    back-projected pixels, s1 = d / f inside (all three neighbours at d / f), the
    disc axis is -z inside and points to the camera on the border."""
    say("insertion: plane closed form")
    W, H, f, d = 40, 30, 200.0, 0.5
    cam = {"width": W, "height": H, "fx": f, "fy": f, "cx": (W - 1) / 2, "cy": (H - 1) / 2,
           "R": np.eye(3, dtype=np.float32), "t": np.zeros(3, np.float32)}
    K = np.random.default_rng(1).uniform(size=(3, H, W)).astype(np.float32)
    z = np.zeros((H, W), np.float32)
    got, pix, n = _gpu(P, cam, (K + 0.1, K, z, np.full((H, W), d, np.float32), z))
    assert n == W * H and np.array_equal(pix, np.arange(W * H))
    jj, ii = pix // W, pix % W
    np.testing.assert_allclose(got["mean"][0], (ii - cam["cx"]) * d / f, atol=1e-7)
    np.testing.assert_allclose(got["mean"][1], (jj - cam["cy"]) * d / f, atol=1e-7)
    inner = (ii > 0) & (ii < W - 1) & (jj > 0) & (jj < H - 1)
    np.testing.assert_allclose(got["log_scale"][0, inner], np.log(d / f), atol=5e-6)
    np.testing.assert_allclose(got["log_scale"][2, inner], np.log(d / f) + np.log(0.1), atol=5e-6)
    az = _rot_z(got["quat"])
    np.testing.assert_allclose(az[:, inner], np.array([[0.0], [0.0], [-1.0]]) * np.ones((1, inner.sum())), atol=1e-6)
    p = got["mean"][:, ~inner]
    np.testing.assert_allclose(az[:, ~inner], -p / np.linalg.norm(p, axis=0), atol=1e-6)


def test_insertion_full_size_sampled(P, O):
    """Room at 1280x720: the sample decisions and order on every pixel (the reference
    mask), and 300 sampled Gaussians recomputed by the reference over the whole-frame
    mask (its draw takes only those 300 pixels; the mask does not depend on the draw)."""
    say("insertion: room 1280x720, sampled")
    scene, cam = synth.scene_room(), _room_cam(1280, 720)
    inputs = synth.insertion_inputs(scene, cam, device=DEV)
    C, K, Wg, D, r = inputs
    mask = O.insertion_mask(C, K, Wg, D)
    take = mask & (r < np.float32(0.25))
    wpix = np.flatnonzero(take.reshape(-1))
    got, pix, n_taken = _gpu(P, cam.as_dict(), inputs)
    assert n_taken == wpix.size > 10000
    np.testing.assert_array_equal(pix, wpix)
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(wpix.size, 300, replace=False))
    r_sel = np.ones_like(r)
    r_sel.reshape(-1)[wpix[sel]] = 0.0
    want, opix = O.insert_gaussians(cam.as_dict(), C, K, Wg, D, r_sel)
    np.testing.assert_array_equal(opix, wpix[sel])
    _compare({k: v[:, sel] for k, v in got.items()}, want, cam.as_dict())
