"""Pins of the oracle's projection and compositing (CPU only).

Each check comes from outside the oracle: closed forms of the EWA footprint,
library routines (scipy rotations), invariants of the over-operator, special
cases that reduce to the SDF image, and a dense brute-force renderer."""
import math

import numpy as np
import pytest
import torch

from tests import dense_ref
from tests.tiny_cases import RCfg, tiny_case


DIL = float(np.float32(0.3))  # the low-pass term as the float32 config field holds it


def _cfg(O, **kw):
    return O.RenderCfg(**kw)


def _one_gaussian(mean, log_scale, quat=(1, 0, 0, 0), logit=2.0, rgb=(0.9, 0.2, 0.1)):
    return {"mean": np.asarray(mean, np.float32).reshape(3, 1),
            "log_scale": np.asarray(log_scale, np.float32).reshape(3, 1),
            "quat": np.asarray(quat, np.float32).reshape(4, 1),
            "opacity_logit": np.asarray([logit], np.float32),
            "rgb": np.asarray(rgb, np.float32).reshape(3, 1)}


def _cam(W=64, H=48, f=60.0, R=np.eye(3), t=np.zeros(3), cx=None, cy=None):
    return {"width": W, "height": H, "fx": f, "fy": f, "cx": W / 2 if cx is None else cx,
            "cy": H / 2 if cy is None else cy, "R": np.asarray(R, np.float32), "t": np.asarray(t, np.float32)}


# ----------------------------------------------------------------- projection
def test_isotropic_on_axis_footprint(oracle):
    """Eq. 3 footprint of an isotropic Gaussian on the optical axis: Sigma_2D = (f s / z)^2 I + 0.3 I."""
    f, z, s = 60.0, 2.0, 0.05
    g = _one_gaussian([0, 0, z], [math.log(s)] * 3)
    P = oracle.project(_cfg(oracle), g, _cam(f=f))
    s32 = float(np.float32(math.log(s)))
    expect = (f * math.exp(s32) / z) ** 2 + DIL
    assert P["valid"][0]
    np.testing.assert_allclose(P["cov"][0], [expect, 0.0, expect], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(P["m"][0], [32.0, 24.0], atol=1e-12)
    assert P["depth"][0] == pytest.approx(z)


def test_isotropic_off_axis_footprint(oracle):
    """Off axis with fx = fy = f: Sigma_2D = s^2 f^2/z^2 [[1+x^2/z^2, xy/z^2],[xy/z^2, 1+y^2/z^2]] + 0.3 I."""
    f = 55.0
    for (x, y, z) in [(0.4, -0.3, 1.7), (-0.8, 0.5, 2.5), (0.1, 0.9, 1.1)]:
        ls = np.float32(math.log(0.04))
        s = math.exp(float(ls))
        g = _one_gaussian([x, y, z], [ls] * 3, quat=(0.3, -0.5, 0.2, 0.7))
        P = oracle.project(_cfg(oracle), g, _cam(f=f))
        x, y, z = (float(np.float32(v)) for v in (x, y, z))
        k = s * s * f * f / (z * z)
        expect = [k * (1 + x * x / z ** 2) + DIL, k * x * y / z ** 2, k * (1 + y * y / z ** 2) + DIL]
        np.testing.assert_allclose(P["cov"][0], expect, rtol=1e-10)


def test_conic_is_inverse(oracle):
    case = tiny_case(1, M=40)
    P = oracle.project(_cfg(oracle), case["gauss"], case["cam"])
    for k in np.nonzero(P["valid"])[0]:
        a, b, c = P["conic"][k]
        A, B, C = P["cov"][k]
        np.testing.assert_allclose(np.array([[a, b], [b, c]]) @ np.array([[A, B], [B, C]]), np.eye(2), atol=1e-9)


def test_footprint_matches_linearised_projection(oracle):
    """Sigma_2D equals J_num Sigma_3D J_num^T + 0.3 I where J_num is the central-difference Jacobian of
    the exact pinhole map mu -> pi(R mu + t), and Sigma_3D is built with scipy's rotation of the
    (w, x, y, z) quaternion (a library pin of the quaternion and rotation conventions)."""
    from scipy.spatial.transform import Rotation
    case = tiny_case(2, M=25)
    cam, g = case["cam"], case["gauss"]
    P = oracle.project(_cfg(oracle), g, cam)
    R = cam["R"].astype(np.float64)
    t = cam["t"].astype(np.float64)

    def pix(mu):
        p = R @ mu + t
        return np.array([cam["fx"] * p[0] / p[2] + cam["cx"], cam["fy"] * p[1] / p[2] + cam["cy"]])

    for k in np.nonzero(P["valid"])[0]:
        mu = g["mean"][:, k].astype(np.float64)
        h = 1e-6
        Jn = np.stack([(pix(mu + h * e) - pix(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        w, x, y, z = g["quat"][:, k].astype(np.float64)
        Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
        s = np.exp(g["log_scale"][:, k].astype(np.float64))
        S3 = Rq @ np.diag(s ** 2) @ Rq.T
        S2 = Jn @ S3 @ Jn.T + DIL * np.eye(2)
        np.testing.assert_allclose(P["cov"][k], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(P["m"][k], pix(mu), rtol=1e-12)


def test_rigid_motion_invariance(oracle):
    """Moving world and camera by the same rigid motion leaves every 2D quantity unchanged."""
    case = tiny_case(3, M=20)
    cam, g = case["cam"], case["gauss"]
    from tests.tiny_cases import rot_xyz
    Q = rot_xyz(0.3, -0.2, 0.5)
    s = np.array([0.1, -0.2, 0.05])
    g2 = dict(g)
    g2["mean"] = (Q @ g["mean"].astype(np.float64) + s[:, None]).astype(np.float32)
    # quaternion of Q composed with each Gaussian's rotation
    from scipy.spatial.transform import Rotation
    qq = []
    for k in range(g["quat"].shape[1]):
        w, x, y, z = g["quat"][:, k].astype(np.float64)
        r = Rotation.from_matrix(Q) * Rotation.from_quat([x, y, z, w])
        x2, y2, z2, w2 = r.as_quat()
        qq.append([w2, x2, y2, z2])
    g2["quat"] = np.asarray(qq, np.float32).T
    R = cam["R"].astype(np.float64)
    cam2 = dict(cam)
    cam2["R"] = (R @ Q.T).astype(np.float32)
    cam2["t"] = (cam["t"] - R @ Q.T @ s).astype(np.float32)
    P1 = oracle.project(_cfg(oracle), g, cam)
    P2 = oracle.project(_cfg(oracle), g2, cam2)
    v = P1["valid"] & P2["valid"]
    assert v.sum() > 10
    np.testing.assert_allclose(P1["cov"][v], P2["cov"][v], rtol=2e-4, atol=1e-5)
    np.testing.assert_allclose(P1["m"][v], P2["m"][v], rtol=1e-5, atol=1e-4)


def test_box_contains_support(oracle):
    """Every pixel where sigma exp(-q/2) >= 1/255 lies inside the reported box (brute force)."""
    case = tiny_case(4, M=30, W=80, H=60, log_scale=-2.2)
    cfg = _cfg(oracle)
    P = oracle.project(cfg, case["gauss"], case["cam"])
    jj, ii = np.meshgrid(np.arange(-20, 80), np.arange(-20, 100), indexing="ij")
    for k in np.nonzero(P["valid"])[0]:
        a, b, c = P["conic"][k]
        dx = ii - P["m"][k, 0]
        dy = jj - P["m"][k, 1]
        al = P["sigma"][k] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        inside = al >= 1 / 255
        if not inside.any():
            continue
        x0, x1, y0, y1 = P["box"][k]
        assert ii[inside].min() >= x0 - 1e-9 and ii[inside].max() <= x1 + 1e-9
        assert jj[inside].min() >= y0 - 1e-9 and jj[inside].max() <= y1 + 1e-9


def test_near_plane_cull(oracle):
    g = _one_gaussian([0, 0, 0.15], [-3] * 3)
    P = oracle.project(_cfg(oracle), g, _cam())
    assert not P["valid"][0]


# ---------------------------------------------------------------- compositing
@pytest.mark.parametrize("mode", [0, 1])
def test_no_gaussians_gives_sdf_image(oracle, mode):
    """SDF-only rendering: with M = 0, C* = C_t and D* = D_t (Eq. 4 with W_G = 0)."""
    case = tiny_case(5, M=1)
    g = {k: v[..., :0] for k, v in case["gauss"].items()}
    r = oracle.render(_cfg(oracle, mode=mode), g, case["cam"], case["base_rgb"], case["base_depth"])
    np.testing.assert_array_equal(r["rgb"], case["base_rgb"].reshape(3, -1).astype(np.float64))
    np.testing.assert_array_equal(r["depth"], case["base_depth"].reshape(-1).astype(np.float64))


@pytest.mark.parametrize("mode", [0, 1])
def test_all_occluded_gives_sdf_image(oracle, mode):
    """Gaussians behind the SDF surface (d_i >= D_t + eps) are culled by the depth test of Eq. 1-2."""
    case = tiny_case(6, M=20, invalid_frac=0.0)
    base_depth = np.full_like(case["base_depth"], 0.8)  # all Gaussians are at 1.0 .. 2.4 m
    r = oracle.render(_cfg(oracle, mode=mode, eps_cull=0.1), case["gauss"], case["cam"], case["base_rgb"],
                      base_depth)
    np.testing.assert_array_equal(r["rgb"], case["base_rgb"].reshape(3, -1).astype(np.float64))
    assert (r["n"] == 0).all()


@pytest.mark.parametrize("mode", [0, 1])
def test_single_gaussian_closed_form(oracle, mode):
    """One isotropic Gaussian on the axis over a constant base: alpha(x) = sigma exp(-r^2 / (2 v))
    with v = (f s/z)^2 + 0.3; sorted: C = alpha c + (1-alpha) C_t; sort-free: (C_t + alpha c)/(1+alpha)."""
    W, H, f, z = 64, 48, 60.0, 1.5
    ls = np.float32(math.log(0.03))
    g = _one_gaussian([0, 0, z], [ls] * 3, logit=1.0, rgb=(0.9, 0.2, 0.4))
    cam = _cam(W, H, f)
    Ct = np.array([0.1, 0.5, 0.7], np.float32)
    base_rgb = np.broadcast_to(Ct[:, None, None], (3, H, W)).astype(np.float32).copy()
    base_depth = np.full((H, W), 3.0, np.float32)
    r = oracle.render(_cfg(oracle, mode=mode), g, cam, base_rgb, base_depth)
    v = (f * math.exp(float(ls)) / z) ** 2 + DIL
    sig = 1 / (1 + math.exp(-1.0))
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    r2 = (ii - W / 2) ** 2 + (jj - H / 2) ** 2
    a = sig * np.exp(-r2 / (2 * v))
    a = np.where(a >= 1 / 255, a, 0.0).reshape(-1)
    c = np.array([0.9, 0.2, 0.4], np.float32).astype(np.float64)
    if mode == 0:
        expC = a[None, :] * c[:, None] + (1 - a[None, :]) * Ct.astype(np.float64)[:, None]
        expD = a * z + (1 - a) * 3.0
    else:
        expC = (Ct.astype(np.float64)[:, None] + a[None, :] * c[:, None]) / (1 + a[None, :])
        expD = (3.0 + a * z) / (1 + a)
    np.testing.assert_allclose(r["rgb"], expC, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["depth"], expD, rtol=1e-12)


def test_transmittance_invariants(oracle):
    """T_final in [0,1]; with every Gaussian of one colour c, C* = c (1 - T) + T C_t, i.e. the
    Gaussian weights and T_final sum to one; and with T_min off, T_final = prod (1 - alpha_i) over the
    contributors, an order-independent product computed here by unsorted summation of logs."""
    case = tiny_case(7, M=40, log_scale=-2.3)
    g = dict(case["gauss"])
    cval = np.float32(0.625)
    g["rgb"] = np.full_like(g["rgb"], cval)
    cfg = _cfg(oracle, T_min=0.0, eps_cull=0.05)
    r = oracle.render(cfg, g, case["cam"], case["base_rgb"], case["base_depth"])
    T = r["T"]
    assert (T >= 0).all() and (T <= 1).all()
    Ct = case["base_rgb"].reshape(3, -1).astype(np.float64)
    np.testing.assert_allclose(r["rgb"], float(cval) * (1 - T)[None] + T[None] * Ct, rtol=1e-12, atol=1e-13)
    # unsorted per-pixel product
    P = oracle.project(cfg, g, case["cam"])
    W, H = case["cam"]["width"], case["cam"]["height"]
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    bd = case["base_depth"].reshape(-1)
    thr = (np.where(bd > 0, bd, np.float32(np.inf)) + np.float32(cfg.eps_cull)).astype(np.float32)
    logT = np.zeros(W * H)
    for k in np.nonzero(P["valid"])[0]:
        a, b, c = P["conic"][k]
        dx = ii.reshape(-1) - P["m"][k, 0]
        dy = jj.reshape(-1) - P["m"][k, 1]
        al = P["sigma"][k] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        use = (al >= 1 / 255) & (P["depth32"][k] < thr)
        al = np.minimum(al, cfg.alpha_max)
        logT += np.where(use, np.log1p(-al), 0.0)
    np.testing.assert_allclose(T, np.exp(logT), rtol=1e-10)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_dense_bruteforce(oracle, mode, seed):
    """The oracle equals an independent dense renderer (all pairs, one global depth permutation,
    cumulative-product transmittance) on tiny inputs, in both modes."""
    case = tiny_case(seed, M=30)
    cfg = RCfg(mode=mode, eps_cull=0.02)
    r = oracle.render(_cfg(oracle, mode=mode, eps_cull=0.02), case["gauss"], case["cam"], case["base_rgb"],
                      case["base_depth"])
    with torch.no_grad():
        C, D = dense_ref.render(dense_ref.to_params(case["gauss"]), case["cam"], case["base_rgb"],
                                case["base_depth"], cfg)
    assert (r["flag"] == 0).all()
    np.testing.assert_allclose(r["rgb"], C.reshape(3, -1).numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(r["depth"], D.reshape(-1).numpy(), rtol=1e-11, atol=1e-12)
    assert (r["n"] > 0).sum() > 50


def test_pixel_list_equals_full_image(oracle):
    case = tiny_case(8, M=30)
    cfg = _cfg(oracle)
    full = oracle.render(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    pix = np.array([0, 17, 333, 599, 1199], np.int32)
    part = oracle.render(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], pix=pix)
    np.testing.assert_array_equal(part["rgb"], full["rgb"][:, pix])
    np.testing.assert_array_equal(part["depth"], full["depth"][pix])


def test_sorted_order_matters_and_is_front_to_back(oracle):
    """Two coincident-footprint Gaussians at different depths: the nearer one is composited first,
    C = a1 c1 + (1-a1) a2 c2 + (1-a1)(1-a2) C_t, independently of their index order."""
    W, H, f = 16, 12, 30.0
    ls = np.float32(math.log(0.05))
    for swap in (False, True):
        z = [1.0, 2.0] if not swap else [2.0, 1.0]
        cols = [(1, 0, 0), (0, 0, 1)] if not swap else [(0, 0, 1), (1, 0, 0)]
        g = {"mean": np.array([[0, 0], [0, 0], z], np.float32), "log_scale": np.full((3, 2), ls, np.float32),
             "quat": np.array([[1, 1], [0, 0], [0, 0], [0, 0]], np.float32),
             "opacity_logit": np.array([0.5, 0.5], np.float32), "rgb": np.array(cols, np.float32).T.copy()}
        cam = _cam(W, H, f)
        base = np.zeros((3, H, W), np.float32)
        r = oracle.render(_cfg(oracle), g, cam, base, np.full((H, W), 5.0, np.float32), pix=np.array([6 * W + 8]))
        sig = 1 / (1 + math.exp(-0.5))
        a1 = sig  # at the centre pixel
        assert r["rgb"][0, 0] == pytest.approx(a1, rel=1e-12)
        assert r["rgb"][2, 0] == pytest.approx((1 - a1) * sig, rel=1e-12)
