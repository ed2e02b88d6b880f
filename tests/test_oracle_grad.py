"""Pins of the oracle's analytic gradients (CPU only).

(i)  autograd of the independent dense float64 renderer,
(ii) central finite differences of the oracle's own forward pass in float64,
     under the active-set rule (a sampled parameter counts only when the set of
     contributing (pixel, Gaussian) pairs is the same at theta + h and theta - h),
(iii) an exact identity between the camera-translation gradient and the sum of
     the mean gradients.
"""
import numpy as np
import pytest
import torch

from tests import dense_ref
from tests.tiny_cases import RCfg, tiny_case

KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


def _upstream(case, seed):
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    W, H = case["cam"]["width"], case["cam"]["height"]
    return rng.normal(size=(3, W * H)), rng.normal(size=W * H)


def _autograd(case, cfg, gC, gD):
    params = dense_ref.to_params(case["gauss"], requires_grad=True)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    C, D = dense_ref.render(params, case["cam"], case["base_rgb"], case["base_depth"], cfg, xi=xi)
    L = (C.reshape(3, -1) * torch.as_tensor(gC)).sum() + (D.reshape(-1) * torch.as_tensor(gD)).sum()
    L.backward()
    out = {k: params[k].grad.numpy() for k in KEYS}
    out["pose"] = xi.grad.numpy()
    return out


def _normwise(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_hand_adjoints_match_autograd(oracle, mode, seed):
    case = tiny_case(seed, M=30, log_scale=-2.4)
    rc = RCfg(mode=mode, eps_cull=0.03)
    cfg = oracle.RenderCfg(mode=mode, eps_cull=0.03)
    gC, gD = _upstream(case, seed)
    an = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    ag = _autograd(case, rc, gC, gD)
    for k in KEYS + ("pose",):
        assert _normwise(an[k], ag[k]) < 1e-9, (k, _normwise(an[k], ag[k]))


def test_capped_alpha_has_no_alpha_gradient(oracle):
    """With every opacity saturated above alpha_max, only colour and depth carry gradient."""
    case = tiny_case(9, M=20, log_scale=-2.0)
    g = dict(case["gauss"])
    g["opacity_logit"] = np.full_like(g["opacity_logit"], 9.0)  # sigma ~ 0.99988 > 0.99
    cfg = oracle.RenderCfg(mode=0, eps_cull=0.03, T_min=0.0)
    W, H = case["cam"]["width"], case["cam"]["height"]
    # probe only the centres, where alpha = sigma > alpha_max
    P = oracle.project(cfg, g, case["cam"])
    gC, gD = np.zeros((3, W * H)), np.zeros(W * H)
    an = oracle.render_bwd(cfg, g, case["cam"], case["base_rgb"], case["base_depth"], gC + 1.0, gD)
    ag = _autograd({**case, "gauss": g}, RCfg(mode=0, eps_cull=0.03, T_min=0.0), gC + 1.0, gD)
    for k in KEYS + ("pose",):
        assert _normwise(an[k], ag[k]) < 1e-9, k
    assert P["valid"].any()


def _render_sum(oracle, cfg, case, g, cam, gC, gD):
    r = oracle.render(cfg, g, cam, case["base_rgb"], case["base_depth"])
    return float((r["rgb"] * gC).sum() + (r["depth"] * gD).sum()), r


def _pose_cam(cam, xi):
    """Camera after the left perturbation T <- Exp(xi) T (exact exponential), in float32."""
    from scipy.spatial.transform import Rotation
    rho, phi = np.asarray(xi[:3]), np.asarray(xi[3:])
    Rphi = Rotation.from_rotvec(phi).as_matrix()
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    V = np.eye(3) if th < 1e-12 else (np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K)
    R = cam["R"].astype(np.float64)
    t = cam["t"].astype(np.float64)
    c2 = dict(cam)
    c2["R"] = (Rphi @ R).astype(np.float32)
    c2["t"] = (Rphi @ t + V @ rho).astype(np.float32)
    return c2


@pytest.mark.parametrize("mode", [0, 1])
def test_central_differences(oracle, mode):
    """Central differences of the float64 forward, h = 2^-13 (exact in float32 for |theta| < 1024),
    on 64 seeded parameters, tolerance 1e-2 relative to max(|g_an|, |g_fd|)."""
    case = tiny_case(11, M=24, log_scale=-2.3)
    cfg = oracle.RenderCfg(mode=mode, eps_cull=0.03)
    gC, gD = _upstream(case, 11)
    an = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    rng = np.random.Generator(np.random.PCG64(5))
    h = 2.0 ** -13
    checked = 0
    tried = 0
    while checked < 64 and tried < 2000:
        tried += 1
        k = KEYS[rng.integers(0, len(KEYS))]
        arr = case["gauss"][k]
        idx = tuple(rng.integers(0, s) for s in arr.shape)
        gmax = np.abs(an[k]).max()
        if abs(an[k][idx]) < 1e-3 * gmax:
            continue
        gp, gm = {kk: v.copy() for kk, v in case["gauss"].items()}, {kk: v.copy() for kk, v in case["gauss"].items()}
        gp[k][idx] = np.float32(arr[idx] + h)
        gm[k][idx] = np.float32(arr[idx] - h)
        assert float(gp[k][idx]) - float(arr[idx]) == h
        Lp, rp = _render_sum(oracle, cfg, case, gp, case["cam"], gC, gD)
        Lm, rm = _render_sum(oracle, cfg, case, gm, case["cam"], gC, gD)
        if not (np.array_equal(rp["n"], rm["n"]) and np.array_equal(rp["order"], rm["order"])
                and (rp["flag"] == 0).all() and (rm["flag"] == 0).all()):
            continue  # active set changed between the two evaluations
        fd = (Lp - Lm) / (2 * h)
        ref = max(abs(fd), abs(an[k][idx]))
        assert abs(fd - an[k][idx]) <= 1e-2 * ref, (k, idx, fd, an[k][idx])
        checked += 1
    assert checked == 64
    # The six pose parameters (camera perturbed with the exact exponential map).  A pose change moves
    # every footprint, so the active-set rule is applied per pixel: the upstream adjoint is kept only
    # at pixels whose contributors, their depth order and flags agree at +h and -h (gradients add
    # over pixels).
    for j in range(6):
        hp = 1e-4 if j < 3 else 2e-4
        xi = np.zeros(6)
        xi[j] = hp
        cp, cm = _pose_cam(case["cam"], xi), _pose_cam(case["cam"], -xi)
        rp = oracle.render(cfg, case["gauss"], cp, case["base_rgb"], case["base_depth"])
        rm = oracle.render(cfg, case["gauss"], cm, case["base_rgb"], case["base_depth"])
        keep = (rp["n"] == rm["n"]) & (rp["order"] == rm["order"]) & (rp["flag"] == 0) & (rm["flag"] == 0)
        assert keep.mean() > 0.9
        gCk, gDk = gC * keep[None], gD * keep
        fd = (float((rp["rgb"] * gCk).sum() + (rp["depth"] * gDk).sum()) -
              float((rm["rgb"] * gCk).sum() + (rm["depth"] * gDk).sum())) / (2 * hp)
        ank = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gCk,
                                gDk)["pose"][j]
        ref = max(abs(fd), abs(ank))
        assert abs(fd - ank) <= 1e-2 * ref, (j, fd, ank)


@pytest.mark.parametrize("mode", [0, 1])
def test_translation_gradient_is_rotated_mean_gradient(oracle, mode):
    """Translating the camera by rho in its own frame moves every centre by rho and changes nothing
    else, exactly as moving every mean by R^T rho does; so dL/drho = R sum_i dL/dmu_i."""
    case = tiny_case(12, M=30)
    cfg = oracle.RenderCfg(mode=mode, eps_cull=0.03)
    gC, gD = _upstream(case, 12)
    an = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    R = case["cam"]["R"].astype(np.float64)
    # R is a float32 rotation, orthogonal to ~1e-7, hence the tolerance
    np.testing.assert_allclose(an["pose"][:3], R @ an["mean"].sum(axis=1), rtol=1e-6, atol=1e-12)


def test_pixel_subset_gradients_add_up(oracle):
    """Gradients are additive over pixels: the full image equals the sum over a partition."""
    case = tiny_case(13, M=30)
    cfg = oracle.RenderCfg(mode=0, eps_cull=0.03)
    gC, gD = _upstream(case, 13)
    full = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    n = gD.shape[0]
    parts = [np.arange(0, n, 3), np.arange(1, n, 3), np.arange(2, n, 3)]
    acc = None
    for p in parts:
        r = oracle.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC[:, p],
                              gD[p], pix=p.astype(np.int32))
        acc = r if acc is None else {k: acc[k] + r[k] for k in acc}
    for k in KEYS + ("pose",):
        np.testing.assert_allclose(acc[k], full[k], rtol=1e-10, atol=1e-14)
