"""Per-view pose perturbation and the auxiliary per-pixel output of the render.

* pose_xi != 0: the view is rendered from Exp(xi) T_cw (compared with the FP64
  reference at that camera), and the returned gradient is dL/dxi at xi: against
  the reference's left-perturbation gradient at the perturbed camera times the
  transposed left Jacobian of SE(3) (taken here by central differences of the
  matrix exponential and logarithm, independently of the library), and against
  central differences of the FP64 reference over xi.
* out_aux: the final transmittance (sorted mode) or the Gaussian weight W_G of
  Eq. 2 (sort-free mode), against the reference's per-pixel values.
"""
import numpy as np
import pytest
import torch
from scipy.linalg import expm, logm

from tests.gpu_util import DEV, cfg_pair, h, normwise, say, t
from tests.tiny_cases import tiny_case

pytestmark = pytest.mark.gpu
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


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


def _hat(xi):
    rho, phi = xi[:3], xi[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    X[:3, 3] = rho
    return X


def _vee(X):
    return np.array([X[0, 3], X[1, 3], X[2, 3], X[2, 1], X[0, 2], X[1, 0]])


def _cam_at(cam, xi):
    """Camera Exp(xi) T_cw, composed in float64 (scipy expm) and stored in float32."""
    T = np.eye(4)
    T[:3, :3] = np.asarray(cam["R"], np.float64).reshape(3, 3)
    T[:3, 3] = np.asarray(cam["t"], np.float64)
    T2 = expm(_hat(np.asarray(xi, np.float64))) @ T
    c = dict(cam)
    c["R"] = T2[:3, :3].astype(np.float32)
    c["t"] = T2[:3, 3].astype(np.float32)
    return c


def _left_jacobian_fd(xi, e=1e-6):
    """J with Exp(xi + d) = Exp(J d) Exp(xi) to first order, by central differences of log."""
    E0inv = np.linalg.inv(expm(_hat(xi)))
    J = np.zeros((6, 6))
    for i in range(6):
        d = np.zeros(6)
        d[i] = e
        lp = _vee(np.real(logm(expm(_hat(xi + d)) @ E0inv)))
        lm = _vee(np.real(logm(expm(_hat(xi - d)) @ E0inv)))
        J[:, i] = (lp - lm) / (2 * e)
    return J


XI0 = np.array([0.012, -0.008, 0.010, 0.015, -0.020, 0.010])


@pytest.mark.parametrize("mode", [0, 1])
def test_pose_xi_render_and_gradient(P, O, mode):
    say(f"pose_xi != 0: forward and gradient, mode {mode}")
    case = tiny_case(7, M=60, W=53, H=37, log_scale=-2.4)
    gc, oc = cfg_pair(P, O, mode=mode, eps=0.03)
    W, H = case["cam"]["width"], case["cam"]["height"]
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]))
    ws = P.Workspace(gc, 60, [view.cam], device=DEV)
    gd = {k: t(v) for k, v in case["gauss"].items()}
    xi = t(XI0.reshape(1, 6))
    P.render_fwd(gc, gd, [view], ws, pose_xi=xi)
    cam_p = _cam_at(case["cam"], XI0)
    r = O.render(oc, case["gauss"], cam_p, case["base_rgb"], case["base_depth"])
    keep = r["flag"] == 0
    assert keep.mean() > 0.99 and (r["n"] > 0).sum() > 200
    assert normwise(h(view.out_rgb).reshape(3, -1), r["rgb"], keep) < 1e-4
    assert normwise(h(view.out_depth).reshape(-1), r["depth"], keep) < 1e-4
    # explicit upstream adjoints; zero where a reference decision is within rounding of a threshold
    rng = np.random.Generator(np.random.PCG64(77))
    gC = rng.normal(size=(3, W * H)) * keep
    gD = rng.normal(size=W * H) * keep
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(1, 6, device=DEV)
    P.render_bwd(gc, gd, [view], ws, grads, dpose, dL_drgb=[t(gC).reshape(3, H, W)],
                 dL_ddepth=[t(gD).reshape(H, W)], pose_xi=xi)
    torch.cuda.synchronize()
    got = h(dpose)[0].astype(np.float64)
    # (a) the reference's gradient of the left perturbation at Exp(xi0) T, mapped by J_l(xi0)^T
    ref = O.render_bwd(oc, case["gauss"], cam_p, case["base_rgb"], case["base_depth"], gC, gD)
    want = _left_jacobian_fd(XI0).T @ ref["pose"]
    assert normwise(got, want) < 1e-3, (got, want)
    for k in KEYS:  # the Gaussian gradients are those at the perturbed camera
        assert normwise(h(grads[k]), ref[k]) < 1e-3, k
    # (b) central differences of the FP64 reference over xi (per-pixel active-set rule)
    for j in range(6):
        hp = 1e-4 if j < 3 else 2e-4
        d = np.zeros(6)
        d[j] = hp
        rp = O.render(oc, case["gauss"], _cam_at(case["cam"], XI0 + d), case["base_rgb"], case["base_depth"])
        rm = O.render(oc, case["gauss"], _cam_at(case["cam"], XI0 - d), case["base_rgb"], case["base_depth"])
        ok = (rp["n"] == rm["n"]) & (rp["order"] == rm["order"]) & (rp["flag"] == 0) & (rm["flag"] == 0)
        assert ok.mean() > 0.9
        fd = (float((rp["rgb"] * gC * ok).sum() + (rp["depth"] * gD * ok).sum()) -
              float((rm["rgb"] * gC * ok).sum() + (rm["depth"] * gD * ok).sum())) / (2 * hp)
        # the GPU gradient with the same pixels' adjoints
        dp2 = torch.zeros(1, 6, device=DEV)
        P.render_bwd(gc, gd, [view], ws, P.zeros_like_gaussians(gd), dp2, dL_drgb=[t(gC * ok).reshape(3, H, W)],
                     dL_ddepth=[t(gD * ok).reshape(H, W)], pose_xi=xi)
        torch.cuda.synchronize()
        an = float(h(dp2)[0, j])
        assert abs(fd - an) <= 1e-2 * max(abs(fd), abs(an)), (j, fd, an)


def test_pose_xi_through_autograd(P, O):
    """RenderLoss with a non-zero pose_xi: the loss is the reference loss at Exp(xi) T, its pose
    gradient is J_l(xi)^T times the reference's gradient of the loss at that camera, and a step of
    xi against the gradient lowers the reference loss."""
    say("pose_xi through RenderLoss")
    case = tiny_case(8, M=60, W=53, H=37, log_scale=-2.4)
    gc, oc = cfg_pair(P, O, eps=0.03)
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]), t(case["target_rgb"]),
                  t(case["target_depth"]))
    sess = P.Session(gc, [view], 60, device=DEV)
    params = {k: t(v).requires_grad_(True) for k, v in case["gauss"].items()}
    xi = t(XI0.reshape(1, 6)).requires_grad_(True)
    loss = P.RenderLoss.apply(*(params[k] for k in KEYS), xi, sess)
    loss.backward()
    cam_p = _cam_at(case["cam"], XI0)
    r = O.render(oc, case["gauss"], cam_p, case["base_rgb"], case["base_depth"])
    L, grgb, gdep, _ = O.loss(oc, 53, 37, r["rgb"], r["depth"], case["target_rgb"], case["target_depth"],
                              case["base_depth"])
    assert abs(loss.item() - L) <= 1e-4 * L
    ref = O.render_bwd(oc, case["gauss"], cam_p, case["base_rgb"], case["base_depth"], grgb, gdep)
    g = h(xi.grad)[0].astype(np.float64)
    assert normwise(g, _left_jacobian_fd(XI0).T @ ref["pose"]) < 1e-3
    for k in KEYS:
        assert normwise(h(params[k].grad), ref[k]) < 1e-3, k
    step = -1e-3 * g / np.linalg.norm(g)
    rs = O.render(oc, case["gauss"], _cam_at(case["cam"], XI0 + step), case["base_rgb"], case["base_depth"])
    Ls = O.loss(oc, 53, 37, rs["rgb"], rs["depth"], case["target_rgb"], case["target_depth"], case["base_depth"],
                want_grad=False)[0]
    assert Ls < L
    # None for pose_xi: no pose gradient is returned and the camera is used as it is
    loss0 = P.RenderLoss.apply(*(params[k] for k in KEYS), None, sess)
    r0 = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    L0 = O.loss(oc, 53, 37, r0["rgb"], r0["depth"], case["target_rgb"], case["target_depth"], case["base_depth"],
                want_grad=False)[0]
    assert abs(loss0.item() - L0) <= 1e-4 * L0


@pytest.mark.parametrize("mode", [0, 1])
def test_out_aux(P, O, mode):
    """out_aux holds T_final (sorted mode) or W_G (sort-free mode); views without it are unchanged."""
    say(f"out_aux, mode {mode}")
    cases = [tiny_case(9, M=80, W=53, H=37, log_scale=-2.4), tiny_case(10, M=80, W=40, H=30, log_scale=-2.4)]
    gc, oc = cfg_pair(P, O, mode=mode, eps=0.03)
    g = cases[0]["gauss"]
    views = [P.View(c["cam"], t(c["base_rgb"]), t(c["base_depth"]),
                    out_aux=torch.full((c["cam"]["height"], c["cam"]["width"]), -1.0, device=DEV) if i == 0 else None)
             for i, c in enumerate(cases)]
    ws = P.Workspace(gc, 80, [v.cam for v in views], device=DEV)
    P.render_fwd(gc, {k: t(v) for k, v in g.items()}, views, ws)
    torch.cuda.synchronize()
    c = cases[0]
    r = O.render(oc, g, c["cam"], c["base_rgb"], c["base_depth"])
    keep = r["flag"] == 0
    ref = r["T"] if mode == 0 else r["W"]
    got = h(views[0].out_aux).reshape(-1)
    assert normwise(got, ref, keep) < 1e-4
    assert np.abs(got - ref)[keep].max() < 1e-4 * max(1.0, np.abs(ref).max())
    if mode == 0:
        assert (got[keep] <= 1.0).all() and (got[keep] >= 0.0).all() and (got[keep] < 1.0).any()
    else:
        assert (got[keep] > 0.0).any()
