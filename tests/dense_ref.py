"""Dense float64 PyTorch renderer used as an independent pin of the oracle.

It is written from the same definitions as the oracle but by another route:
every (pixel, Gaussian) pair is evaluated as one dense matrix, the depth order
is one global ``torch.sort``-style permutation, transmittance is a cumulative
product, and derivatives come from autograd rather than hand adjoints.  Only
tiny inputs are rendered with it.  It does not import the oracle.
"""
from __future__ import annotations

import numpy as np
import torch


def _f32_row(R, t, r, p):
    """binary32 row r of R p + t with the evaluation order used for decisions."""
    R = np.asarray(R, np.float32).reshape(3, 3)
    t = np.asarray(t, np.float32)
    a = np.float32(R[r, 0]) * p[0]
    b = np.float32(R[r, 1]) * p[1]
    s = (a + b).astype(np.float32)
    c = np.float32(R[r, 2]) * p[2]
    s = (s + c).astype(np.float32)
    return (s + np.float32(t[r])).astype(np.float32)


def depth32(mean32, R, t):
    p = [np.asarray(mean32[k], np.float32) for k in range(3)]
    return _f32_row(R, t, 2, p)


def hat(v):
    z = torch.zeros((), dtype=v.dtype)
    return torch.stack([torch.stack([z, -v[2], v[1]]), torch.stack([v[2], z, -v[0]]),
                        torch.stack([-v[1], v[0], z])])


def quat_rot(q):
    qn = q / q.norm(dim=0, keepdim=True)
    w, x, y, z = qn
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)  # [M,3,3]


def sh_real(L, d):
    """Real spherical harmonics of bands 1..L at the unit directions d [3,M] (torch), built
    from the associated Legendre functions: Y_l^m = N_lm P_l^|m|(z) times the real or
    imaginary part of (x + i y)^|m| (which is sin^|m| theta e^{i |m| phi}), with the
    Condon-Shortley phase, sqrt(2) for m != 0, sine terms for m < 0, and m = -l .. l within
    each band.  Returns [K,M]."""
    import math
    from numpy.polynomial import legendre as leg
    from numpy.polynomial import polynomial as poly
    x, y, z = d
    out = []
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            a = abs(m)
            # d^a/dz^a P_l(z) in the power basis
            c = leg.leg2poly(leg.legder([0] * l + [1], a))
            q = sum(float(ck) * z ** k for k, ck in enumerate(c))
            re, im = torch.ones_like(x), torch.zeros_like(x)
            for _ in range(a):  # (x + i y)^a
                re, im = re * x - im * y, re * y + im * x
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - a) / math.factorial(l + a))
            cs = (-1) ** a
            if m < 0:
                out.append(math.sqrt(2) * N * cs * q * im)
            elif m == 0:
                out.append(N * q)
            else:
                out.append(math.sqrt(2) * N * cs * q * re)
    return torch.stack(out)


def render(params, cam, base_rgb, base_depth, cfg, xi=None):
    """params: dict of float64 tensors (mean [3,M], log_scale [3,M], quat [4,M], opacity_logit [M],
    rgb [3,M]) holding float32-representable values; cam: dict; base_rgb [3,H,W], base_depth [H,W]
    float32 numpy; cfg: object with mode, eps_cull, dilation, alpha_min, alpha_max, T_min, z_near.
    xi: optional float64 tensor (6,) pose perturbation (rho, phi) applied as T <- Exp(xi) T
    (to first order, which is exact for derivatives at xi = 0).
    Returns C [3,H,W], D [H,W] (float64 tensors)."""
    W, H = cam["width"], cam["height"]
    M = params["opacity_logit"].shape[0]
    R = torch.as_tensor(np.asarray(cam["R"], np.float32).reshape(3, 3).astype(np.float64))
    t = torch.as_tensor(np.asarray(cam["t"], np.float32).astype(np.float64))
    fx, fy, cx, cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))
    if xi is None:
        xi = torch.zeros(6, dtype=torch.float64)
    rho, phi = xi[:3], xi[3:]
    Rp = (torch.eye(3, dtype=torch.float64) + hat(phi)) @ R

    mu = params["mean"]
    pc = (torch.eye(3, dtype=torch.float64) + hat(phi)) @ (R @ mu + t[:, None]) + rho[:, None]  # [3,M]
    x, y, z = pc
    # decisions in binary32
    z32 = depth32(params["mean"].detach().numpy().astype(np.float32), cam["R"], cam["t"])
    valid = z32 >= np.float32(cfg.z_near)

    Rq = quat_rot(params["quat"])
    s = torch.exp(params["log_scale"])  # [3,M]
    S3 = Rq @ torch.diag_embed(s.T ** 2) @ Rq.transpose(1, 2)  # [M,3,3]
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * x / z ** 2], -1),
                     torch.stack([zero, fy / z, -fy * y / z ** 2], -1)], -2)  # [M,2,3]
    Wm = J @ Rp
    S2 = Wm @ S3 @ Wm.transpose(1, 2) + cfg.dilation * torch.eye(2, dtype=torch.float64)
    A, B, C = S2[:, 0, 0], 0.5 * (S2[:, 0, 1] + S2[:, 1, 0]), S2[:, 1, 1]
    det = A * C - B * B
    ca, cb, cc = C / det, -B / det, A / det
    mx = fx * x / z + cx
    my = fy * y / z + cy
    sig = torch.sigmoid(params["opacity_logit"])
    valid = valid & (det.detach().numpy() > 0) & (255.0 * sig.detach().numpy() > 1.0)

    jj, ii = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    px = torch.as_tensor(ii.reshape(-1))[:, None]
    py = torch.as_tensor(jj.reshape(-1))[:, None]
    dx = px - mx[None, :]
    dy = py - my[None, :]
    power = -0.5 * (ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy)
    raw = sig[None, :] * torch.exp(power)  # [P,M]

    bd = np.asarray(base_depth, np.float32).reshape(-1)
    dvalid = bd > 0
    dcull = np.where(dvalid, bd, np.float32(np.inf)).astype(np.float32)
    thr = (dcull + np.float32(cfg.eps_cull)).astype(np.float32)
    cand = (z32[None, :] < thr[:, None]) & valid[None, :] & (raw.detach().numpy() >= cfg.alpha_min)
    cand_t = torch.as_tensor(cand)
    Ct = torch.as_tensor(np.asarray(base_rgb, np.float32).reshape(3, -1).astype(np.float64))  # [3,P]
    Dt = torch.as_tensor(bd.astype(np.float64))
    rgb = params["rgb"]  # [3,M]
    if params.get("sh") is not None:
        # view-dependent bands (3DGS): the unit direction from the perturbed camera's centre
        # o = -Rp^T tp (tp its translation, to first order in xi) to the centre
        tp = (torch.eye(3, dtype=torch.float64) + hat(phi)) @ t + rho
        v = mu + (Rp.T @ tp)[:, None]
        dirs = v / v.norm(dim=0, keepdim=True)
        K = params["sh"].shape[1]
        L = {3: 1, 8: 2, 15: 3}[K]
        rgb = rgb + (params["sh"] * sh_real(L, dirs)[None]).sum(dim=1)

    if cfg.mode == 0:
        alpha = torch.where(raw > cfg.alpha_max, torch.full_like(raw, cfg.alpha_max), raw)
        alpha = torch.where(cand_t, alpha, torch.zeros_like(alpha))
        order = np.lexsort((np.arange(M), z32))  # by depth32, ties by index
        a = alpha[:, order]
        one_minus = 1.0 - a
        Tincl = torch.cumprod(one_minus, dim=1)
        keep = torch.as_tensor((Tincl.detach().numpy() >= cfg.T_min) if cfg.T_min > 0 else np.ones(a.shape, bool))
        a = torch.where(keep, a, torch.zeros_like(a))
        Tincl = torch.cumprod(1.0 - a, dim=1)
        Texcl = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], dim=1)
        w = a * Texcl
        Tf = Tincl[:, -1] if M > 0 else torch.ones(H * W, dtype=torch.float64)
        col = w @ rgb[:, order].T  # [P,3]
        dep = w @ z[order]
        Cs = col.T + Tf[None, :] * Ct
        Ds = torch.where(torch.as_tensor(dvalid), dep + Tf * Dt, torch.zeros_like(Dt))
    else:
        a = torch.where(cand_t, raw, torch.zeros_like(raw))
        Wg = a.sum(dim=1)
        Cs = (Ct + (a @ rgb.T).T) / (1 + Wg)[None, :]
        Ds = torch.where(torch.as_tensor(dvalid), (Dt + a @ z) / (1 + Wg), torch.zeros_like(Dt))
    return Cs.reshape(3, H, W), Ds.reshape(H, W)


def to_params(g, requires_grad=False):
    out = {}
    for k in ("mean", "log_scale", "quat", "opacity_logit", "rgb", "sh"):
        if k in g:
            out[k] = torch.tensor(np.asarray(g[k], np.float32).astype(np.float64), requires_grad=requires_grad)
    return out
