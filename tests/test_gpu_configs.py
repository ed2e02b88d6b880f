"""GPU checks at the sizes of two workloads:

* Differentiation (640x480, 50,000 Gaussians on the room): the gradients of the loss
  returned by RenderLoss (torch.autograd) for 16 seeded Gaussians against the FP64
  reference's analytic gradients (each Gaussian's support box re-rendered by the
  reference, with the loss's adjoint there), and central differences of the FP64
  reference loss (h = 1e-4) on 64 parameters of those Gaussians, re-rendering only the
  parameter's support box, under the active-set rule (same contributors in the same depth
  order, no flags and the same residual signs at +h and -h; otherwise the next seeded
  parameter is drawn), tolerance
  1e-2 of max(|analytic|, |difference|).  The backward recomputes the per-pixel
  transmittance (nothing per pixel is stored by the forward besides T_final).
* Large streaming map (512^3 at 5 mm, 1,000,000 Gaussians, 4 keyframes at 1280x720):
  fusion of the 4 frames at every lattice point, the raycast of the 4 views on sampled
  pixels, one batched iteration (forward with the fused loss, backward with Adam in its
  epilogue) with the forward on 150 sampled pixels per view, the gradients of an upstream
  placed on those pixels, and the Adam update of every parameter.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, cfg_pair, gauss_dev, h, normwise, report_flags, say, t

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
    O.lib()
    return O


def _seed(scene, W, H, M):
    cams = synth.orbit_cameras(0, W, H, frames=list(range(0, 100, 10)))
    depths = [synth.render_frame(scene, c)[0] for c in cams]
    return synth.seed_gaussians(scene, cams, depths, M)


# ---------------------------------------------------------------- differentiation
def test_differentiation_640x480_50k(P, O):
    say("differentiation: 640x480, 50k Gaussians")
    W, H, M = 640, 480, 50_000
    scene = synth.scene_room(256)
    cam = synth.orbit_cameras(0, W, H, frames=[0])[0]
    d, c = synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=0)
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    ref = O.fuse(grid, O.new_volume(grid), cam.as_dict(), d, c)
    rd, rc, _ = O.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), cam.as_dict())
    base_rgb = rc.reshape(3, H, W).astype(np.float32)
    base_depth = rd.reshape(H, W).astype(np.float32)
    gauss = _seed(scene, W, H, M)
    camd = cam.as_dict()
    gc, oc = cfg_pair(P, O, eps=scene.voxel)
    view = P.View(camd, t(base_rgb), t(base_depth), t(c), t(d))
    sess = P.Session(gc, [view], M, device=DEV)
    params = {k: t(v).requires_grad_(True) for k, v in gauss.items()}
    xi = torch.zeros(1, 6, device=DEV, requires_grad=True)
    loss = P.RenderLoss.apply(*(params[k] for k in KEYS), xi, sess)
    loss.backward()
    torch.cuda.synchronize()
    got = {k: h(params[k].grad).reshape(ROWS[k], M) for k in KEYS}
    C_gpu, D_gpu = h(view.out_rgb).reshape(3, -1), h(view.out_depth).reshape(-1)
    # the fused loss equals the L1 of the GPU's images (a property at any size)
    om = (d.reshape(-1) > 0) & (base_depth.reshape(-1) > 0)
    L_img = np.abs(C_gpu.astype(np.float64) - c.reshape(3, -1)).mean() + \
        np.abs(D_gpu.astype(np.float64)[om] - d.reshape(-1)[om]).mean()
    assert abs(loss.item() - L_img) <= 1e-4 * L_img

    proj = O.project(oc, gauss, camd)
    box = proj["box"]  # xmin, xmax, ymin, ymax of the support
    inside = proj["valid"] & (box[:, 0] > 2) & (box[:, 1] < W - 3) & (box[:, 2] > 2) & (box[:, 3] < H - 3)
    inside &= (box[:, 1] - box[:, 0]) * (box[:, 3] - box[:, 2]) < 60 * 60

    def box_pixels(g, margin=2):
        x0, x1 = int(np.floor(box[g, 0])) - margin, int(np.ceil(box[g, 1])) + margin
        y0, y1 = int(np.floor(box[g, 2])) - margin, int(np.ceil(box[g, 3])) + margin
        jj, ii = np.mgrid[max(y0, 0):min(y1, H - 1) + 1, max(x0, 0):min(x1, W - 1) + 1]
        return (jj * W + ii).reshape(-1).astype(np.int32)

    def box_loss(g_params, pix):
        """The loss restricted to the pixels `pix` (every other pixel set to its target, so its
        residual and adjoint are zero), its adjoints there, and the render of those pixels."""
        r = O.render(oc, g_params, camd, base_rgb, base_depth, pix=pix)
        rgb_full = c.reshape(3, -1).astype(np.float64).copy()
        dep_full = d.reshape(-1).astype(np.float64).copy()
        rgb_full[:, pix] = r["rgb"]
        dep_full[pix] = r["depth"]
        L, grgb, gdep, _ = O.loss(oc, W, H, rgb_full, dep_full, c, d, base_depth)
        return L, grgb[:, pix], gdep[pix], r

    rng = np.random.Generator(np.random.PCG64(3))
    cands = rng.permutation(np.flatnonzero(inside))
    done_g, checked, tried = 0, 0, 0
    for g in cands:
        if done_g == 16:
            break
        pix = box_pixels(g)
        L0, grgb, gdep, r0 = box_loss(gauss, pix)
        res = np.abs(r0["rgb"] - c.reshape(3, -1)[:, pix])
        if (r0["flag"] != 0).any() or res.min() < 1e-5:
            continue  # a decision or a residual sign near rounding in the box: draw the next one
        ref_g = O.render_bwd(oc, gauss, camd, base_rgb, base_depth, grgb, gdep, pix=pix)
        ref_g = {k: ref_g[k].reshape(ROWS[k], M)[:, g] for k in KEYS}
        if np.abs(ref_g["rgb"]).max() < 1e-9:
            continue  # the Gaussian contributes to no pixel: draw the next one
        done_g += 1
        for k in KEYS:
            a, b = got[k][:, g], ref_g[k]
            assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-12, (g, k, a, b)
        # central differences on 4 parameters of this Gaussian (components whose reference
        # gradient is at least 1e-3 of the Gaussian's largest in that attribute)
        n_here = 0
        while n_here < 4 and tried < 600:
            tried += 1
            k = KEYS[rng.integers(0, len(KEYS))]
            row = int(rng.integers(0, ROWS[k]))
            if abs(ref_g[k][row]) < 1e-3 * np.abs(ref_g[k]).max() or ref_g[k][row] == 0.0:
                continue
            an = float(got[k][row, g])
            gp = {kk: v.copy() for kk, v in gauss.items()}
            gm = {kk: v.copy() for kk, v in gauss.items()}
            arr_p = gp[k].reshape(ROWS[k], M)
            arr_m = gm[k].reshape(ROWS[k], M)
            arr_p[row, g] = np.float32(float(arr_p[row, g]) + 1e-4)
            arr_m[row, g] = np.float32(float(arr_m[row, g]) - 1e-4)
            step = float(arr_p[row, g]) - float(arr_m[row, g])
            Lp, _, _, rp = box_loss(gp, pix)
            Lm, _, _, rm = box_loss(gm, pix)
            same = np.array_equal(rp["n"], rm["n"]) and (rp["flag"] == 0).all() and (rm["flag"] == 0).all()
            same = same and np.array_equal(rp["order"], rm["order"])  # no two depths swapped places
            same = same and np.array_equal(np.sign(rp["rgb"] - c.reshape(3, -1)[:, pix]),
                                           np.sign(rm["rgb"] - c.reshape(3, -1)[:, pix]))
            same = same and np.array_equal(np.sign(rp["depth"] - d.reshape(-1)[pix]),
                                           np.sign(rm["depth"] - d.reshape(-1)[pix]))
            if not same:
                continue  # the active set changed between +h and -h
            fd = (Lp - Lm) / step
            assert abs(fd - an) <= 1e-2 * max(abs(fd), abs(an)), (g, k, row, fd, an)
            n_here += 1
            checked += 1
    assert done_g == 16 and checked == 64, (done_g, checked)


# ---------------------------------------------------------------- large streaming map
def test_large_map_iteration_512_1m(P, O):
    say("large map: 512^3, 1M Gaussians, 4 keyframes")
    frames = [0, 10, 20, 30]
    scene, fr = synth.workload_room_frames(n=512, frames=frames)
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=DEV)
    for cam, d, c in fr:
        P.fuse(vol, cam.as_dict(), t(d), t(c))
    outs = P.raycast(vol, [cam.as_dict() for cam, _, _ in fr], z_near=0.2)
    torch.cuda.synchronize()
    say("large map: reference fusion of the 4 frames")
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    ref = O.new_volume(grid)
    for cam, d, c in fr:
        O.fuse(grid, ref, cam.as_dict(), d, c)
    np.testing.assert_array_equal(h(vol.weight), ref["weight"].astype(np.float32))
    upd = ref["weight"] > 0
    assert upd.sum() > 5_000_000
    # binary32 camera-frame depth of a voxel: a 3-term dot product over coordinates up to ~3 m,
    # rounded to ~3u * 5 m ~ 1e-6 m, i.e. ~5e-5 of the 2 cm truncation; the running average
    # keeps it there.  Bound: the 1e-4 relative tolerance of the tsdf's range [-1, 1].
    assert np.abs(h(vol.tsdf)[upd] - ref["tsdf"][upd]).max() < 1e-4
    t32, c32 = ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32)
    del ref
    rng = np.random.Generator(np.random.PCG64(81))
    for (cam, _, _), (gd_, gc_) in zip(fr, outs):
        pix = np.sort(rng.choice(1280 * 720, 200, replace=False)).astype(np.int32)
        rd, rc, rk = O.raycast(grid, t32, c32, cam.as_dict(), z_near=0.2, pix=pix)
        gdep = h(gd_).reshape(-1)[pix]
        both = (gdep > 0) & (rk >= 0)
        assert ((gdep > 0) == (rk >= 0)).mean() >= 0.99     # the GPU marched its own binary32 volume
        assert np.abs(gdep[both] - rd[both]).max() <= 1e-3 * rd[both].max()
    del t32, c32
    say("large map: one batched iteration, 1M Gaussians")
    M = 1_000_000
    gauss = _seed(scene, 1280, 720, M)
    gc, oc = cfg_pair(P, O, eps=scene.voxel, tile=(16, 32, 256, 2))
    views_np = []
    for cam, d, c in fr:
        bd, bc = synth.render_frame(scene, cam)  # analytic SDF-surface stand-in, identical on both sides
        views_np.append({"cam": cam.as_dict(), "base_rgb": bc, "base_depth": bd, "target_rgb": c, "target_depth": d})
    views = [P.View(v["cam"], t(v["base_rgb"]), t(v["base_depth"]), t(v["target_rgb"]), t(v["target_depth"]))
             for v in views_np]
    ws = P.Workspace(gc, M, [v.cam for v in views], device=DEV)
    gd = gauss_dev(gauss)
    loss = torch.zeros(1, device=DEV)
    P.render_fwd(gc, gd, views, ws, out_loss=loss)
    torch.cuda.synchronize()
    assert ws.status() == 0
    ups_rgb, ups_dep, refs = [], [], None
    for v, vn in zip(views, views_np):
        pix = np.sort(rng.choice(1280 * 720, 150, replace=False)).astype(np.int32)
        r = O.render(oc, gauss, vn["cam"], vn["base_rgb"], vn["base_depth"], pix=pix)
        keep = r["flag"] == 0
        assert keep.mean() > 0.95
        C = h(v.out_rgb).reshape(3, -1)
        D = h(v.out_depth).reshape(-1)
        assert normwise(C[:, pix], r["rgb"], keep) < 1e-4
        assert normwise(D[pix], r["depth"], keep) < 1e-4
        report_flags("large map view", keep, C[:, pix], r["rgb"])
        gC = np.zeros((3, 1280 * 720), np.float32)
        gD = np.zeros(1280 * 720, np.float32)
        ps = pix[keep]
        gC[:, ps] = rng.normal(size=(3, ps.size))
        gD[ps] = rng.normal(size=ps.size)
        ups_rgb.append(t(gC).reshape(3, 720, 1280))
        ups_dep.append(t(gD).reshape(720, 1280))
        rg = O.render_bwd(oc, gauss, vn["cam"], vn["base_rgb"], vn["base_depth"], gC[:, ps], gD[ps], pix=ps)
        refs = rg if refs is None else {k: refs[k] + rg[k] if k != "pose" else np.vstack([refs[k], rg[k]])
                                        for k in refs}
    # backward with Adam in its epilogue on that upstream: the gradients, then every parameter
    opt = P.Adam(gd)
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(4, 6, device=DEV)
    P.render_bwd_adam(gc, gd, views, ws, opt, grads=grads, dpose=dpose, dL_drgb=ups_rgb, dL_ddepth=ups_dep)
    torch.cuda.synchronize()
    for k in KEYS:
        assert normwise(h(grads[k]), refs[k]) < 1e-3, k
    assert normwise(h(dpose), refs["pose"]) < 1e-3
    # Adam (first step) from the reference gradient on the reference side, elementwise where
    # the update does not hinge on the gradient's own error.  The first step moves a
    # parameter by lr g / (|g| + eps), whose sensitivity to g is lr eps / (|g| + eps)^2: a
    # gradient element off by up to its own size (tiny elements can be, under the normwise
    # 1e-3 bound of the gradient) moves the update by up to lr eps / |g|.  Elements where
    # that exceeds a tenth of the update's tolerance (gradients below ~1e-8; Gaussians seen
    # through a transmittance near T_min at one sampled pixel) and sign flips of near-zero
    # gradients are counted, not compared.
    f32 = lambda x: float(np.float32(x))
    eps = f32(1e-15)
    for k in KEYS:
        p = gauss[k].astype(np.float64).reshape(-1).copy()
        gr = refs[k].reshape(-1).astype(np.float64)
        lr = f32(O.PAPER_LR[k])
        O.adam(p, gr, np.zeros_like(p), np.zeros_like(p), lr, 1, b1=f32(0.9), b2=f32(0.999), eps=eps)
        got = h(gd[k]).astype(np.float64).reshape(-1)
        p0 = gauss[k].astype(np.float64).reshape(-1)
        # 1e-6 relative on both terms of p = p0 - step (the step carries its own roundings,
        # and p0 - step cancels where p0 ~ lr), plus one rounding of p0
        tol = 1e-6 * (np.abs(p) + np.abs(p0 - p)) + 2.0 ** -23 * np.abs(p0)
        same = np.sign(h(grads[k]).reshape(-1)) == np.sign(gr)
        with np.errstate(divide="ignore"):
            firm = same & (lr * eps / np.abs(gr) <= 0.1 * tol)
        bad = np.flatnonzero(firm & ~(np.abs(got - p) <= tol))
        for b in bad[:8]:
            say(f"  adam {k} element {b}: p0 {p0[b]!r} gpu {got[b]!r} ref {p[b]!r} "
                f"g_ref {gr[b]!r} g_gpu {h(grads[k]).reshape(-1)[b]!r}")
        assert bad.size == 0, (k, bad.size)
        nz = gr != 0
        assert (~same).sum() <= max(3, 1e-3 * nz.sum()), (k, (~same).sum(), nz.sum())
        soft = same & nz & ~firm
        say(f"  adam {k}: {firm.sum()} compared, {soft.sum()} with the update sensitive to the gradient's "
            f"error, {(~same).sum()} sign flips")
        assert soft.sum() <= 0.1 * nz.sum(), (k, soft.sum(), nz.sum())  # most elements are compared
