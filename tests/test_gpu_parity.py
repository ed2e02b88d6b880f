"""GPU parity of every entry point of libgps against the FP64 reference implementation.

All inputs are seeded and synthetic; the HIP path is called through the C ABI
(ctypes binding) and compared with the reference on the same inputs.
Tolerances: images, depths, loss 1e-4 relative (normwise over pixels whose
reference decisions are not within rounding of a threshold), gradients 1e-3
relative (normwise per tensor), Adam 1e-6 relative elementwise; integer
decisions (fusion pixel, raycast hit/miss, weights) bit-exact.
"""
import math

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, cfg_pair, gauss_dev, h, normwise, report_flags, say, t
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


@pytest.fixture(scope="module")
def small():
    return synth.workload_small()


def _second_small_camera():
    c = np.full(3, 0.02 * 63 / 2)
    eye = c + 1.5 * np.array([math.cos(2.2) * math.cos(0.5), math.sin(2.2) * math.cos(0.5), math.sin(0.5)])
    R, tt = synth.look_at(eye, c + np.array([0.05, -0.03, 0.0]))
    return synth.Camera(160, 120, 150.0, 150.0, 80.0, 60.0, R, tt)


# ------------------------------------------------------------------- fusion
def test_fuse_parity_small(P, O, small):
    say("fuse parity: 64^3, two 160x120 frames")
    sc = small["scene"]
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, device=DEV)
    ref = O.new_volume(grid)
    cam2 = _second_small_camera()
    d2, c2 = synth.render_frame(sc, cam2)
    for cam, d, c in ((small["cam"], small["depth"], small["rgb"]), (cam2, d2, c2)):
        P.fuse(vol, cam.as_dict(), t(d), t(c))
        O.fuse(grid, ref, cam.as_dict(), d, c)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h(vol.weight), ref["weight"].astype(np.float32))
    np.testing.assert_array_equal(h(vol.rgb_weight), ref["rgb_weight"].astype(np.float32))
    assert (ref["weight"] > 0).sum() > 5000
    assert np.abs(h(vol.tsdf) - ref["tsdf"]).max() < 2e-5
    assert np.abs(h(vol.rgb) - ref["rgb"]).max() < 2e-5
    assert normwise(h(vol.tsdf), ref["tsdf"]) < 1e-5


def test_fuse_weight_cap(P, O, small):
    sc = small["scene"]
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 2.0)
    vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, max_weight=2.0, device=DEV)
    ref = O.new_volume(grid)
    for _ in range(4):
        P.fuse(vol, small["cam"].as_dict(), t(small["depth"]), t(small["rgb"]))
        O.fuse(grid, ref, small["cam"].as_dict(), small["depth"], small["rgb"])
    torch.cuda.synchronize()
    assert h(vol.weight).max() == 2.0
    np.testing.assert_array_equal(h(vol.weight), ref["weight"].astype(np.float32))
    assert np.abs(h(vol.tsdf) - ref["tsdf"]).max() < 2e-5


# ------------------------------------------------------------------ raycast
def _fused_small(O, small):
    sc = small["scene"]
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    ref = O.new_volume(grid)
    O.fuse(grid, ref, small["cam"].as_dict(), small["depth"], small["rgb"])
    cam2 = _second_small_camera()
    d2, c2 = synth.render_frame(sc, cam2)
    O.fuse(grid, ref, cam2.as_dict(), d2, c2)
    return grid, ref


@pytest.mark.parametrize("bricks", [False, True])
def test_raycast_parity_small(P, O, small, bricks):
    say(f"raycast parity: 64^3, bricks={bricks}")
    sc = small["scene"]
    grid, ref = _fused_small(O, small)
    t32, c32 = ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32)
    vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, device=DEV, skip_bricks=bricks)
    vol.tsdf.copy_(t(t32))
    vol.rgb.copy_(t(c32))
    cams = [small["cam"], _second_small_camera()]
    outs = P.raycast(vol, [c.as_dict() for c in cams], z_near=0.2)
    torch.cuda.synchronize()
    for cam, (gd, gc) in zip(cams, outs):
        rd, rc, rk = O.raycast(grid, t32, c32, cam.as_dict(), z_near=0.2)
        gd, gc = h(gd).reshape(-1), h(gc).reshape(3, -1)
        np.testing.assert_array_equal(gd > 0, rk >= 0)  # the same rays hit
        hit = rk >= 0
        assert hit.sum() > 1000
        assert np.abs(gd[hit] - rd[hit]).max() <= 1e-4 * rd[hit].max()
        assert normwise(gd, rd) < 1e-5
        # colour: 1e-4 normwise; elementwise the stripe edges turn depth rounding (~1e-6 m) into
        # colour differences of up to slope * 1e-6, hence the looser elementwise bound
        assert normwise(gc, rc) < 1e-4
        assert np.abs(gc - rc).max() < 1e-3
        assert (gc[:, ~hit] == 0).all()


def test_raycast_bricks_do_not_change_result(P, O, small):
    sc = small["scene"]
    _, ref = _fused_small(O, small)
    outs = []
    for bricks in (False, True):
        vol = P.Volume(sc.dims, sc.origin, sc.voxel, sc.trunc, device=DEV, skip_bricks=bricks)
        vol.tsdf.copy_(t(ref["tsdf"]))
        vol.rgb.copy_(t(ref["rgb"]))
        outs.append([h(x) for x in P.raycast(vol, [small["cam"].as_dict()])[0]])
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def _brick_minima(tsdf):
    """Minimum over the 9^3 lattice points [8b, 8b + 8] (clipped) of each brick, then over
    each 4^3 group of bricks; tsdf indexed [z, y, x]."""
    nz, ny, nx = tsdf.shape
    B = [(n + 7) // 8 for n in (nx, ny, nz)]
    bm = np.empty((B[2], B[1], B[0]), np.float32)
    for k in range(B[2]):
        for j in range(B[1]):
            for i in range(B[0]):
                bm[k, j, i] = tsdf[8 * k:8 * k + 9, 8 * j:8 * j + 9, 8 * i:8 * i + 9].min()
    S = [(b + 3) // 4 for b in B]
    sm = np.empty((S[2], S[1], S[0]), np.float32)
    for k in range(S[2]):
        for j in range(S[1]):
            for i in range(S[0]):
                sm[k, j, i] = bm[4 * k:4 * k + 4, 4 * j:4 * j + 4, 4 * i:4 * i + 4].min()
    return bm.reshape(-1), sm.reshape(-1)


@pytest.mark.parametrize("dims", [(64, 64, 64), (70, 45, 37), (4100, 3, 10)],
                         ids=["64^3", "ragged", "long-rows"])
def test_brick_minima(P, dims):
    """The brick and superbrick minima the raycast rebuilds, against their definition, on
    random values: a whole lattice, ragged edges in every axis, and rows longer than the
    row kernel takes (the per-brick kernel)."""
    nx, ny, nz = dims
    rng = np.random.Generator(np.random.PCG64(31))
    vals = rng.uniform(-1.0, 1.0, (nz, ny, nx)).astype(np.float32)
    vol = P.Volume(dims, (0.0, 0.0, 0.0), 0.02, 0.08, device=DEV, skip_bricks=True)
    vol.tsdf.copy_(t(vals.reshape(-1)))
    cam = synth.Camera(64, 48, 60.0, 60.0, 32.0, 24.0, np.eye(3, dtype=np.float32),
                       np.array([-0.3, -0.3, -1.0], np.float32))
    P.raycast(vol, [cam.as_dict()], z_near=0.2)
    torch.cuda.synchronize()
    bm, sm = _brick_minima(vals)
    got = h(vol.brick_min)
    np.testing.assert_array_equal(got[:bm.size], bm)
    np.testing.assert_array_equal(got[bm.size:bm.size + sm.size], sm)


# ------------------------------------------------------------ render fwd
TILES = [(16, 16, 256, 1), (8, 8, 128, 1), (16, 16, 128, 2), (16, 16, 512, 4), (16, 32, 256, 2), (16, 32, 128, 1),
         (32, 16, 128, 2)]


def _render_gpu(P, gc, g, views_np, targets=True):
    views = []
    for vn in views_np:
        views.append(P.View(vn["cam"], t(vn["base_rgb"]), t(vn["base_depth"]),
                            t(vn["target_rgb"]) if targets else None, t(vn["target_depth"]) if targets else None))
    M = int(np.asarray(g["opacity_logit"]).size)
    ws = P.Workspace(gc, M, [v.cam for v in views], device=DEV)
    gd = gauss_dev(g)
    loss = torch.zeros(1, device=DEV)
    P.render_fwd(gc, gd, views, ws, out_loss=loss if targets else None)
    return views, ws, gd, loss


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tile", TILES)
def test_render_fwd_parity_tiny(P, O, mode, tile):
    say(f"render fwd parity tiny: mode={mode} tile={tile}")
    for seed in (0, 1, 2):
        case = tiny_case(seed, M=60, W=53, H=37, log_scale=-2.4)
        gc, oc = cfg_pair(P, O, mode=mode, eps=0.03, tile=tile)
        views, ws, _, loss = _render_gpu(P, gc, case["gauss"], [case])
        torch.cuda.synchronize()
        assert ws.status() == 0
        r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
        keep = r["flag"] == 0
        assert keep.mean() > 0.99
        C, D = h(views[0].out_rgb).reshape(3, -1), h(views[0].out_depth).reshape(-1)
        assert normwise(C, r["rgb"], keep) < 1e-4
        assert normwise(D, r["depth"], keep) < 1e-4
        assert np.abs(C - r["rgb"])[:, keep].max() < 1e-4
        assert (r["n"] > 0).sum() > 200
        L, _, _, _ = O.loss(oc, case["cam"]["width"], case["cam"]["height"], r["rgb"], r["depth"],
                            case["target_rgb"], case["target_depth"], case["base_depth"], want_grad=False)
        assert abs(loss.item() - L) <= 1e-4 * abs(L)


@pytest.mark.parametrize("mode", [0, 1])
def test_render_fwd_parity_small_scene(P, O, small, mode):
    say(f"render fwd parity: 160x120, 2000 Gaussians, mode={mode}")
    sc, cam = small["scene"], small["cam"]
    grid, ref = _fused_small(O, small)
    rd, rc, _ = O.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), cam.as_dict())
    vn = {"cam": cam.as_dict(), "base_rgb": rc.reshape(3, 120, 160), "base_depth": rd.reshape(120, 160),
          "target_rgb": small["rgb"], "target_depth": small["depth"]}
    gc, oc = cfg_pair(P, O, mode=mode, eps=sc.voxel)
    views, ws, _, loss = _render_gpu(P, gc, small["gauss"], [vn])
    torch.cuda.synchronize()
    r = O.render(oc, small["gauss"], cam.as_dict(), vn["base_rgb"].astype(np.float32),
                 vn["base_depth"].astype(np.float32))
    keep = r["flag"] == 0
    C, D = h(views[0].out_rgb).reshape(3, -1), h(views[0].out_depth).reshape(-1)
    assert normwise(C, r["rgb"], keep) < 1e-4 and normwise(D, r["depth"], keep) < 1e-4
    report_flags(f"small scene mode {mode}", keep, C, r["rgb"])
    L, _, _, om = O.loss(oc, 160, 120, r["rgb"], r["depth"], small["rgb"], small["depth"],
                         vn["base_depth"].astype(np.float32), want_grad=False)
    assert abs(loss.item() - L) <= 1e-4 * abs(L)
    st = ws.stats()
    assert st["status"] == 0 and st["n_instances"] > 0 and st["view_omega"][0] == om


# ------------------------------------------------------------ render bwd
def _explicit_upstream(case, seed, flags=None):
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    W, H = case["cam"]["width"], case["cam"]["height"]
    gC = rng.normal(size=(3, H * W)).astype(np.float32)
    gD = rng.normal(size=H * W).astype(np.float32)
    if flags is not None:  # ambiguous decisions in the reference: no upstream there
        gC[:, flags != 0] = 0
        gD[flags != 0] = 0
    return gC, gD


def _grads_gpu(P, gc, gd, views, ws, up=None, scale=None):
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(len(views), 6, device=DEV)
    if up is None:
        P.render_bwd(gc, gd, views, ws, grads, dpose, loss_scale=scale)
    else:
        P.render_bwd(gc, gd, views, ws, grads, dpose, dL_drgb=[t(u[0]).reshape(views[i].out_rgb.shape)
                                                                for i, u in enumerate(up)],
                     dL_ddepth=[t(u[1]).reshape(views[i].out_depth.shape) for i, u in enumerate(up)])
    torch.cuda.synchronize()
    out = {k: h(v) for k, v in grads.items()}
    out["pose"] = h(dpose)
    return out


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tile", [(16, 16, 256, 1), (8, 8, 512, 1), (16, 16, 256, 4), (16, 32, 256, 2)])
def test_render_bwd_parity_explicit(P, O, mode, tile):
    say(f"render bwd parity (explicit upstream): mode={mode} tile={tile}")
    for seed in (0, 1):
        case = tiny_case(seed, M=60, W=53, H=37, log_scale=-2.4)
        gc, oc = cfg_pair(P, O, mode=mode, eps=0.03, tile=tile)
        views, ws, gd, _ = _render_gpu(P, gc, case["gauss"], [case])
        r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
        gC, gD = _explicit_upstream(case, seed, r["flag"])
        got = _grads_gpu(P, gc, gd, views, ws, up=[(gC, gD)])
        ref = O.render_bwd(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
        for k in KEYS:
            assert normwise(got[k], ref[k]) < 1e-3, (k, normwise(got[k], ref[k]))
        assert normwise(got["pose"][0], ref["pose"]) < 1e-3


@pytest.mark.parametrize("mode", [0, 1])
def test_render_bwd_parity_fused_loss(P, O, small, mode):
    say(f"render bwd parity (fused loss): 160x120, mode={mode}")
    sc, cam = small["scene"], small["cam"]
    grid, ref = _fused_small(O, small)
    rd, rc, _ = O.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), cam.as_dict())
    vn = {"cam": cam.as_dict(), "base_rgb": rc.reshape(3, 120, 160).astype(np.float32),
          "base_depth": rd.reshape(120, 160).astype(np.float32), "target_rgb": small["rgb"],
          "target_depth": small["depth"]}
    gc, oc = cfg_pair(P, O, mode=mode, eps=sc.voxel)
    views, ws, gd, loss = _render_gpu(P, gc, small["gauss"], [vn])
    scale = torch.full((1,), 2.0, device=DEV)
    got = _grads_gpu(P, gc, gd, views, ws, scale=scale)
    r = O.render(oc, small["gauss"], cam.as_dict(), vn["base_rgb"], vn["base_depth"])
    L, grgb, gdep, _ = O.loss(oc, 160, 120, r["rgb"], r["depth"], small["rgb"], small["depth"], vn["base_depth"],
                              scale=2.0)
    refg = O.render_bwd(oc, small["gauss"], cam.as_dict(), vn["base_rgb"], vn["base_depth"], grgb, gdep)
    for k in KEYS:
        assert normwise(got[k], refg[k]) < 1e-3, (k, normwise(got[k], refg[k]))
    assert normwise(got["pose"][0], refg["pose"]) < 1e-3


def test_autograd_function(P, O):
    """RenderLoss through torch.autograd matches the reference loss and gradients."""
    case = tiny_case(4, M=60, W=53, H=37, log_scale=-2.4)
    gc, oc = cfg_pair(P, O, eps=0.03)
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]), t(case["target_rgb"]),
                  t(case["target_depth"]))
    sess = P.Session(gc, [view], 60, device=DEV)
    params = {k: t(v).requires_grad_(True) for k, v in case["gauss"].items()}
    xi = torch.zeros(1, 6, device=DEV, requires_grad=True)
    loss = P.RenderLoss.apply(params["mean"], params["log_scale"], params["quat"], params["opacity_logit"],
                              params["rgb"], xi, sess)
    (3.0 * loss).backward()
    r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    L, grgb, gdep, _ = O.loss(oc, 53, 37, r["rgb"], r["depth"], case["target_rgb"], case["target_depth"],
                              case["base_depth"], scale=3.0)
    assert abs(loss.item() - L) <= 1e-4 * L
    ref = O.render_bwd(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], grgb, gdep)
    for k in KEYS:
        assert normwise(h(params[k].grad), ref[k]) < 1e-3, k
    assert normwise(h(xi.grad)[0], ref["pose"]) < 1e-3


# ------------------------------------------------------------ multi-view
def test_multiview_one_call(P, O):
    """Views of different sizes in one call equal the per-view reference; the loss is their mean."""
    say("multi-view parity: 3 views of different sizes")
    cases = [tiny_case(20, M=50, W=53, H=37), tiny_case(21, M=50, W=40, H=30), tiny_case(22, M=50, W=71, H=19)]
    g = cases[0]["gauss"]
    gc, oc = cfg_pair(P, O, eps=0.03)
    views, ws, gd, loss = _render_gpu(P, gc, g, cases)
    got = _grads_gpu(P, gc, gd, views, ws)
    Ls, acc = [], None
    for c, v in zip(cases, views):
        r = O.render(oc, g, c["cam"], c["base_rgb"], c["base_depth"])
        keep = r["flag"] == 0
        assert normwise(h(v.out_rgb).reshape(3, -1), r["rgb"], keep) < 1e-4
        L, grgb, gdep, _ = O.loss(oc, c["cam"]["width"], c["cam"]["height"], r["rgb"], r["depth"], c["target_rgb"],
                                  c["target_depth"], c["base_depth"], scale=1.0 / 3)
        Ls.append(L)
        rg = O.render_bwd(oc, g, c["cam"], c["base_rgb"], c["base_depth"], grgb, gdep)
        acc = rg if acc is None else {k: acc[k] + rg[k] if k != "pose" else np.vstack([acc[k], rg[k]]) for k in acc}
    assert abs(loss.item() - np.mean(Ls)) <= 1e-4 * np.mean(Ls)
    for k in KEYS:
        assert normwise(got[k], acc[k]) < 1e-3, k
    assert normwise(got["pose"], acc["pose"].reshape(3, 6)) < 1e-3


# ------------------------------------------------------------------- adam
def test_adam_parity(P, O):
    rng = np.random.Generator(np.random.PCG64(31))
    n = 10007  # ragged: not a multiple of 4 -> scalar path
    shapes = {"a": 4096, "b": n}
    for name, size in shapes.items():
        p0 = rng.normal(size=size).astype(np.float32)
        p, m, v = t(p0), torch.zeros(size, device=DEV), torch.zeros(size, device=DEV)
        rp, rm, rv = p0.astype(np.float64), np.zeros(size), np.zeros(size)
        for step in range(1, 4):
            g = (rng.normal(size=size) * 10 ** rng.uniform(-4, 1, size)).astype(np.float32)
            p_old, m_old = rp.copy(), rm.copy()
            P.adam_step([(p, t(g), m, v, 1e-3)], step)
            # the C ABI takes lr, beta1, beta2 and eps as binary32: the reference gets those values
            # (beta2 = 0.999 rounds to 0.99900001287, so 1 - beta2 differs from 0.001 by 1.3e-5)
            f32 = lambda x: float(np.float32(x))
            O.adam(rp, g.astype(np.float64), rm, rv, f32(1e-3), step, b1=f32(0.9), b2=f32(0.999), eps=f32(1e-15))
            torch.cuda.synchronize()
            # compare from identical inputs (the reference state is reset to the GPU's after each
            # step), element by element, 1e-6 relative (of the result, and of the step where
            # p - step cancels); the only extra allowance is one binary32 rounding of the terms
            # that cancel (p - step, b1 m + (1 - b1) g)
            ulp = 2.0 ** -23
            assert (np.abs(h(p) - rp) <= 1e-6 * (np.abs(rp) + np.abs(p_old - rp)) + ulp * np.abs(p_old)).all()
            assert (np.abs(h(m) - rm) <= 1e-6 * np.abs(rm) + ulp * (0.9 * np.abs(m_old) + 0.1 * np.abs(g))).all()
            assert (np.abs(h(v) - rv) <= 1e-6 * np.abs(rv)).all()
            rp, rm, rv = h(p).astype(np.float64), h(m).astype(np.float64), h(v).astype(np.float64)


def test_adam_device_counter(P):
    """With a device step counter the bias correction follows the counter, which advances by one."""
    p1, p2 = t(np.ones(64)), t(np.ones(64))
    g = t(np.full(64, 0.5))
    m1, v1, m2, v2 = (torch.zeros(64, device=DEV) for _ in range(4))
    ctr = torch.zeros(1, dtype=torch.int32, device=DEV)
    for step in range(1, 4):
        P.adam_step([(p1, g, m1, v1, 0.01)], 0, step_counter=ctr)
        P.adam_step([(p2, g, m2, v2, 0.01)], step)
    torch.cuda.synchronize()
    assert int(ctr.item()) == 3
    np.testing.assert_array_equal(h(p1), h(p2))


# ---------------------------------------------------- determinism / edges
def test_bitwise_determinism(P, O, small):
    sc, cam = small["scene"], small["cam"]
    grid, ref = _fused_small(O, small)
    rd, rc, _ = O.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), cam.as_dict())
    vn = {"cam": cam.as_dict(), "base_rgb": rc.reshape(3, 120, 160), "base_depth": rd.reshape(120, 160),
          "target_rgb": small["rgb"], "target_depth": small["depth"]}
    gc, _ = cfg_pair(P, O, eps=sc.voxel)
    runs = []
    for _ in range(2):
        views, ws, gd, loss = _render_gpu(P, gc, small["gauss"], [vn])
        got = _grads_gpu(P, gc, gd, views, ws)
        runs.append((h(views[0].out_rgb), h(loss), got))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    for k in KEYS + ("pose",):
        np.testing.assert_array_equal(runs[0][2][k], runs[1][2][k])


@pytest.mark.parametrize("mode", [0, 1])
def test_no_gaussians_and_all_culled(P, O, mode):
    case = tiny_case(5, M=30, W=53, H=37)
    gc, _ = cfg_pair(P, O, mode=mode, eps=0.03)
    g0 = {k: v[..., :0].copy() for k, v in case["gauss"].items()}
    views, ws, gd, _ = _render_gpu(P, gc, g0, [case])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h(views[0].out_rgb), case["base_rgb"])
    bd = np.where(case["base_depth"] > 0, case["base_depth"], 0).astype(np.float32)
    np.testing.assert_array_equal(h(views[0].out_depth), bd)
    occl = dict(case)
    occl["base_depth"] = np.full_like(case["base_depth"], 0.5)
    views, ws, gd, _ = _render_gpu(P, gc, case["gauss"], [occl])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h(views[0].out_rgb), case["base_rgb"])
    assert ws.stats()["pairs_contrib"] == 0
    got = _grads_gpu(P, gc, gd, views, ws)
    for k in KEYS:
        assert (got[k] == 0).all()


def test_capacity_overflow_is_reported_and_recoverable(P, O):
    case = tiny_case(6, M=60, W=53, H=37, log_scale=-2.0)
    gc, oc = cfg_pair(P, O, eps=0.03, max_instances=8)
    views, ws, gd, _ = _render_gpu(P, gc, case["gauss"], [case])
    torch.cuda.synchronize()
    st = ws.stats()
    assert st["status"] == -3 and st["n_instances"] > 8
    gc2, _ = cfg_pair(P, O, eps=0.03, max_instances=int(st["n_instances"]))
    views2, ws2, _, _ = _render_gpu(P, gc2, case["gauss"], [case])
    torch.cuda.synchronize()
    assert ws2.status() == 0
    r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    assert normwise(h(views2[0].out_rgb).reshape(3, -1), r["rgb"], r["flag"] == 0) < 1e-4


@pytest.mark.parametrize("with_pose", [True, False])
def test_overflowed_backward_changes_nothing(P, O, with_pose):
    """A backward (with Adam in its epilogue) on an overflowed workspace reads no slot: gradients and
    dpose are zero, parameters, moments and the step counter are unchanged."""
    say(f"overflowed backward with Adam: pose {with_pose}")
    case = tiny_case(6, M=60, W=53, H=37, log_scale=-2.0)
    gc, _ = cfg_pair(P, O, eps=0.03, max_instances=8)
    views, ws, gd, _ = _render_gpu(P, gc, case["gauss"], [case])
    opt = P.Adam(gd)
    for k in KEYS:  # non-trivial moments, so an update would move them
        opt.m[k].fill_(0.01)
        opt.v[k].fill_(0.02)
    opt.counter.fill_(5)
    before = {k: (gd[k].clone(), opt.m[k].clone(), opt.v[k].clone()) for k in KEYS}
    grads = {k: torch.full_like(v, 7.0) for k, v in gd.items()}
    dpose = torch.full((1, 6), 7.0, device=DEV) if with_pose else None
    P.render_bwd_adam(gc, gd, views, ws, opt, grads=grads, dpose=dpose)
    torch.cuda.synchronize()
    assert ws.status() == -3
    for k in KEYS:
        assert torch.equal(gd[k], before[k][0]) and torch.equal(opt.m[k], before[k][1]), k
        assert torch.equal(opt.v[k], before[k][2]), k
        assert (grads[k] == 0).all(), k
    if with_pose:
        assert (dpose == 0).all()
    assert int(opt.counter.item()) == 5
    # the plain backward on the overflowed workspace: zero gradients as well
    got = _grads_gpu(P, gc, gd, views, ws)
    for k in KEYS + ("pose",):
        assert (got[k] == 0).all(), k


def test_bad_device_pointer_kind_is_refused(P):
    with pytest.raises(ValueError):
        P.gps._ptr(torch.zeros(4), "cpu tensor")


@pytest.mark.parametrize("M", [3000, 9000])
def test_long_tile_lists(P, O, M):
    """Tiles holding more than 512 (LDS block sort) and more than 8192 (global-memory sort)
    instances composite in the same order as the reference."""
    say(f"long tile lists: M={M}")
    # M > 8192 on a single 16x16 tile puts every instance into that tile's list
    W, H = (32, 24) if M <= 8192 else (16, 16)
    case = tiny_case(40, M=M, W=W, H=H, f=30.0, log_scale=-1.6, invalid_frac=0.0)
    case["base_depth"][:] = 3.0
    gc, oc = cfg_pair(P, O, eps=0.03)
    views, ws, gd, _ = _render_gpu(P, gc, case["gauss"], [case])
    torch.cuda.synchronize()
    st = ws.stats()
    assert st["status"] == 0
    if M > 8192:
        assert st["sort_fallback"] > 0
    r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    keep = r["flag"] == 0
    assert keep.mean() > 0.95
    assert normwise(h(views[0].out_rgb).reshape(3, -1), r["rgb"], keep) < 1e-4
    gC, gD = _explicit_upstream(case, 40, r["flag"])
    got = _grads_gpu(P, gc, gd, views, ws, up=[(gC, gD)])
    ref = O.render_bwd(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    for k in KEYS:
        assert normwise(got[k], ref[k]) < 1e-3, (k, normwise(got[k], ref[k]))


# ------------------------------------------------------------- graph / tuner
@pytest.mark.parametrize("fused_adam", [False, True])
def test_graph_replay_matches_eager(P, O, fused_adam):
    """A captured iteration (forward + backward + Adam) replayed several times, with eager work and
    synchronisation between replays, gives bitwise the eager parameters after every replay, also
    after a new camera pose is uploaded."""
    from paper_2509_11574_amd.graph import IterationGraph
    case = tiny_case(7, M=80, W=53, H=37, log_scale=-2.4)
    gc, _ = cfg_pair(P, O, eps=0.03)
    cam2 = dict(case["cam"])
    cam2["t"] = (case["cam"]["t"] + np.array([0.01, -0.02, 0.015])).astype(np.float32)

    def setup():
        params = gauss_dev(case["gauss"])
        view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]), t(case["target_rgb"]),
                      t(case["target_depth"]))
        view2 = P.View(cam2, view.base_rgb, view.base_depth, view.target_rgb, view.target_depth)
        ws = P.Workspace(gc, 80, [case["cam"]], device=DEV)
        return params, view, view2, ws, P.zeros_like_gaussians(params), P.Adam(params), torch.zeros(1, device=DEV)

    params, view, view2, ws, grads, opt, loss = setup()
    snaps = []
    for i in range(5):
        v = view if i < 3 else view2
        P.render_fwd(gc, params, [v], ws, out_loss=loss)
        P.render_bwd(gc, params, [v], ws, grads)
        opt.step(grads)
        snaps.append({k: h(x) for k, x in params.items()})
    params, view, view2, ws, grads, opt, loss = setup()
    g = IterationGraph(gc, params, [view], ws, grads, opt, loss, fused_adam=fused_adam)
    for i in range(5):
        if i == 3:
            g.set_views([view2])
        g.replay()
        torch.cuda.synchronize()
        _ = torch.randn(4096, device=DEV).sum().item()  # eager work between replays
        assert ws.status() == 0
        for k in KEYS:
            np.testing.assert_array_equal(h(params[k]), snaps[i][k])


def test_autotune_picks_a_compiled_config(P, O, tmp_path, monkeypatch):
    from paper_2509_11574_amd import autotune
    monkeypatch.setenv("GPS_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    case = tiny_case(8, M=80, W=53, H=37)
    gc, _ = cfg_pair(P, O, eps=0.03)
    params = gauss_dev(case["gauss"])
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]), t(case["target_rgb"]),
                  t(case["target_depth"]))
    cfgs = [(16, 16, 256, 1), (8, 8, 128, 1), (16, 16, 256, 4)]
    best, ms = autotune.autotune(gc, params, [view], configs=cfgs, reps=2)
    assert (best.tile_w, best.tile_h, best.batch, best.pix_per_thread) in cfgs and len(ms) == 3
    best2, _ = autotune.autotune(gc, params, [view], configs=cfgs, reps=2)  # from the cache
    assert (best2.tile_w, best2.tile_h, best2.batch, best2.pix_per_thread) == \
        (best.tile_w, best.tile_h, best.batch, best.pix_per_thread)
