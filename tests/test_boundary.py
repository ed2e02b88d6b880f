"""The C-ABI library loads, exports every entry point include/gps.h declares, and
rejects bad arguments synchronously, before touching the device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2509_11574_amd as P
    if not os.path.exists(P.gps.LIB_PATH):
        from paper_2509_11574_amd import build
        build.build()
    P.lib()
    return P


def _declared():
    src = open(os.path.join(ROOT, "include", "gps.h")).read()
    return sorted(set(re.findall(r"\b(gps_[a-z_]+)\s*\(", src)))


def test_header_declares_the_path_calls():
    names = _declared()
    for n in ("gps_fuse", "gps_raycast", "gps_render_fwd", "gps_render_bwd", "gps_adam_step"):
        assert n in names


def test_every_declared_symbol_is_exported(P):
    L = P.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(P.gps.EXPORTS) <= set(_declared())


def test_abi_version_and_status_strings(P):
    L = P.lib()
    assert L.gps_abi_version() == 5
    assert L.gps_status_string(0) == b"ok"
    assert b"capacity" in L.gps_status_string(-3)


def test_level_camera_matches_the_reference(P):
    """gps_level_camera (a host call) against the reference tracker's own level intrinsics."""
    from oracle import icp as OI
    cam = {"width": 1280, "height": 720, "fx": 1200.0, "fy": 1190.0, "cx": 639.7, "cy": 360.2,
           "R": np.eye(3), "t": np.zeros(3)}
    for lvl in range(4):
        got, ref = P.gps.level_camera(cam, lvl), OI.level_camera(cam, lvl)
        assert (got["width"], got["height"]) == (ref["width"], ref["height"])
        for k in ("fx", "fy", "cx", "cy"):
            assert got[k] == np.float32(ref[k]), (lvl, k)
    with pytest.raises(P.GpsError):
        P.gps.level_camera(cam, 17)
    with pytest.raises(P.GpsError):
        P.gps.level_camera({**cam, "width": 3, "height": 3}, 2)


def test_default_cfg(P):
    c = P.gps.RenderCfgS()
    P.lib().gps_render_cfg_default(ctypes.byref(c))
    assert (c.tile_w, c.tile_h, c.batch, c.pix_per_thread, c.mode) == (16, 16, 256, 1, 0)
    assert c.alpha_min == pytest.approx(1 / 255) and c.dilation == pytest.approx(0.3)


def _cam(W=64, H=48):
    return {"width": W, "height": H, "fx": 50.0, "fy": 50.0, "cx": W / 2, "cy": H / 2, "R": np.eye(3), "t": np.zeros(3)}


def test_workspace_size_grows_with_work(P):
    cfg = P.RenderCfg()
    a = P.workspace_size(cfg, 1000, [_cam()])
    b = P.workspace_size(cfg, 100000, [_cam()])
    c = P.workspace_size(cfg, 1000, [_cam(), _cam(320, 240)])
    assert 0 < a < b and a < c


@pytest.mark.parametrize("field,value", [("tile_w", 12), ("batch", 100), ("pix_per_thread", 3)])
def test_unsupported_tile_config(P, field, value):
    cfg = P.RenderCfg()
    setattr(cfg, field, value)
    with pytest.raises(P.GpsError) as e:
        P.workspace_size(cfg, 1000, [_cam()])
    assert e.value.status == -6


@pytest.mark.parametrize("field,value", [("mode", 2), ("alpha_min", 0.0), ("alpha_max", 1.0), ("z_near", 0.0),
                                         ("eps_cull", float("nan")), ("max_instances", -5)])
def test_invalid_cfg(P, field, value):
    cfg = P.RenderCfg()
    setattr(cfg, field, value)
    with pytest.raises(P.GpsError) as e:
        P.workspace_size(cfg, 1000, [_cam()])
    assert e.value.status == -1


def test_invalid_cameras_and_counts(P):
    cfg = P.RenderCfg()
    for bad in (_cam(0, 10), {**_cam(), "fx": 0.0}, {**_cam(), "cx": float("inf")}):
        with pytest.raises(P.GpsError):
            P.workspace_size(cfg, 10, [bad])
    with pytest.raises(P.GpsError):
        P.workspace_size(cfg, -1, [_cam()])
    with pytest.raises(ValueError):
        P.gps._views_array([])


def test_null_pointers_rejected_before_launch(P):
    L = P.lib()
    cam = P.camera(_cam())
    vol = P.gps.VolumeS()
    vol.nx = vol.ny = vol.nz = 8
    vol.voxel, vol.trunc, vol.max_weight = 0.1, 0.4, 100.0
    assert L.gps_fuse(ctypes.byref(vol), ctypes.byref(cam), None, None, None) == -1
    assert L.gps_raycast(ctypes.byref(vol), ctypes.byref(cam), 1, None, None, 0.2, 0.0, None) == -1
    cfg = P.RenderCfg().struct()
    g = P.gps.GaussiansS()
    g.count = 10  # non-zero count with null arrays
    v = (P.gps.ViewS * 1)()
    assert L.gps_render_fwd(ctypes.byref(cfg), ctypes.byref(g), v, 1, None, 0, None, None) == -1
    assert L.gps_render_bwd(ctypes.byref(cfg), ctypes.byref(g), v, 1, None, None, None, None, None, None, 0,
                            None) == -1
    grp = (P.gps.AdamGroupS * 1)()
    grp[0].n = 5
    assert L.gps_adam_step(grp, 1, 1, None, 0.9, 0.999, 1e-15, None) == -1
    assert L.gps_adam_step(grp, 0, 1, None, 0.9, 0.999, 1e-15, None) == -1
    assert L.gps_adam_step(grp, 9, 1, None, 0.9, 0.999, 1e-15, None) == -1
    # eps must be positive and finite, as for the backward with Adam in its epilogue
    # (with eps = 0 an element whose gradients were all zero would become 0/0)
    empty = (P.gps.AdamGroupS * 1)()
    empty[0].n = 0
    for bad_eps in (0.0, -1e-8, float("nan"), float("inf")):
        assert L.gps_adam_step(empty, 1, 1, None, 0.9, 0.999, bad_eps, None) == -1
    st = ctypes.c_int32(0)
    assert L.gps_device_status(None, 0, ctypes.byref(st), None) == -1


def test_oracle_and_product_are_independent():
    """The product package never imports the reference implementation, and vice versa."""
    pkg = os.path.join(ROOT, "paper_2509_11574_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).lower() or f == "__init__.py", f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2509_11574_amd" not in txt and "gps.h" not in txt, f


def test_removal_defaults_and_argument_checks(P):
    """Gaussian removal (Eq. 8): the default thresholds are the paper's; bad
    arguments are refused before anything is launched."""
    L = P.lib()
    c = P.gps.RemovalCfgS()
    L.gps_removal_cfg_default(ctypes.byref(c))
    assert (c.min_opacity, c.max_scale, c.min_scale) == pytest.approx((0.005, 0.1, 0.003))
    n = ctypes.c_size_t(0)
    assert L.gps_removal_workspace_size(1000, ctypes.byref(n)) == 0 and n.value >= 2 * 4 * 4
    assert L.gps_removal_workspace_size(-1, ctypes.byref(n)) == -1
    sets = (P.gps.GaussiansS * 1)()
    outs = (P.gps.GaussiansS * 1)()
    assert L.gps_remove_gaussians(ctypes.byref(c), sets, outs, 0, None, None, 0, None) == -1   # no set
    assert L.gps_remove_gaussians(ctypes.byref(c), sets, outs, 5, None, None, 0, None) == -1   # too many sets
    bad = P.gps.RemovalCfgS(0.005, 0.001, 0.003)                                             # min > max scale
    assert L.gps_remove_gaussians(ctypes.byref(bad), sets, outs, 1, None, None, 0, None) == -1
    sets[0].count = 10                                                                        # null arrays
    assert L.gps_remove_gaussians(ctypes.byref(c), sets, outs, 1, None, None, 0, None) == -1


def test_insertion_defaults_and_argument_checks(P):
    """Gaussian insertion (Eq. 6, App. A): the defaults are the paper's constants;
    bad arguments are refused before anything is launched."""
    L = P.lib()
    c = P.gps.InsertCfgS()
    L.gps_insert_cfg_default(ctypes.byref(c))
    assert (c.delta_c, c.delta_w, c.fraction, c.scale_cap, c.flat_ratio, c.opacity) == pytest.approx(
        (0.05, 4.0, 0.25, 0.1, 0.1, 0.5))
    n = ctypes.c_size_t(0)
    assert L.gps_insertion_workspace_size(64, 48, ctypes.byref(n)) == 0 and n.value >= 4 * 64 * 48
    assert L.gps_insertion_workspace_size(0, 48, ctypes.byref(n)) == -1
    assert L.gps_insertion_workspace_size(1 << 16, 1 << 16, ctypes.byref(n)) == -1    # beyond 2^30 pixels
    cam = P.camera(_cam())
    g = P.gps.GaussiansS()
    buf = (ctypes.c_float * 4)()
    img = ctypes.cast(buf, ctypes.c_void_p)
    cnt = ctypes.c_int32(0)

    def call(cfg, g=g, ws_bytes=1 << 20):
        return L.gps_insert_gaussians(ctypes.byref(cfg), ctypes.byref(cam), img, img, img, img, img, ctypes.byref(g),
                                      None, ctypes.byref(cnt), None, ws_bytes, None)
    assert call(c) == -1                                                   # no workspace
    for field, value in (("fraction", 1.5), ("opacity", 1.0), ("scale_cap", 0.0), ("flat_ratio", 1.5),
                         ("delta_w", 0.0), ("delta_c", float("nan"))):
        bad = P.gps.InsertCfgS.from_buffer_copy(c)
        setattr(bad, field, value)
        assert call(bad) == -1, field
    g.count = 10                                                           # capacity without arrays
    assert call(c) == -1
    assert L.gps_insert_gaussians(ctypes.byref(c), ctypes.byref(cam), None, img, img, img, img, ctypes.byref(g),
                                  None, ctypes.byref(cnt), None, 0, None) == -1


def test_icp_argument_checks(P):
    """Camera tracking (Eq. 5): bad arguments are refused before anything is launched."""
    L = P.lib()
    n = ctypes.c_size_t(0)
    assert L.gps_icp_workspace_size(160, 120, ctypes.byref(n)) == 0 and n.value >= 29 * 4 * 75
    assert L.gps_icp_workspace_size(0, 120, ctypes.byref(n)) == -1
    buf = (ctypes.c_float * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.gps_depth_downsample(p, 1, 4, p, None) == -1              # width below 2
    assert L.gps_depth_downsample(None, 4, 4, p, None) == -1
    cam = P.camera(_cam())
    sysb = (ctypes.c_double * 29)()
    sp = ctypes.cast(sysb, ctypes.c_void_p)
    assert L.gps_icp_reduce(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.1, sp, None, 1 << 20, None) == -1
    assert L.gps_icp_reduce(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.0, sp, p, 1 << 20, None) == -1
    assert L.gps_icp_reduce(ctypes.byref(cam), None, ctypes.byref(cam), p, p, 0.1, sp, p, 1 << 20, None) == -1
    bad = P.camera({**_cam(), "fx": 0.0})
    assert L.gps_icp_reduce(ctypes.byref(cam), p, ctypes.byref(bad), p, p, 0.1, sp, p, 1 << 20, None) == -1
    assert L.gps_icp_solve(None, p, None, None) == -1 and L.gps_icp_solve(sp, None, None, None) == -1
    # the fused step: the reduce's checks (pose, depth, threshold, workspace)
    assert L.gps_icp_step(ctypes.byref(cam), p, ctypes.byref(cam), p, None, 0.1, sp, None, sp, 1 << 20, None) == -1
    assert L.gps_icp_step(ctypes.byref(cam), None, ctypes.byref(cam), p, p, 0.1, sp, None, sp, 1 << 20, None) == -1
    assert L.gps_icp_step(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.0, sp, None, sp, 1 << 20, None) == -1
    assert L.gps_icp_step(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.1, sp, None, None, 1 << 20, None) == -1
    # the variant without a workspace checks the same arguments
    assert L.gps_icp_reduce_noalloc(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.0, sp, None) == -1
    assert L.gps_icp_reduce_noalloc(ctypes.byref(cam), None, ctypes.byref(cam), p, p, 0.1, sp, None) == -1
    assert L.gps_icp_reduce_noalloc(ctypes.byref(cam), p, ctypes.byref(bad), p, p, 0.1, sp, None) == -1
    assert L.gps_icp_reduce_noalloc(ctypes.byref(cam), p, ctypes.byref(cam), p, p, 0.1, None, None) == -1


def test_fused_adam_argument_checks(P):
    """The backward with Adam in its epilogue refuses a missing Adam block, moments of the
    wrong count, non-finite learning rates and betas outside [0, 1) before any launch
    (status -1).  Every call here fails its argument checks, so nothing reaches a device."""
    L = P.lib()
    rc = P.RenderCfg()
    cfg = rc.struct()
    g = P.gps.GaussiansS()
    v = (P.gps.ViewS * 1)()
    v[0].cam = P.camera(_cam())
    img = ctypes.cast((ctypes.c_float * (4 * 64 * 48))(), ctypes.c_void_p)   # host stand-ins: never read
    for f in ("base_rgb", "base_depth", "target_rgb", "target_depth", "out_rgb", "out_depth"):
        setattr(v[0], f, img)
    nbytes = P.workspace_size(rc, 0, [_cam()])
    raw = (ctypes.c_uint8 * (nbytes + 256))()
    wsp = ctypes.c_void_p((ctypes.addressof(raw) + 255) & ~255)

    def call(af):
        return L.gps_render_bwd_adam(ctypes.byref(cfg), ctypes.byref(g), v, 1, None, None, None, None, None,
                                     ctypes.byref(af) if af is not None else None, wsp, nbytes, None)
    assert call(None) == -1
    good = P.gps.AdamFusedS()
    good.lr_mean = good.lr_log_scale = good.lr_quat = good.lr_opacity = good.lr_rgb = 1e-3
    good.beta1, good.beta2, good.eps, good.step = 0.9, 0.999, 1e-15, 1
    for field, value in (("lr_quat", float("nan")), ("beta1", 1.0), ("beta2", -0.1), ("eps", 0.0), ("step", 0)):
        bad = P.gps.AdamFusedS.from_buffer_copy(good)
        setattr(bad, field, value)
        assert call(bad) == -1, field
    bad = P.gps.AdamFusedS.from_buffer_copy(good)
    bad.m.count = 5                                        # moments of another size
    assert call(bad) == -1


def test_hash_argument_checks(P):
    """Voxel-block hash (Sec. 3.2.1): bad volumes and arguments are refused before any launch."""
    L = P.lib()
    from paper_2509_11574_amd.gps import HashVolumeS
    buf = (ctypes.c_float * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)

    def vol(**kw):
        s = HashVolumeS()
        s.nx = s.ny = s.nz = 64
        s.voxel, s.trunc, s.max_weight = 0.02, 0.08, 100.0
        s.n_buckets, s.capacity = 1024, 256
        for name in ("keys", "slots", "block_key", "state", "visible", "block_min", "tsdf", "weight", "rgb",
                     "rgb_weight"):
            setattr(s, name, p)
        for k, v in kw.items():
            setattr(s, k, v)
        return s

    cam = P.camera(_cam())
    cams = (P.gps.Camera * 1)(cam)
    ptrs = (ctypes.c_void_p * 1)(p.value)
    for bad in (dict(n_buckets=1000), dict(n_buckets=1), dict(capacity=0), dict(voxel=0.0), dict(trunc=-1.0),
                dict(nx=1), dict(keys=None), dict(tsdf=None), dict(state=None), dict(max_weight=0.5)):
        v = vol(**bad)
        assert L.gps_hash_reset(ctypes.byref(v), None) == -1, bad
        assert L.gps_hash_fuse(ctypes.byref(v), ctypes.byref(cam), p, p, None) == -1, bad
        assert L.gps_hash_raycast(ctypes.byref(v), cams, 1, ptrs, ptrs, 0.2, 0.0, None, 0, None) == -1, bad
    v = vol()
    assert L.gps_hash_fuse(ctypes.byref(v), ctypes.byref(cam), None, p, None) == -1
    assert L.gps_hash_fuse(ctypes.byref(v), None, p, p, None) == -1
    assert L.gps_hash_raycast(ctypes.byref(v), cams, 0, ptrs, ptrs, 0.2, 0.0, None, 0, None) == -1
    assert L.gps_hash_raycast(ctypes.byref(v), cams, 1, ptrs, ptrs, -0.1, 0.0, None, 0, None) == -1
    assert L.gps_hash_raycast(ctypes.byref(v), cams, 1, None, ptrs, 0.2, 0.0, None, 0, None) == -1
    # a depth-range scratch shorter than 2 floats per 16x16 tile of the views
    need = 2 * ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    assert L.gps_hash_raycast(ctypes.byref(v), cams, 1, ptrs, ptrs, 0.2, 0.0, p, need - 1, None) == -1
