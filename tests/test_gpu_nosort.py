"""GPU parity of the sort-free blend without any depth sort (GPS_RENDER_NO_SORT; Sec. 3.1,
Eq. 1, 2, 4: the blend does not depend on the order of the Gaussians).

The lists are composited in the order the binning emitted them and every record of a
list is visited.  Checked against the reference's sort-free render and gradients (the
same tolerances as the sorted lists), against the sorted-list sort-free render of the
same call (equal up to the rounding of the sums' order), on tile lists long enough to
need the block sort in sorted mode (which this mode never launches), with the
per-Gaussian backward of Appendix B, over repeated calls (equal up to rounding), and
refused in the sorted over-compositing mode.
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import DEV, cfg_pair, gauss_dev, h, normwise, say, t
from tests.tiny_cases import tiny_case

pytestmark = pytest.mark.gpu
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
TILES = [(16, 16, 256, 1), (8, 8, 128, 1), (16, 32, 256, 2), (16, 16, 512, 4), (32, 16, 128, 2)]


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


def _run(P, gc, g, case, up):
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]))
    M = int(np.asarray(g["opacity_logit"]).size)
    ws = P.Workspace(gc, M, [case["cam"]], device=DEV)
    gd = gauss_dev(g)
    P.render_fwd(gc, gd, [view], ws)
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(1, 6, device=DEV)
    H, W = case["base_depth"].shape
    P.render_bwd(gc, gd, [view], ws, grads, dpose, dL_drgb=[t(up[0]).reshape(3, H, W)],
                 dL_ddepth=[t(up[1]).reshape(H, W)])
    torch.cuda.synchronize()
    assert ws.status() == 0
    out = {k: h(v) for k, v in grads.items()}
    out["pose"] = h(dpose)[0]
    return h(view.out_rgb).reshape(3, -1), h(view.out_depth).reshape(-1), out, ws.stats()


def _upstream(case, seed, flags):
    rng = np.random.Generator(np.random.PCG64(700 + seed))
    H, W = case["base_depth"].shape
    gC = rng.normal(size=(3, H * W)).astype(np.float32)
    gD = rng.normal(size=H * W).astype(np.float32)
    gC[:, flags != 0] = 0
    gD[flags != 0] = 0
    return gC, gD


def _check(P, O, case, tile, per_gaussian=False, seed=0):
    g = case["gauss"]
    gc, oc = cfg_pair(P, O, mode=1, eps=0.03, tile=tile, no_sort=True, bwd_per_gaussian=per_gaussian)
    r = O.render(oc, g, case["cam"], case["base_rgb"], case["base_depth"])
    keep = r["flag"] == 0
    up = _upstream(case, seed, r["flag"])
    C, D, got, st = _run(P, gc, g, case, up)
    assert normwise(C, r["rgb"], keep) < 1e-4 and normwise(D, r["depth"], keep) < 1e-4
    ref = O.render_bwd(oc, g, case["cam"], case["base_rgb"], case["base_depth"], *up)
    for k in KEYS:
        assert normwise(got[k], ref[k]) < 1e-3, (k, normwise(got[k], ref[k]))
    assert normwise(got["pose"], ref["pose"]) < 1e-3
    # the sorted-list sort-free render of the same input: the same sums in another order
    gs, _ = cfg_pair(P, O, mode=1, eps=0.03, tile=tile, bwd_per_gaussian=per_gaussian)
    C2, D2, got2, _ = _run(P, gs, g, case, up)
    assert np.abs(C - C2).max() <= 1e-5 * max(1.0, np.abs(C2).max())
    assert np.abs(D - D2).max() <= 1e-5 * max(1.0, np.abs(D2).max())
    for k in KEYS:
        assert normwise(got[k], got2[k]) < 1e-4, k
    return st


@pytest.mark.parametrize("tile", TILES)
def test_nosort_parity_tiny(P, O, tile):
    say(f"sort-free without sort: tiny cases, tile {tile}")
    for seed in (0, 1, 2):
        _check(P, O, tiny_case(seed, M=60, W=53, H=37, log_scale=-2.4), tile, seed=seed)


def test_nosort_parity_small_scene_and_repeats(P, O):
    say("sort-free without sort: 160x120 scene, 2000 Gaussians, repeated calls")
    w = synth.workload_small()
    grid = None
    from oracle import oracle as Om
    sc, cam = w["scene"], w["cam"].as_dict()
    grid = Om.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    ref = Om.fuse(grid, Om.new_volume(grid), cam, w["depth"], w["rgb"])
    rd, rc, _ = Om.raycast(grid, ref["tsdf"].astype(np.float32), ref["rgb"].astype(np.float32), cam)
    case = {"cam": cam, "gauss": w["gauss"], "base_rgb": rc.reshape(3, 120, 160).astype(np.float32),
            "base_depth": rd.reshape(120, 160).astype(np.float32)}
    _check(P, O, case, (16, 16, 256, 1))
    gc, oc = cfg_pair(P, O, mode=1, eps=0.03, no_sort=True)
    r = O.render(oc, case["gauss"], cam, case["base_rgb"], case["base_depth"])
    up = _upstream(case, 5, r["flag"])
    runs = [_run(P, gc, case["gauss"], case, up) for _ in range(3)]
    for C, D, got, _ in runs[1:]:
        assert np.abs(C - runs[0][0]).max() <= 1e-5 and np.abs(D - runs[0][1]).max() <= 1e-5
        for k in KEYS:
            assert normwise(got[k], runs[0][2][k]) < 1e-4


@pytest.mark.parametrize("M", [3000, 9000])
def test_nosort_long_lists(P, O, M):
    say(f"sort-free without sort: long tile lists, M={M}")
    W, H = (32, 24) if M <= 8192 else (16, 16)
    case = tiny_case(40, M=M, W=W, H=H, f=30.0, log_scale=-1.6, invalid_frac=0.0)
    case["base_depth"][:] = 3.0
    st = _check(P, O, case, (16, 16, 256, 1))
    assert st["sort_fallback"] == 0  # no sort of any kind ran


def test_nosort_with_the_per_gaussian_backward(P, O):
    say("sort-free without sort: per-Gaussian backward (App. B)")
    _check(P, O, tiny_case(3, M=60, W=53, H=37, log_scale=-2.4), (16, 16, 256, 1), per_gaussian=True)


def test_nosort_refused_in_sorted_mode(P, O):
    gc, _ = cfg_pair(P, O, mode=0, eps=0.03, no_sort=True)
    case = tiny_case(0, M=10)
    with pytest.raises(P.GpsError):
        P.Workspace(gc, 10, [case["cam"]], device=DEV)
