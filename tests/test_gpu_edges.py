"""GPU parity on inputs that reach the renderer's edge cases.

* Opacity cap: opacity logits of 8 to 12 (sigma > 0.9996) on wide Gaussians, so that
  alpha = sigma exp(-q/2) exceeds alpha_max = 0.99 near their centres: the forward
  (alpha capped, sorted mode) and the backward (no alpha gradient through a capped
  value) against the reference.
* Tile lists at the boundaries of the per-tile sort: one screen tile holding exactly
  509 to 513 instances (the register sort of one wavefront takes lists below 511 keys,
  the block sort the others) and 8,192 / 8,193 instances (the LDS sort's capacity and
  the global-memory sort above it), forward and backward, at the default tile and at
  the benchmarked 16x32 tile.
"""
import numpy as np
import pytest
import torch

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


def _run(P, gc, case, gC, gD):
    W, H = case["cam"]["width"], case["cam"]["height"]
    view = P.View(case["cam"], t(case["base_rgb"]), t(case["base_depth"]))
    M = case["gauss"]["opacity_logit"].size
    ws = P.Workspace(gc, M, [view.cam], device=DEV)
    gd = {k: t(v) for k, v in case["gauss"].items()}
    P.render_fwd(gc, gd, [view], ws)
    grads = P.zeros_like_gaussians(gd)
    dpose = torch.zeros(1, 6, device=DEV)
    P.render_bwd(gc, gd, [view], ws, grads, dpose, dL_drgb=[t(gC).reshape(3, H, W)], dL_ddepth=[t(gD).reshape(H, W)])
    torch.cuda.synchronize()
    st = ws.stats()
    assert st["status"] == 0
    out = {k: h(v) for k, v in grads.items()}
    out["pose"] = h(dpose)[0]
    return h(view.out_rgb).reshape(3, -1), h(view.out_depth).reshape(-1), out, st


def _check(O, oc, case, C, D, got, gC, gD):
    r = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    keep = r["flag"] == 0
    assert keep.mean() > 0.85
    assert normwise(C, r["rgb"], keep) < 1e-4
    assert normwise(D, r["depth"], keep) < 1e-4
    # the adjoints given are already zero where the reference flags a decision near a threshold
    ref = O.render_bwd(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    return r, keep, ref


@pytest.mark.parametrize("tile", [(16, 16, 256, 1), (16, 32, 256, 2)])
def test_opacity_cap_reached(P, O, tile):
    say(f"opacity cap reached: tile {tile}")
    case = tiny_case(31, M=60, W=53, H=37, log_scale=-1.6)
    rng = np.random.default_rng(31)
    case["gauss"]["opacity_logit"] = rng.uniform(8.0, 12.0, 60).astype(np.float32)
    case["base_depth"][:] = 3.0
    gc, oc = cfg_pair(P, O, eps=0.03, tile=tile)
    W, H = 53, 37
    gC = rng.normal(size=(3, W * H))
    gD = rng.normal(size=W * H)
    # the reference decides which pixels are near a threshold; their adjoints are set to zero
    r0 = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    keep0 = r0["flag"] == 0
    gC, gD = gC * keep0, gD * keep0
    C, D, got, _ = _run(P, gc, case, gC, gD)
    r, keep, ref = _check(O, oc, case, C, D, got, gC, gD)
    for k in KEYS:
        assert normwise(got[k], ref[k]) < 1e-3, (k, normwise(got[k], ref[k]))
    assert normwise(got["pose"], ref["pose"]) < 1e-3
    # the cap is active: without it (alpha_max just below 1) the reference image differs
    oc_nocap = O.RenderCfg(mode=0, eps_cull=0.03, alpha_max=1.0 - 1e-7)
    r_nocap = O.render(oc_nocap, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    changed = np.abs(r_nocap["rgb"] - r["rgb"]).max(axis=0) > 1e-6
    assert changed.sum() >= 20, changed.sum()


@pytest.mark.parametrize("tile", [(16, 16, 256, 1), (16, 32, 256, 2)])
@pytest.mark.parametrize("n_keys", [509, 510, 511, 512, 513, 8192, 8193])
def test_tile_list_length_boundaries(P, O, tile, n_keys):
    """A frame of exactly one screen tile: every Gaussian overlaps it, so the tile's list
    holds exactly n_keys instances (no depth cull: the base is far behind)."""
    say(f"tile list of {n_keys} keys: tile {tile}")
    W, H = tile[0], tile[1]
    case = tiny_case(40 + n_keys % 7, M=n_keys, W=W, H=H, f=30.0, log_scale=-1.2, invalid_frac=0.0)
    rng = np.random.default_rng(n_keys)
    # low opacities (sigma about 0.011) so that long lists are composited, and no transmittance
    # stop, so that every list runs to its end
    case["gauss"]["opacity_logit"] = rng.normal(-4.5, 0.2, n_keys).astype(np.float32)
    case["base_depth"][:] = 3.0
    gc, oc = cfg_pair(P, O, eps=0.03, tile=tile, T_min=0.0)
    r0 = O.render(oc, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    gC = rng.normal(size=(3, W * H)) * (r0["flag"] == 0)
    gD = rng.normal(size=W * H) * (r0["flag"] == 0)
    C, D, got, st = _run(P, gc, case, gC, gD)
    assert st["n_instances"] == n_keys and st["n_tiles"] == 1
    assert (st["sort_fallback"] > 0) == (n_keys > 8192)
    r, keep, ref = _check(O, oc, case, C, D, got, gC, gD)
    assert r["n"][keep].mean() > 0.2 * n_keys  # long per-pixel lists: the order matters
    for k in KEYS:
        assert normwise(got[k], ref[k]) < 1e-3, (k, normwise(got[k], ref[k]))
