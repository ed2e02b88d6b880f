"""One keyframe of map maintenance (Sec. 3.2.2) on top of the C ABI: the map's
Gaussians with their Adam state, insertion of new Gaussians where the sort-free
render of Eq. 1-4 leaves a high colour error and a low Gaussian weight (Eq. 6,
App. A), and removal (Eq. 8).  The arithmetic is in libgps.so (render, insertion,
removal kernels); this module only concatenates and swaps device tensors."""
from __future__ import annotations

from dataclasses import replace

import torch

from . import gps


class GaussianMap:
    """Planar device tensors of the map's Gaussians (and SH bands, if any) and an Adam state
    over them.  New Gaussians start with zero moments; the step counter is shared."""

    def __init__(self, params: dict, opt: gps.Adam | None = None):
        self.params = {k: v.contiguous() for k, v in params.items()}
        self.opt = opt if opt is not None else gps.Adam(self.params)
        self.opt.params = self.params

    @property
    def count(self) -> int:
        return int(self.params["opacity_logit"].numel())

    def _set(self, params: dict, m: dict, v: dict):
        for k in gps.gauss_keys(self.params):
            self.params[k] = params[k].contiguous()
            self.opt.m[k] = m[k].contiguous()
            self.opt.v[k] = v[k].contiguous()

    def append(self, new: dict) -> int:
        """Appends the Gaussians of `new` (planar tensors, the Gaussians along the last axis)
        after the existing ones; the SH bands of new Gaussians start at zero when `new` has
        none."""
        n = int(new["opacity_logit"].numel())
        if n == 0:
            return 0
        p, m, v = {}, {}, {}
        for k in gps.gauss_keys(self.params):
            old = self.params[k]
            add = new.get(k)
            if add is None:
                add = torch.zeros(*old.shape[:-1], n, dtype=old.dtype, device=old.device)
            add = add.to(torch.float32).reshape(*old.shape[:-1], n)
            p[k] = torch.cat([old, add], dim=-1)
            z = torch.zeros_like(add)
            m[k] = torch.cat([self.opt.m[k], z], dim=-1)
            v[k] = torch.cat([self.opt.v[k], z], dim=-1)
        self._set(p, m, v)
        return n

    def prune(self, min_opacity=0.005, max_scale=0.1, min_scale=0.003) -> int:
        """Removal of Eq. 8 with both Adam moments as companion sets; returns the kept count."""
        kept, (m, v), n = gps.remove_gaussians(self.params, [self.opt.m, self.opt.v], min_opacity, max_scale,
                                               min_scale)
        self._set(kept, m, v)
        return n


def insert_from_render(gmap: GaussianMap, cfg: gps.RenderCfg, view: gps.View, rand: torch.Tensor,
                       ws: gps.Workspace | None = None, capacity=None):
    """Renders `view` with the sort-free blend (mode 1) over its SDF image, taking C* and
    the Gaussian weight W_G (Eq. 2), inserts new Gaussians where Eq. 6 holds, and
    appends them to the map.  Returns (new Gaussians, their pixels, n_taken)."""
    cfg1 = replace(cfg, mode=1, views_preset=False)
    c = gps.camera(view.cam)
    dev = view.base_depth.device
    if view.out_aux is None:
        view.out_aux = torch.empty(c.height, c.width, dtype=torch.float32, device=dev)
    if ws is None:
        ws = gps.Workspace(cfg1, max(gmap.count, 1), [view.cam], device=dev)
    gps.render_fwd(cfg1, gmap.params, [view], ws)
    new, pix, n_taken = gps.insert_gaussians(view.cam, view.out_rgb, view.target_rgb, view.out_aux,
                                             view.base_depth, rand, capacity=capacity,
                                             sh_degree=gps.sh_degree(gmap.params))
    gmap.append(new)
    return new, pix, n_taken
