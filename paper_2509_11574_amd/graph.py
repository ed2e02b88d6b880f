"""One optimisation iteration -- render forward with the fused loss, backward and
Adam (a separate launch, or in the backward's epilogue with fused_adam) --
captured once as a HIP graph (torch.cuda.CUDAGraph on ROCm) and replayed.

The captured kernels read the view table (cameras and image pointers) from the
workspace, so new camera poses, base images or target images are taken by
uploading a table (`set_views`, outside the graph; it also takes the per-tile
maxima of the base depths) before replaying; views must keep their sizes.  The Adam step counter lives on the device.  Nothing in the captured
sequence allocates memory or reads device data on the host.
"""
from __future__ import annotations

from dataclasses import replace

import torch

from . import gps as G


class IterationGraph:
    def __init__(self, cfg: G.RenderCfg, params: dict, views, ws: G.Workspace, grads: dict, opt: G.Adam,
                 loss: torch.Tensor, dpose: torch.Tensor | None = None, fused_adam: bool = False):
        if opt.counter is None:
            raise ValueError("graph replay needs Adam with a device step counter")
        self.cfg_upload = replace(cfg, views_preset=False)
        self.cfg = replace(cfg, views_preset=True)
        self.params, self.ws, self.grads, self.opt, self.loss, self.dpose = params, ws, grads, opt, loss, dpose
        self.fused_adam = fused_adam
        self.views = list(views)
        self.set_views(self.views)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._iteration()

    def _iteration(self):
        G.render_fwd(self.cfg, self.params, self.views, self.ws, out_loss=self.loss)
        if self.fused_adam:  # Adam in the epilogue of the backward (gps_render_bwd_adam)
            G.render_bwd_adam(self.cfg, self.params, self.views, self.ws, self.opt, grads=self.grads,
                              dpose=self.dpose)
        else:
            G.render_bwd(self.cfg, self.params, self.views, self.ws, self.grads, self.dpose)
            self.opt.step(self.grads)

    def set_views(self, views):
        """Upload the table of `views` (same sizes as at capture) for the next replays."""
        G.views_upload(self.cfg_upload, self.params, list(views), self.ws)

    def replay(self):
        self.graph.replay()
