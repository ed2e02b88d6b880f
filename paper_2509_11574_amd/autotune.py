"""Autotuner for the compositing kernels: screen tile (8x8, 16x16, 16x32, 32x16) x
Gaussians staged per LDS batch (128, 256, 512) x pixels per lane (1, 2, 4).

Every combination compiled into libgps is timed on the caller's real workload
(render forward + backward on the given views), with HIP events on the current
stream; the fastest is returned and cached per (device architecture, view
sizes, Gaussian count bucket, mode).  All combinations compute the same
function; they differ only in summation order and speed.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import replace

import torch

from . import gps as G

_CACHE_ENV = "GPS_AUTOTUNE_CACHE"


def _cache_path():
    p = os.environ.get(_CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gps_mi355x", "autotune.json")


def shape_key(views, n_gaussians: int, mode: int) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    sizes = "+".join(f"{G.camera(v.cam).width}x{G.camera(v.cam).height}" for v in views)
    mb = 2 ** max(0, round(math.log2(max(1, n_gaussians))))
    return f"{arch}|{sizes}|M~{mb}|mode{mode}"


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def time_config(cfg: G.RenderCfg, params: dict, views, reps: int = 5, warmup: int = 2) -> float:
    """Median ms of one render forward + backward (fused loss) with this configuration."""
    M = int(params["opacity_logit"].numel())
    dev = params["mean"].device
    ws = G.Workspace(cfg, M, [v.cam for v in views], device=dev)
    grads = G.zeros_like_gaussians(params)
    loss = torch.zeros(1, device=dev)
    for _ in range(warmup):
        G.render_fwd(cfg, params, views, ws, out_loss=loss)
        G.render_bwd(cfg, params, views, ws, grads)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        G.render_fwd(cfg, params, views, ws, out_loss=loss)
        G.render_bwd(cfg, params, views, ws, grads)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    if ws.status() != 0:
        return float("inf")
    times.sort()
    return times[len(times) // 2]


def autotune(cfg: G.RenderCfg, params: dict, views, configs=None, reps: int = 5, use_cache: bool = True):
    """Returns (best RenderCfg, {"16x16x256x1": ms, ...}).  The views must carry targets."""
    M = int(params["opacity_logit"].numel())
    key = shape_key(views, M, cfg.mode)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        tw, th, b, ppt = db[key]["best"]
        return replace(cfg, tile_w=tw, tile_h=th, batch=b, pix_per_thread=ppt), db[key]["ms"]
    configs = configs or G.TILE_CONFIGS
    timings = {}
    for (tw, th, b, ppt) in configs:
        c = replace(cfg, tile_w=tw, tile_h=th, batch=b, pix_per_thread=ppt, views_preset=False)
        timings[f"{tw}x{th}x{b}x{ppt}"] = round(time_config(c, params, views, reps=reps), 4)
    best = min(timings, key=timings.get)
    tw, th, b, ppt = (int(x) for x in best.split("x"))
    if use_cache:
        db[key] = {"best": [tw, th, b, ppt], "ms": timings}
        _store(db)
    return replace(cfg, tile_w=tw, tile_h=th, batch=b, pix_per_thread=ppt), timings
