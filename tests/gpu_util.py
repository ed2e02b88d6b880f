"""Helpers shared by the GPU parity tests (input marshalling and comparisons only)."""
from __future__ import annotations

import sys

import numpy as np
import torch

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(DEV)


def h(x):
    return x.detach().float().cpu().numpy()


def normwise(a, b, mask=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def cfg_pair(P, O, mode=0, eps=0.02, tile=(16, 16, 256, 1), **kw):
    gpu_only = {k: kw.pop(k) for k in ("max_instances", "no_sort", "bwd_per_gaussian", "views_preset") if k in kw}
    gc = P.RenderCfg(tile_w=tile[0], tile_h=tile[1], batch=tile[2], pix_per_thread=tile[3], mode=mode,
                     eps_cull=eps, **kw, **gpu_only)
    oc = O.RenderCfg(mode=mode, eps_cull=eps, **kw)
    return gc, oc


def gauss_dev(g):
    return {k: t(v) for k, v in g.items()}


def report_flags(tag, keep, got, want, tol=1e-3):
    """Prints how many pixels the reference flagged (a 1/255, cap or transmittance decision
    within rounding reach) and, of those, how many the GPU decided the other way (its value
    differs from the reference's beyond tol): the flip count of the comparison."""
    got = np.asarray(got, np.float64).reshape(-1, keep.size)
    want = np.asarray(want, np.float64).reshape(-1, keep.size)
    differ = np.abs(got - want).max(axis=0) > tol * max(1.0, float(np.abs(want).max()))
    flips = int((differ & ~keep).sum())
    say(f"  {tag}: {int((~keep).sum())} of {keep.size} pixels flagged, {flips} flipped")
    return flips
