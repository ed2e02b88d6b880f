"""Pins of the reference implementation of Gaussian removal (Sec. 3.2.2, Eq. 8).

The reference decides on the stored parameters in binary32 (opacity logit
against logit(delta_sigma), largest log-scale against ln(delta_s_max) and
ln(delta_s_min)); these tests tie that rule to the definition in the paper
(sigmoid and exp evaluated in binary64) and to hand-built cases, one criterion
at a time, and check that the kept Gaussians keep their order and that
companion arrays follow the same rows.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _set(o, scales):
    scales = np.asarray(scales, np.float64).reshape(3, -1)
    M = scales.shape[1]
    rng = np.random.default_rng(0)
    return {"mean": rng.normal(size=(3, M)).astype(np.float32), "log_scale": np.log(scales).astype(np.float32),
            "quat": rng.normal(size=(4, M)).astype(np.float32), "opacity_logit": np.asarray(o, np.float32),
            "rgb": rng.uniform(size=(3, M)).astype(np.float32)}


def test_defaults_are_the_paper_thresholds():
    r = GOLD["removal"]
    assert O.REMOVAL_DEFAULTS == {"min_opacity": r["delta_sigma"], "max_scale": r["delta_s_max"],
                                  "min_scale": r["delta_s_min"]}


def test_each_criterion_alone():
    logit = lambda s: np.log(s / (1 - s))
    ok = 0.01  # a scale that no criterion removes
    cases = [  # (opacity, (s1, s2, s3), kept)
        (0.5, (ok, ok, ok), True),
        (0.004, (ok, ok, ok), False),       # sigma < delta_sigma
        (0.006, (ok, ok, ok), True),
        (0.5, (0.11, ok, ok), False),        # largest scale above delta_s_max
        (0.5, (ok, 0.11, 0.0001), False),    # ... whichever axis it is on
        (0.5, (0.09, ok, ok), True),
        (0.5, (0.0029, 0.001, 0.002), False),  # largest scale below delta_s_min
        (0.5, (0.0031, 0.001, 0.002), True),   # a small axis alone does not remove
    ]
    g = _set([logit(c[0]) for c in cases], np.array([c[1] for c in cases]).T)
    assert O.removal_keep(g).tolist() == [c[2] for c in cases]


def test_binary32_rule_agrees_with_the_definition():
    """Away from the rounding of the thresholds, comparing stored parameters
    decides as comparing sigmoid(o) and exp(l) in binary64 does."""
    rng = np.random.default_rng(5)
    M = 20000
    o = rng.normal(-4.0, 2.5, M).astype(np.float32)
    ls = rng.normal(-4.5, 1.5, (3, M)).astype(np.float32)
    g = _set(np.zeros(M), np.ones((3, M)))
    g["opacity_logit"], g["log_scale"] = o, ls
    keep = O.removal_keep(g)
    sig = 1.0 / (1.0 + np.exp(-o.astype(np.float64)))
    smax = np.exp(ls.astype(np.float64)).max(axis=0)
    ref = ~((sig < 0.005) | (smax > 0.1) | (smax < 0.003))
    near = (np.abs(sig / 0.005 - 1) < 1e-5) | (np.abs(smax / 0.1 - 1) < 1e-5) | (np.abs(smax / 0.003 - 1) < 1e-5)
    assert 0 < keep.sum() < M and (~keep).sum() > 1000
    assert np.array_equal(keep[~near], ref[~near])


def test_order_and_companions():
    rng = np.random.default_rng(9)
    M = 500
    g = _set(rng.normal(-3, 3, M), np.exp(rng.normal(-4.5, 1.5, (3, M))))
    m = {k: rng.normal(size=v.shape).astype(np.float32) for k, v in g.items()}
    kept, (mk,), idx = O.remove_gaussians(g, [m])
    assert np.all(np.diff(idx) > 0) and idx.size == O.removal_keep(g).sum()
    for k in g:
        rows = g[k].reshape(-1, M)
        assert np.array_equal(kept[k], rows[:, idx])
        assert np.array_equal(mk[k], m[k].reshape(-1, M)[:, idx])


@pytest.mark.parametrize("which", ["none", "all"])
def test_degenerate_sets(which):
    M = 7
    if which == "none":
        g = _set(np.zeros(M), np.full((3, M), 0.01))
    else:
        g = _set(np.full(M, -9.0), np.full((3, M), 0.01))
    kept, _, idx = O.remove_gaussians(g)
    assert idx.size == (M if which == "none" else 0)
    assert kept["mean"].shape == (3, idx.size)
