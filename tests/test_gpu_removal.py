"""GPU parity of Gaussian removal (Sec. 3.2.2, Eq. 8) against the reference.

Bit-exact: the kept set, its order, the companion rows and the count.  Inputs
straddle every threshold, including parameters exactly at the binary32
thresholds (kept: the tests are strict), with sizes that leave a ragged last
block, plus the empty set and sets where everything or nothing is removed.
"""
import numpy as np
import pytest
import torch

from tests.gpu_util import DEV, say

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
    return O


def _random_set(M, seed):
    rng = np.random.default_rng(seed)
    g = {k: rng.normal(size=(ROWS[k], M)).astype(np.float32) for k in KEYS}
    g["opacity_logit"] = rng.normal(-4.0, 2.5, M).astype(np.float32)
    g["log_scale"] = rng.normal(-4.5, 1.5, (3, M)).astype(np.float32)
    return g


def _dev(g):
    return {k: torch.as_tensor(v.reshape(-1) if ROWS[k] == 1 else v).to(DEV) for k, v in g.items()}


def _check(P, O, g, companions):
    kept, comps, n = P.remove_gaussians(_dev(g), [_dev(c) for c in companions])
    torch.cuda.synchronize()
    rk, rcomps, idx = O.remove_gaussians(g, companions)
    assert n == idx.size
    for k in KEYS:
        assert np.array_equal(kept[k].cpu().numpy().reshape(ROWS[k], n), rk[k]), k
        for c, rc in zip(comps, rcomps):
            assert np.array_equal(c[k].cpu().numpy().reshape(ROWS[k], n), rc[k]), k
    return n


@pytest.mark.parametrize("M", [1, 255, 1000, 4097, 100_000])
def test_removal_parity(P, O, M):
    say(f"removal parity: M={M}")
    g = _random_set(M, M)
    m, v = _random_set(M, M + 1), _random_set(M, M + 2)
    t_o, t_hi, t_lo = O.removal_thresholds()
    if M >= 1000:  # parameters exactly at and one ulp around the thresholds
        g["opacity_logit"][:3] = [t_o, np.nextafter(t_o, np.float32(-np.inf)), np.nextafter(t_o, np.float32(np.inf))]
        g["log_scale"][:, 3:9] = np.float32(-4.0)
        g["log_scale"][0, 3:6] = [t_hi, np.nextafter(t_hi, np.float32(np.inf)), np.nextafter(t_hi, np.float32(-np.inf))]
        g["log_scale"][:, 6:9] = [[t_lo, np.nextafter(t_lo, np.float32(-np.inf)), np.nextafter(t_lo, np.float32(np.inf))]] * 3
        g["opacity_logit"][3:9] = 0.0
    n = _check(P, O, g, [m, v])
    if M >= 1000:
        assert 0 < n < M


def test_removal_degenerate(P, O):
    say("removal: empty set, nothing removed, everything removed")
    g0 = _random_set(0, 3)
    assert _check(P, O, g0, []) == 0
    keep_all = _random_set(600, 4)
    keep_all["opacity_logit"][:] = 0.0
    keep_all["log_scale"][:] = np.float32(np.log(0.01))
    assert _check(P, O, keep_all, [_random_set(600, 5)]) == 600
    drop_all = _random_set(600, 6)
    drop_all["opacity_logit"][:] = -9.0
    assert _check(P, O, drop_all, []) == 0
