"""Pins of the reference's view-dependent colour (Sec. 3.1: SH coefficients per
Gaussian, following 3DGS; App. C: learning rate 0.0005 for the bands above 0).

* The basis: the reference's bands 1..3 equal scipy's spherical harmonics in real form
  (Condon-Shortley phase, sqrt(2) Re / Im for m > 0 / m < 0, m = -l .. l), on random
  directions; so does the dense renderer's basis, built another way (Legendre
  polynomials); orthonormality on the sphere (quadrature); the basis derivatives
  against central differences of the basis polynomials.
* The render and its gradient with SH of degree 1, 2 and 3, both modes: forward values
  and every gradient (coefficients, the mean through the view direction, the pose)
  against the dense float64 renderer and autograd; degree 0 coefficients (none) leave
  the render unchanged; rotating the coefficients' view out of the picture (all bands
  zero) gives the degree-0 render.
"""
import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle import oracle as O
from tests import dense_ref
from tests.tiny_cases import RCfg, tiny_case

KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb", "sh")


def _sph(m, l, theta, phi):
    try:
        return np.asarray(sp.sph_harm_y(l, m, theta, phi))
    except AttributeError:  # older scipy
        return np.asarray(sp.sph_harm(m, l, phi, theta))


def _scipy_real(L, d):
    theta, phi = np.arccos(np.clip(d[2], -1, 1)), np.arctan2(d[1], d[0])
    out = []
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            if m < 0:
                out.append(np.sqrt(2) * _sph(-m, l, theta, phi).imag)
            elif m == 0:
                out.append(_sph(0, l, theta, phi).real)
            else:
                out.append(np.sqrt(2) * _sph(m, l, theta, phi).real)
    return np.array(out)


def test_basis_matches_scipy_and_is_orthonormal():
    rng = np.random.Generator(np.random.PCG64(4))
    d = rng.normal(size=(3, 50))
    d /= np.linalg.norm(d, axis=0)
    want = _scipy_real(3, d)
    got = np.stack([O.sh_basis(3, d[:, j])[0] for j in range(d.shape[1])], axis=1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    np.testing.assert_allclose(dense_ref.sh_real(3, torch.as_tensor(d)).numpy(), want, rtol=0, atol=1e-13)
    for L, K in ((1, 3), (2, 8)):
        assert O.sh_basis(L, d[:, 0])[0].shape == (K,)
        np.testing.assert_array_equal(O.sh_basis(L, d[:, 0])[0], got[:K, 0])
    # orthonormality (Gauss-Legendre in cos(theta) x uniform in phi, exact for these degrees)
    zq, wq = np.polynomial.legendre.leggauss(12)
    ph = np.arange(24) * 2 * np.pi / 24
    Z, PH = np.meshgrid(zq, ph, indexing="ij")
    Wt = np.outer(wq, np.full(24, 2 * np.pi / 24)).reshape(-1)
    s = np.sqrt(1 - Z ** 2)
    dirs = np.stack([s * np.cos(PH), s * np.sin(PH), Z]).reshape(3, -1)
    Y = np.stack([O.sh_basis(3, dirs[:, j])[0] for j in range(dirs.shape[1])], axis=1)
    np.testing.assert_allclose((Y * Wt) @ Y.T, np.eye(15), atol=1e-12)


def test_basis_derivatives_by_central_differences():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(5):
        d = rng.normal(size=3)
        Y, dY = O.sh_basis(3, d)  # the polynomials, off the sphere too
        for a in range(3):
            e = np.zeros(3)
            e[a] = 1e-6
            fd = (O.sh_basis(3, d + e)[0] - O.sh_basis(3, d - e)[0]) / 2e-6
            np.testing.assert_allclose(dY[:, a], fd, rtol=1e-7, atol=1e-8)


def _sh_case(seed, L, M=25):
    case = tiny_case(seed, M=M, log_scale=-2.4)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    g = dict(case["gauss"])
    g["sh"] = (0.3 * rng.normal(size=(3, O.SH_COEFFS[L], M))).astype(np.float32)
    case["gauss"] = g
    return case


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("L", [1, 2, 3])
def test_sh_render_and_gradients_match_autograd(mode, L):
    case = _sh_case(L + 10 * mode, L)
    cfg = O.RenderCfg(mode=mode, eps_cull=0.03)
    rc = RCfg(mode=mode, eps_cull=0.03)
    r = O.render(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"])
    params = dense_ref.to_params(case["gauss"], requires_grad=True)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    C, D = dense_ref.render(params, case["cam"], case["base_rgb"], case["base_depth"], rc, xi=xi)
    keep = r["flag"] == 0
    np.testing.assert_allclose(r["rgb"][:, keep], C.detach().numpy().reshape(3, -1)[:, keep], rtol=0, atol=1e-12)
    rng = np.random.Generator(np.random.PCG64(7))
    W, H = case["cam"]["width"], case["cam"]["height"]
    gC, gD = rng.normal(size=(3, W * H)) * keep, rng.normal(size=W * H) * keep
    Ls = (C.reshape(3, -1) * torch.as_tensor(gC)).sum() + (D.reshape(-1) * torch.as_tensor(gD)).sum()
    Ls.backward()
    an = O.render_bwd(cfg, case["gauss"], case["cam"], case["base_rgb"], case["base_depth"], gC, gD)
    assert np.abs(an["sh"]).max() > 0
    for k in KEYS:
        ag = params[k].grad.numpy()
        assert np.linalg.norm(an[k] - ag) <= 1e-9 * np.linalg.norm(ag), (k, np.linalg.norm(an[k] - ag))
    assert np.linalg.norm(an["pose"] - xi.grad.numpy()) <= 1e-9 * np.linalg.norm(xi.grad.numpy())


def test_zero_bands_give_the_degree0_render():
    case = _sh_case(3, 3)
    g0 = {k: v for k, v in case["gauss"].items() if k != "sh"}
    gz = dict(case["gauss"])
    gz["sh"] = np.zeros_like(gz["sh"])
    cfg = O.RenderCfg(eps_cull=0.03)
    a = O.render(cfg, g0, case["cam"], case["base_rgb"], case["base_depth"])
    b = O.render(cfg, gz, case["cam"], case["base_rgb"], case["base_depth"])
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["depth"], b["depth"])
