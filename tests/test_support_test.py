"""The support-ellipse culling of the compositing kernels (SupportTest, render_common.h)
replayed on the CPU in binary32: a rectangle it rejects holds no pixel whose opacity
reaches alpha_min by the per-pixel test (the binary32 steps of eval_alpha), on random
Gaussians (isotropic to strongly elongated, low to high opacity, rotated) against random
rectangles near their support.  This is the property the kernels rely on to skip a
record for a whole tile or wavefront; the GPU parity tests check the compiled kernels
pixel by pixel.  Also: the test rejects a good share of the rectangles the bounding box
would keep."""
import numpy as np

F = np.float32
L2E = F(1.4426950408889634)


def fma(a, b, c):
    return F(np.float64(a) * np.float64(b) + np.float64(c))


def record(rng):
    """A projected Gaussian as the kernels store it: centre, the exponent's coefficients
    (-0.5 a, -b, -0.5 c) log2 e of the conic, log2 sigma, and the padded box half-extents."""
    s1, s2 = np.exp(rng.uniform(-0.5, 3.5, 2))
    th = rng.uniform(0, np.pi)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    S = R @ np.diag([s1 * s1, s2 * s2]) @ R.T + 0.3 * np.eye(2)
    A, B, C = F(S[0, 0]), F(S[0, 1]), F(S[1, 1])
    det = F(A * C - B * B)
    idet = F(1.0) / det
    sig = F(1.0 / (1.0 + np.exp(-rng.normal(0.0, 2.0))))
    amin = F(1.0 / 255.0)
    if not sig > amin:
        return None
    kappa = F(2.0) * F(np.log(sig / amin))
    rx, ry = F(np.sqrt(kappa * A)) + F(1), F(np.sqrt(kappa * C)) + F(1)
    mx, my = F(rng.uniform(0, 64)), F(rng.uniform(0, 64))
    qa, qb, qc = F(-0.5) * L2E * (C * idet), L2E * (B * idet), F(-0.5) * L2E * (A * idet)
    return dict(mx=mx, my=my, A=qa, B=qb, C=qc, l2s=F(np.log2(sig)), rx=rx, ry=ry, amin=amin)


def meets(r, x0, y0, w, h):
    """SupportTest::meets, step for step in binary32."""
    kx = F(-0.5) * r["B"] * (F(1.0) / r["A"])
    ky = F(-0.5) * r["B"] * (F(1.0) / r["C"])
    need = (F(np.log2(r["amin"])) - r["l2s"]) * F(1.0001) - F(1e-4)
    X0, X1 = F(x0 - 1.0) - r["mx"], F(x0 + w) - r["mx"]
    Y0, Y1 = F(y0 - 1.0) - r["my"], F(y0 + h) - r["my"]
    if X0 <= 0 <= X1 and Y0 <= 0 <= Y1:
        return True

    def at(dx, dy):
        return F(dx * F(r["A"] * dx + r["B"] * dy)) + F(r["C"] * dy * dy)

    e = [at(X0, min(max(ky * X0, Y0), Y1)), at(X1, min(max(ky * X1, Y0), Y1)),
         at(min(max(kx * Y0, X0), X1), Y0), at(min(max(kx * Y1, X0), X1), Y1)]
    return not (max(e) < need)


def pixel_passes(r, px, py):
    """eval_alpha's binary32 steps and the alpha_min test."""
    dx, dy = F(F(px) - r["mx"]), F(F(py) - r["my"])
    pw = fma(r["A"], F(dx * dx), fma(r["B"], F(dx * dy), fma(r["C"], F(dy * dy), r["l2s"])))
    return F(2.0) ** pw >= r["amin"]


def test_rejected_rectangles_hold_no_contributing_pixel():
    rng = np.random.Generator(np.random.PCG64(21))
    rejected = box_kept = 0
    for _ in range(3000):
        r = record(rng)
        if r is None:
            continue
        for _ in range(6):
            w, h = (8, 16) if rng.uniform() < 0.5 else (16, 32)
            x0 = int(np.floor(r["mx"] + rng.uniform(-1.3, 1.3) * float(r["rx"]))) - w // 2
            y0 = int(np.floor(r["my"] + rng.uniform(-1.3, 1.3) * float(r["ry"]))) - h // 2
            in_box = not (r["mx"] + r["rx"] < x0 or r["mx"] - r["rx"] > x0 + w - 1 or
                          r["my"] + r["ry"] < y0 or r["my"] - r["ry"] > y0 + h - 1)
            if meets(r, F(x0), F(y0), F(w), F(h)):
                continue
            rejected += 1
            box_kept += in_box
            for py in range(y0, y0 + h):
                for px in range(x0, x0 + w):
                    assert not pixel_passes(r, px, py), (r, x0, y0, px, py)
    assert rejected > 2000 and box_kept > 200, (rejected, box_kept)
