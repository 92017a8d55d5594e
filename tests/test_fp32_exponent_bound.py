"""The blend stage's FP32 exponent and its per-Gaussian error bound.

The blend kernel evaluates the log2-domain exponent of Eq. 2 in FP32 on the
conic's principal axes, q = ql - a1 u^2 - a2 v^2, and decides alpha >= alpha_low
from it unless q lies within a per-Gaussian bound of log2(alpha_low), where it
re-decides in FP64. This file restates that arithmetic in NumPy float32 (each
operation rounded as the kernel's) and the bound's formula, and checks the
bound against the exact (FP64) exponent on random and adversarial Gaussians:
thin footprints (axis ratios up to 10^5) at every angle, centres far from the
pixel. It pins the error analysis, not the kernel's code, which the GPU parity
tests check end to end."""
import math

import numpy as np

U0 = 2.0 ** -24
Q_LOW = math.log2(1.0 / 255.0)
H = 0.5 / math.log(2.0)  # P = h * (conic quadratic form), h = log2(e) / 2


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def fma32(a, b, c):
    # a*b of two float32 values is exact in float64; one float64 rounding of
    # the sum then the float32 rounding (within the bound's slack)
    return f32(a * b + c)


def principal_axes(pa, pb, pg):
    tau = np.where(pb != 0, (pg - pa) / np.where(pb != 0, 2 * pb, 1), 0.0)
    t = np.where(pb != 0, np.where(tau >= 0, 1.0, -1.0) / (np.abs(tau) + np.sqrt(1 + tau * tau)), 0.0)
    c = 1 / np.sqrt(1 + t * t)
    return c, t * c, pa - t * pb, pg + t * pb


def bound(a1, a2, ql):
    """Returns (dq, ok): the bound at the region's edge and whether the
    off-region condition holds (else the kernel decides in FP64 only)."""
    d0 = 0.02
    ra = np.sqrt(a1) + np.sqrt(a2)
    amin = np.minimum(a1, a2)
    k1 = 1.5 * U0 * (8 * math.sqrt(2) * ra / np.sqrt(amin) + 6)
    k2 = 1.5 * U0 * 20 * ra
    k0 = 1.5 * U0 * 3 * np.abs(ql)
    m = ql - Q_LOW
    pm = np.maximum(m + d0, 0)
    dq = k1 * pm + k2 * np.sqrt(pm) + k0
    A, B = 1 - k1, k2
    sp, ss = np.sqrt(pm), B / (2 * A)
    fmin = np.where(sp >= ss, A * pm - B * sp - m, -m - B * B / (4 * A))
    band = dq + 2.0 ** -19
    ok = (dq <= 2.0 ** -8) & (A > 0.5) & (fmin > 2 * band + k0 + 2.0 ** -19)
    return dq, ok


def fp32_exponent(X, Y, fx, fy, c, s, a1, a2, ql):
    """The kernel's sequence: staging rounds the quadrant-relative centre and
    the coefficients to float32, then each operation rounds."""
    Xf, Yf = f32(X), f32(Y)
    dx, dy = f32(Xf - fx), f32(Yf - fy)
    cf, sf, a1f, a2f, qlf = f32(c), f32(s), f32(a1), f32(a2), f32(ql)
    u = fma32(cf, dx, -f32(sf * dy))
    v = fma32(sf, dx, f32(cf * dy))
    return fma32(-f32(a1f * u), u, fma32(-f32(a2f * v), v, qlf))


def draw(rng, n, max_ratio):
    """Random Gaussians seen from a pixel: P's eigenvalues, its angle,
    log2-opacity, the centre relative to an 8 x 8 quadrant and the pixel's
    offset in it."""
    big = np.exp(rng.uniform(math.log(1e-4), math.log(3.0), n))
    small = big / np.exp(rng.uniform(0, math.log(max_ratio), n))
    th = rng.uniform(0, math.pi, n)
    ct, st = np.cos(th), np.sin(th)
    pa = small * ct * ct + big * st * st
    pg = small * st * st + big * ct * ct
    pb = (small - big) * ct * st
    ql = rng.uniform(Q_LOW - 1.0, 0.0, n)
    fx = rng.integers(0, 8, n).astype(np.float64)
    fy = rng.integers(0, 8, n).astype(np.float64)
    # offsets: mostly inside the alpha_low ellipse, some on its edge, some beyond
    c, s, a1, a2 = principal_axes(pa, pb, pg)
    target = np.maximum(ql - Q_LOW, 0) * rng.choice([0.3, 0.99, 1.0, 1.01, 3.0], n) + rng.uniform(0, 0.05, n)
    ang = rng.uniform(0, 2 * math.pi, n)
    uu = np.sqrt(target / a1) * np.cos(ang)
    vv = np.sqrt(target / a2) * np.sin(ang)
    dx = c * uu + s * vv
    dy = -s * uu + c * vv
    X = dx + fx + rng.uniform(-0.5, 0.5, n) * 1e-3  # centre relative to the quadrant
    Y = dy + fy + rng.uniform(-0.5, 0.5, n) * 1e-3
    return pa, pb, pg, ql, X, Y, fx, fy


def check(rng, n, max_ratio):
    pa, pb, pg, ql, X, Y, fx, fy = draw(rng, n, max_ratio)
    c, s, a1, a2 = principal_axes(pa, pb, pg)
    dxe, dye = X - fx, Y - fy
    q_exact = ql - (pa * dxe * dxe + 2 * pb * dxe * dye + pg * dye * dye)
    q32 = fp32_exponent(X, Y, fx, fy, c, s, a1, a2, ql)
    dq, ok = bound(a1, a2, ql)
    inside = q_exact >= Q_LOW - 0.02
    err = np.abs(q32 - q_exact)
    band = dq + 2.0 ** -19
    # where the kernel trusts FP32, the error stays within the bound inside
    # the region, and outside it FP32 stays below the candidate threshold
    assert np.all(err[ok & inside] <= dq[ok & inside]), np.max((err / dq)[ok & inside])
    assert np.all(q32[ok & ~inside] < Q_LOW - 2 * band[ok & ~inside])
    return ok.mean(), np.median(dq[ok]), np.max((err / dq)[ok & inside])


def test_principal_axes_diagonalise_the_conic():
    rng = np.random.default_rng(0)
    pa, pb, pg, *_ = draw(rng, 1000, 1e3)
    c, s, a1, a2 = principal_axes(pa, pb, pg)
    d = rng.normal(size=(2, 1000)) * 10
    u = c * d[0] - s * d[1]
    v = s * d[0] + c * d[1]
    lhs = pa * d[0] ** 2 + 2 * pb * d[0] * d[1] + pg * d[1] ** 2
    np.testing.assert_allclose(a1 * u * u + a2 * v * v, lhs, rtol=1e-9)
    assert np.all(a1 > 0) and np.all(a2 > 0)


def test_bound_holds_for_ordinary_gaussians():
    rng = np.random.default_rng(1)
    frac_ok, med, worst = check(rng, 400_000, 10.0)
    assert frac_ok > 0.999
    assert worst < 1.0 and med < 1e-4


def test_bound_holds_for_thin_gaussians():
    rng = np.random.default_rng(2)
    frac_ok, med, worst = check(rng, 400_000, 1e5)
    assert frac_ok > 0.9  # the thinnest far-reaching ones fall back to FP64
    assert worst < 1.0


def test_bound_is_not_vacuous():
    """The bound is within a small factor of errors that do occur, so it
    neither hides a mistake in the analysis nor sends most pixels to FP64."""
    rng = np.random.default_rng(3)
    pa, pb, pg, ql, X, Y, fx, fy = draw(rng, 200_000, 100.0)
    c, s, a1, a2 = principal_axes(pa, pb, pg)
    dxe, dye = X - fx, Y - fy
    q_exact = ql - (pa * dxe * dxe + 2 * pb * dxe * dye + pg * dye * dye)
    err = np.abs(fp32_exponent(X, Y, fx, fy, c, s, a1, a2, ql) - q_exact)
    dq, ok = bound(a1, a2, ql)
    inside = ok & (q_exact >= Q_LOW - 0.02)
    assert np.max(err[inside] / dq[inside]) > 1e-3
