"""Pins of the SSIM used by the load-balancing training experiment
(bench._ssim: 11 x 11 Gaussian window of sigma 1.5, zero padding,
C1 = 0.01^2, C2 = 0.03^2). CPU only.

With zero padding, a pixel p sees the part w(p) of the window's mass that
falls inside the image. For two constant images a = c1, b = c2 that gives,
per pixel, mu_a = c1 w, mu_b = c2 w, sigma_a^2 = c1^2 w (1 - w),
sigma_b^2 = c2^2 w (1 - w), sigma_ab = c1 c2 w (1 - w), so SSIM(p) is a closed
form in w(p), which is computed here from the separable window in NumPy."""
import math

import numpy as np
import pytest


def _ssim():
    import bench
    return bench._ssim


def _window_mass(h, w):
    x = np.arange(11) - 5.0
    g = np.exp(-x * x / (2 * 1.5 ** 2))
    g /= g.sum()

    def inside(n):
        out = np.zeros(n)
        for p in range(n):
            for k in range(11):
                if 0 <= p + k - 5 < n:
                    out[p] += g[k]
        return out

    return inside(h)[:, None] * inside(w)[None, :]


def test_identical_images_give_one():
    import torch
    rng = np.random.default_rng(0)
    img = torch.tensor(rng.uniform(0, 1, size=(3, 24, 31)))
    assert abs(float(_ssim()(img, img.clone())) - 1.0) < 1e-12


@pytest.mark.parametrize("c1v,c2v", [(0.5, 0.5), (0.5, 0.25), (0.9, 0.1), (0.2, 0.0)])
def test_constant_images_closed_form(c1v, c2v):
    import torch
    h, w = 20, 27
    a = torch.full((3, h, w), c1v, dtype=torch.float64)
    b = torch.full((3, h, w), c2v, dtype=torch.float64)
    m = _window_mass(h, w)
    k1, k2 = 0.01 ** 2, 0.03 ** 2
    num = (2 * c1v * c2v * m * m + k1) * (2 * c1v * c2v * m * (1 - m) + k2)
    den = ((c1v ** 2 + c2v ** 2) * m * m + k1) * ((c1v ** 2 + c2v ** 2) * m * (1 - m) + k2)
    expect = float((num / den).mean())
    assert abs(float(_ssim()(a, b)) - expect) < 1e-10


def test_structure_term_of_a_contrast_inversion_is_negative():
    """An image against its inversion (1 - x): the covariance term changes
    sign, so the SSIM of a textured image is negative."""
    import torch
    rng = np.random.default_rng(1)
    x = rng.uniform(0.2, 0.8, size=(3, 32, 32))
    a = torch.tensor(x)
    b = torch.tensor(1.0 - x)
    assert float(_ssim()(a, b)) < 0.0
    assert math.isfinite(float(_ssim()(a, b)))
