"""Pins for the SSIM and PSNR used to compare VDI renderings with DVR.

Checked against closed forms (constant images, constant offsets), an explicit
per-window evaluation of the definition with the 2D window as an outer
product (independent of the separable filtering), and identity/symmetry.
"""
import math

import numpy as np
import pytest

from paper_2206_14503_amd import quality


def test_ssim_of_an_image_with_itself_is_one():
    rng = np.random.default_rng(1)
    img = rng.uniform(0, 1, (40, 50, 4))
    assert quality.ssim(img, img) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("a,b", [(0.2, 0.2), (0.2, 0.5), (0.0, 0.9), (0.7, 0.3)])
def test_ssim_of_constant_images(a, b):
    """No variance: the structure term is C2/C2 = 1, leaving the luminance term
    (2ab + C1) / (a^2 + b^2 + C1)."""
    x = np.full((20, 30, 4), a)
    y = np.full((20, 30, 4), b)
    c1 = 0.01 ** 2
    assert quality.ssim(x, y) == pytest.approx((2 * a * b + c1) / (a * a + b * b + c1), abs=1e-12)


def test_ssim_map_matches_the_windowed_definition():
    """At sampled positions, means, variances and covariance summed explicitly
    over the 11x11 window with weights outer(g, g)."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (30, 34))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    m = quality.ssim_map(x, y)
    assert m.shape == (20, 24)
    g = quality.gaussian_window()
    w2 = np.outer(g, g)
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    for (i, j) in [(0, 0), (5, 17), (19, 23), (11, 3)]:
        px, py = x[i:i + 11, j:j + 11], y[i:i + 11, j:j + 11]
        mx, my = (w2 * px).sum(), (w2 * py).sum()
        vx, vy = (w2 * (px - mx) ** 2).sum(), (w2 * (py - my) ** 2).sum()
        cxy = (w2 * (px - mx) * (py - my)).sum()
        ref = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
        assert m[i, j] == pytest.approx(ref, abs=1e-12)


def test_ssim_is_symmetric_and_below_one_for_different_images():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (24, 24, 4))
    y = rng.uniform(0, 1, (24, 24, 4))
    assert quality.ssim(x, y) == pytest.approx(quality.ssim(y, x), abs=1e-14)
    assert quality.ssim(x, y) < 0.5


def test_gaussian_window():
    g = quality.gaussian_window()
    assert g.size == 11 and g.sum() == pytest.approx(1.0, abs=1e-15)
    assert g[0] / g[5] == pytest.approx(math.exp(-25 / (2 * 1.5 ** 2)), rel=1e-12)


def test_psnr_closed_forms():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 0.5, (16, 16, 4))
    assert quality.psnr(x, x) == math.inf
    assert quality.psnr(x, x + 0.1) == pytest.approx(-20 * math.log10(0.1), abs=1e-9)
    flat = x.reshape(-1, 4)
    assert quality.psnr(flat, flat + 0.01, height=16) == pytest.approx(40.0, abs=1e-9)
