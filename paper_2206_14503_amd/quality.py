"""Image quality of VDI renderings against direct volume rendering.

The paper compares VDI renderings at viewpoint deviations with DVR by SSIM
(Wang, Bovik, Sheikh and Simoncelli, 2004) and by PSNR (Sec. 7).  Both are
evaluation metrics on downloaded images, computed here in fp64 with numpy.

SSIM at one window position, for images x and y of dynamic range L:

    (2 mu_x mu_y + C1) (2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1) (s_x^2 + s_y^2 + C2))

with C1 = (0.01 L)^2, C2 = (0.03 L)^2, and the means, variances and
covariance weighted by an 11x11 Gaussian window of standard deviation 1.5
(weights summing to one).  It is evaluated at every position where the window
fits inside the image and averaged; a colour image's SSIM is the mean over its
R, G and B channels.  Images are premultiplied RGBA [H, W, 4] (or [H*W, 4] with
the height given); the RGB of premultiplied colour is the image over black.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

K1, K2 = 0.01, 0.03


def gaussian_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """1D Gaussian weights, normalised to sum one (the 2D window is their outer product)."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    w = np.exp(-(r * r) / (2.0 * sigma * sigma))
    return w / w.sum()


def _filter_valid(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted window sums of a 2D image at every position where the window fits."""
    n = w.size
    h, wd = img.shape
    rows = sum(w[t] * img[:, t:wd - n + 1 + t] for t in range(n))
    return sum(w[t] * rows[t:h - n + 1 + t, :] for t in range(n))


def ssim_map(x: np.ndarray, y: np.ndarray, data_range: float = 1.0, size: int = 11,
             sigma: float = 1.5) -> np.ndarray:
    """SSIM of two 2D images at every valid window position."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.shape != y.shape or x.ndim != 2 or min(x.shape) < size:
        raise ValueError("two 2D images of equal shape, at least the window size")
    w = gaussian_window(size, sigma)
    c1, c2 = (K1 * data_range) ** 2, (K2 * data_range) ** 2
    mx, my = _filter_valid(x, w), _filter_valid(y, w)
    sxx = _filter_valid(x * x, w) - mx * mx
    syy = _filter_valid(y * y, w) - my * my
    sxy = _filter_valid(x * y, w) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def _rgb(img: np.ndarray, height: Optional[int]) -> np.ndarray:
    img = np.asarray(img, np.float64)
    if img.ndim == 2:
        if height is None:
            raise ValueError("a [H*W, 4] image needs its height")
        img = img.reshape(height, -1, img.shape[-1])
    return img[..., :3]


def ssim(a: np.ndarray, b: np.ndarray, height: Optional[int] = None, data_range: float = 1.0) -> float:
    """Mean SSIM over the R, G and B channels of two RGBA images."""
    x, y = _rgb(a, height), _rgb(b, height)
    return float(np.mean([ssim_map(x[..., c], y[..., c], data_range).mean() for c in range(3)]))


def psnr(a: np.ndarray, b: np.ndarray, height: Optional[int] = None, data_range: float = 1.0) -> float:
    """Peak signal-to-noise ratio (dB) over the R, G and B channels."""
    x, y = _rgb(a, height), _rgb(b, height)
    mse = float(np.mean((x - y) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(data_range * data_range / mse)
