"""Stage quality measure of the progressive display (host-side evaluation).

SSIM of a stage's reconstruction against the point-wise hologram's, the score
the paper tabulates per stage (Sec. 3).  Standard SSIM (Wang et al., IEEE TIP
2004): 11 x 11 Gaussian window, sigma 1.5, C1 = (0.01 R)^2, C2 = (0.03 R)^2,
mean over the windows inside the image.  Separable weighted window sums,
float64, NumPy; runs on the host on amplitudes copied back from the GPU.
"""

import numpy as np


def _weights(size, sigma):
    t = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    return g / g.sum()


def _window_mean(img, g):
    # weighted mean over every size x size window that fits: rows, then columns
    v = np.lib.stride_tricks.sliding_window_view(img, g.size, axis=0) @ g
    return np.lib.stride_tricks.sliding_window_view(v, g.size, axis=1) @ g


def ssim(x, y, data_range, size=11, sigma=1.5):
    """Mean SSIM of two equally shaped real images (both at least size x size)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or min(x.shape) < size:
        raise ValueError("ssim needs two images of one shape, at least the window size")
    g = _weights(size, sigma)
    mx, my = _window_mean(x, g), _window_mean(y, g)
    vx = _window_mean(x * x, g) - mx * mx
    vy = _window_mean(y * y, g) - my * my
    cxy = _window_mean(x * y, g) - mx * my
    c1 = (0.01 * data_range) ** 2
    c2 = (0.03 * data_range) ** 2
    num = (2.0 * mx * my + c1) * (2.0 * cxy + c2)
    den = (mx * mx + my * my + c1) * (vx + vy + c2)
    return float(np.mean(num / den))
