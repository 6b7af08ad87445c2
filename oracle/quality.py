"""Structural similarity (oracle; test infrastructure only).

The paper scores each progressive stage by the SSIM of its reconstruction
against the point-wise hologram's (Sec. 3, Table 3).  SSIM (Wang, Bovik,
Sheikh, Simoncelli, IEEE TIP 2004): over every 11 x 11 window with Gaussian
weights (sigma 1.5), with weighted means mu, variances s^2 and covariance s_xy,

    SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
    C1 = (0.01 R)^2, C2 = (0.03 R)^2, R the data range,

averaged over the windows that fit inside the image.  Written here with a 2D
'valid' convolution by the full 2D window (scipy.signal), FP64.
"""

import numpy as np
from scipy.signal import convolve2d


def gaussian_window(size=11, sigma=1.5):
    t = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def ssim(x, y, data_range, size=11, sigma=1.5):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = gaussian_window(size, sigma)

    def wavg(img):
        return convolve2d(img, w[::-1, ::-1], mode="valid")

    mx, my = wavg(x), wavg(y)
    sxx = wavg(x * x) - mx * mx
    syy = wavg(y * y) - my * my
    sxy = wavg(x * y) - mx * my
    c1 = (0.01 * data_range) ** 2
    c2 = (0.03 * data_range) ** 2
    m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(m.mean())
