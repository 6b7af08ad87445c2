"""Pins of the SSIM used to score progressive stages (oracle/quality.py) and of
the package's host-side implementation (paper_2211_09938_amd/quality.py).

Closed forms: an image against itself scores 1; two constant images c1, c2
score (2 c1 c2 + C1) / (c1^2 + c2^2 + C1) (the structure term is 1 when both
variances vanish); the score is symmetric; more noise scores lower.  The two
implementations (2D convolution vs separable window sums) agree to 1e-12.
"""

import numpy as np
import pytest

from oracle import quality as oq
from paper_2211_09938_amd import quality as pq


@pytest.mark.parametrize("impl", [oq.ssim, pq.ssim])
def test_identity_and_constants(impl):
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (40, 33))
    assert abs(impl(x, x, 1.0) - 1.0) <= 1e-12
    c1, c2, r = 0.3, 0.7, 1.0
    a, b = np.full((20, 20), c1), np.full((20, 20), c2)
    k1 = (0.01 * r) ** 2
    want = (2 * c1 * c2 + k1) / (c1 * c1 + c2 * c2 + k1)
    assert abs(impl(a, b, r) - want) <= 1e-12


@pytest.mark.parametrize("impl", [oq.ssim, pq.ssim])
def test_symmetry_and_monotone_in_noise(impl):
    rng = np.random.default_rng(2)
    yy, xx = np.mgrid[0:64, 0:64]
    x = np.exp(-((yy - 30) ** 2 + (xx - 25) ** 2) / 200.0)
    n = rng.standard_normal(x.shape)
    y1, y2 = x + 0.02 * n, x + 0.1 * n
    assert abs(impl(x, y1, 1.0) - impl(y1, x, 1.0)) <= 1e-12
    assert 1.0 > impl(x, y1, 1.0) > impl(x, y2, 1.0)


def test_package_matches_oracle():
    rng = np.random.default_rng(3)
    for shape in [(11, 11), (37, 52), (128, 96)]:
        x = rng.uniform(0, 2, shape)
        y = x + rng.normal(0, 0.3, shape)
        assert abs(pq.ssim(x, y, 2.0) - oq.ssim(x, y, 2.0)) <= 1e-12


def test_rejects_small_or_mismatched_images():
    with pytest.raises(ValueError):
        pq.ssim(np.zeros((10, 20)), np.zeros((10, 20)), 1.0)
    with pytest.raises(ValueError):
        pq.ssim(np.zeros((20, 20)), np.zeros((20, 21)), 1.0)
