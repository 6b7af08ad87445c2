"""Pins of the oracle's Haar transform and saliency masks against closed forms.

Nothing here calls the GPU library.  Each check is derived from the definition
of the averaging Haar basis (Sec. 2, Eq. 2; algorithm step 1) or of the block
maximum quantiser (step 1), not by re-running the oracle's own code.
"""

import numpy as np
import pytest

from oracle import haar, saliency
from paper_2211_09938_amd import scenes

SHAPES = [(8, 8), (16, 24), (32, 16), (40, 56)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_perfect_reconstruction_bit_exact_on_dyadic_inputs(shape, levels):
    a = scenes.dyadic(np.random.default_rng(7), *shape).astype(np.float64)
    c = haar.analysis(a, levels)
    assert np.array_equal(haar.synthesis(c, levels), a)


@pytest.mark.parametrize("shape", SHAPES)
def test_perfect_reconstruction_random(shape):
    a = np.random.default_rng(3).standard_normal(shape)
    r = haar.synthesis(haar.analysis(a, 3), 3)
    assert np.max(np.abs(r - a)) <= 1e-15 * np.max(np.abs(a)) * 8


def _block(a, y0, x0, h, w):
    return a[y0:y0 + h, x0:x0 + w]


@pytest.mark.parametrize("shape", [(16, 24), (24, 16)])
def test_coefficients_equal_half_block_mean_differences(shape):
    """Every averaging-Haar coefficient in closed form, by brute force over blocks.

    Level-l coefficient at (j, i) belongs to the 2^l block with corner
    (j 2^l, i 2^l).  With m(.) the mean over a (sub)block:
      LL = m(block);  V = (m(left) - m(right)) / 2;  H = (m(top) - m(bottom)) / 2;
      D = (m(TL) - m(TR) - m(BL) + m(BR)) / 4.
    """
    a = np.random.default_rng(11).standard_normal(shape)
    ny, nx = shape
    levels = 3
    c = haar.analysis(a, levels)
    for level in range(1, levels + 1):
        b, hb = 1 << level, 1 << (level - 1)
        h, w = ny >> level, nx >> level
        for j in range(h):
            for i in range(w):
                y0, x0 = j * b, i * b
                tl = _block(a, y0, x0, hb, hb).mean()
                tr = _block(a, y0, x0 + hb, hb, hb).mean()
                bl = _block(a, y0 + hb, x0, hb, hb).mean()
                br = _block(a, y0 + hb, x0 + hb, hb, hb).mean()
                v = ((tl + bl) / 2 - (tr + br) / 2) / 2
                hh = ((tl + tr) / 2 - (bl + br) / 2) / 2
                d = (tl - tr - bl + br) / 4
                assert c[j, w + i] == pytest.approx(v, abs=1e-13)
                assert c[h + j, i] == pytest.approx(hh, abs=1e-13)
                assert c[h + j, w + i] == pytest.approx(d, abs=1e-13)
                if level == levels:
                    assert c[j, i] == pytest.approx(_block(a, y0, x0, b, b).mean(), abs=1e-13)


def test_constant_image_has_zero_details_and_mean_approximation():
    a = np.full((32, 48), 0.375)
    c = haar.analysis(a, 3)
    approx = c[0:4, 0:6].copy()
    c[0:4, 0:6] = 0.0
    assert np.all(c == 0.0)
    assert np.all(approx == 0.375)


@pytest.mark.parametrize("band", ["V", "H", "D"])
@pytest.mark.parametrize("level", [1, 2, 3])
def test_single_basis_function_gives_single_unit_coefficient(band, level):
    """A unit-height +-1 Haar pattern analyses to exactly one coefficient of value 1."""
    ny, nx = 24, 32
    b, hb = 1 << level, 1 << (level - 1)
    j, i = 1, 2
    a = np.zeros((ny, nx))
    y0, x0 = j * b, i * b
    sx = np.r_[np.ones(hb), -np.ones(hb)]
    sy = np.r_[np.ones(hb), -np.ones(hb)]
    one = np.ones(b)
    pat = {"V": np.outer(one, sx), "H": np.outer(sy, one), "D": np.outer(sy, sx)}[band]
    a[y0:y0 + b, x0:x0 + b] = pat
    c = haar.analysis(a, 3)
    h, w = ny >> level, nx >> level
    pos = {"V": (j, w + i), "H": (h + j, i), "D": (h + j, w + i)}[band]
    expect = np.zeros_like(c)
    expect[pos] = 1.0
    assert np.array_equal(c, expect)


def test_maxpool_matches_loops():
    s = np.random.default_rng(5).random((24, 40))
    for level in (1, 2, 3):
        b = 1 << level
        p = saliency.maxpool(s, level)
        for j in range(24 // b):
            for i in range(40 // b):
                assert p[j, i] == s[j * b:(j + 1) * b, i * b:(i + 1) * b].max()


def test_threshold_is_strict_and_levels_map_fine_to_coarse():
    s = np.zeros((16, 16))
    s[5, 9] = 0.7  # exactly the level-2 threshold
    m1, m2, m3 = saliency.detail_masks(s, 3)  # thresholds 0.9, 0.7, 0.5
    assert not m1.any()          # 0.7 is not more than 0.9
    assert not m2.any()          # 0.7 is not more than 0.7
    assert m3.sum() == 1 and m3[5 // 8, 9 // 8]
    s[5, 9] = 0.95
    m1, m2, m3 = saliency.detail_masks(s, 3)
    assert m1.sum() == 1 and m1[2, 4]
    assert m2.sum() == 1 and m2[1, 2]
    assert m3.sum() == 1 and m3[0, 1]


def test_default_thresholds_follow_paper_order(golden_dir):
    import os

    vals = None
    with open(os.path.join(golden_dir, "paper_counts.txt")) as f:
        for line in f:
            if line.startswith("thresholds"):
                vals = [float(v) for v in line.split()[1:]]
    # low to high wavelet level: level-1 details, level-2, level-3, then the approximation (0)
    assert tuple(vals[:3]) == saliency.default_thresholds(3)
    assert vals[3] == 0.0


def test_masking_zeroes_only_unsalient_details():
    a = np.random.default_rng(2).standard_normal((16, 16))
    c = haar.analysis(a, 3)
    masks = [np.zeros((8, 8), bool), np.zeros((4, 4), bool), np.zeros((2, 2), bool)]
    masks[0][3, 4] = True
    cm = saliency.apply_masks(c, masks, 3)
    keep = np.zeros_like(c, dtype=bool)
    keep[0:2, 0:2] = True                    # approximation always kept
    keep[3, 8 + 4] = keep[8 + 3, 4] = keep[8 + 3, 8 + 4] = True
    assert np.array_equal(cm, np.where(keep, c, 0.0))
