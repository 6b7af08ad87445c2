"""Saliency quantisation and detail masking (oracle, test infrastructure).

Paper, algorithm step 1: the saliency map is quantised to 2, 4 and 8 times
smaller sizes by taking the maximum per block, so that each quantised map has
the size of the wavelet output of its level.  Steps 3-5 refine only blocks whose
saliency is *more than* a threshold; Sec. 3 lists the thresholds 0.9, 0.7, 0.5, 0
"for low to high levels".

Readings taken here (the paper does not pin them down):
* level-l detail coefficients (l = 1 finest) are kept where
  maxpool_{2^l}(S) > t_l, the mask living at coefficient resolution;
* the thresholds map low-to-high onto level 1, 2, 3 details and the level-3
  approximation: t = (0.9, 0.7, 0.5) for the details, and the approximation is
  used everywhere ("saliency more than 0 ... all foreground and background");
* comparisons are strict; for other level counts every detail threshold is 0.5.
"""

import numpy as np

DEFAULT_THRESHOLDS_3 = (0.9, 0.7, 0.5)


def default_thresholds(levels):
    if levels == 3:
        return DEFAULT_THRESHOLDS_3
    return tuple([0.5] * levels)


def maxpool(sal, level):
    """Block maximum over 2^level x 2^level blocks (float64 result)."""
    s = np.asarray(sal, dtype=np.float64)
    b = 1 << level
    ny, nx = s.shape
    return s.reshape(ny // b, b, nx // b, b).max(axis=(1, 3))


def detail_masks(sal, levels, thresholds=None):
    """Boolean keep-masks M_l, l = 1..levels, each (ny/2^l, nx/2^l)."""
    if thresholds is None:
        thresholds = default_thresholds(levels)
    if len(thresholds) != levels:
        raise ValueError("need one threshold per detail level")
    return [maxpool(sal, l) > float(thresholds[l - 1]) for l in range(1, levels + 1)]


def apply_masks(c, masks, levels):
    """Zero the level-l detail coefficients where M_l is False.

    The coarsest approximation square is never masked.
    """
    from .haar import detail_slices

    out = np.array(c, dtype=np.float64, copy=True)
    ny, nx = out.shape
    for level in range(1, levels + 1):
        keep = masks[level - 1]
        for sl in detail_slices(ny, nx, level).values():
            out[sl] = np.where(keep, out[sl], 0.0)
    return out
