"""Averaging Haar wavelet analysis and synthesis (oracle, test infrastructure).

Paper: Sec. 2, Eq. 2 -- an object is a linear combination of Haar basis
functions; level 1 splits it into L, H, V, D and L is split again, recursively.
Algorithm step 1 applies three levels (L -> LL -> LLL), each level a quarter of
the size of the previous one.

Reading of the paper (it names no normalisation): the *averaging* Haar pair

    lo = (a + b) / 2,    hi = (a - b) / 2          (analysis)
    a  = lo + hi,        b  = lo - hi              (synthesis)

so that the coarsest approximation value is the mean of its 2^L x 2^L block
(the "intensity" that step 2 multiplies a block fringe by) and every basis
function is a unit-height +-1 block pattern.

2D order and layout (Mallat): at each level transform along x (columns of the
row-major array) first, then along y, and store, inside the top-left
2h x 2w square of the coefficient array,

    [0:h, 0:w]   LL  (lo_y lo_x)     [0:h, w:2w]   V (lo_y hi_x)
    [h:2h, 0:w]  H   (hi_y lo_x)     [h:2h, w:2w]  D (hi_y hi_x)

and recurse on the LL square.  Arrays are indexed [y, x].
"""

import numpy as np


def _split_x(a):
    """One analysis step along x: returns (lo, hi), each half as wide."""
    even = a[:, 0::2]
    odd = a[:, 1::2]
    return (even + odd) / 2.0, (even - odd) / 2.0


def _split_y(a):
    """One analysis step along y: returns (lo, hi), each half as tall."""
    even = a[0::2, :]
    odd = a[1::2, :]
    return (even + odd) / 2.0, (even - odd) / 2.0


def _merge_x(lo, hi):
    out = np.empty((lo.shape[0], 2 * lo.shape[1]), dtype=np.float64)
    out[:, 0::2] = lo + hi
    out[:, 1::2] = lo - hi
    return out


def _merge_y(lo, hi):
    out = np.empty((2 * lo.shape[0], lo.shape[1]), dtype=np.float64)
    out[0::2, :] = lo + hi
    out[1::2, :] = lo - hi
    return out


def check_shape(ny, nx, levels):
    if levels < 1:
        raise ValueError("levels must be >= 1")
    if ny % (1 << levels) or nx % (1 << levels):
        raise ValueError("both sides must be divisible by 2**levels")


def analysis(a, levels):
    """Multi-level 2D averaging Haar analysis W(a), Mallat layout (float64)."""
    a = np.asarray(a, dtype=np.float64)
    ny, nx = a.shape
    check_shape(ny, nx, levels)
    c = np.zeros((ny, nx), dtype=np.float64)
    ll = a
    h, w = ny, nx
    for _ in range(levels):
        lo_x, hi_x = _split_x(ll)
        ll_new, h_band = _split_y(lo_x)  # lo_y lo_x, hi_y lo_x
        v_band, d_band = _split_y(hi_x)  # lo_y hi_x, hi_y hi_x
        h, w = h // 2, w // 2
        c[0:h, w:2 * w] = v_band
        c[h:2 * h, 0:w] = h_band
        c[h:2 * h, w:2 * w] = d_band
        ll = ll_new
    c[0:h, 0:w] = ll
    return c


def synthesis(c, levels):
    """Inverse of :func:`analysis` (S = W^-1), float64."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    check_shape(ny, nx, levels)
    h, w = ny >> levels, nx >> levels
    ll = c[0:h, 0:w].copy()
    for _ in range(levels):
        v_band = c[0:h, w:2 * w]
        h_band = c[h:2 * h, 0:w]
        d_band = c[h:2 * h, w:2 * w]
        lo_x = _merge_y(ll, h_band)
        hi_x = _merge_y(v_band, d_band)
        ll = _merge_x(lo_x, hi_x)
        h, w = 2 * h, 2 * w
    return ll


def detail_slices(ny, nx, level):
    """Slices of the V, H and D quadrants of detail level ``level`` (1 = finest)."""
    h, w = ny >> level, nx >> level
    return {
        "V": (slice(0, h), slice(w, 2 * w)),
        "H": (slice(h, 2 * h), slice(0, w)),
        "D": (slice(h, 2 * h), slice(w, 2 * w)),
    }


def approx_slice(ny, nx, levels):
    return (slice(0, ny >> levels), slice(0, nx >> levels))
