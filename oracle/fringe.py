"""1D block fringes of the Haar basis blocks (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2: a level-l coefficient spreads over a 2^l x 2^l block of object points,
and the look-up table holds the hologram of such a block.  Under the Fresnel
form of Eq. 1 the kernel of an integer offset (dy, dx) is the product
k(dy) k(dx) with k(m) = exp(i pi p^2 m^2 / (lambda z)) (``fresnel.kernel_2d``
with dx = 0), so the hologram of a uniform block (the lo band) or of a block
whose first half is +1 and second half -1 along an axis (the hi band) factors
into the 1D sums

    g_lo[m] = sum_{u < 2^l} k(m - u)
    g_hi[m] = sum_{u < 2^(l-1)} k(m - u) - sum_{2^(l-1) <= u < 2^l} k(m - u)

of the offset m = pixel - block start, with g = k at level 0.  FP64 throughout;
the angle of k reaches a few million radians at the largest offsets, where its
FP64 rounding is below 1e-9 rad.
"""

import numpy as np

from . import fresnel


def kernel_1d(m, lam, pitch, z):
    """k(m) for integer offsets m (complex128)."""
    m = np.asarray(m, dtype=np.float64)
    return fresnel.kernel_2d(m, np.zeros_like(m), lam, pitch, z)


def block_fringe(m, level, band, lam, pitch, z):
    """g_lo (band 0) or g_hi (band 1) of a 2^level block at offsets m (complex128)."""
    m = np.asarray(m, dtype=np.int64)
    b = 1 << level
    out = np.zeros(m.shape, dtype=np.complex128)
    for u in range(b):
        sign = 1.0 if (band == 0 or u < b // 2) else -1.0
        out += sign * kernel_1d(m - u, lam, pitch, z)
    return out


def table(n_pix, level, band, lam, pitch, z, prefactor=1.0):
    """One axis's table as the library lays it out: entry i holds g[i - n_pix] for
    i in [0, 2 n_pix), times a layer constant (Eq. 1's prefactor, or 1), and zero
    where no block of that level fits the axis (offsets below -(n_pix - 2^level))."""
    m = np.arange(2 * n_pix, dtype=np.int64) - n_pix
    g = block_fringe(m, level, band, lam, pitch, z) * prefactor
    g[m < -(n_pix - (1 << level))] = 0.0
    return g
