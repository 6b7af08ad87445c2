"""Pins of the 1D block fringes (oracle/fringe.py).

No GPU.  The fringe of a level is pinned to the 2D direct sum of the Fresnel
form (oracle/fresnel.py, itself pinned to zone plates): the hologram of a unit
2^l x 2^l block equals g_lo(y - q0) g_lo(x - p0), and that of a block whose
left half is +1 and right half -1 equals g_lo(y - q0) g_hi(x - p0).  A zone
plate with lambda z / p^2 = 64 fixes the kernel's values, and level 0 is the
kernel itself.
"""

import numpy as np
import pytest

from oracle import fresnel, fringe

LAM, PITCH = 532e-9, 8e-6


@pytest.mark.parametrize("level", [1, 2, 3])
def test_block_holograms_factor_into_the_fringes(level):
    z = 0.05
    b = 1 << level
    n = 24
    q0, p0 = 2 * b, b
    obj_lo = np.zeros((n, n))
    obj_lo[q0:q0 + b, p0:p0 + b] = 1.0
    obj_hi = obj_lo.copy()
    obj_hi[q0:q0 + b, p0 + b // 2:p0 + b] = -1.0
    ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    h_lo = fresnel.direct_sum(obj_lo, LAM, PITCH, z, ys.ravel(), xs.ravel(), workers=1).reshape(n, n)
    h_hi = fresnel.direct_sum(obj_hi, LAM, PITCH, z, ys.ravel(), xs.ravel(), workers=1).reshape(n, n)
    gy = fringe.block_fringe(np.arange(n) - q0, level, 0, LAM, PITCH, z)
    glo = fringe.block_fringe(np.arange(n) - p0, level, 0, LAM, PITCH, z)
    ghi = fringe.block_fringe(np.arange(n) - p0, level, 1, LAM, PITCH, z)
    assert np.allclose(h_lo, np.outer(gy, glo), rtol=0, atol=1e-11)
    assert np.allclose(h_hi, np.outer(gy, ghi), rtol=0, atol=1e-11)


def test_zone_plate_values_and_level_zero():
    z = 64 * PITCH * PITCH / LAM  # lambda z / p^2 = 64: phase pi m^2 / 64
    k = fringe.kernel_1d(np.array([0, 4, 8, -8, 16]), LAM, PITCH, z)
    assert np.allclose(k, [1, np.exp(1j * np.pi / 4), -1, -1, 1], atol=1e-13)
    m = np.arange(-40, 40)
    assert np.array_equal(fringe.block_fringe(m, 0, 0, LAM, PITCH, z), fringe.kernel_1d(m, LAM, PITCH, z))


def test_table_layout_and_support():
    n, level = 32, 2
    t = fringe.table(n, level, 1, LAM, PITCH, 0.2, prefactor=2.0 - 1.0j)
    m = np.arange(2 * n) - n
    inside = m >= -(n - (1 << level))
    assert np.all(t[~inside] == 0)
    ref = (2.0 - 1.0j) * fringe.block_fringe(m[inside], level, 1, LAM, PITCH, 0.2)
    assert np.allclose(t[inside], ref, rtol=0, atol=1e-14)
