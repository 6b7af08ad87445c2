"""Pins of the progressive stage outputs of the oracle (Sec. 2 steps 2-5, Sec. 3 display).

Closed forms that do not use the Haar code:
* with every block salient, stage j shows the object averaged over blocks of
  side 2^(L-j) (the approximation of level L-j), so stage 0 is the 8 x 8 block
  mean and stage L the object itself;
* with no salient block every stage equals stage 0;
* with one salient pixel, the increment of stage j (level l = L-j+1) is zero
  outside the 2^l x 2^l block that holds the pixel.
"""

import numpy as np
import pytest

from oracle import fresnel, progressive


def block_mean(a, b):
    ny, nx = a.shape
    m = a.reshape(ny // b, b, nx // b, b).mean(axis=(1, 3))
    return np.repeat(np.repeat(m, b, axis=0), b, axis=1)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_all_salient_stage_is_block_mean(levels):
    rng = np.random.default_rng(11)
    a = rng.uniform(0.0, 1.0, (32, 48))
    for j in range(levels + 1):
        got = progressive.stage_reconstruction(a, None, levels, j)
        assert np.max(np.abs(got - block_mean(a, 1 << (levels - j)))) <= 1e-14


def test_no_salient_block_keeps_every_stage_at_the_block_mean():
    rng = np.random.default_rng(12)
    a = rng.uniform(0.0, 1.0, (24, 40))
    sal = np.zeros_like(a)
    for j in range(4):
        got = progressive.stage_reconstruction(a, sal, 3, j)
        assert np.max(np.abs(got - block_mean(a, 8))) <= 1e-14


def test_one_salient_pixel_confines_each_increment_to_its_block():
    rng = np.random.default_rng(13)
    a = rng.uniform(0.0, 1.0, (32, 32))
    sal = np.zeros_like(a)
    q0, p0 = 13, 22
    sal[q0, p0] = 1.0
    prev = progressive.stage_reconstruction(a, sal, 3, 0)
    for j in range(1, 4):
        cur = progressive.stage_reconstruction(a, sal, 3, j)
        b = 1 << (3 - j + 1)
        inc = cur - prev
        outside = np.ones_like(a, dtype=bool)
        outside[(q0 // b) * b:(q0 // b + 1) * b, (p0 // b) * b:(p0 // b + 1) * b] = False
        assert np.all(inc[outside] == 0.0)
        assert np.any(inc[~outside] != 0.0)
        prev = cur
    assert np.array_equal(prev, progressive.masked_reconstruction(a, sal, 3))


def test_stage_holograms_are_holograms_of_the_stage_objects():
    rng = np.random.default_rng(14)
    ny, nx = 16, 24
    obj = rng.uniform(0.0, 1.0, (ny, nx))
    layer = (rng.uniform(0, 1, (ny, nx)) > 0.5).astype(np.uint8)
    z = (0.15, 0.25)
    lam, pitch = 532e-9, 8e-6
    st = progressive.stage_holograms(obj, z, lam, pitch, 3, None, layer, workers=1)
    assert st.shape == (4, ny, nx)
    ys, xs = fresnel.grid_pixels(ny, nx)
    for j in range(4):
        ref = np.zeros(ny * nx, dtype=np.complex128)
        for d in range(2):
            a_d = np.where(layer == d, obj, 0.0)
            ref += fresnel.direct_sum(block_mean(a_d, 1 << (3 - j)), lam, pitch, z[d], ys, xs,
                                      workers=1)
        assert np.max(np.abs(st[j].ravel() - ref)) <= 1e-9 * max(1.0, np.max(np.abs(ref)))
    full = progressive.hologram(obj, z, lam, pitch, 3, None, layer, workers=1)
    assert np.max(np.abs(st[3] - full)) <= 1e-9 * np.max(np.abs(full))
