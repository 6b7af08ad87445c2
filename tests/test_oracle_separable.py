"""Pins of the separable window evaluation (oracle/separable.py).

It must equal the direct 2D point sum (oracle/progressive.py, itself pinned to
closed forms in test_oracle_hologram.py) on small scenes, for windows that do
not start at the origin, non-square objects, several layers, graded saliency
and the Eq. 1 prefactor; and it must reproduce the analytic zone plate of a
single point far from the window.
"""

import numpy as np
import pytest

from oracle import progressive, separable
from paper_2211_09938_amd import scenes


def direct_window(s, y0, x0, h, w, **kw):
    ys, xs = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    sal = None if s.saliency is None else s.saliency.astype(np.float64)
    v = progressive.hologram(s.obj.astype(np.float64), s.z, s.lam, s.pitch, s.levels, sal,
                             s.layer, pixels=(ys.ravel(), xs.ravel()), workers=1, **kw)
    return v.reshape(h, w)


@pytest.mark.parametrize("shape,planes,win", [
    ((40, 48), 1, (0, 0, 40, 48)),
    ((40, 48), 2, (8, 5, 17, 30)),
    ((64, 32), 3, (31, 0, 33, 32)),
])
def test_window_equals_direct_sum(shape, planes, win):
    s = scenes.random_scene(71 + planes, *shape, planes=planes, fraction=0.3)
    y0, x0, h, w = win
    got = separable.window(s.obj, s.z, s.lam, s.pitch, s.levels, s.saliency.astype(np.float64),
                           s.layer, y0=y0, x0=x0, h=h, w=w)
    ref = direct_window(s, y0, x0, h, w)
    assert progressive.rel_l2(got, ref) <= 1e-12


def test_window_with_thresholds_and_prefactor_equals_direct_sum():
    rng = np.random.default_rng(5)
    s = scenes.random_scene(90, 48, 40, planes=2, fraction=None)
    s.saliency = rng.uniform(0.0, 1.0, s.obj.shape).astype(np.float32)
    th = (0.8, 0.4, 0.2)
    got = separable.window(s.obj, s.z, s.lam, s.pitch, 3, s.saliency.astype(np.float64), s.layer,
                           thresholds=th, y0=3, x0=7, h=20, w=11, eq1_prefactor=True)
    ref = direct_window(s, 3, 7, 20, 11, thresholds=th, eq1_prefactor=True)
    assert progressive.rel_l2(got, ref) <= 1e-12


def test_single_point_far_window_is_the_zone_plate():
    # all-salient single point: the hologram is the sampled chirp itself (|H| = 1)
    ny, nx, q0, p0, z = 96, 80, 70, 9, 0.15
    obj = np.zeros((ny, nx))
    obj[q0, p0] = 1.0
    got = separable.window(obj, (z,), scenes.WAVELENGTH, scenes.PITCH, 3, None, None,
                           y0=0, x0=40, h=24, w=40)
    yy, xx = np.meshgrid(np.arange(0, 24), np.arange(40, 80), indexing="ij")
    th = np.pi * scenes.PITCH ** 2 * ((yy - q0) ** 2 + (xx - p0) ** 2) / (scenes.WAVELENGTH * z)
    assert np.max(np.abs(got - np.exp(1j * th))) <= 1e-12


def test_several_windows_share_one_reconstruction():
    s = scenes.random_scene(77, 48, 64, planes=2, fraction=0.3)
    sal = s.saliency.astype(np.float64)
    corners = [(0, 0), (10, 33), (32, 48)]
    ws = separable.windows(s.obj, s.z, s.lam, s.pitch, 3, sal, s.layer, corners=corners, h=16, w=16)
    for (y0, x0), got in zip(corners, ws):
        assert progressive.rel_l2(got, direct_window(s, y0, x0, 16, 16)) <= 1e-12


@pytest.mark.parametrize("shape,levels,fraction", [((32, 32), 3, 0.3), ((24, 40), 2, 0.5),
                                                  ((48, 16), 3, None)])
def test_separable_loss_chain_equals_direct_sum_chain(shape, levels, fraction):
    # the full-size chain (products of kernel matrices) against the chain of direct
    # 2D sums in oracle.gradient, itself pinned by central finite differences
    from oracle import gradient

    s = scenes.random_scene(510 + shape[0], *shape, fraction=fraction, levels=levels)
    target = scenes.blobs(np.random.default_rng(41), *shape, 4, sigma_px=(2, 5), scale_ref=32)
    sal = None if s.saliency is None else s.saliency.astype(np.float64)
    ref_loss, ref_grad = gradient.loss_and_grad(s.obj.astype(np.float64), target, s.z[0], s.lam,
                                                s.pitch, levels, sal, workers=1)
    loss, grad, u = separable.loss_and_grad(s.obj.astype(np.float64), target, s.z[0], s.lam,
                                            s.pitch, levels, sal)
    assert loss == pytest.approx(ref_loss, rel=1e-12)
    assert progressive.rel_l2(grad, ref_grad) <= 1e-12
    ref_u = gradient.fresnel_backpropagate(
        progressive.hologram(s.obj.astype(np.float64), s.z, s.lam, s.pitch, levels, sal,
                             workers=1), s.lam, s.pitch, s.z[0], workers=1)
    assert progressive.rel_l2(u, ref_u) <= 1e-12
