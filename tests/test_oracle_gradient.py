"""Pins of the oracle's adjoint, Fresnel back-propagation and loss gradient.

No GPU.  Checks: explicit dense transposes of the linear maps, the dot-product
(adjoint) identity, central finite differences of the full loss chain, and the
closed-form back-propagation of a zone plate (a geometric series).
"""

import numpy as np
import pytest

from oracle import gradient, haar, progressive, saliency
from paper_2211_09938_amd import scenes

LAM, PITCH = 532e-9, 8e-6


def _dense(op, n_in_shape):
    n = int(np.prod(n_in_shape))
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(np.asarray(op(e.reshape(n_in_shape))).ravel())
    return np.array(cols).T


def test_masked_reconstruction_is_self_adjoint_and_matches_transposes():
    ny, nx = 16, 8
    sal = (np.random.default_rng(1).random((ny, nx)) > 0.6).astype(float)
    masks = saliency.detail_masks(sal, 3)
    W = _dense(lambda a: haar.analysis(a, 3), (ny, nx))
    S = _dense(lambda c: haar.synthesis(c, 3), (ny, nx))
    M = np.diag(saliency.apply_masks(np.ones((ny, nx)), masks, 3).ravel())
    P = _dense(lambda a: progressive.masked_reconstruction(a, sal, 3), (ny, nx))
    assert np.allclose(P, S @ M @ W, atol=1e-14)
    assert np.allclose(P, P.T, atol=1e-14)
    assert np.allclose(W.T @ M @ S.T, P, atol=1e-14)


def test_backward_satisfies_dot_product_identity():
    rng = np.random.default_rng(2)
    ny, nx = 16, 16
    z = [0.03, 0.06]
    layer = (rng.random((ny, nx)) > 0.5).astype(np.uint8)
    sal = (rng.random((ny, nx)) > 0.5).astype(float)
    a = rng.random((ny, nx))
    g = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    h = progressive.hologram(a, z, LAM, PITCH, 3, sal, layer, eq1_prefactor=True)
    ga = gradient.grad_object(g, z, LAM, PITCH, 3, sal, layer, eq1_prefactor=True)
    lhs = np.real(np.vdot(g, h))          # Re <G, H> = dL/dA . A for the linear loss
    rhs = float(np.sum(ga * a))
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_block_gradient_equals_full_gradient():
    rng = np.random.default_rng(3)
    ny, nx = 16, 24
    z = [0.03, 0.05]
    layer = (rng.random((ny, nx)) > 0.5).astype(np.uint8)
    sal = (rng.random((ny, nx)) > 0.4).astype(float)
    g = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    full = gradient.grad_object(g, z, LAM, PITCH, 3, sal, layer)
    blocks = [(0, 0), (1, 2), (0, 1)]
    part = gradient.grad_object_blocks(g, z, LAM, PITCH, blocks, 3, sal, layer)
    for k, (by, bx) in enumerate(blocks):
        assert np.allclose(part[k], full[by * 8:(by + 1) * 8, bx * 8:(bx + 1) * 8], atol=1e-12)


def test_loss_gradient_matches_central_finite_differences():
    s = scenes.random_scene(4, 32, 32, fraction=0.3)
    target = scenes.blobs(np.random.default_rng(40), 32, 32, 4, sigma_px=(2, 5), scale_ref=32)
    obj = s.obj.astype(np.float64)
    z = 0.02
    loss, grad = gradient.loss_and_grad(obj, target, z, LAM, PITCH, 3, s.saliency, workers=1)

    def f(a):
        h = progressive.hologram(a, [z], LAM, PITCH, 3, s.saliency, workers=1)
        u = gradient.fresnel_backpropagate(h, LAM, PITCH, z, workers=1)
        return gradient.amplitude_loss(u, target)[0]

    h = 1e-6
    rng = np.random.default_rng(5)
    for k in rng.choice(32 * 32, 10, replace=False):
        e = np.zeros(32 * 32)
        e[k] = h
        e = e.reshape(32, 32)
        fd = (f(obj + e) - f(obj - e)) / (2 * h)
        assert fd == pytest.approx(grad.ravel()[k], rel=1e-5, abs=1e-9 * abs(loss))
    for _ in range(2):
        v = rng.standard_normal((32, 32))
        fd = (f(obj + h * v) - f(obj - h * v)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(grad * v)), rel=1e-6)


def test_backpropagated_zone_plate_is_a_geometric_series():
    ny, nx = 16, 24
    z = 0.05
    q0, p0 = 5, 17
    a = np.zeros((ny, nx))
    a[q0, p0] = 1.0
    h = progressive.full_hologram(a, [z], LAM, PITCH)
    u = gradient.fresnel_backpropagate(h, LAM, PITCH, z)
    c = np.pi * PITCH ** 2 / (LAM * z)

    def series(n, m0, m):
        # sum_y exp(i c ((y - m0)^2 - (y - m)^2)) = exp(i c (m0^2 - m^2)) sum_y exp(2 i c y (m - m0))
        theta = 2 * c * (m - m0)
        pre = np.exp(1j * c * (m0 * m0 - m * m))
        if abs(np.exp(1j * theta) - 1) < 1e-15:
            return pre * n
        return pre * (np.exp(1j * theta * n) - 1) / (np.exp(1j * theta) - 1)

    ref = np.array([[series(ny, q0, q) * series(nx, p0, p) for p in range(nx)] for q in range(ny)])
    ref /= ny * nx
    assert u[q0, p0] == pytest.approx(1.0, abs=1e-12)
    assert np.max(np.abs(u - ref)) < 1e-12


def test_backpropagation_adjoint_identity():
    rng = np.random.default_rng(6)
    ny, nx = 12, 16
    hf = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    gu = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    u = gradient.fresnel_backpropagate(hf, LAM, PITCH, 0.04)
    gh = gradient.fresnel_backpropagate_adjoint(gu, LAM, PITCH, 0.04)
    assert np.real(np.vdot(gu, u)) == pytest.approx(np.real(np.vdot(gh, hf)), rel=1e-12)
