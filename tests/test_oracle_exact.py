"""Pins of the exact-distance Eq. 1 sum (oracle/exact.py).

* on axis, one point of unit amplitude gives exp(i k z) / z (closed form);
* far from a small object, the exact sum tends to the paraxial one times the
  constant exp(i k z) / z: at z = 2 m and a 12-pixel object the phase of the
  next term of the expansion, k rho^4 / (8 z^3), is below 1e-9 rad, so the
  two agree to 1e-7 relative;
* at a short distance they differ by an amount the next term predicts;
* mirror symmetry of a symmetric object.
"""

import numpy as np

from oracle import exact, fresnel, progressive

LAM, PITCH = 532e-9, 8e-6


def test_on_axis_point_is_spherical_wave_constant():
    amp = np.zeros((8, 8))
    amp[3, 5] = 1.0
    z = 0.173
    v = exact.direct_sum_exact(amp, LAM, PITCH, z, [3], [5])
    assert abs(v[0] - np.exp(2j * np.pi * z / LAM) / z) <= 1e-12 / z


def test_far_field_tends_to_paraxial_form():
    rng = np.random.default_rng(3)
    amp = rng.uniform(0, 1, (12, 12))
    z = 2.0
    ys, xs = fresnel.grid_pixels(12, 12)
    ex = exact.direct_sum_exact(amp, LAM, PITCH, z, ys, xs)
    par = fresnel.direct_sum(amp, LAM, PITCH, z, ys, xs, workers=1) * fresnel.prefactor(LAM, z)
    assert progressive.rel_l2(ex, par) <= 1e-7


def test_near_field_difference_matches_next_term():
    # one point: exact phase - paraxial phase = k (r - z - rho^2 / (2z)) ~ -k rho^4 / (8 z^3)
    amp = np.zeros((1, 64))
    amp[0, 0] = 1.0
    z = 0.02
    xs = np.arange(64)
    ex = exact.direct_sum_exact(amp, LAM, PITCH, z, np.zeros(64), xs)
    par = fresnel.direct_sum(amp, LAM, PITCH, z, np.zeros(64), xs, workers=1) * fresnel.prefactor(LAM, z)
    rho = PITCH * xs
    k = 2 * np.pi / LAM
    dphi = np.angle(ex / par)
    pred = -k * rho ** 4 / (8 * z ** 3)
    big = np.abs(pred) > 1e-3
    assert np.all(np.abs(dphi[big] - pred[big]) <= 0.05 * np.abs(pred[big]))
    assert np.max(np.abs(np.abs(ex) * np.sqrt(z * z + rho ** 2) - 1.0)) <= 1e-12


def test_mirror_symmetry():
    rng = np.random.default_rng(4)
    half = rng.uniform(0, 1, (8, 4))
    amp = np.concatenate([half, half[:, ::-1]], axis=1)  # symmetric about the column centre
    ys, xs = fresnel.grid_pixels(8, 8)
    v = exact.direct_sum_exact(amp, LAM, PITCH, 0.05, ys, xs).reshape(8, 8)
    assert np.max(np.abs(v - v[:, ::-1])) <= 1e-9 * np.max(np.abs(v))


def test_hologram_exact_uses_the_masked_reconstruction():
    rng = np.random.default_rng(5)
    obj = rng.uniform(0, 1, (16, 16))
    sal = np.zeros((16, 16))
    sal[2:6, 9:13] = 1.0
    h = exact.hologram_exact(obj, (0.1,), LAM, PITCH, 3, sal)
    a_hat = progressive.masked_reconstruction(obj, sal, 3)
    ys, xs = fresnel.grid_pixels(16, 16)
    ref = exact.direct_sum_exact(a_hat, LAM, PITCH, 0.1, ys, xs).reshape(16, 16)
    assert np.array_equal(h, ref)
