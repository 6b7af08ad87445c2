"""Pins of the angular-spectrum oracle (oracle/angular.py).

* brute force: on small grids (odd and even sides) the FFT form equals the
  DFT written out as explicit double sums over pixels and frequencies;
* paraxial limit: the transfer phase differs from 2 pi z / lambda -
  pi lambda z (fx^2 + fy^2) by its next expansion term, -2 pi (z / lambda) s^2 / 8,
  s = lambda^2 (fx^2 + fy^2) (a dropped term, wrong sign or a wrong frequency
  scale shows there);
* evanescent components are cut: |T| = 0 beyond 1 / lambda, 1 inside;
* group and inverse laws, z = 0 identity, Parseval;
* refocus: at z = N pitch^2 / lambda the Fresnel chirp of the hot path's
  point hologram is N-periodic and the inverse method turns it back into the
  point, up to the energy that the non-paraxial phase remainder phi of the
  transfer can move (at most phi^2 of it).
"""

import numpy as np
import pytest

from oracle import angular, progressive

LAM, PITCH = 532e-9, 8e-6


def brute(field, lam, pitch, z):
    f = np.asarray(field, dtype=np.complex128)
    ny, nx = f.shape
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    out = np.zeros_like(f)
    t = angular.transfer(ny, nx, lam, pitch, z)
    for ky in range(ny):
        for kx in range(nx):
            e = np.exp(-2j * np.pi * (ky * y / ny + kx * x / nx))
            g = np.sum(f * e) * t[ky, kx]
            out += g * np.conj(e)
    return out / (ny * nx)


@pytest.mark.parametrize("shape,z", [((5, 6), 0.01), ((8, 7), -0.003), ((6, 12), 0.2)])
def test_fft_form_equals_explicit_dft(shape, z):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    pitch = 2e-6
    got = angular.propagate(f, LAM, pitch, z)
    assert np.max(np.abs(got - brute(f, LAM, pitch, z))) <= 1e-12 * np.max(np.abs(got))


def test_frequencies_follow_dft_order():
    assert np.allclose(angular.frequencies(6, 1.0), np.fft.fftfreq(6))
    assert np.allclose(angular.frequencies(7, 0.5), np.fft.fftfreq(7, 0.5))


@pytest.mark.parametrize("z", [0.2, -0.05])
def test_transfer_paraxial_limit(z):
    ny, nx = 64, 48
    t = angular.transfer(ny, nx, LAM, PITCH, z)
    fy = np.fft.fftfreq(ny, PITCH)[:, None]
    fx = np.fft.fftfreq(nx, PITCH)[None, :]
    f2 = fx * fx + fy * fy
    parax = np.exp(1j * (2 * np.pi * z / LAM - np.pi * LAM * z * f2))
    s = LAM * LAM * f2
    rest = np.angle(t * np.conj(parax))
    want = -2 * np.pi * (z / LAM) * s * s / 8
    assert np.all(np.abs(rest - want) <= 0.05 * np.abs(want) + 1e-9)
    assert np.max(np.abs(want)) > 1e-3  # the term is visible at these sizes


def test_evanescent_components_are_cut():
    pitch = 0.2e-6  # bins reach 1 / (2 pitch) = 2.5e6 / m > 1 / lambda
    ny, nx = 16, 16
    t = angular.transfer(ny, nx, LAM, pitch, 1e-6)
    fy = np.fft.fftfreq(ny, pitch)[:, None]
    fx = np.fft.fftfreq(nx, pitch)[None, :]
    ev = fx * fx + fy * fy > 1.0 / LAM ** 2
    assert ev.any() and (~ev).any()
    assert np.all(t[ev] == 0)
    assert np.allclose(np.abs(t[~ev]), 1.0, atol=1e-14)
    y, x = np.mgrid[0:ny, 0:nx]
    wave = np.exp(2j * np.pi * (7 * y / ny + 7 * x / nx))  # an evanescent bin
    assert ev[7, 7]
    assert np.max(np.abs(angular.propagate(wave, LAM, pitch, 1e-6))) <= 1e-12


def test_group_inverse_identity_and_parseval():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((32, 40)) + 1j * rng.standard_normal((32, 40))
    z1, z2 = 0.07, 0.13
    a = angular.propagate(angular.propagate(f, LAM, PITCH, z1), LAM, PITCH, z2)
    b = angular.propagate(f, LAM, PITCH, z1 + z2)
    # FP64 rounds the transfer phase 2 pi z / lambda (about 2.4e6 rad) to ~3e-10
    assert progressive.rel_l2(a, b) <= 1e-9
    back = angular.reconstruct(angular.propagate(f, LAM, PITCH, 0.2), LAM, PITCH, 0.2)
    assert progressive.rel_l2(back, f) <= 1e-9
    assert progressive.rel_l2(angular.propagate(f, LAM, PITCH, 0.0), f) <= 1e-14
    g = angular.propagate(f, LAM, PITCH, 0.3)
    assert abs(np.sum(np.abs(g) ** 2) / np.sum(np.abs(f) ** 2) - 1) <= 1e-12


@pytest.mark.parametrize("q0,p0,pitch", [(20, 41, PITCH), (0, 63, PITCH), (33, 5, 32e-6)])
def test_point_hologram_refocuses_onto_the_point(q0, p0, pitch):
    n = 64
    z = n * pitch * pitch / LAM
    obj = np.zeros((n, n))
    obj[q0, p0] = 1.0
    # the hot path's hologram of one point (every detail kept)
    h = progressive.hologram(obj, (z,), LAM, pitch, 3, workers=1)
    # at this distance the chirp exp(i pi m^2 / n) is n-periodic: the hologram
    # is exactly the periodic field the DFT sees
    yy, xx = np.mgrid[0:n, 0:n]
    dy = (yy - q0 + n // 2) % n - n // 2
    dx = (xx - p0 + n // 2) % n - n // 2
    hp = np.exp(1j * np.pi * pitch ** 2 * (dy ** 2 + dx ** 2) / (LAM * z))
    assert np.max(np.abs(hp - h)) <= 1e-9
    # its DFT is G exp(-i pi (ky^2 + kx^2) / n), |G| = n, which the paraxial
    # inverse transfer cancels exactly; the true transfer leaves a phase
    # remainder below phi = 2 pi (z / lambda) s^2 / 8 / (1 - s) at the corner
    # bin s = lambda^2 / (2 pitch^2), so at most phi^2 of the energy leaves the point
    s = LAM * LAM / (2 * pitch * pitch)
    phi = 2 * np.pi * (z / LAM) * s * s / 8 / (1 - s)
    u = angular.reconstruct(h, LAM, pitch, z)
    a = np.abs(u)
    assert np.unravel_index(np.argmax(a), a.shape) == (q0, p0)
    assert abs(np.sum(a * a) - n * n) <= 1e-9 * n * n
    assert a[q0, p0] ** 2 >= (1 - phi * phi) * n * n
    assert phi < (0.06 if pitch == PITCH else 4e-3)
