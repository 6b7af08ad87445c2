"""GPU parity of the angular-spectrum propagation (cgh_angular_spectrum), the
inverse method the paper reconstructs its holograms with.

Bar: rel-L2 <= 1e-5 against the FP64 oracle (oracle/angular.py) for every side
form the kernels take (2^a and 3 * 2^a, 2 to 4096, both FFT directions through
the forward and inverse distances), in place, with evanescent bins, at the full
2048^2 and the maximum 4096^2; and the refocus of the hot path's point hologram.
Inputs are seeded: white complex noise, unit-modulus random-phase fields
(hologram-like), and the oracle's own point hologram.
"""

import numpy as np
import pytest

from oracle import angular, progressive

from helpers import rel_l2

pytestmark = pytest.mark.gpu
LAM, PITCH = 532e-9, 8e-6


def run(f, lam, pitch, z, inplace=False):
    import torch

    from paper_2211_09938_amd import cgh

    t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.complex64)).cuda()
    out = cgh.angular_spectrum(t, lam, pitch, z, out=t if inplace else None)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


def noise(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("shape,z", [
    ((2, 4), 0.1), ((3, 6), -0.05), ((8, 8), 0.2), ((12, 48), -0.2), ((96, 64), 0.15),
    ((256, 256), -0.2), ((768, 1536), 0.2), ((4096, 64), -0.1), ((64, 4096), 0.1),
    ((3072, 24), 0.3),
])
def test_matches_oracle(shape, z):
    f = noise(shape, shape[0] * 7919 + shape[1])
    got = run(f, LAM, PITCH, z)
    ref = angular.propagate(f.astype(np.complex128), LAM, PITCH, z)
    err = rel_l2(got, ref)
    print(shape, z, "rel-L2 %.2e" % err)
    assert err <= 1e-5


def test_in_place_equals_out_of_place_and_round_trip():
    f = noise((192, 128), 5)
    a = run(f, LAM, PITCH, 0.2)
    b = run(f, LAM, PITCH, 0.2, inplace=True)
    assert np.array_equal(a, b)
    back = run(a.astype(np.complex64), LAM, PITCH, -0.2)
    assert rel_l2(back, f.astype(np.complex128)) <= 1e-5


def test_evanescent_bins():
    pitch = 0.2e-6
    f = noise((32, 48), 9)
    got = run(f, LAM, pitch, 2e-6)
    assert rel_l2(got, angular.propagate(f.astype(np.complex128), LAM, pitch, 2e-6)) <= 1e-5
    y, x = np.mgrid[0:16, 0:16]
    wave = np.exp(2j * np.pi * (7 * y / 16 + 7 * x / 16))  # an evanescent bin
    assert np.max(np.abs(run(wave, LAM, pitch, 1e-6))) <= 1e-6


@pytest.mark.parametrize("n", [2048, 4096])
def test_full_size_random_phase(n):
    rng = np.random.default_rng(n)
    f = np.exp(2j * np.pi * rng.random((n, n))).astype(np.complex64)
    got = run(f, LAM, PITCH, -0.2)
    err = rel_l2(got, angular.propagate(f.astype(np.complex128), LAM, PITCH, -0.2))
    print(n, "rel-L2 %.2e" % err)
    assert err <= 1e-5


def test_point_hologram_refocuses():
    n, q0, p0 = 64, 37, 12
    z = n * PITCH * PITCH / LAM
    obj = np.zeros((n, n))
    obj[q0, p0] = 1.0
    h = progressive.hologram(obj, (z,), LAM, PITCH, 3, workers=1)
    from paper_2211_09938_amd import cgh
    import torch

    t = torch.from_numpy(h.astype(np.complex64)).cuda()
    u = cgh.reconstruct(t, LAM, PITCH, z).cpu().numpy().astype(np.complex128)
    assert rel_l2(u, angular.reconstruct(h.astype(np.complex64), LAM, PITCH, z)) <= 1e-5
    a = np.abs(u)
    s = LAM * LAM / (2 * PITCH * PITCH)
    phi = 2 * np.pi * (z / LAM) * s * s / 8 / (1 - s)
    assert np.unravel_index(np.argmax(a), a.shape) == (q0, p0)
    assert a[q0, p0] ** 2 >= (1 - phi * phi) * n * n * (1 - 1e-5)
