"""Angular-spectrum propagation (oracle; test infrastructure only).

The paper reconstructs its holograms with the inverse angular-spectrum method
at the scene's own parameters (Sec. 2, closing paragraph of the method; the
reconstructions of Fig. 4 and the SSIM of Table 3 come from it).  The angular
spectrum of a sampled field f (ny x nx, pixel pitch p) propagated over a
distance z is (Goodman, Introduction to Fourier Optics, Sec. 3.10)

    U = IDFT2( DFT2(f) * T ),   T(fx, fy) = exp( i 2 pi z sqrt(1/lambda^2 - fx^2 - fy^2) )

with fx = kx / (nx p), kx in [-nx/2, nx/2) in DFT order (likewise fy), and
T = 0 for the evanescent components fx^2 + fy^2 > 1/lambda^2.  The inverse
method, from the hologram plane back to the object plane, is the same
operator with z -> -z.  The sign convention matches the hot path's Fresnel
kernel exp(+i pi r^2 / (lambda z)): propagating a point over +z with this
transfer gives, in the paraxial limit, exactly that chirp (times the constant
exp(i k z) / (i lambda z) and the pixel area), so the hologram of a point
refocuses onto the point under z -> -z.

Readings: the grid is the hologram's own (no zero padding, so the DFT's
periodic wrap-around is part of the operator); DFT2 unnormalised and IDFT2
normalised by 1/(ny nx), as numpy defines them.

Written with numpy's FFT (a library primitive standing for the DFT), complex128.
"""

import numpy as np


def frequencies(n, pitch):
    """Spatial frequencies (cycles per metre) of the n DFT bins, DFT order."""
    k = np.arange(n)
    k = np.where(k < (n + 1) // 2, k, k - n)
    return k / (n * pitch)


def transfer(ny, nx, lam, pitch, z):
    """Angular-spectrum transfer function on the (ny, nx) DFT grid, complex128."""
    fy = frequencies(ny, pitch)[:, None]
    fx = frequencies(nx, pitch)[None, :]
    arg = 1.0 / (lam * lam) - fx * fx - fy * fy
    prop = arg >= 0.0
    phase = 2.0 * np.pi * z * np.sqrt(np.where(prop, arg, 0.0))
    return np.where(prop, np.exp(1j * phase), 0.0)


def propagate(field, lam, pitch, z):
    """Field after free-space propagation over z (metres; negative: backwards)."""
    f = np.asarray(field, dtype=np.complex128)
    ny, nx = f.shape
    return np.fft.ifft2(np.fft.fft2(f) * transfer(ny, nx, lam, pitch, z))


def reconstruct(hologram, lam, pitch, z):
    """Inverse angular-spectrum reconstruction of a hologram recorded at distance z."""
    return propagate(hologram, lam, pitch, -z)
