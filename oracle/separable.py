"""The same progressive hologram over a rectangular window, evaluated separably (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The Fresnel kernel of Eq. 1 in its paraxial form depends on the lateral offset
only through (dy^2 + dx^2), so it is the product of a y factor and an x factor:

    exp(i pi p^2 (dy^2 + dx^2) / (lambda z)) = k_z(dy) * k_z(dx),
    k_z(m) = exp(i pi p^2 m^2 / (lambda z)).

For one layer the direct 2D sum over points is therefore a product of three
matrices, H[Y, X] = K_y[Y, :] . Ahat . K_x[X, :]^T with K[m, q] = k_z(m - q),
and a window of the hologram needs only the window's rows of K_y and columns
of K_x.  Ahat is the masked reconstruction of the layer (Eq. 3, steps 2-5),
from ``progressive.masked_reconstruction``.  The matrix products are NumPy's
FP64 BLAS; everything else is float64 / complex128.

It computes nothing that ``progressive.hologram`` does not; it is pinned to it
(the direct sum) in the test suite and serves where the direct sum would take
minutes: windows of 2048 x 2048 objects and full 1024 x 1024 holograms.
"""

import numpy as np

from . import fresnel, progressive


def kernel_rows(rows, n, lam, pitch, z):
    """K[r, q] = k_z(rows[r] - q) for q in [0, n), complex128 (len(rows), n)."""
    d = np.asarray(rows, dtype=np.float64)[:, None] - np.arange(n, dtype=np.float64)[None, :]
    th = np.pi * pitch * pitch * (d * d) / (lam * z)
    return np.cos(th) + 1j * np.sin(th)


def windows(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
            thresholds=None, corners=((0, 0),), h=None, w=None, eq1_prefactor=False):
    """Hologram windows [y0:y0+h, x0:x0+w] for every (y0, x0) in ``corners``.

    Each layer's masked reconstruction is formed once and shared by the windows.
    Returns a list of complex128 (h, w) arrays.
    """
    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    outs = []
    for (y0, x0) in corners:
        hh = ny - y0 if h is None else h
        ww = nx - x0 if w is None else w
        outs.append(np.zeros((hh, ww), dtype=np.complex128))
    for d, a_d in enumerate(progressive.layer_split(obj, layer_index, len(z))):
        if not np.any(a_d):
            continue
        a_hat = progressive.masked_reconstruction(a_d, saliency_map, levels, thresholds)
        for (y0, x0), out in zip(corners, outs):
            hh, ww = out.shape
            ky = kernel_rows(np.arange(y0, y0 + hh), ny, lam, pitch, z[d])
            kx = kernel_rows(np.arange(x0, x0 + ww), nx, lam, pitch, z[d])
            # (K_y Ahat) with a real Ahat: two real products (contiguous operands,
            # so that NumPy hands them to BLAS)
            left = (np.ascontiguousarray(ky.real) @ a_hat
                    + 1j * (np.ascontiguousarray(ky.imag) @ a_hat))
            part = left @ np.ascontiguousarray(kx.T)
            if eq1_prefactor:
                part = part * fresnel.prefactor(lam, z[d])
            out += part
    return outs


def window(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
           thresholds=None, y0=0, x0=0, h=None, w=None, eq1_prefactor=False):
    """Hologram window [y0:y0+h, x0:x0+w] of the progressive hologram, complex128 (h, w)."""
    return windows(obj, z, lam, pitch, levels, saliency_map, layer_index, thresholds,
                   corners=((y0, x0),), h=h, w=w, eq1_prefactor=eq1_prefactor)[0]


# ---------------------------------------------------------------- differentiable form, full size
#
# The same chain as ``gradient.loss_and_grad`` (single layer at z, Fresnel
# back-propagation, loss sum (|U| - T)^2), with every 2D kernel sum written as
# matrix products.  The kernel matrix K[m, q] = k_z(m - q) is symmetric, so
#
#   hologram          H   = K_y Ahat K_x^T                      (Ahat real)
#   back-propagation  U   = s conj(K_y)^T H conj(K_x)            s = 1 / (ny nx)
#   loss cotangent    g_U = 2 (|U| - T) U / |U|                  (0 where U = 0)
#   adjoint of U      g_H = s K_y g_U K_x^T
#   back-projection   R   = Re( K_y^T conj(g_H) K_x )
#   gradient          dL/dA = S M W (R)                          (self-adjoint)
#
# where conj(g_H) is the conjugate of the cotangent because the real loss
# depends on H through Re(conj(g_H) dH).  Pinned to the direct-sum chain of
# ``gradient`` on small sides; at 1024 x 1024 it takes seconds.


def full_kernel(n, lam, pitch, z):
    """K[m, q] = k_z(m - q) over a whole side of n pixels, complex128 (n, n)."""
    return kernel_rows(np.arange(n), n, lam, pitch, z)


def loss_and_grad(obj, target, z, lam, pitch, levels=3, saliency_map=None, thresholds=None):
    """(loss, dL/dA, U) of the single-layer reconstruction loss, all in float64."""
    from . import gradient

    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    ky = full_kernel(ny, lam, pitch, z)
    kx = full_kernel(nx, lam, pitch, z)
    a_hat = progressive.masked_reconstruction(obj, saliency_map, levels, thresholds)
    h = (np.ascontiguousarray(ky.real) @ a_hat + 1j * (np.ascontiguousarray(ky.imag) @ a_hat))
    h = h @ np.ascontiguousarray(kx.T)
    s = 1.0 / float(ny * nx)
    u = s * (np.ascontiguousarray(np.conj(ky).T) @ h @ np.conj(kx))
    loss, g_u = gradient.amplitude_loss(u, target)
    g_h = s * (ky @ g_u @ np.ascontiguousarray(kx.T))
    r = np.real(np.ascontiguousarray(ky.T) @ np.conj(g_h) @ kx)
    grad = progressive.masked_reconstruction(r, saliency_map, levels, thresholds)
    return loss, grad, u
