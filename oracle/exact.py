"""Eq. 1 with the exact distance (oracle; test infrastructure only).

Paper, Sec. 2, Eq. 1: the object wave at hologram pixel (x, y) is the sum over
object points i of A_i / r_i * exp(j k r_i), k = 2 pi / lambda, with r_i the
distance from the point to the pixel.  Reading of the garbled distance term:
the hologram lies in the plane z = 0 and layer d at distance z_d, so

    r = sqrt( pitch^2 ((x - p)^2 + (y - q)^2) + z_d^2 ).

The hot path uses the paraxial (Fresnel) form of this sum; this module
evaluates the exact one, point by point in FP64, so that the error of the
approximation can be measured.  The object whose points are summed is the
same masked reconstruction of each layer as in ``progressive``.
"""

import numpy as np

from . import fresnel, progressive


def direct_sum_exact(amp, lam, pitch, z, ys, xs, block=65536):
    """sum over nonzero points of amp[q, p] / r * exp(i 2 pi r / lambda) at pixels (ys, xs)."""
    amp = np.asarray(amp, dtype=np.float64)
    qs, ps = np.nonzero(amp)
    a = amp[qs, ps]
    qs = qs.astype(np.float64)
    ps = ps.astype(np.float64)
    ys = np.asarray(ys, dtype=np.float64).ravel()
    xs = np.asarray(xs, dtype=np.float64).ravel()
    out = np.zeros(ys.shape[0], dtype=np.complex128)
    if qs.shape[0] == 0:
        return out
    step = max(1, block // qs.shape[0])
    for s in range(0, ys.shape[0], step):
        dy = ys[s:s + step, None] - qs[None, :]
        dx = xs[s:s + step, None] - ps[None, :]
        r = np.sqrt(pitch * pitch * (dx * dx + dy * dy) + z * z)
        th = 2.0 * np.pi * r / lam
        w = a[None, :] / r
        out[s:s + step] = (w * np.cos(th)).sum(axis=1) + 1j * (w * np.sin(th)).sum(axis=1)
    return out


def hologram_exact(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
                   thresholds=None, pixels=None):
    """Exact-distance hologram of the masked reconstruction of every layer, complex128."""
    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    if pixels is None:
        ys, xs = fresnel.grid_pixels(ny, nx)
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    out = np.zeros(ys.shape[0], dtype=np.complex128)
    for d, a_d in enumerate(progressive.layer_split(obj, layer_index, len(z))):
        a_hat = progressive.masked_reconstruction(a_d, saliency_map, levels, thresholds)
        out += direct_sum_exact(a_hat, lam, pitch, z[d], ys, xs)
    return out.reshape(ny, nx) if pixels is None else out
