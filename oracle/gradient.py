"""Adjoint of the progressive hologram and Fresnel back-propagation (oracle).

The paper computes holograms only; the differentiable form is an extension.
Everything here follows from the forward definition in ``progressive`` by the
chain rule, in float64:

Forward, per layer d:  H = sum_d P_d * K_d( Ahat_d ),  Ahat_d = S M W (A * [layer == d])
where K_d is the direct 2D Fresnel sum of Eq. 1 (Fresnel form).

Cotangent convention: for a real loss L of a complex H, the incoming gradient
is G = dL/dRe(H) + i dL/dIm(H).  Then dL/dx = Re( sum conj(G) dH/dx ) for a real
input x, so

    R_d[q, p]      = Re( P_d * sum_{y,x} conj(G[y, x]) * kernel_d(y - q, x - p) )
    dL/dA_d        = (S M W)^T R_d
    dL/dA[q, p]    = dL/dA_d[q, p] with d = layer[q, p].

For the averaging Haar pair, W^T = S * Lambda and S^T = Lambda^-1 * W with
Lambda = diag(4^-l) (l the level of each coefficient), so (S M W)^T = S M W:
the masked reconstruction operator is self-adjoint.  ``grad_object`` uses that
identity; the tests check it against explicit dense transposes.

Fresnel back-propagation (reconstruction on the object plane, single layer at z):

    U[q, p] = 1/(ny*nx) * sum_{y,x} conj(kernel(y - q, x - p)) * H[y, x]

Its adjoint maps g_U to g_H[y, x] = 1/(ny*nx) * sum_{q,p} kernel(y - q, x - p) g_U[q, p].
Loss L = sum (|U| - T)^2 has cotangent g_U = 2 (|U| - T) U / |U| (0 where U = 0).
The paper reconstructs with the angular spectrum method instead; the Fresnel
form keeps the reconstruction on the same kernel as the forward pass.
"""

import numpy as np

from . import fresnel, progressive


def backproject(grad_h, lam, pitch, z, pixels, eq1_prefactor=False, workers=None):
    """R at object pixels ``pixels`` = (qs, ps) for one layer (float64 array)."""
    qs, ps = (np.asarray(v).ravel() for v in pixels)
    r = fresnel.direct_sum(np.conj(np.asarray(grad_h, dtype=np.complex128)), lam, pitch, z,
                           qs, ps, workers=workers)
    if eq1_prefactor:
        r = r * fresnel.prefactor(lam, z)
    return np.real(r)


def grad_object(grad_h, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
                thresholds=None, eq1_prefactor=False, workers=None):
    """Full dL/dA (ny, nx) float64 for cotangent ``grad_h`` (ny, nx complex)."""
    grad_h = np.asarray(grad_h, dtype=np.complex128)
    ny, nx = grad_h.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    qs, ps = fresnel.grid_pixels(ny, nx)
    out = np.zeros((ny, nx), dtype=np.float64)
    for d in range(len(z)):
        r = backproject(grad_h, lam, pitch, z[d], (qs, ps), eq1_prefactor, workers).reshape(ny, nx)
        g_d = progressive.masked_reconstruction(r, saliency_map, levels, thresholds)
        if layer_index is None:
            out += g_d
        else:
            out += np.where(np.asarray(layer_index) == d, g_d, 0.0)
    return out


def grad_object_blocks(grad_h, z, lam, pitch, blocks, levels=3, saliency_map=None,
                       layer_index=None, thresholds=None, eq1_prefactor=False, workers=None):
    """dL/dA on selected 2^levels x 2^levels blocks only.

    The masked reconstruction operator acts within each aligned 2^levels block,
    so the gradient on a block needs R only on that block.  ``blocks`` is a list
    of (by, bx) block indices; returns an array (len(blocks), b, b).
    """
    grad_h = np.asarray(grad_h, dtype=np.complex128)
    b = 1 << levels
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    out = np.zeros((len(blocks), b, b), dtype=np.float64)
    for k, (by, bx) in enumerate(blocks):
        ys, xs = fresnel.grid_pixels(b, b)
        ys = ys + by * b
        xs = xs + bx * b
        sal = None
        if saliency_map is not None:
            sal = np.asarray(saliency_map)[by * b:(by + 1) * b, bx * b:(bx + 1) * b]
        for d in range(len(z)):
            r = backproject(grad_h, lam, pitch, z[d], (ys, xs), eq1_prefactor, workers).reshape(b, b)
            g_d = progressive.masked_reconstruction(r, sal, levels, thresholds)
            if layer_index is None:
                out[k] += g_d
            else:
                li = np.asarray(layer_index)[by * b:(by + 1) * b, bx * b:(bx + 1) * b]
                out[k] += np.where(li == d, g_d, 0.0)
    return out


def fresnel_backpropagate(field, lam, pitch, z, pixels=None, workers=None):
    """U = 1/(ny nx) * conjugate-kernel direct sum of ``field`` (complex)."""
    field = np.asarray(field, dtype=np.complex128)
    ny, nx = field.shape
    if pixels is None:
        qs, ps = fresnel.grid_pixels(ny, nx)
    else:
        qs, ps = (np.asarray(v).ravel() for v in pixels)
    u = np.conj(fresnel.direct_sum(np.conj(field), lam, pitch, z, qs, ps, workers=workers))
    u = u / float(ny * nx)
    return u.reshape(ny, nx) if pixels is None else u


def fresnel_backpropagate_adjoint(grad_u, lam, pitch, z, pixels=None, workers=None):
    """Adjoint of :func:`fresnel_backpropagate` applied to ``grad_u``."""
    grad_u = np.asarray(grad_u, dtype=np.complex128)
    ny, nx = grad_u.shape
    if pixels is None:
        ys, xs = fresnel.grid_pixels(ny, nx)
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    g = fresnel.direct_sum(grad_u, lam, pitch, z, ys, xs, workers=workers) / float(ny * nx)
    return g.reshape(ny, nx) if pixels is None else g


def amplitude_loss(u, target):
    """L = sum (|U| - T)^2 and its cotangent g_U = 2 (|U| - T) U / |U|."""
    u = np.asarray(u, dtype=np.complex128)
    mag = np.abs(u)
    diff = mag - np.asarray(target, dtype=np.float64)
    loss = float(np.sum(diff * diff))
    phase = np.where(mag > 0, u / np.where(mag > 0, mag, 1.0), 0.0)
    return loss, 2.0 * diff * phase


def loss_and_grad(obj, target, z, lam, pitch, levels=3, saliency_map=None, thresholds=None,
                  workers=None):
    """Single-layer reconstruction loss and dL/dA for the differentiable form."""
    h = progressive.hologram(obj, [z], lam, pitch, levels, saliency_map, None, thresholds,
                             workers=workers)
    u = fresnel_backpropagate(h, lam, pitch, z, workers=workers)
    loss, g_u = amplitude_loss(u, target)
    g_h = fresnel_backpropagate_adjoint(g_u, lam, pitch, z, workers=workers)
    grad = grad_object(g_h, [z], lam, pitch, levels, saliency_map, None, thresholds,
                       workers=workers)
    return loss, grad
