"""Progressive saliency-guided hologram, plain definition (oracle).

Paper, Sec. 2: by linearity (Eq. 3) the hologram of an object is the sum of the
holograms of its Haar basis functions times their coefficients.  Steps 2-5 keep
the level-3 approximation for every block and add the detail ("residual map")
contribution of level l only where the quantised saliency exceeds that level's
threshold.  The 3D extension splits the scene into depth layers, each with its
own fringe (Sec. 2, last paragraph).

The result is, exactly, the Fresnel hologram of a masked reconstruction of each
layer, which is what this module computes:

    A_d    = A * [layer == d]                      (pixel-exact layer split)
    Ahat_d = S( M (.) W(A_d) )                     (W analysis, S synthesis, M masks)
    H      = sum_d P_d * sum_points Ahat_d[q, p] * kernel_d(y - q, x - p)

with P_d = 1, or exp(i k z_d) / z_d when the Eq. 1 prefactor is requested.
The same saliency masks apply to every layer.  Inputs are promoted to float64.
"""

import numpy as np

from . import fresnel, haar, saliency


def masked_reconstruction(amp, sal, levels, thresholds=None):
    """Ahat = S(M (.) W(amp)); ``sal`` None means every block is salient."""
    amp = np.asarray(amp, dtype=np.float64)
    c = haar.analysis(amp, levels)
    if sal is not None:
        masks = saliency.detail_masks(sal, levels, thresholds)
        c = saliency.apply_masks(c, masks, levels)
    return haar.synthesis(c, levels)


def stage_reconstruction(amp, sal, levels, stage, thresholds=None):
    """Object of progressive stage ``stage`` (0..levels) of one layer.

    Sec. 2, steps 2-5, and the progressive display of Sec. 3: stage 0 shows the
    coarsest approximation alone (every block, step 2); stage j adds the salient
    details of levels levels, levels-1, ..., levels-j+1 (steps 3-5 in order), so
    stage ``levels`` is ``masked_reconstruction``.
    """
    amp = np.asarray(amp, dtype=np.float64)
    c = haar.analysis(amp, levels)
    if sal is not None:
        masks = saliency.detail_masks(sal, levels, thresholds)
    else:
        masks = [np.ones((amp.shape[0] >> l, amp.shape[1] >> l), dtype=bool)
                 for l in range(1, levels + 1)]
    masks = [m if l > levels - stage else np.zeros_like(m)
             for l, m in zip(range(1, levels + 1), masks)]
    c = saliency.apply_masks(c, masks, levels)
    return haar.synthesis(c, levels)


def layer_split(obj, layer_index, n_layers):
    obj = np.asarray(obj, dtype=np.float64)
    if layer_index is None:
        return [obj]
    li = np.asarray(layer_index)
    return [np.where(li == d, obj, 0.0) for d in range(n_layers)]


def hologram(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
             thresholds=None, pixels=None, eq1_prefactor=False, workers=None):
    """Progressive hologram of ``obj`` (ny, nx), complex128.

    ``z`` is a sequence of layer distances (metres); ``layer_index`` maps each
    pixel to a layer (None: all pixels in layer 0).  ``pixels`` is None for the
    full (ny, nx) hologram, or a pair (ys, xs) of coordinate arrays, in which
    case a flat array of those pixel values is returned.
    """
    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    if pixels is None:
        ys, xs = fresnel.grid_pixels(ny, nx)
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    out = np.zeros(ys.shape[0], dtype=np.complex128)
    for d, a_d in enumerate(layer_split(obj, layer_index, len(z))):
        a_hat = masked_reconstruction(a_d, saliency_map, levels, thresholds)
        part = fresnel.direct_sum(a_hat, lam, pitch, z[d], ys, xs, workers=workers)
        if eq1_prefactor:
            part = part * fresnel.prefactor(lam, z[d])
        out += part
    if pixels is None:
        return out.reshape(ny, nx)
    return out


def stage_holograms(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
                    thresholds=None, pixels=None, eq1_prefactor=False, workers=None):
    """The levels + 1 cumulative stage holograms (see ``stage_reconstruction``).

    Returns complex128 of shape (levels + 1, ny, nx), or (levels + 1, len(ys))
    when ``pixels`` is given.
    """
    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    if pixels is None:
        ys, xs = fresnel.grid_pixels(ny, nx)
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    out = np.zeros((levels + 1, ys.shape[0]), dtype=np.complex128)
    for d, a_d in enumerate(layer_split(obj, layer_index, len(z))):
        for j in range(levels + 1):
            a_hat = stage_reconstruction(a_d, saliency_map, levels, j, thresholds)
            part = fresnel.direct_sum(a_hat, lam, pitch, z[d], ys, xs, workers=workers)
            if eq1_prefactor:
                part = part * fresnel.prefactor(lam, z[d])
            out[j] += part
    if pixels is None:
        return out.reshape(levels + 1, ny, nx)
    return out


def full_hologram(obj, z, lam, pitch, layer_index=None, pixels=None, eq1_prefactor=False,
                  workers=None):
    """The fully point-wise hologram (every point with its own 1x1 fringe)."""
    obj = np.asarray(obj, dtype=np.float64)
    ny, nx = obj.shape
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    if pixels is None:
        ys, xs = fresnel.grid_pixels(ny, nx)
    else:
        ys, xs = (np.asarray(v).ravel() for v in pixels)
    out = np.zeros(ys.shape[0], dtype=np.complex128)
    for d, a_d in enumerate(layer_split(obj, layer_index, len(z))):
        part = fresnel.direct_sum(a_d, lam, pitch, z[d], ys, xs, workers=workers)
        if eq1_prefactor:
            part = part * fresnel.prefactor(lam, z[d])
        out += part
    if pixels is None:
        return out.reshape(ny, nx)
    return out


def rel_l2(approx, exact):
    """||approx - exact||_2 / ||exact||_2 over all given entries (complex)."""
    approx = np.asarray(approx, dtype=np.complex128)
    exact = np.asarray(exact, dtype=np.complex128)
    den = np.linalg.norm(exact.ravel())
    num = np.linalg.norm((approx - exact).ravel())
    return float(num / den) if den > 0 else float(num)
