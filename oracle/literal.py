"""Paper-literal progressive hologram and operator accounting (oracle).

This is a second, independent form of the progressive hologram, written the way
algorithm steps 2-5 of Sec. 2 describe it, in the image domain:

* step 2: every point of the coarsest approximation image (the 2^L x 2^L block
  means) fetches the fringe of a uniform 2^L x 2^L block of unit points, shifts
  it to the block position, multiplies by the point's intensity and adds it to
  the hologram plane;
* steps 3-5: the residual map between two consecutive approximation levels
  (finer image minus the coarser one replicated 2x2) is processed the same way
  with half-size block fringes, but only where the level's quantised saliency
  mask is set (mask expanded 2x2 to the residual's resolution).

The block fringes are a look-up table computed with Eq. 1 in its Fresnel form
(the hologram of one uniform b x b block at the origin, over every offset of the
plane).  An *operator* is one multiply + shift + add of such a block fringe
(Sec. 3).  At 256 x 256 the coarsest step costs (256/8)^2 = 1024 operators and a
fully point-wise hologram N*M = 65,536 (Sec. 3).

Approximation images here are block means (reshape + mean), not the Haar
recursion of ``haar``, so the two forms share no arithmetic.
"""

import numpy as np

from . import fresnel, saliency


def block_mean(img, b):
    ny, nx = img.shape
    return img.reshape(ny // b, b, nx // b, b).mean(axis=(1, 3))


def replicate2(img):
    return np.repeat(np.repeat(img, 2, axis=0), 2, axis=1)


def block_fringe(b, ny, nx, lam, pitch, z):
    """Fringe of a uniform b x b block of unit points with its corner at (0, 0).

    Returned over offsets dy in [-(ny-b), ny-1], dx in [-(nx-b), nx-1];
    element [dy + ny - b, dx + nx - b].
    """
    dys = np.arange(-(ny - b), ny)
    dxs = np.arange(-(nx - b), nx)
    out = np.zeros((dys.size, dxs.size), dtype=np.complex128)
    for u in range(b):
        for v in range(b):
            out += fresnel.kernel_2d(dys[:, None] - u, dxs[None, :] - v, lam, pitch, z)
    return out


def _add_blocks(holo, values, b, lut):
    """H += value * shift(LUT_b) for every nonzero entry of ``values``."""
    ny, nx = holo.shape
    for (j, i) in zip(*np.nonzero(values)):
        y0, x0 = j * b, i * b
        # offset (y - y0) for y in [0, ny) lands at index y - y0 + ny - b
        holo += values[j, i] * lut[ny - b - y0: 2 * ny - b - y0, nx - b - x0: 2 * nx - b - x0]


def layer_hologram_literal(amp, lam, pitch, z, levels, sal, thresholds=None):
    """Returns (hologram, ops) for one depth layer; ops[0] is step 2, then steps 3.. ."""
    amp = np.asarray(amp, dtype=np.float64)
    ny, nx = amp.shape
    masks = None
    if sal is not None:
        masks = saliency.detail_masks(sal, levels, thresholds)
    holo = np.zeros((ny, nx), dtype=np.complex128)
    ops = []
    top = 1 << levels
    coarse = block_mean(amp, top)
    _add_blocks(holo, coarse, top, block_fringe(top, ny, nx, lam, pitch, z))
    ops.append(coarse.size)
    for level in range(levels, 0, -1):
        b = 1 << (level - 1)
        finer = block_mean(amp, b) if b > 1 else amp
        resid = finer - replicate2(block_mean(amp, 1 << level))
        keep = np.ones(resid.shape, dtype=bool) if masks is None else replicate2(masks[level - 1])
        _add_blocks(holo, np.where(keep, resid, 0.0), b, block_fringe(b, ny, nx, lam, pitch, z))
        ops.append(int(keep.sum()))
    return holo, ops


def hologram_literal(obj, z, lam, pitch, levels=3, saliency_map=None, layer_index=None,
                     thresholds=None):
    """Multi-layer sum of :func:`layer_hologram_literal`; returns (H, ops per layer)."""
    obj = np.asarray(obj, dtype=np.float64)
    z = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    layers = [obj] if layer_index is None else [np.where(np.asarray(layer_index) == d, obj, 0.0)
                                                for d in range(len(z))]
    holo = np.zeros(obj.shape, dtype=np.complex128)
    all_ops = []
    for d, a_d in enumerate(layers):
        h, ops = layer_hologram_literal(a_d, lam, pitch, z[d], levels, saliency_map, thresholds)
        holo += h
        all_ops.append(ops)
    return holo, all_ops


def operator_counts(ny, nx, levels, saliency_map=None, thresholds=None):
    """Per-step operator counts (step 2 first) and their running totals.

    Counts follow the paper's accounting: one operator per processed point of
    the approximation image (all of them), then one per point of each residual
    map where the level's mask is set.  Also returns the point-wise count ny*nx.
    """
    top = 1 << levels
    steps = [(ny // top) * (nx // top)]
    if saliency_map is None:
        for level in range(levels, 0, -1):
            b = 1 << (level - 1)
            steps.append((ny // b) * (nx // b))
    else:
        masks = saliency.detail_masks(saliency_map, levels, thresholds)
        for level in range(levels, 0, -1):
            steps.append(int(replicate2(masks[level - 1]).sum()))
    return steps, list(np.cumsum(steps)), ny * nx
