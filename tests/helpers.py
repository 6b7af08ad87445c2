"""Shared test helpers: run the GPU path and the oracle on the same seeded scene."""

import numpy as np

from oracle import fresnel, progressive


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def gpu_hologram(scene, precision="fp32", thresholds=None, **kw):
    import torch

    from paper_2211_09938_amd import cgh

    obj = to_dev(scene.obj)
    sal = None if scene.saliency is None else to_dev(scene.saliency)
    lay = None if scene.layer is None else to_dev(scene.layer)
    h = cgh.progressive_hologram(obj, scene.z, scene.lam, scene.pitch, scene.levels, sal, lay,
                                 thresholds=thresholds, precision=precision, **kw)
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.complex128)


def oracle_hologram(scene, pixels=None, thresholds=None, eq1_prefactor=False):
    sal = None if scene.saliency is None else scene.saliency.astype(np.float64)
    return progressive.hologram(scene.obj.astype(np.float64), scene.z, scene.lam, scene.pitch,
                                scene.levels, sal, scene.layer, thresholds, pixels=pixels,
                                eq1_prefactor=eq1_prefactor)


def sample_pixels(ny, nx, seed, n_random=192, crop=16):
    """A seeded crop, random pixels and the four corners."""
    rng = np.random.default_rng(seed)
    c = min(crop, ny, nx)
    y0 = int(rng.integers(0, ny - c + 1))
    x0 = int(rng.integers(0, nx - c + 1))
    cy, cx = fresnel.grid_pixels(ny, nx, y0, x0, c, c)
    ry = rng.integers(0, ny, n_random)
    rx = rng.integers(0, nx, n_random)
    ky = np.array([0, 0, ny - 1, ny - 1])
    kx = np.array([0, nx - 1, 0, nx - 1])
    return np.concatenate([cy, ry, ky]), np.concatenate([cx, rx, kx])


def rel_l2(a, b):
    return progressive.rel_l2(a, b)
