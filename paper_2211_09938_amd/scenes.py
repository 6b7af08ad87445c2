"""Seeded synthetic scenes (the only module shared by the oracle checks and the GPU path).

It holds no hologram arithmetic: it only draws inputs.  The paper evaluates on
three natural images of a public saliency dataset with saliency maps from a
trained detector (Sec. 3); neither is available, so seeded synthetic scenes of
the same kind stand in for them: smooth bright objects (Gaussian blobs, optional
uniform noise), binary saliency masks made of ellipses covering a target
fraction of the area, and, for the 3D extension, a smooth depth map quantised to
a few planes.

RNG: ``numpy.random.default_rng(seed)`` (PCG64).  Every array handed to the GPU
is float32 / uint8; the oracle receives float64 copies of the same float32 values.
"""

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

WAVELENGTH = 532e-9
PITCH = 8e-6


@dataclass
class Scene:
    obj: np.ndarray                      # (ny, nx) float32 amplitudes
    saliency: Optional[np.ndarray]       # (ny, nx) float32 in [0, 1], or None
    z: Tuple[float, ...]                 # layer distances, metres
    layer: Optional[np.ndarray] = None   # (ny, nx) uint8 layer ids, or None (one layer)
    lam: float = WAVELENGTH
    pitch: float = PITCH
    levels: int = 3
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.obj.shape


def blobs(rng, ny, nx, count=6, noise=0.0, sigma_px=(4.0, 12.0), scale_ref=128):
    """clip(sum_i a_i exp(-r_i^2 / (2 sigma_i^2)) [+ U(0, noise)], 0, 1) as float32."""
    n_ref = max(ny, nx)
    a = rng.uniform(0.5, 1.0, count)
    cx = rng.uniform(0, nx, count)
    cy = rng.uniform(0, ny, count)
    sig = rng.uniform(sigma_px[0], sigma_px[1], count) * (n_ref / scale_ref)
    yy = np.arange(ny, dtype=np.float64)[:, None]
    xx = np.arange(nx, dtype=np.float64)[None, :]
    img = np.zeros((ny, nx), dtype=np.float64)
    for i in range(count):
        img += a[i] * np.exp(-(((xx - cx[i]) ** 2) + ((yy - cy[i]) ** 2)) / (2.0 * sig[i] ** 2))
    if noise > 0:
        img += rng.uniform(0.0, noise, (ny, nx))
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def ellipse_mask(rng, ny, nx, fraction, count=1, tol=0.01):
    """Union of ``count`` rotated ellipses whose area is ``fraction`` (+-tol) of the plane.

    Centres ~ U(0.3, 0.7) of each side, angle ~ U(0, pi), axis ratio ~ U(0.5, 1);
    a common semi-axis scale is found by bisection.  Returns float32 0/1.
    """
    cy = rng.uniform(0.3 * ny, 0.7 * ny, count)
    cx = rng.uniform(0.3 * nx, 0.7 * nx, count)
    th = rng.uniform(0.0, np.pi, count)
    ratio = rng.uniform(0.5, 1.0, count)
    def union(scale, step):
        yy = np.arange(0, ny, step, dtype=np.float64)[:, None] + 0.5
        xx = np.arange(0, nx, step, dtype=np.float64)[None, :] + 0.5
        m = np.zeros((yy.shape[0], xx.shape[1]), dtype=bool)
        for i in range(count):
            dy, dx = yy - cy[i], xx - cx[i]
            u = dx * np.cos(th[i]) + dy * np.sin(th[i])
            v = -dx * np.sin(th[i]) + dy * np.cos(th[i])
            a = scale
            b = scale * ratio[i]
            m |= (u / a) ** 2 + (v / b) ** 2 <= 1.0
        return m

    # bisect the common scale on a grid of at most ~256 x 256 samples, then
    # draw the mask at full resolution with the scale found
    step = max(1, max(ny, nx) // 256)
    lo, hi = 0.0, 2.0 * max(ny, nx)
    mid = hi
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        f = union(mid, step).mean()
        if abs(f - fraction) <= tol:
            break
        if f < fraction:
            lo = mid
        else:
            hi = mid
    return union(mid, 1).astype(np.float32)


def smooth_depth_layers(rng, ny, nx, planes, z_range=(0.1, 0.3)):
    """Smooth depth map quantised to ``planes`` layers (nearest, ties down) and their z."""
    n_ref = max(ny, nx)
    b = rng.uniform(-1.0, 1.0, 4)
    rho = rng.uniform(0.25 * n_ref, 0.5 * n_ref, 4)
    cy = rng.uniform(0, ny, 4)
    cx = rng.uniform(0, nx, 4)
    yy = np.arange(ny, dtype=np.float64)[:, None]
    xx = np.arange(nx, dtype=np.float64)[None, :]
    dep = np.zeros((ny, nx), dtype=np.float64)
    for i in range(4):
        dep += b[i] * np.exp(-((xx - cx[i]) ** 2 + (yy - cy[i]) ** 2) / (2.0 * rho[i] ** 2))
    span = dep.max() - dep.min()
    dep = (dep - dep.min()) / (span if span > 0 else 1.0)
    if planes == 1:
        return np.zeros((ny, nx), dtype=np.uint8), (0.5 * (z_range[0] + z_range[1]),)
    layer = np.minimum(planes - 1, np.floor(dep * (planes - 1) + 0.5)).astype(np.uint8)
    z = tuple(float(v) for v in np.linspace(z_range[0], z_range[1], planes))
    return layer, z


def dyadic(rng, ny, nx, bits=16):
    """Values k / 2^bits in [0, 1]: every Haar sum and halving of them is exact in float32."""
    return (rng.integers(0, (1 << bits) + 1, (ny, nx)) / float(1 << bits)).astype(np.float32)


# ---------------------------------------------------------------- named workloads

def tiny(seed=1, n=128):
    """128 x 128, one plane at 0.2 m, 6 blobs, one ellipse over ~25% of the area."""
    rng = np.random.default_rng(seed)
    obj = blobs(rng, n, n, 6, noise=0.0)
    sal = ellipse_mask(rng, n, n, 0.25, count=1)
    return Scene(obj, sal, (0.2,), None, name=f"tiny{n}")


def plane_1024(seed=2, n=1024):
    """1024 x 1024, one plane at 0.2 m, blobs + U(0, 0.1) noise, 3 ellipses over ~30%."""
    rng = np.random.default_rng(seed)
    obj = blobs(rng, n, n, 6, noise=0.1)
    sal = ellipse_mask(rng, n, n, 0.30, count=3)
    return Scene(obj, sal, (0.2,), None, name=f"plane{n}")


def depth_2048(seed=3, n=2048, planes=8):
    """2048 x 2048, smooth depth quantised to 8 planes in 0.1-0.3 m, blobs + noise, ~20% saliency."""
    rng = np.random.default_rng(seed)
    obj = blobs(rng, n, n, 6, noise=0.1)
    sal = ellipse_mask(rng, n, n, 0.20, count=1)
    layer, z = smooth_depth_layers(rng, n, n, planes)
    return Scene(obj, sal, z, layer, name=f"depth{n}x{planes}")


def batched(seed=4, count=64, sides=(256, 512, 768, 1024, 1536, 2048), max_planes=4):
    """Uneven batch: sides uniform over ``sides``, 1-4 planes, saliency 5-60% from 1-3 ellipses."""
    scenes = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        n = int(rng.choice(sides))
        planes = int(rng.integers(1, max_planes + 1))
        frac = float(rng.uniform(0.05, 0.6))
        k = int(rng.integers(1, 4))
        obj = blobs(rng, n, n, 6, noise=0.1)
        sal = ellipse_mask(rng, n, n, frac, count=k)
        layer, z = smooth_depth_layers(rng, n, n, planes)
        scenes.append(Scene(obj, sal, z, layer if planes > 1 else None, name=f"batch{i}_{n}x{planes}"))
    return scenes


def differentiable(seed=5, target_seed=50, n=1024):
    """1024 x 1024 amplitudes and a blob target image, one plane at 0.2 m, ~30% saliency."""
    rng = np.random.default_rng(seed)
    obj = blobs(rng, n, n, 6, noise=0.0)
    sal = ellipse_mask(rng, n, n, 0.30, count=1)
    target = blobs(np.random.default_rng(target_seed), n, n, 6, noise=0.0)
    return Scene(obj, sal, (0.2,), None, name=f"grad{n}", extra={"target": target})


def random_scene(seed, ny, nx, planes=1, fraction=0.3, levels=3, lam=WAVELENGTH, pitch=PITCH,
                 z_range=(0.1, 0.3)):
    """Generic seeded scene of any (ny, nx) for parity sweeps and ragged shapes."""
    rng = np.random.default_rng(seed)
    obj = blobs(rng, ny, nx, 6, noise=0.1, sigma_px=(2.0, 6.0), scale_ref=max(ny, nx, 64))
    sal = ellipse_mask(rng, ny, nx, fraction, count=2) if fraction is not None else None
    if planes > 1:
        layer, z = smooth_depth_layers(rng, ny, nx, planes, z_range)
    else:
        layer, z = None, (0.2,)
    return Scene(obj, sal, z, layer, lam, pitch, levels, name=f"rand{seed}_{ny}x{nx}x{planes}")
