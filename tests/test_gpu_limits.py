"""GPU parity at the size limits of the ABI: the largest side (16384) and the
largest layer count (256), against the FP64 oracle.
"""

import os
import time

import numpy as np
import pytest

from oracle import separable
from paper_2211_09938_amd import scenes

from helpers import gpu_hologram, oracle_hologram, rel_l2, sample_pixels

pytestmark = pytest.mark.gpu
os.environ.setdefault("ORACLE_WORKERS", "8")


def big_scene(n=16384, seed=601):
    """Smooth object as a product of two 1D blob profiles (cheap at 16384^2) and a
    rectangular salient region of ~5% of the area, one plane at 0.2 m."""
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64)
    prof = []
    for _ in range(2):
        c = rng.uniform(0, n, 3)
        w = rng.uniform(0.02, 0.1, 3) * n
        prof.append(np.clip(sum(np.exp(-(t - c[i]) ** 2 / (2 * w[i] ** 2)) for i in range(3)), 0, 1))
    obj = (prof[0][:, None] * prof[1][None, :]).astype(np.float32)
    sal = np.zeros((n, n), dtype=np.float32)
    y0, x0 = (int(v) for v in rng.integers(0, n // 2, 2))
    sal[y0:y0 + n // 5, x0:x0 + n // 4] = 1.0
    return scenes.Scene(obj, sal, (0.2,), None, name=f"big{n}")


# split forms: the model-derived bounds of the forward parity tests (4 x 2^-16 for
# BF16; the FP32 bar for FP16, whose split error lies below FP32 accumulation)
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16_split", 4 * 2.0 ** -16),
                                           ("fp16_split", 1e-5)])
def test_largest_side_16384(precision, tol):
    # bf16_split: the one-workgroup-per-CU split kernel over 8192 tiles without split-K
    t0 = time.time()
    s = big_scene()
    print(f"scene {time.time() - t0:.1f} s", flush=True)
    h = gpu_hologram(s, precision=precision)
    print(f"gpu {time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(16384)
    corners = [(0, 0), (16384 - 16, 16384 - 16)] + [tuple(int(v) for v in rng.integers(0, 16384 - 16, 2))]
    refs = separable.windows(s.obj.astype(np.float64), s.z, s.lam, s.pitch, 3,
                             s.saliency.astype(np.float64), None, corners=corners, h=16, w=16)
    for (y0, x0), ref in zip(corners, refs):
        err = rel_l2(h[y0:y0 + 16, x0:x0 + 16], ref)
        print(f"16384^2 {precision} window ({y0}, {x0}): rel-L2 {err:.2e} "
              f"({time.time() - t0:.1f} s)", flush=True)
        assert err <= tol


def test_largest_layer_count_256():
    rng = np.random.default_rng(256)
    s = scenes.random_scene(602, 64, 64, planes=1, fraction=0.4)
    s.layer = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    s.z = tuple(float(v) for v in np.linspace(0.05, 0.3, 256))
    h = gpu_hologram(s)
    ys, xs = sample_pixels(64, 64, seed=5, n_random=64)
    err = rel_l2(h[ys, xs], oracle_hologram(s, pixels=(ys, xs)))
    print(f"256 layers: rel-L2 {err:.2e}")
    assert err <= 1e-5
