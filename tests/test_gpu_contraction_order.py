"""GPU parity of the per-(layer, level) contraction order.

Eq. 3's superposition of one layer and level, Fy Cb Fx^T, can be contracted
rows-first (T = Cb Fx^T, then Fy T^T: the second contraction sums over the
square's nonzero rows) or columns-first (T' = Cb^T Fy^T, then T'^T Fx^T: it sums
over the nonzero columns).  The library takes, per layer and level, the order
with the shorter padded K.  These tests pin the K it reports to the support of
the oracle's masked coefficients (exact integers, on dyadic objects where every
Haar sum is exact in FP32) and check holograms of scenes that use both orders
against the FP64 oracle.
"""

import os

import numpy as np
import pytest

from paper_2211_09938_amd import scenes

from helpers import gpu_hologram, oracle_hologram, rel_l2, sample_pixels, support, to_dev

pytestmark = pytest.mark.gpu
os.environ.setdefault("ORACLE_WORKERS", "8")

FP32_TOL = 1e-5
SPLIT_MODEL = {"bf16_split": 4 * 2.0 ** -16, "fp16_split": 1e-5}


def pad16(v):
    return (v + 15) // 16 * 16


def expected_k(scene):
    k_active = k_padded = 0
    orders = set()
    for rows, cols in support(scene):
        cf = pad16(cols) < pad16(rows)
        k_active += cols if cf else rows
        k_padded += pad16(cols) if cf else pad16(rows)
        if rows:
            orders.add("columns" if cf else "rows")
    return k_active, k_padded, orders


def stripes(seed=71, ny=200, nx=328):
    """Non-square, three layers: a vertical stripe (few columns: columns-first), a
    horizontal stripe (few rows: rows-first) and the rest; dyadic amplitudes."""
    rng = np.random.default_rng(seed)
    obj = scenes.dyadic(rng, ny, nx).astype(np.float32)
    layer = np.full((ny, nx), 2, dtype=np.uint8)
    layer[24:64, :] = 1
    layer[:, 16:56] = 0
    sal = scenes.ellipse_mask(rng, ny, nx, 0.3)
    sal[:, 8:64] = 1.0  # the vertical stripe's detail is salient at every level
    return scenes.Scene(obj, sal, (0.08, 0.12, 0.16), layer, name="stripes")


def dyadic_depth_2048():
    s = scenes.depth_2048()
    s.obj = scenes.dyadic(np.random.default_rng(2049), 2048, 2048).astype(np.float32)
    return s


def gpu_k(scene, precision="fp32"):
    import torch

    from paper_2211_09938_amd import cgh as m

    ny, nx = scene.obj.shape
    ws = torch.empty(m.workspace_size(ny, nx, len(scene.z), 3, precision), dtype=torch.uint8,
                     device="cuda")
    lay = None if scene.layer is None else to_dev(scene.layer)
    sal = None if scene.saliency is None else to_dev(scene.saliency)
    m.progressive_hologram(to_dev(scene.obj), scene.z, scene.lam, scene.pitch, 3, sal, lay,
                           precision=precision, workspace=ws)
    st = m.workspace_stats(ws, ny, nx, len(scene.z), 3, precision)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("case", ["stripes", "ragged", "depth2048"])
def test_k_of_the_second_contraction_matches_oracle_support(case):
    if case == "stripes":
        s = stripes()
    elif case == "ragged":
        s = scenes.random_scene(72, 72, 136, planes=3, fraction=0.4)
        s.obj = scenes.dyadic(np.random.default_rng(72), 72, 136).astype(np.float32)
    else:
        s = dyadic_depth_2048()
    k_active, k_padded, orders = expected_k(s)
    if case in ("stripes", "depth2048"):
        assert orders == {"rows", "columns"}  # the scene exercises both orders
    st = gpu_k(s)
    print(f"{case}: k_active {st['k_active']} (oracle {k_active}), "
          f"k_padded {st['k_padded']} (oracle {k_padded}), orders {sorted(orders)}")
    assert st["k_active"] == k_active
    assert st["k_padded"] == k_padded


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_TOL),
                                           ("bf16_split", SPLIT_MODEL["bf16_split"]),
                                           ("fp16_split", SPLIT_MODEL["fp16_split"])])
def test_both_orders_non_square_full_hologram(precision, tol):
    s = stripes()
    h = gpu_hologram(s, precision=precision)
    err = rel_l2(h, oracle_hologram(s))
    print(f"stripes 200x328 {precision}: rel-L2 {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("precision", ["fp32", "bf16_split"])
def test_columns_first_only_scene(precision):
    # a single vertical-stripe layer on a tall scene: every level columns-first
    rng = np.random.default_rng(73)
    ny, nx = 264, 96
    obj = np.zeros((ny, nx), dtype=np.float32)
    obj[:, 40:56] = scenes.dyadic(rng, ny, 16)
    s = scenes.Scene(obj, scenes.ellipse_mask(rng, ny, nx, 0.5), (0.1,), None, name="column")
    _, _, orders = expected_k(s)
    assert orders == {"columns"}
    h = gpu_hologram(s, precision=precision)
    err = rel_l2(h, oracle_hologram(s))
    print(f"column-only 264x96 {precision}: rel-L2 {err:.3e}")
    assert err <= (FP32_TOL if precision == "fp32" else SPLIT_MODEL[precision])


def first_dense_tiles(ny, nx, planes, tm, levels=3):
    """Tiles of the first contraction with every row and column active, in the order
    with more of them, at tm x 128 tiles (the library's bound for choosing 128-column
    tiles, with which the first contraction generates its fringe operand from the
    operand-format tables instead of reading a gathered panel)."""
    t = 0
    for l in range(1, levels + 1):
        sy, sx = ny >> (l - 1), nx >> (l - 1)
        t += max(-(-sy // tm) * -(-nx // 128), -(-sx // tm) * -(-ny // 128))
    return t * planes


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_TOL),
                                           ("bf16_split", SPLIT_MODEL["bf16_split"]),
                                           ("fp16_split", SPLIT_MODEL["fp16_split"])])
def test_generated_fringe_operand_on_ragged_tiles(precision, tol):
    # 1000 x 1096 (neither a multiple of 128) in 6 planes: 128-column tiles whose last
    # column of tiles runs past the image, and both contraction orders
    ny, nx, planes = 1000, 1096, 6
    assert first_dense_tiles(ny, nx, planes, 64 if precision == "fp32" else 128) >= 512
    s = scenes.random_scene(1096, ny, nx, planes=planes, fraction=0.3)
    h = gpu_hologram(s, precision=precision)
    ys, xs = sample_pixels(ny, nx, seed=11, n_random=128, crop=8)
    err = rel_l2(h[ys, xs], oracle_hologram(s, pixels=(ys, xs)))
    print(f"1000x1096x6 {precision}: rel-L2 {err:.3e} on {len(ys)} pixels")
    assert err <= tol
