"""GPU parity of the paper-literal residual-map form (cgh_literal_hologram).

Against the oracle's own literal form (oracle/literal.py: block means, residual
maps, shifted block fringes) and, at 1024^2, against the separable FP64 window
of the progressive hologram.  Bars: rel-L2 <= 1e-5 (FP32), <= 1e-3 (split).
"""

import os

import numpy as np
import pytest

from oracle import literal
from paper_2211_09938_amd import scenes

from helpers import gpu_hologram, rel_l2, to_dev

pytestmark = pytest.mark.gpu
os.environ.setdefault("ORACLE_WORKERS", "8")


def gpu_literal(s, precision="fp32", **kw):
    import torch

    from paper_2211_09938_amd import cgh

    sal = None if s.saliency is None else to_dev(s.saliency)
    lay = None if s.layer is None else to_dev(s.layer)
    h = cgh.literal_hologram(to_dev(s.obj), s.z, s.lam, s.pitch, s.levels, sal, lay,
                             precision=precision, **kw)
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.complex128)


def oracle_literal(s, eq1_prefactor=False):
    from oracle import fresnel

    sal = None if s.saliency is None else s.saliency.astype(np.float64)
    h, _ = literal.hologram_literal(s.obj.astype(np.float64), s.z, s.lam, s.pitch, s.levels, sal,
                                    s.layer)
    if eq1_prefactor:  # per-layer constant: recompute layer by layer
        z = list(s.z)
        layers = [s.obj.astype(np.float64)] if s.layer is None else [
            np.where(s.layer == d, s.obj, 0.0) for d in range(len(z))]
        h = sum(literal.layer_hologram_literal(a, s.lam, s.pitch, z[d], s.levels, sal)[0] *
                fresnel.prefactor(s.lam, z[d]) for d, a in enumerate(layers))
    return h


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16_split", 1e-3),
                                           ("fp16_split", 1e-3)])
@pytest.mark.parametrize("case", ["tiny64", "ragged3", "levels2"])
def test_literal_matches_oracle_literal(case, precision, tol):
    if case == "tiny64":
        s = scenes.tiny(n=64)
    elif case == "ragged3":
        s = scenes.random_scene(501, 40, 72, planes=3, fraction=0.4)
    else:
        s = scenes.random_scene(502, 48, 32, planes=2, levels=2)
    err = rel_l2(gpu_literal(s, precision), oracle_literal(s))
    print(f"literal {case} {precision}: rel-L2 {err:.2e}")
    assert err <= tol


def test_literal_prefactor_accumulate_and_agreement_with_coefficient_form():
    import torch

    from paper_2211_09938_amd import cgh

    s = scenes.random_scene(503, 64, 96, planes=2, fraction=0.3)
    lit = gpu_literal(s, eq1_prefactor=True)
    assert rel_l2(lit, oracle_literal(s, eq1_prefactor=True)) <= 1e-5
    coef = gpu_hologram(s, eq1_prefactor=True)
    assert rel_l2(lit, coef) <= 1e-5
    out = torch.from_numpy(lit.astype(np.complex64)).cuda()
    cgh.literal_hologram(to_dev(s.obj), s.z, s.lam, s.pitch, 3, to_dev(s.saliency),
                         to_dev(s.layer), eq1_prefactor=True, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), 2 * lit) <= 1e-6


def test_literal_plane_1024_full():
    from oracle import separable

    s = scenes.plane_1024()
    got = gpu_literal(s)
    ref = separable.window(s.obj.astype(np.float64), s.z, s.lam, s.pitch, 3,
                           s.saliency.astype(np.float64), None)
    err = rel_l2(got, ref)
    print(f"literal plane1024 full: rel-L2 {err:.2e}")
    assert err <= 1e-5
