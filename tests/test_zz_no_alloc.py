"""GPU test of the allocation-free entry point (cgh_progressive_hologram_noalloc).

It takes its scratch from the library's static device array instead of a
workspace, and runs the same kernels as cgh_progressive_hologram, so on the same
arguments the two must agree bit for bit (which is also inside the FP32 bar of
1e-5 and the split forms' bar).  Two calls in a row, the second on a smaller
problem, so that the second runs on the first one's leftovers in the array; a
request beyond the array's size is rejected without touching the output.
"""

import ctypes

import numpy as np
import pytest

from paper_2211_09938_amd import scenes

from helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu


def cgh():
    from paper_2211_09938_amd import cgh as m

    return m


def _both(s, precision):
    import torch

    obj = to_dev(s.obj)
    sal = None if s.saliency is None else to_dev(s.saliency)
    lay = None if s.layer is None else to_dev(s.layer)
    ref = cgh().progressive_hologram(obj, s.z, s.lam, s.pitch, s.levels, sal, lay,
                                     precision=precision)
    out = torch.full((obj.shape[0], obj.shape[1]), 7.0 + 7.0j, dtype=torch.complex64,
                     device=obj.device)
    got = cgh().progressive_hologram_noalloc(obj, s.z, s.lam, s.pitch, s.levels, sal, lay,
                                             precision=precision, out=out)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    cases = [
        # the 1024 x 1024 single-plane workload at its full size (115.5 MiB of scratch)
        (scenes.plane_1024(), "fp32", 1e-5),
        # then a smaller, ragged three-plane scene in a split form, on the first call's leftovers
        (scenes.random_scene(501, 264, 200, planes=3), "bf16_split", 1e-3),
    ]
    for s, precision, tol in cases:
        print(f"noalloc {s.shape} {precision}", flush=True)
        got, ref = _both(s, precision)
        assert np.isfinite(got).all()
        assert rel_l2(got, ref) <= tol
        assert np.array_equal(got, ref), "same kernels and split: expected bit-identical results"


def test_noalloc_rejects_requests_beyond_the_static_scratch():
    import torch

    n = 2048
    obj = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    out = torch.full((n, n), 3.0 + 1.0j, dtype=torch.complex64, device="cuda")
    z = (ctypes.c_double * 1)(0.2)
    st = cgh().lib().cgh_progressive_hologram_noalloc(
        ctypes.c_void_p(obj.data_ptr()), None, 1, z, None, None, 532e-9, 8e-6, n, n, 3, 0, 0,
        ctypes.c_void_p(out.data_ptr()), None)
    assert st == 8  # CGH_ERROR_SCRATCH_LIMIT
    torch.cuda.synchronize()
    assert torch.all(out == (3.0 + 1.0j))
