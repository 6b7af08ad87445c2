"""The single-scene forward pass captured into a HIP graph (torch.cuda.graph).

cgh_progressive_hologram enqueues kernels only (no memset, copy or
synchronisation), so a caller can capture it once and replay it.  The graph is
replayed three times with eager forward passes of another scene and
synchronisations between the replays; every replay must equal the eager result
bit for bit (the kernels are deterministic).
"""

import pytest

from paper_2211_09938_amd import scenes

from helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16_split"])
def test_forward_graph_replays_match_eager(precision):
    import torch

    from paper_2211_09938_amd import cgh

    s = scenes.random_scene(77, 264, 200, planes=3)   # split-K and partial tiles
    o = scenes.random_scene(78, 128, 136, planes=2)   # eager work between replays
    dev = torch.device("cuda:0")

    def setup(sc):
        ws = torch.empty(cgh.workspace_size(*sc.obj.shape, len(sc.z), sc.levels, precision),
                         dtype=torch.uint8, device=dev)
        out = torch.empty(sc.obj.shape, dtype=torch.complex64, device=dev)
        args = (to_dev(sc.obj), sc.z, sc.lam, sc.pitch, sc.levels, to_dev(sc.saliency),
                to_dev(sc.layer))
        return lambda: cgh.progressive_hologram(*args, precision=precision, out=out,
                                                workspace=ws), out

    run, out = setup(s)
    run_other, out_other = setup(o)
    run()
    run_other()
    torch.cuda.synchronize()
    ref = out.clone()
    ref_other = out_other.clone()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for r in range(3):
        out.zero_()
        run_other()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"
        assert torch.equal(out_other, ref_other)
