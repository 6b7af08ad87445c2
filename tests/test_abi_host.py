"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function that include/cgh.h declares, and
reject invalid arguments on the host before anything is enqueued -- which is why
these calls work without a GPU: validation never reaches a HIP call.
"""

import ctypes
import os

import pytest

from paper_2211_09938_amd import cgh

pytestmark = pytest.mark.skipif(not os.path.exists(cgh.LIB_PATH), reason="libcgh.so not built")

OK, INVALID, SHAPE, UNSUP, OOM, WS, HIP, INTERNAL, SCRATCH_LIMIT = range(9)
P = ctypes.c_void_p
BOGUS = P(0x1000)  # never dereferenced: validation fails first


def test_every_declared_function_is_exported():
    lib = cgh.lib()
    names = cgh.header_functions()
    assert "cgh_progressive_hologram" in names and "cgh_hologram_backward" in names
    assert "cgh_haar_dwt" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in cgh.SIGNATURES, name


def test_status_strings():
    lib = cgh.lib()
    for code in range(9):
        assert lib.cgh_status_string(code).decode().startswith(cgh.STATUS[code])
    assert lib.cgh_status_string(99) == b"CGH_ERROR_UNKNOWN"
    assert lib.cgh_version() >= 100


def ws_size(ny, nx, layers=1, levels=3, prec=0):
    out = ctypes.c_size_t(0)
    st = cgh.lib().cgh_workspace_size(ny, nx, layers, levels, prec, ctypes.byref(out))
    return st, out.value


def test_workspace_size_rules():
    st, b = ws_size(128, 128)
    assert st == OK and b > 128 * 128 * 8
    st2, b2 = ws_size(2048, 2048, 8)
    assert st2 == OK and b2 > b
    assert ws_size(0, 64)[0] == OK and ws_size(0, 64)[1] == 0
    assert ws_size(100, 64)[0] == SHAPE          # 100 not divisible by 8
    assert ws_size(64, 64, 1, 0)[0] == SHAPE     # levels < 1
    assert ws_size(64, 64, 1, 4)[0] == UNSUP     # more levels than implemented
    assert ws_size(64, 64, 0)[0] == INVALID      # no layer
    assert ws_size(64, 64, 257)[0] == INVALID
    assert ws_size(64, 64, 1, 3, 7)[0] == INVALID
    assert ws_size(32768, 64)[0] == SHAPE        # beyond the side limit
    assert cgh.lib().cgh_workspace_size(64, 64, 1, 3, 0, None) == INVALID


def call_forward(**over):
    z = (ctypes.c_double * 1)(0.2)
    args = dict(obj=BOGUS, layer=None, n_layers=1, z=z, sal=None, thr=None, lam=532e-9,
                pitch=8e-6, ny=64, nx=64, levels=3, prec=0, flags=0, ws=BOGUS, ws_bytes=1 << 40,
                out=BOGUS)
    args.update(over)
    return cgh.lib().cgh_progressive_hologram(
        args["obj"], args["layer"], args["n_layers"], args["z"], args["sal"], args["thr"],
        args["lam"], args["pitch"], args["ny"], args["nx"], args["levels"], args["prec"],
        args["flags"], args["ws"], args["ws_bytes"], args["out"], None)


@pytest.mark.parametrize("over,code", [
    (dict(obj=None), INVALID),
    (dict(out=None), INVALID),
    (dict(z=None), INVALID),
    (dict(z=(ctypes.c_double * 1)(-0.2)), INVALID),
    (dict(z=(ctypes.c_double * 1)(float("nan"))), INVALID),
    (dict(lam=0.0), INVALID),
    (dict(lam=float("inf")), INVALID),
    (dict(pitch=-1.0), INVALID),
    (dict(n_layers=2), INVALID),                      # two layers need a layer map
    (dict(n_layers=0), INVALID),
    (dict(thr=(ctypes.c_float * 3)(0.9, 1.5, 0.5)), INVALID),
    (dict(thr=(ctypes.c_float * 3)(0.9, float("nan"), 0.5)), INVALID),
    (dict(flags=8), INVALID),
    (dict(prec=5), INVALID),
    (dict(ny=60), SHAPE),
    (dict(levels=0), SHAPE),
    (dict(levels=4), UNSUP),
    (dict(ny=32768), SHAPE),
    (dict(ws=None), WS),
    (dict(ws_bytes=1024), WS),
])
def test_forward_rejects_invalid_arguments(over, code):
    assert call_forward(**over) == code


@pytest.mark.parametrize("over,code", [
    (dict(obj=None), INVALID),
    (dict(out=None), INVALID),
    (dict(flags=1), INVALID),                         # accumulate is rejected for stages
    (dict(lam=-1.0), INVALID),
    (dict(ny=60), SHAPE),
    (dict(ws_bytes=1024), WS),
])
def test_stages_rejects_invalid_arguments(over, code):
    z = (ctypes.c_double * 1)(0.2)
    args = dict(obj=BOGUS, layer=None, n_layers=1, z=z, sal=None, thr=None, lam=532e-9,
                pitch=8e-6, ny=64, nx=64, levels=3, prec=0, flags=0, ws=BOGUS, ws_bytes=1 << 40,
                out=BOGUS)
    args.update(over)
    assert cgh.lib().cgh_progressive_stages(
        args["obj"], args["layer"], args["n_layers"], args["z"], args["sal"], args["thr"],
        args["lam"], args["pitch"], args["ny"], args["nx"], args["levels"], args["prec"],
        args["flags"], args["ws"], args["ws_bytes"], args["out"], None) == code
    assert cgh.lib().cgh_progressive_stages(None, None, 1, z, None, None, 532e-9, 8e-6, 0, 64, 3,
                                            0, 0, None, 0, None, None) == OK


def test_literal_validation():
    lib = cgh.lib()
    z = (ctypes.c_double * 1)(0.2)
    base = [BOGUS, None, 1, z, None, None, 532e-9, 8e-6, 64, 64, 3, 0, 0, BOGUS, 1 << 40, BOGUS,
            None]
    for idx, val, code in [(0, None, INVALID), (15, None, INVALID), (8, 60, SHAPE),
                           (14, 16, WS), (11, 9, INVALID), (12, 8, INVALID), (2, 2, INVALID)]:
        a = list(base)
        a[idx] = val
        assert lib.cgh_literal_hologram(*a) == code, (idx, val)


def test_fused_validation():
    lib = cgh.lib()
    z = (ctypes.c_double * 1)(0.2)
    base = [BOGUS, None, 1, z, None, None, 532e-9, 8e-6, 64, 64, 3, 0, 0, BOGUS, 1 << 40, BOGUS,
            None]
    for idx, val, code in [(0, None, INVALID), (15, None, INVALID), (8, 60, SHAPE),
                           (14, 16, WS), (11, 9, INVALID), (12, 8, INVALID), (2, 2, INVALID),
                           (6, 0.0, INVALID), (10, 0, SHAPE)]:
        a = list(base)
        a[idx] = val
        assert lib.cgh_fused_hologram(*a) == code, (idx, val)
    a = list(base)
    a[8] = 0
    assert lib.cgh_fused_hologram(*a) == OK


def test_exact_validation():
    lib = cgh.lib()
    z = (ctypes.c_double * 1)(0.2)
    base = [BOGUS, None, 1, z, None, None, 532e-9, 8e-6, 64, 64, 3, 0, BOGUS, 1 << 40, BOGUS, None]
    for idx, val, code in [(11, 2, INVALID),      # the Eq. 1 prefactor is inherent
                           (11, 8, INVALID),      # unknown flag
                           (0, None, INVALID), (14, None, INVALID), (8, 60, SHAPE),
                           (13, 16, WS), (6, 0.0, INVALID)]:
        a = list(base)
        a[idx] = val
        assert lib.cgh_exact_hologram(*a) == code, (idx, val)
    a = list(base)
    a[8], a[0], a[14], a[12], a[13] = 0, None, None, None, 0
    assert lib.cgh_exact_hologram(*a) == OK


def test_forward_empty_problem_is_a_no_op():
    assert call_forward(ny=0, obj=None, out=None, ws=None, ws_bytes=0) == OK
    assert call_forward(nx=0, obj=None, out=None, ws=None, ws_bytes=0) == OK


def test_backward_and_backprop_validation():
    lib = cgh.lib()
    z = (ctypes.c_double * 1)(0.2)
    base = [BOGUS, None, 1, z, None, None, 532e-9, 8e-6, 64, 64, 3, 0, 0, BOGUS, 1 << 40, BOGUS, None]
    a = list(base)
    a[12] = 1  # accumulate is meaningless for a gradient
    assert lib.cgh_hologram_backward(*a) == INVALID
    a = list(base)
    a[0] = None
    assert lib.cgh_hologram_backward(*a) == INVALID
    a = list(base)
    a[14] = 16
    assert lib.cgh_hologram_backward(*a) == WS
    assert lib.cgh_fresnel_backpropagate(BOGUS, 64, 64, 532e-9, 8e-6, 0.0, 0, 0, BOGUS, 1 << 40,
                                         BOGUS, None) == INVALID
    assert lib.cgh_fresnel_backpropagate(BOGUS, 64, 63, 532e-9, 8e-6, 0.2, 0, 0, BOGUS, 1 << 40,
                                         BOGUS, None) == SHAPE
    assert lib.cgh_fresnel_backpropagate(BOGUS, 64, 64, 532e-9, 8e-6, 0.2, 0, 0, BOGUS, 16,
                                         P(0x2000), None) == WS
    assert lib.cgh_fresnel_backpropagate(BOGUS, 64, 64, 532e-9, 8e-6, 0.2, 0, 0, BOGUS, 1 << 40,
                                         BOGUS, None) == INVALID  # in-place is rejected


def test_haar_validation():
    lib = cgh.lib()
    assert lib.cgh_haar_dwt(BOGUS, 64, 60, 3, BOGUS, None) == SHAPE
    assert lib.cgh_haar_dwt(None, 64, 64, 3, BOGUS, None) == INVALID
    assert lib.cgh_haar_dwt(BOGUS, 64, 64, 3, BOGUS, None) == INVALID  # aliasing in/out
    assert lib.cgh_haar_idwt(BOGUS, 64, 64, 0, P(0x2000), None) == SHAPE
    assert lib.cgh_haar_dwt(None, 0, 64, 3, None, None) == OK


def _scene_array(n=1, **over):
    arr = (cgh.SceneDesc * n)()
    z = (ctypes.c_double * 1)(0.2)
    for i in range(n):
        arr[i].object = BOGUS
        arr[i].layer_index = None
        arr[i].n_layers = 1
        arr[i].z = ctypes.cast(z, ctypes.POINTER(ctypes.c_double))
        arr[i].saliency = None
        arr[i].ny = 64
        arr[i].nx = 64
        arr[i].hologram = P(0x2000)
        for k, v in over.items():
            setattr(arr[i], k, v)
    return arr, z


def plan_create(arr, n, levels=3, lam=532e-9, pitch=8e-6, prec=0, flags=0):
    handle = ctypes.c_void_p()
    st = cgh.lib().cgh_plan_create(arr, n, levels, lam, pitch, None, prec, flags, None, None,
                                   ctypes.byref(handle))
    return st, handle


def test_plan_validation_and_forced_allocation_failure(monkeypatch):
    lib = cgh.lib()
    arr, z = _scene_array(3)
    assert lib.cgh_plan_create(None, 3, 3, 532e-9, 8e-6, None, 0, 0, None, None,
                               ctypes.byref(ctypes.c_void_p())) == INVALID
    assert lib.cgh_plan_create(arr, 3, 3, 532e-9, 8e-6, None, 0, 0, None, None, None) == INVALID
    assert plan_create(arr, 0)[0] == INVALID
    assert plan_create(arr, 3, flags=1)[0] == INVALID        # accumulate is per call, not per plan
    assert plan_create(arr, 3, lam=-1.0)[0] == INVALID
    assert plan_create(arr, 3, levels=4)[0] == UNSUP
    bad, z2 = _scene_array(2, ny=60)
    assert plan_create(bad, 2)[0] == SHAPE
    bad, z3 = _scene_array(2, object=None)
    assert plan_create(bad, 2)[0] == INVALID
    bad, z4 = _scene_array(2, n_layers=2)                    # two layers need a layer map
    assert plan_create(bad, 2)[0] == INVALID
    monkeypatch.setenv("CGH_TEST_FAIL_ALLOC", "1")
    st, h = plan_create(arr, 3)
    assert st == OOM and not h.value
    assert lib.cgh_plan_execute(None, None) == INVALID
    assert lib.cgh_plan_destroy(None) == INVALID
    assert lib.cgh_plan_get_info(None, None) == INVALID


def test_angular_spectrum_validation():
    lib = cgh.lib()
    ws_bytes = lib.cgh_angular_spectrum_workspace_size
    assert ws_bytes(2048, 2048) >= 2048 * 2048 * 8 + 2 * 2048 * 8
    assert ws_bytes(768, 1536) >= 768 * 1536 * 8
    for bad in [(5, 8), (8, 10), (8192, 8), (8, 6144), (1, 8), (0, 8)]:
        assert ws_bytes(*bad) == 0, bad

    def call(ny=64, nx=64, lam=532e-9, pitch=8e-6, z=-0.2, field=BOGUS, ws=BOGUS, nbytes=1 << 30,
             out=BOGUS):
        return lib.cgh_angular_spectrum(field, ny, nx, lam, pitch, z, ws, nbytes, out, None)

    assert call(ny=0) == OK and call(nx=0, field=None) == OK
    assert call(ny=-4) == SHAPE
    assert call(ny=100) == SHAPE and call(nx=5) == SHAPE and call(nx=8192) == SHAPE
    assert call(lam=0.0) == INVALID and call(pitch=-1.0) == INVALID
    assert call(z=float("inf")) == INVALID and call(z=float("nan")) == INVALID
    assert call(field=None) == INVALID and call(out=None) == INVALID
    assert call(ws=None) == WS and call(nbytes=ws_bytes(64, 64) - 1) == WS


LAYOUT_SHAPES = [(8, 8, 1, 1), (16, 24, 3, 3), (64, 64, 1, 3), (128, 128, 2, 3), (264, 200, 3, 3),
                 (520, 136, 2, 3), (1024, 1024, 1, 3), (1024, 512, 4, 2), (2048, 2048, 8, 3),
                 (2048, 2048, 1, 1), (4096, 256, 2, 3), (16384, 16384, 1, 3), (256, 256, 256, 3)]


@pytest.mark.parametrize("ny,nx,layers,levels", LAYOUT_SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "bf16_split", "fp16_split"])
def test_workspace_layout_holds_every_path(ny, nx, layers, levels, prec):
    """Every path's scratch fits the shared region and the second contraction's
    split-K partials fit the reserved partial holograms (a split beyond them once
    wrote past the workspace); the launch paths check the same conditions and
    return CGH_ERROR_INTERNAL otherwise."""
    lay = cgh.workspace_layout(ny, nx, layers, levels, prec)
    assert lay["total"] == cgh.workspace_size(ny, nx, layers, levels, prec)
    assert 1 <= lay["split_second"] <= lay["split_reserved"] <= 16
    plane = ny * nx * 8
    if lay["split_reserved"] > 1:
        assert lay["partial_bytes"] >= lay["split_reserved"] * plane
    else:
        assert lay["partial_bytes"] == 0
    for key in ("forward_bytes", "backward_bytes", "literal_bytes", "fused_bytes",
                "backprop_bytes"):
        if key == "backprop_bytes" and (layers, levels) != (1, 1):
            continue  # back-propagation runs on the (1 layer, 1 level) layout
        assert lay[key] <= lay["shared_bytes"], key
    assert lay["shared_bytes"] + lay["partial_bytes"] <= lay["total"]


def test_workspace_layout_rejects_what_workspace_size_rejects():
    assert cgh.lib().cgh_workspace_layout(100, 64, 1, 3, 0, cgh.ctypes.byref(cgh.LayoutInfo())) == SHAPE
    assert cgh.lib().cgh_workspace_layout(64, 64, 1, 3, 0, None) == INVALID
    assert cgh.workspace_layout(0, 64)["total"] == 0


def call_noalloc(**over):
    z = (ctypes.c_double * 8)(*([0.2] * 8))
    args = dict(obj=BOGUS, layer=None, n_layers=1, z=z, sal=None, thr=None, lam=532e-9,
                pitch=8e-6, ny=64, nx=64, levels=3, prec=0, flags=0, out=BOGUS)
    args.update(over)
    return cgh.lib().cgh_progressive_hologram_noalloc(
        args["obj"], args["layer"], args["n_layers"], args["z"], args["sal"], args["thr"],
        args["lam"], args["pitch"], args["ny"], args["nx"], args["levels"], args["prec"],
        args["flags"], args["out"], None)


@pytest.mark.parametrize("over,code", [
    (dict(obj=None), INVALID),
    (dict(out=None), INVALID),
    (dict(lam=-1.0), INVALID),
    (dict(ny=100), SHAPE),
    (dict(prec=5), INVALID),
    (dict(flags=8), INVALID),
    (dict(ny=0), OK),
    # beyond the static scratch: rejected on the host, nothing enqueued
    (dict(ny=2048, nx=2048), SCRATCH_LIMIT),
    (dict(ny=1024, nx=1024, n_layers=2, layer=BOGUS), SCRATCH_LIMIT),
    (dict(ny=16384, nx=16384, prec=1), SCRATCH_LIMIT),
])
def test_noalloc_validation_and_scratch_limit(over, code):
    assert call_noalloc(**over) == code
