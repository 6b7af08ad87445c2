"""Thin Python binding of libcgh (ctypes): argument marshalling only.

Every step of the hologram path runs in the HIP library; PyTorch supplies
device memory (its caching allocator) and the current stream.  Functions take
CUDA (ROCm) tensors, check dtype / device / contiguity, allocate the outputs and
the workspace with torch, and pass raw pointers plus
``torch.cuda.current_stream().cuda_stream`` across the C ABI.  A non-zero
status raises ``RuntimeError`` with the library's status string.

The library is loaded on first use; if it is not built the call fails loudly
(there is no fallback implementation).
"""

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgh.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "cgh.h")

PRECISIONS = {"fp32": 0, "bf16_split": 1, "fp16_split": 2}
FLAG_ACCUMULATE = 1
FLAG_EQ1_PREFACTOR = 2

STATUS = {
    0: "CGH_SUCCESS",
    1: "CGH_ERROR_INVALID_VALUE",
    2: "CGH_ERROR_SHAPE",
    3: "CGH_ERROR_UNSUPPORTED",
    4: "CGH_ERROR_OUT_OF_MEMORY",
    5: "CGH_ERROR_WORKSPACE",
    6: "CGH_ERROR_HIP",
    7: "CGH_ERROR_INTERNAL",
    8: "CGH_ERROR_SCRATCH_LIMIT",
}
NOALLOC_SCRATCH_BYTES = 128 << 20  # CGH_NOALLOC_SCRATCH_BYTES

_lock = threading.Lock()
_lib = None

_c_int, _c_uint, _c_double = ctypes.c_int, ctypes.c_uint, ctypes.c_double
_vp, _sz = ctypes.c_void_p, ctypes.c_size_t

SIGNATURES = {
    "cgh_status_string": (ctypes.c_char_p, [_c_int]),
    "cgh_last_hip_error": (_c_int, []),
    "cgh_version": (_c_int, []),
    "cgh_haar_dwt": (_c_int, [_vp, _c_int, _c_int, _c_int, _vp, _vp]),
    "cgh_haar_idwt": (_c_int, [_vp, _c_int, _c_int, _c_int, _vp, _vp]),
    "cgh_workspace_size": (_c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_sz)]),
    "cgh_workspace_layout": (_c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp]),
    "cgh_progressive_hologram": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double,
                                          _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _sz, _vp,
                                          _vp]),
    "cgh_progressive_hologram_noalloc": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double,
                                                  _c_double, _c_int, _c_int, _c_int, _c_int,
                                                  _c_uint, _vp, _vp]),
    "cgh_progressive_stages": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double,
                                        _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _sz, _vp,
                                        _vp]),
    "cgh_literal_hologram": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double,
                                      _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _sz, _vp,
                                      _vp]),
    "cgh_fused_hologram": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double,
                                      _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _sz, _vp,
                                      _vp]),
    "cgh_exact_hologram": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double, _c_int,
                                    _c_int, _c_int, _c_uint, _vp, _sz, _vp, _vp]),
    "cgh_hologram_backward": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _c_double, _c_double,
                                       _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _sz, _vp, _vp]),
    "cgh_fresnel_backpropagate": (_c_int, [_vp, _c_int, _c_int, _c_double, _c_double, _c_double,
                                           _c_int, _c_int, _vp, _sz, _vp, _vp]),
    "cgh_angular_spectrum_workspace_size": (_sz, [_c_int, _c_int]),
    "cgh_angular_spectrum": (_c_int, [_vp, _c_int, _c_int, _c_double, _c_double, _c_double, _vp,
                                      _sz, _vp, _vp]),
    "cgh_profile_enable": (_c_int, [_c_int]),
    "cgh_profile_stages": (_c_int, [_c_uint]),
    "cgh_profile_read": (_c_int, [ctypes.POINTER(_c_double), ctypes.POINTER(ctypes.c_longlong),
                                  _c_int]),
    "cgh_workspace_stats": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp]),
    "cgh_mfma_peak": (_c_int, [_c_int, _c_int, _c_int, _c_int, _vp, ctypes.POINTER(_c_double), _vp]),
    "cgh_plan_create": (_c_int, [_vp, _c_int, _c_int, _c_double, _c_double, _vp, _c_int, _c_uint,
                                 ctypes.c_char_p, _vp, ctypes.POINTER(_vp)]),
    "cgh_plan_execute": (_c_int, [_vp, _vp]),
    "cgh_plan_destroy": (_c_int, [_vp]),
    "cgh_plan_get_info": (_c_int, [_vp, _vp]),
    "cgh_plan_get_stats": (_c_int, [_vp, _vp, _vp]),
}


class SceneDesc(ctypes.Structure):
    """Mirror of cgh_scene."""

    _fields_ = [
        ("object", _vp),
        ("layer_index", _vp),
        ("n_layers", _c_int),
        ("z", ctypes.POINTER(_c_double)),
        ("saliency", _vp),
        ("ny", _c_int),
        ("nx", _c_int),
        ("hologram", _vp),
    ]


class PlanInfo(ctypes.Structure):
    """Mirror of cgh_plan_info."""

    _fields_ = [
        ("n_scenes", _c_int),
        ("first_tile", _c_int * 2),
        ("second_tile", _c_int * 2),
        ("from_cache", _c_int),
        ("persistent_grid", _c_int),
        ("tune_ms_first", _c_double),
        ("tune_ms_second", _c_double),
        ("device_bytes", _sz),
    ]

class LayoutInfo(ctypes.Structure):
    """Mirror of cgh_layout_info."""

    _fields_ = [
        ("total", _sz),
        ("shared_bytes", _sz),
        ("partial_bytes", _sz),
        ("split_reserved", _c_int),
        ("split_second", _c_int),
        ("forward_bytes", _sz),
        ("backward_bytes", _sz),
        ("backprop_bytes", _sz),
        ("literal_bytes", _sz),
        ("fused_bytes", _sz),
        ("lut_x_offset", _sz),
        ("lut_y_offset", _sz),
        ("gen_x_offset", _sz),
        ("gen_y_offset", _sz),
        ("koff_row_offset", _sz),
        ("koff_col_offset", _sz),
    ]


STAGES = ("coef", "lut", "plan", "first", "second", "reduce")


class Stats(ctypes.Structure):
    """Mirror of cgh_stats."""

    _fields_ = [
        ("k_active", ctypes.c_longlong),
        ("k_padded", ctypes.c_longlong),
        ("k_total", ctypes.c_longlong),
        ("k_tile", ctypes.c_int),
        ("split_k", ctypes.c_int),
        ("flops_first", ctypes.c_double),
        ("flops_second", ctypes.c_double),
        ("flops_second_issued", ctypes.c_double),
        ("operators", ctypes.c_longlong * 4),
        ("operators_pointwise", ctypes.c_longlong),
    ]

    def as_dict(self):
        out = {name: getattr(self, name) for name, _ in self._fields_}
        out["operators"] = list(out["operators"])
        return out


class CghError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().cgh_status_string(status).decode()
        if status == 6:
            msg += f" (hipError {lib().cgh_last_hip_error()})"
        super().__init__(f"{where}: {msg}")


def lib():
    """The loaded libcgh (ctypes.CDLL) with argument types set."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(
                        f"libcgh.so is not built ({LIB_PATH}); run python -m paper_2211_09938_amd.build")
                handle = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(handle, name)
                    fn.restype = res
                    fn.argtypes = args
                _lib = handle
    return _lib


def _check(status, where):
    if status != 0:
        raise CghError(status, where)


# ------------------------------------------------------------------ helpers

def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_tensor(t, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    return ctypes.c_void_p(t.data_ptr())


def _precision(p):
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        return PRECISIONS[p]
    return int(p)


def workspace_size(ny, nx, n_layers=1, levels=3, precision="fp32"):
    out = ctypes.c_size_t(0)
    _check(lib().cgh_workspace_size(ny, nx, n_layers, levels, _precision(precision), ctypes.byref(out)),
           "cgh_workspace_size")
    return out.value


def workspace_layout(ny, nx, n_layers=1, levels=3, precision="fp32"):
    """How the workspace of a problem is divided (cgh_workspace_layout), as a dict."""
    info = LayoutInfo()
    _check(lib().cgh_workspace_layout(ny, nx, n_layers, levels, _precision(precision),
                                      ctypes.byref(info)), "cgh_workspace_layout")
    return {name: getattr(info, name) for name, _ in info._fields_}


def _workspace(nbytes, device, workspace=None):
    torch = _torch()
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace too small")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def _host_doubles(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def _host_floats(vals):
    if vals is None:
        return None
    return (ctypes.c_float * len(vals))(*[float(v) for v in vals])


# --------------------------------------------------------------- operations

def haar_dwt(x, levels=3):
    """Averaging-Haar Mallat coefficients of a (ny, nx) float32 GPU tensor."""
    torch = _torch()
    ny, nx = x.shape
    px = _dev_tensor(x, torch.float32, "x")
    out = torch.empty_like(x)
    _check(lib().cgh_haar_dwt(px, ny, nx, levels, ctypes.c_void_p(out.data_ptr()), _stream()),
           "cgh_haar_dwt")
    return out


def haar_idwt(c, levels=3):
    torch = _torch()
    ny, nx = c.shape
    pc = _dev_tensor(c, torch.float32, "coeffs")
    out = torch.empty_like(c)
    _check(lib().cgh_haar_idwt(pc, ny, nx, levels, ctypes.c_void_p(out.data_ptr()), _stream()),
           "cgh_haar_idwt")
    return out


def progressive_hologram(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                         thresholds=None, precision="fp32", eq1_prefactor=False, out=None,
                         accumulate=False, workspace=None):
    """Complex64 (ny, nx) hologram of ``obj`` (float32, GPU); see cgh_progressive_hologram."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    prec = _precision(precision)
    nbytes = workspace_size(ny, nx, len(zs), levels, prec)
    ws = _workspace(nbytes, obj.device, workspace)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an existing `out`")
        out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_EQ1_PREFACTOR if eq1_prefactor else 0)
    _check(lib().cgh_progressive_hologram(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, prec, flags, ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), p_out, _stream()), "cgh_progressive_hologram")
    return out


def progressive_hologram_noalloc(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                                 thresholds=None, precision="fp32", eq1_prefactor=False, out=None,
                                 accumulate=False):
    """As :func:`progressive_hologram`, through cgh_progressive_hologram_noalloc: the library
    takes its scratch from its own static device array (no workspace); ``out`` may be given
    so that nothing is allocated here either."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an existing `out`")
        out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_EQ1_PREFACTOR if eq1_prefactor else 0)
    _check(lib().cgh_progressive_hologram_noalloc(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, _precision(precision), flags, p_out, _stream()),
        "cgh_progressive_hologram_noalloc")
    return out


def progressive_stages(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                       thresholds=None, precision="fp32", eq1_prefactor=False, out=None,
                       workspace=None):
    """Complex64 (levels + 1, ny, nx) cumulative stage holograms; see cgh_progressive_stages."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    prec = _precision(precision)
    nbytes = workspace_size(ny, nx, len(zs), levels, prec)
    ws = _workspace(nbytes, obj.device, workspace)
    if out is None:
        out = torch.empty((levels + 1, ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (levels + 1, ny, nx))
    flags = FLAG_EQ1_PREFACTOR if eq1_prefactor else 0
    _check(lib().cgh_progressive_stages(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, prec, flags, ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), p_out, _stream()), "cgh_progressive_stages")
    return out


def literal_hologram(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                     thresholds=None, precision="fp32", eq1_prefactor=False, out=None,
                     accumulate=False, workspace=None):
    """Complex64 hologram by the paper-literal residual-map form; see cgh_literal_hologram."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    prec = _precision(precision)
    ws = _workspace(workspace_size(ny, nx, len(zs), levels, prec), obj.device, workspace)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an existing `out`")
        out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_EQ1_PREFACTOR if eq1_prefactor else 0)
    _check(lib().cgh_literal_hologram(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, prec, flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        p_out, _stream()), "cgh_literal_hologram")
    return out


def fused_hologram(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                   thresholds=None, precision="fp32", eq1_prefactor=False, out=None,
                   accumulate=False, workspace=None):
    """Complex64 hologram by the dense reconstruct-then-contract form; see cgh_fused_hologram."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    prec = _precision(precision)
    ws = _workspace(workspace_size(ny, nx, len(zs), levels, prec), obj.device, workspace)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an existing `out`")
        out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    flags = (FLAG_ACCUMULATE if accumulate else 0) | (FLAG_EQ1_PREFACTOR if eq1_prefactor else 0)
    _check(lib().cgh_fused_hologram(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, prec, flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        p_out, _stream()), "cgh_fused_hologram")
    return out


def exact_hologram(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                   thresholds=None, out=None, accumulate=False, workspace=None):
    """Complex64 exact-distance Eq. 1 hologram of the masked reconstruction; see cgh_exact_hologram."""
    torch = _torch()
    ny, nx = obj.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_obj = _dev_tensor(obj, torch.float32, "object")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    nbytes = workspace_size(ny, nx, len(zs), levels, 0)
    ws = _workspace(nbytes, obj.device, workspace)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an existing `out`")
        out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    _check(lib().cgh_exact_hologram(
        p_obj, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, FLAG_ACCUMULATE if accumulate else 0,
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), p_out, _stream()), "cgh_exact_hologram")
    return out


def hologram_backward(grad_h, z, lam, pitch, levels=3, saliency=None, layer_index=None,
                      thresholds=None, precision="fp32", eq1_prefactor=False, workspace=None):
    """dL/dA (float32, (ny, nx)) for the complex cotangent ``grad_h``."""
    torch = _torch()
    ny, nx = grad_h.shape
    zs = list(np.atleast_1d(np.asarray(z, dtype=np.float64)))
    p_g = _dev_tensor(grad_h, torch.complex64, "grad_hologram")
    p_sal = None if saliency is None else _dev_tensor(saliency, torch.float32, "saliency", (ny, nx))
    p_lay = None if layer_index is None else _dev_tensor(layer_index, torch.uint8, "layer_index", (ny, nx))
    prec = _precision(precision)
    nbytes = workspace_size(ny, nx, len(zs), levels, prec)
    ws = _workspace(nbytes, grad_h.device, workspace)
    out = torch.empty((ny, nx), dtype=torch.float32, device=grad_h.device)
    flags = FLAG_EQ1_PREFACTOR if eq1_prefactor else 0
    _check(lib().cgh_hologram_backward(
        p_g, p_lay, len(zs), _host_doubles(zs), p_sal, _host_floats(thresholds), float(lam),
        float(pitch), ny, nx, levels, prec, flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        ctypes.c_void_p(out.data_ptr()), _stream()), "cgh_hologram_backward")
    return out


def fresnel_backpropagate(field, lam, pitch, z, adjoint=False, precision="fp32", workspace=None):
    torch = _torch()
    ny, nx = field.shape
    p_in = _dev_tensor(field, torch.complex64, "field")
    prec = _precision(precision)
    nbytes = workspace_size(ny, nx, 1, 1, prec)
    ws = _workspace(nbytes, field.device, workspace)
    out = torch.empty_like(field)
    _check(lib().cgh_fresnel_backpropagate(
        p_in, ny, nx, float(lam), float(pitch), float(z), prec, 1 if adjoint else 0,
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()), _stream()),
        "cgh_fresnel_backpropagate")
    return out


def angular_spectrum(field, lam, pitch, z, out=None, workspace=None):
    """Angular-spectrum propagation of a complex64 field over z (cgh_angular_spectrum);
    ``out`` may be ``field`` (in place)."""
    torch = _torch()
    ny, nx = field.shape
    p_in = _dev_tensor(field, torch.complex64, "field")
    if out is None:
        out = torch.empty_like(field)
    p_out = _dev_tensor(out, torch.complex64, "out", (ny, nx))
    nbytes = lib().cgh_angular_spectrum_workspace_size(ny, nx)
    ws = _workspace(nbytes, field.device, workspace)
    _check(lib().cgh_angular_spectrum(p_in, ny, nx, float(lam), float(pitch), float(z),
                                      ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel() * ws.element_size(), p_out, _stream()),
           "cgh_angular_spectrum")
    return out


def reconstruct(hologram, lam, pitch, z, out=None, workspace=None):
    """Inverse angular-spectrum reconstruction of a hologram recorded at distance z."""
    return angular_spectrum(hologram, lam, pitch, -float(z), out=out, workspace=workspace)


# -------------------------------------------------------------- diagnostics

def profile_enable(on=True):
    _check(lib().cgh_profile_enable(1 if on else 0), "cgh_profile_enable")


def profile_stages(names=None):
    """Stages (names from STAGES) that record event pairs while profiling is on; None: all."""
    mask = 0xFFFFFFFF if names is None else sum(1 << STAGES.index(n) for n in names)
    _check(lib().cgh_profile_stages(mask), "cgh_profile_stages")


def profile_read(reset=True):
    """{stage: (total ms, event pairs)} of the forward stages since the last reset."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_longlong * len(STAGES))()
    _check(lib().cgh_profile_read(ms, n, 1 if reset else 0), "cgh_profile_read")
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


PEAK_KINDS = {"fp32": 0, "bf16": 1, "fp16": 2}


def mfma_peak(kind, blocks=256, iters=4096, zero_operands=False, sink=None):
    """Launches the matrix-core throughput probe (cgh_mfma_peak) on the current
    stream; returns (sink tensor, real flops of the launch)."""
    torch = _torch()
    if sink is None:
        sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    flops = ctypes.c_double(0.0)
    _check(lib().cgh_mfma_peak(PEAK_KINDS[kind], 1 if zero_operands else 0, blocks, iters,
                               _dev_tensor(sink, torch.float32, "sink", (blocks * 256,)),
                               ctypes.byref(flops), _stream()), "cgh_mfma_peak")
    return sink, flops.value


def workspace_stats(workspace, ny, nx, n_layers=1, levels=3, precision="fp32"):
    st = Stats()
    _check(lib().cgh_workspace_stats(ctypes.c_void_p(workspace.data_ptr()), ny, nx, n_layers, levels,
                                     _precision(precision), ctypes.byref(st), _stream()),
           "cgh_workspace_stats")
    return st.as_dict()


# ------------------------------------------------------------ batched plans

class Plan:
    """A batch of scenes planned, tuned and graph-captured once (cgh_plan_*).

    ``scenes`` is a list of dicts with keys ``obj`` (float32 GPU tensor),
    ``z`` (distances), and optionally ``saliency`` and ``layer_index``.  The
    input tensors are referenced by the captured graph and must stay alive and
    unmodified in place only as the caller intends; ``holograms`` holds one
    complex64 output per scene, refreshed by every :meth:`execute`.
    """

    def __init__(self, scenes, lam, pitch, levels=3, thresholds=None, precision="fp32",
                 eq1_prefactor=False, tune_cache=None):
        torch = _torch()
        self._keep = []
        self.holograms = []
        descs = (SceneDesc * len(scenes))()
        for i, sc in enumerate(scenes):
            obj = sc["obj"]
            ny, nx = obj.shape
            zs = list(np.atleast_1d(np.asarray(sc["z"], dtype=np.float64)))
            sal, lay = sc.get("saliency"), sc.get("layer_index")
            out = torch.empty((ny, nx), dtype=torch.complex64, device=obj.device)
            zarr = _host_doubles(zs)
            descs[i].object = _dev_tensor(obj, torch.float32, "object")
            descs[i].layer_index = None if lay is None else _dev_tensor(lay, torch.uint8, "layer_index", (ny, nx))
            descs[i].n_layers = len(zs)
            descs[i].z = ctypes.cast(zarr, ctypes.POINTER(_c_double))
            descs[i].saliency = None if sal is None else _dev_tensor(sal, torch.float32, "saliency", (ny, nx))
            descs[i].ny = ny
            descs[i].nx = nx
            descs[i].hologram = ctypes.c_void_p(out.data_ptr())
            self._keep += [obj, sal, lay, zarr]
            self.holograms.append(out)
        flags = FLAG_EQ1_PREFACTOR if eq1_prefactor else 0
        handle = ctypes.c_void_p()
        cache = None if tune_cache is None else os.fsencode(tune_cache)
        _check(lib().cgh_plan_create(descs, len(scenes), levels, float(lam), float(pitch),
                                     _host_floats(thresholds), _precision(precision), flags, cache,
                                     _stream(), ctypes.byref(handle)), "cgh_plan_create")
        self._handle = handle

    def execute(self):
        _check(lib().cgh_plan_execute(self._handle, _stream()), "cgh_plan_execute")
        return self.holograms

    def info(self):
        inf = PlanInfo()
        _check(lib().cgh_plan_get_info(self._handle, ctypes.byref(inf)), "cgh_plan_get_info")
        return {"n_scenes": inf.n_scenes, "first_tile": tuple(inf.first_tile),
                "second_tile": tuple(inf.second_tile), "from_cache": bool(inf.from_cache),
                "persistent_grid": inf.persistent_grid, "tune_ms_first": inf.tune_ms_first,
                "tune_ms_second": inf.tune_ms_second, "device_bytes": inf.device_bytes}

    def stats(self):
        st = Stats()
        _check(lib().cgh_plan_get_stats(self._handle, ctypes.byref(st), _stream()),
               "cgh_plan_get_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "_handle", None):
            _check(lib().cgh_plan_destroy(self._handle), "cgh_plan_destroy")
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- autograd

def _autograd():
    torch = _torch()

    class ProgressiveHologram(torch.autograd.Function):
        """H = cgh_progressive_hologram(A); backward: cgh_hologram_backward."""

        @staticmethod
        def forward(ctx, obj, z, lam, pitch, levels, saliency, layer_index, thresholds, precision):
            ctx.args = (z, lam, pitch, levels, thresholds, precision)
            ctx.save_for_backward(saliency if saliency is not None else torch.empty(0),
                                  layer_index if layer_index is not None else torch.empty(0))
            ctx.has = (saliency is not None, layer_index is not None)
            return progressive_hologram(obj.contiguous(), z, lam, pitch, levels, saliency,
                                        layer_index, thresholds, precision)

        @staticmethod
        def backward(ctx, grad_h):
            z, lam, pitch, levels, thresholds, precision = ctx.args
            sal, lay = ctx.saved_tensors
            sal = sal if ctx.has[0] else None
            lay = lay if ctx.has[1] else None
            g = hologram_backward(grad_h.contiguous(), z, lam, pitch, levels, sal, lay, thresholds,
                                  precision)
            return g, None, None, None, None, None, None, None, None

    class FresnelBackprop(torch.autograd.Function):
        """U = cgh_fresnel_backpropagate(H); backward: the adjoint propagation."""

        @staticmethod
        def forward(ctx, field, lam, pitch, z, precision):
            ctx.args = (lam, pitch, z, precision)
            return fresnel_backpropagate(field.contiguous(), lam, pitch, z, False, precision)

        @staticmethod
        def backward(ctx, grad_u):
            lam, pitch, z, precision = ctx.args
            return (fresnel_backpropagate(grad_u.contiguous(), lam, pitch, z, True, precision),
                    None, None, None, None)

    return ProgressiveHologram, FresnelBackprop


_fns = None


def autograd_functions():
    global _fns
    if _fns is None:
        _fns = _autograd()
    return _fns


def hologram_fn(obj, z, lam, pitch, levels=3, saliency=None, layer_index=None, thresholds=None,
                precision="fp32"):
    """Differentiable progressive hologram (torch.autograd.Function)."""
    return autograd_functions()[0].apply(obj, z, lam, pitch, levels, saliency, layer_index,
                                         thresholds, precision)


def backprop_fn(field, lam, pitch, z, precision="fp32"):
    """Differentiable Fresnel back-propagation (torch.autograd.Function)."""
    return autograd_functions()[1].apply(field, lam, pitch, z, precision)


def header_functions(path=HEADER_PATH):
    """Names of the functions declared in include/cgh.h."""
    import re

    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgh_[a-z_0-9]+)\s*\(", text)))
