"""GPU parity of the adjoint, the Fresnel back-propagation and the autograd chain.

Compared with the FP64 oracle in ``oracle.gradient``.  Tolerances: relative L2
<= 1e-5 for the linear maps (same FP32 contraction error budget as the forward
pass); 1e-4 for the full loss-gradient chain, whose |U| - T step divides by |U|
and so amplifies relative error where the reconstruction is small.
"""

import os

import numpy as np
import pytest

from oracle import gradient
from paper_2211_09938_amd import scenes

from helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu
os.environ.setdefault("ORACLE_WORKERS", "8")

LIN_TOL = 1e-5
CHAIN_TOL = 1e-4


def cgh():
    from paper_2211_09938_amd import cgh as m

    return m


def _cot(seed, ny, nx):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)


@pytest.mark.parametrize("shape,planes,levels,eq1", [
    ((40, 24), 2, 3, False),
    ((32, 48), 1, 2, True),
    ((136, 72), 3, 3, False),
])
def test_backward_matches_oracle_gradient(shape, planes, levels, eq1):
    import torch

    s = scenes.random_scene(300 + planes, *shape, planes=planes, levels=levels)
    g = _cot(1, *shape)
    lay = None if s.layer is None else to_dev(s.layer)
    ga = cgh().hologram_backward(to_dev(g), s.z, s.lam, s.pitch, levels, to_dev(s.saliency), lay,
                                 eq1_prefactor=eq1)
    torch.cuda.synchronize()
    ref = gradient.grad_object(g.astype(np.complex128), s.z, s.lam, s.pitch, levels,
                               s.saliency.astype(np.float64), s.layer, eq1_prefactor=eq1)
    assert rel_l2(ga.cpu().numpy(), ref) <= LIN_TOL


def test_backward_sampled_blocks_at_1024():
    import torch

    s = scenes.differentiable()
    g = _cot(2, 1024, 1024)
    ga = cgh().hologram_backward(to_dev(g), s.z, s.lam, s.pitch, 3, to_dev(s.saliency))
    torch.cuda.synchronize()
    blocks = [(0, 0), (127, 127), (40, 77), (64, 3)]
    ref = gradient.grad_object_blocks(g.astype(np.complex128), s.z, s.lam, s.pitch, blocks, 3,
                                      s.saliency.astype(np.float64))
    got = np.stack([ga.cpu().numpy()[by * 8:(by + 1) * 8, bx * 8:(bx + 1) * 8] for by, bx in blocks])
    assert rel_l2(got, ref) <= LIN_TOL


@pytest.mark.parametrize("n,planes", [(1024, 1), (512, 3)])
def test_forward_backward_dot_product_identity(n, planes):
    """<F(A), G> = <A, F^H G> at full size (a property that holds at any size)."""
    import torch

    s = scenes.random_scene(400 + planes, n, n, planes=planes)
    g = _cot(3, n, n)
    lay = None if s.layer is None else to_dev(s.layer)
    h = cgh().progressive_hologram(to_dev(s.obj), s.z, s.lam, s.pitch, 3, to_dev(s.saliency), lay)
    ga = cgh().hologram_backward(to_dev(g), s.z, s.lam, s.pitch, 3, to_dev(s.saliency), lay)
    torch.cuda.synchronize()
    lhs = np.real(np.vdot(g.astype(np.complex128), h.cpu().numpy().astype(np.complex128)))
    rhs = float(np.sum(ga.cpu().numpy().astype(np.float64) * s.obj.astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("shape", [(32, 48), (136, 128), (200, 264)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_backpropagation_matches_oracle(shape, adjoint):
    import torch

    f = _cot(4, *shape)
    u = cgh().fresnel_backpropagate(to_dev(f), 532e-9, 8e-6, 0.2, adjoint=adjoint)
    torch.cuda.synchronize()
    fd = f.astype(np.complex128)
    ref = (gradient.fresnel_backpropagate_adjoint if adjoint else gradient.fresnel_backpropagate)(
        fd, 532e-9, 8e-6, 0.2)
    assert rel_l2(u.cpu().numpy(), ref) <= LIN_TOL


@pytest.mark.parametrize("precision,tol", [("fp32", LIN_TOL), ("bf16_split", 1e-3),
                                           ("fp16_split", 1e-3)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_backpropagation_at_1024_sampled(precision, tol, adjoint):
    # the reconstruction of the differentiable workload at its size, sampled pixels
    import torch

    from helpers import sample_pixels

    f = _cot(6, 1024, 1024)
    u = cgh().fresnel_backpropagate(to_dev(f), 532e-9, 8e-6, 0.2, adjoint=adjoint,
                                    precision=precision)
    torch.cuda.synchronize()
    ys, xs = sample_pixels(1024, 1024, seed=6, n_random=96, crop=8)
    fn = gradient.fresnel_backpropagate_adjoint if adjoint else gradient.fresnel_backpropagate
    ref = fn(f.astype(np.complex128), 532e-9, 8e-6, 0.2, pixels=(ys, xs))
    err = rel_l2(u.cpu().numpy()[ys, xs], ref)
    print(f"backprop 1024 {precision} adjoint={adjoint}: rel-L2 {err:.2e}")
    assert err <= tol


def test_autograd_loss_gradient_matches_oracle_chain():
    import torch

    s = scenes.random_scene(500, 32, 32, fraction=0.3)
    target = scenes.blobs(np.random.default_rng(40), 32, 32, 4, sigma_px=(2, 5), scale_ref=32)
    z = s.z[0]
    obj = to_dev(s.obj).requires_grad_(True)
    sal = to_dev(s.saliency)
    h = cgh().hologram_fn(obj, [z], s.lam, s.pitch, 3, sal)
    u = cgh().backprop_fn(h, s.lam, s.pitch, z)
    loss = ((u.abs() - to_dev(target)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref_loss, ref_grad = gradient.loss_and_grad(s.obj.astype(np.float64), target, z, s.lam,
                                                s.pitch, 3, s.saliency.astype(np.float64))
    assert abs(float(loss) - ref_loss) <= CHAIN_TOL * ref_loss
    assert rel_l2(obj.grad.cpu().numpy(), ref_grad) <= CHAIN_TOL


@pytest.mark.parametrize("precision", ["bf16_split", "fp16_split"])
def test_split_precision_backward_and_backprop(precision):
    import torch

    s = scenes.random_scene(310, 40, 56, planes=2)
    g = _cot(5, 40, 56)
    ga = cgh().hologram_backward(to_dev(g), s.z, s.lam, s.pitch, 3, to_dev(s.saliency),
                                 to_dev(s.layer), precision=precision)
    u = cgh().fresnel_backpropagate(to_dev(g), s.lam, s.pitch, 0.2, precision=precision)
    torch.cuda.synchronize()
    ref = gradient.grad_object(g.astype(np.complex128), s.z, s.lam, s.pitch, 3,
                               s.saliency.astype(np.float64), s.layer)
    ref_u = gradient.fresnel_backpropagate(g.astype(np.complex128), s.lam, s.pitch, 0.2)
    assert rel_l2(ga.cpu().numpy(), ref) <= 1e-3
    assert rel_l2(u.cpu().numpy(), ref_u) <= 1e-3


# FP16 split (11-bit halves, range-scaled) is as accurate as FP32 here and takes the
# FP32 chain bar; BF16 split keeps the split forms' 1e-3
@pytest.mark.parametrize("precision,tol", [("fp32", CHAIN_TOL), ("bf16_split", 1e-3),
                                           ("fp16_split", CHAIN_TOL)])
def test_loss_gradient_at_1024_matches_fp64_separable_chain(precision, tol):
    # the differentiable workload at its own size: 1024 x 1024 amplitudes, 30% saliency,
    # loss through |Fresnel back-propagation|, against the FP64 chain of kernel-matrix
    # products (oracle.separable, pinned to the direct-sum chain on small sides)
    import torch

    from oracle import separable

    s = scenes.differentiable()
    target = s.extra["target"]
    z = s.z[0]
    obj = to_dev(s.obj).requires_grad_(True)
    h = cgh().hologram_fn(obj, [z], s.lam, s.pitch, 3, to_dev(s.saliency), precision=precision)
    u = cgh().backprop_fn(h, s.lam, s.pitch, z, precision=precision)
    loss = ((u.abs() - to_dev(target)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref_loss, ref_grad, ref_u = separable.loss_and_grad(
        s.obj.astype(np.float64), target, z, s.lam, s.pitch, 3, s.saliency.astype(np.float64))
    got = obj.grad.cpu().numpy().astype(np.float64)
    e_u = rel_l2(u.detach().cpu().numpy(), ref_u)
    e_g = rel_l2(got, ref_grad)
    e_max = float(np.max(np.abs(got - ref_grad)) / np.max(np.abs(ref_grad)))
    e_loss = abs(float(loss.detach()) - ref_loss) / ref_loss
    print(f"grad1024 {precision}: U rel-L2 {e_u:.2e}, loss {e_loss:.2e}, gradient rel-L2 {e_g:.2e},"
          f" max |diff| / max |grad| {e_max:.2e}")
    assert e_loss <= tol
    assert e_u <= tol
    assert e_g <= tol
    assert e_max <= 10 * tol


@pytest.mark.parametrize("factor", [1e5, 1e-7])
def test_fp16_split_adjoint_and_backprop_outside_unit_range(factor):
    # the cotangent and the back-propagated field are arbitrary in magnitude; the FP16
    # panels are range-scaled by powers of two (exact) and the epilogues undo it
    import torch

    s = scenes.random_scene(311, 48, 40, planes=2)
    g = (_cot(7, 48, 40).astype(np.complex128) * factor).astype(np.complex64)
    ga = cgh().hologram_backward(to_dev(g), s.z, s.lam, s.pitch, 3, to_dev(s.saliency),
                                 to_dev(s.layer), precision="fp16_split")
    u = cgh().fresnel_backpropagate(to_dev(g), s.lam, s.pitch, 0.2, precision="fp16_split")
    torch.cuda.synchronize()
    ref = gradient.grad_object(g.astype(np.complex128), s.z, s.lam, s.pitch, 3,
                               s.saliency.astype(np.float64), s.layer)
    ref_u = gradient.fresnel_backpropagate(g.astype(np.complex128), s.lam, s.pitch, 0.2)
    e_g = rel_l2(ga.cpu().numpy(), ref)
    e_u = rel_l2(u.cpu().numpy(), ref_u)
    print(f"fp16 x{factor:g}: adjoint rel-L2 {e_g:.2e}, back-propagation {e_u:.2e}")
    assert np.isfinite(ga.cpu().numpy()).all() and np.isfinite(u.cpu().numpy()).all()
    assert e_g <= 1e-5 and e_u <= 1e-5
