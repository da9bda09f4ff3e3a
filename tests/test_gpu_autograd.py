"""The differentiable DRT (torch.autograd.Function over the HIP forward and
backprojection): gradients against the explicit transpose of the oracle's
matrix, against central finite differences, and bit-identity with the
non-differentiable entry points."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import FLOAT_TOL, announce, to_dev

pytestmark = pytest.mark.gpu


def _ag():
    from paper_2501_13664_amd import autograd
    return autograd


def _api():
    from paper_2501_13664_amd import api
    return api


def test_backward_is_the_adjoint_bit_for_bit():
    import torch
    ag, api = _ag(), _api()
    N = 32
    f = to_dev(workloads.normal_cube(N, seed=31)).requires_grad_(True)
    gy = to_dev(workloads.normal_weights(api.drt3d_out_shape(N), seed=32))
    announce("autograd backward == adjoint N=32")
    y = ag.drt3d(f)
    assert torch.equal(y.detach(), api.drt3d_forward(f.detach()))
    y.backward(gy)
    assert torch.equal(f.grad, api.drt3d_adjoint(gy))


def test_batched_autograd_matches_per_volume_bit_for_bit():
    import torch
    ag, api = _ag(), _api()
    B, N, mask = 3, 16, 0b011000000110
    f = to_dev(workloads.normal_batch(B, N, seed=33)).requires_grad_(True)
    gy = to_dev(workloads.normal_weights((B,) + api.drt3d_out_shape(N, mask), seed=34))
    announce("autograd batched B=3 N=16")
    y = ag.drt3d(f, mask)
    for b in range(B):
        assert torch.equal(y[b].detach(), api.drt3d_forward(f[b].detach().contiguous(), mask))
    y.backward(gy)
    for b in range(B):
        assert torch.equal(f.grad[b], api.drt3d_adjoint(gy[b].contiguous(), mask))


def test_gradient_against_dense_transpose_n16():
    """loss = sum(W * y^2): grad = 2 R^T (W * R f); also the linear loss sum(W * y),
    grad = R^T W. R is the oracle's explicit matrix; fp64 reference; the error
    is bounded elementwise relative to the same expression over |values|."""
    import torch
    from tests.sparse_ref import drt_matrix
    ag, api = _ag(), _api()
    N, B = 16, 2
    R = drt_matrix(N)
    fb = workloads.normal_batch(B, N, seed=35)
    W = workloads.normal_weights((B,) + api.drt3d_out_shape(N), seed=36)
    f = to_dev(fb).requires_grad_(True)
    Wd = to_dev(W)
    announce("autograd dense transpose N=16 quadratic")
    y = ag.drt3d(f)
    (Wd * y * y).sum().backward()
    got = f.grad.cpu().numpy().astype(np.float64)
    for b in range(B):
        x = fb[b].ravel().astype(np.float64)
        w = W[b].ravel().astype(np.float64)
        ref = 2.0 * (R.T @ (w * (R @ x)))
        bound = 2.0 * (R.T @ (np.abs(w) * (R @ np.abs(x))))
        err = np.abs(got[b].ravel() - ref)
        rel = float(np.max(err / bound))
        nw = float(np.linalg.norm(err) / np.linalg.norm(ref))
        print("b=%d quadratic: elementwise/bound %.3e normwise %.3e" % (b, rel, nw))
        assert rel <= FLOAT_TOL and nw <= FLOAT_TOL
    announce("autograd dense transpose N=16 linear")
    f.grad = None
    (Wd * ag.drt3d(f)).sum().backward()
    got = f.grad.cpu().numpy().astype(np.float64)
    for b in range(B):
        w = W[b].ravel().astype(np.float64)
        ref = R.T @ w
        bound = R.T @ np.abs(w)
        rel = float(np.max(np.abs(got[b].ravel() - ref) / bound))
        print("b=%d linear: elementwise/bound %.3e" % (b, rel))
        assert rel <= FLOAT_TOL


def test_backproject_is_differentiable_both_ways():
    """d<R^T p, u>/dp = R u, and second derivatives go through both Functions."""
    import torch
    ag, api = _ag(), _api()
    N = 8
    p = to_dev(workloads.normal_weights(api.drt3d_out_shape(N), seed=37)).requires_grad_(True)
    u = to_dev(workloads.normal_cube(N, seed=38))
    announce("autograd backproject grad N=8")
    (ag.drt3d_backproject(p) * u).sum().backward()
    assert torch.equal(p.grad, api.drt3d_forward(u))
    f = to_dev(workloads.normal_cube(N, seed=39)).requires_grad_(True)
    y = ag.drt3d(f)
    (g,) = torch.autograd.grad((y * y).sum(), f, create_graph=True)  # g = 2 R^T R f
    (h,) = torch.autograd.grad((g * u).sum(), f)                      # h = 2 R^T R u
    ref = 2.0 * api.drt3d_adjoint(api.drt3d_forward(u))
    assert torch.allclose(h, ref, rtol=1e-5, atol=1e-3)


def test_finite_differences_b8_n128():
    """Batch of 8 N=128 cubes, 12 dodecants, loss = sum(W * y^2), central
    differences with eps = 1e-2 on 64 random voxels, the loss differences
    taken in float64 from the float32 forwards.

    The two float32 forwards round their stage sums differently wherever the
    perturbed voxel enters: each of the 12 N^2 outputs through it carries about
    sqrt(3) roundings of half an ulp of |y| ~ 128 (about 1.3e-5) against a true
    change of 2 eps = 2e-2, so each difference quotient has a relative error of
    about 7e-4 rms, random in sign; over 64 voxels the largest is near 2.5 times
    that (~1.7e-3). The quotients are compared relative to the rms gradient of
    the sample with a bound of 5e-3, three times that model; a wrong factor,
    sign or transposition shows up as an error of order one."""
    import torch
    ag, api = _ag(), _api()
    B, N = 8, 128
    fb = workloads.normal_batch(B, N, seed=5)
    announce("autograd FD B=8 N=128: weights")
    W = to_dev(workloads.normal_weights((B,) + api.drt3d_out_shape(N), seed=6))
    f = to_dev(fb).requires_grad_(True)
    announce("autograd FD B=8 N=128: forward+backward")
    y = ag.drt3d(f)
    (W * y * y).sum().backward()
    grad = f.grad
    vox = workloads.random_voxels(64, B, N, seed=7)
    eps = 1e-2
    fd, an = [], []
    with torch.no_grad():
        for (b, x, yy, z) in vox.tolist():
            announce("autograd FD voxel", b, x, yy, z)
            cube = f[b].detach().clone()
            x0 = cube[x, yy, z].item()
            xp = np.float32(x0 + eps)
            xm = np.float32(x0 - eps)
            cube[x, yy, z] = float(xp)
            yp = api.drt3d_forward(cube).double()
            cube[x, yy, z] = float(xm)
            ym = api.drt3d_forward(cube).double()
            dL = (W[b].double() * (yp - ym) * (yp + ym)).sum().item()
            fd.append(dL / (float(xp) - float(xm)))
            an.append(grad[b, x, yy, z].item())
    fd, an = np.array(fd), np.array(an)
    rms = float(np.sqrt(np.mean(an ** 2)))
    err = float(np.max(np.abs(fd - an)) / rms)
    print("FD: max |fd - grad| / rms(grad) = %.3e (rms grad %.4g)" % (err, rms))
    assert err <= 5e-3
