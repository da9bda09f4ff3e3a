"""GPU parity of the DJT adjoint (Sec. 5.1, eq. (18): the DJT's stage
recursion reversed, i.e. the transpose of eq. (13)) against the oracle's
definition, through the C ABI binding, and of its differentiable pair.

int32 results are bit-exact; float32 within 1e-5 of the FP64 oracle, relative
to J^T(|p|). Projections are random over the whole output array, so entries
outside every line's support (which no voxel reaches) are present and must be
ignored exactly as the definition ignores them."""
import numpy as np
import pytest

import oracle as O
import workloads
from tests.gpu_util import FLOAT_TOL, announce, float_errors, to_dev

pytestmark = pytest.mark.gpu

MASKS = [0xFFF, 0x001, 0b100100100100, 0x0F0, 0x800]


def _api():
    from paper_2501_13664_amd import api
    return api


def _ag():
    from paper_2501_13664_amd import autograd
    return autograd


def _proj(N, mask, seed, lo=-500, hi=500):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(O.count_dodecants(mask), N, N, 2 * N - 1, 2 * N - 1)).astype(np.int32)


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_djt_adjoint_int_small_all_masks(N):
    api = _api()
    for i, mask in enumerate(MASKS):
        p = _proj(N, mask, seed=300 + 10 * N + i)
        announce("djt adjoint int N=%d mask=%#x" % (N, mask))
        got = api.djt3d_adjoint(to_dev(p), mask).cpu().numpy()
        assert np.array_equal(got, O.wrap_int32(O.def_djt_adj(p, N, mask))), "N=%d mask=%#x" % (N, mask)


def test_djt_adjoint_int_n32():
    """N=32 spans several adjoint tiles per pass (63 rows, 16 per tile, a
    ragged last tile) and both pass depths of the plan."""
    api = _api()
    N = 32
    p = _proj(N, 0xFFF, seed=333, lo=-100, hi=100)
    announce("djt adjoint int N=32")
    got = api.djt3d_adjoint(to_dev(p)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.def_djt_adj(p, N)))


def test_djt_adjoint_int_wraps_like_int32():
    api = _api()
    N = 8
    p = _proj(N, 0xFFF, seed=334, lo=2 ** 29, hi=2 ** 31 - 1)
    announce("djt adjoint int wrap N=8")
    got = api.djt3d_adjoint(to_dev(p)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.def_djt_adj(p, N)))


@pytest.mark.parametrize("N", [16, 32])
def test_djt_adjoint_float_tolerance(N):
    api = _api()
    rng = np.random.default_rng(335 + N)
    p = rng.standard_normal((12, N, N, 2 * N - 1, 2 * N - 1)).astype(np.float32)
    announce("djt adjoint f32 N=%d" % N)
    got = api.djt3d_adjoint(to_dev(p)).cpu().numpy()
    ref = O.def_djt_adj(p.astype(np.float64), N)
    rabs = O.def_djt_adj(np.abs(p).astype(np.float64), N)
    nw, el = float_errors(got, ref, rabs)
    print("djt adjoint N=%d normwise %.3e elementwise/J^T|p| %.3e" % (N, nw, el))
    assert nw <= FLOAT_TOL and el <= FLOAT_TOL


def test_djt_adjoint_dot_identity_n64():
    """<J f, p> = <f, J^T p> with both sides on the GPU (int64 sums)."""
    import torch
    api = _api()
    N = 64
    g = torch.Generator(device="cuda")
    g.manual_seed(336)
    f = torch.randint(-20, 20, (N, N, N), generator=g, dtype=torch.int32, device="cuda")
    p = torch.randint(-20, 20, api.djt3d_out_shape(N), generator=g, dtype=torch.int32, device="cuda")
    announce("djt adjoint dot N=64")
    Jf = api.djt3d_forward(f)
    Jtp = api.djt3d_adjoint(p)
    lhs = int((Jf.to(torch.int64) * p).sum())
    rhs = int((f.to(torch.int64) * Jtp).sum())
    assert lhs == rhs


def test_djt_adjoint_dot_identity_n256_one_dodecant():
    """The largest size the DJT takes (its last pass's windows of 8 chunks):
    <J f, p> = <f, J^T p> for one dodecant at N = 256, sums in int64 over
    slices (the projections alone are 68 GB)."""
    import torch
    api = _api()
    N, mask = 256, 0x010
    g = torch.Generator(device="cuda")
    g.manual_seed(337)
    f = torch.randint(0, 4, (N, N, N), generator=g, dtype=torch.int32, device="cuda")
    announce("djt N=256 one dodecant: forward")
    Jf = api.djt3d_forward(f, mask)
    p = torch.randint(-8, 9, Jf.shape, generator=g, dtype=torch.int32, device="cuda")
    announce("djt N=256 one dodecant: adjoint")
    Jtp = api.djt3d_adjoint(p, mask)
    lhs = sum(int((Jf[0, i].to(torch.int64) * p[0, i]).sum()) for i in range(N))
    rhs = int((f.to(torch.int64) * Jtp).sum())
    del Jf, p, Jtp
    torch.cuda.empty_cache()
    assert lhs == rhs


def test_djt_adjoint_ones_closed_form_n64():
    """J^T of the all-ones array is popcount(mask) * N^2 at every voxel: each
    voxel lies on one line per dodecant and slope pair."""
    import torch
    api = _api()
    N = 64
    for mask in (0xFFF, 0b010010010010):
        p = torch.ones(api.djt3d_out_shape(N, mask), dtype=torch.int32, device="cuda")
        announce("djt adjoint ones N=64 mask=%#x" % mask)
        back = api.djt3d_adjoint(p, mask)
        assert bool((back == O.count_dodecants(mask) * N * N).all())


def test_djt_adjoint_batched_matches_single_calls():
    import torch
    api = _api()
    Ns = [16, 8, 32, 16, 4]
    mask = 0b101101101101
    projs = [to_dev(_proj(N, mask, seed=340 + i, lo=-50, hi=50)) for i, N in enumerate(Ns)]
    announce("djt adjoint batched int mixed")
    outs = api.djt3d_adjoint_batched(projs, mask)
    for p, o in zip(projs, outs):
        assert torch.equal(o, api.djt3d_adjoint(p, mask))
    announce("djt adjoint batched int mixed, graph replay")
    outs2 = api.djt3d_adjoint_batched(projs, mask)
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)


def test_djt_adjoint_caller_workspace_and_chunking():
    """The single-volume call with a caller workspace of exactly the queried size."""
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N = 32
    p = to_dev(_proj(N, 0xFFF, seed=345, lo=-9, hi=9))
    nbytes = lib().djt3d_adjoint_workspace_bytes(N, 0xFFF, 0)
    assert nbytes > 0
    ws = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")  # garbage: must not matter
    out = torch.full((N, N, N), 7, dtype=torch.int32, device="cuda")
    announce("djt adjoint caller workspace N=32")
    api.djt3d_adjoint(p, out=out, workspace=ws)
    assert torch.equal(out, api.djt3d_adjoint(p))


# ------------------------------------------------------------------ autograd
def test_djt_backward_is_the_adjoint_bit_for_bit():
    import torch
    ag, api = _ag(), _api()
    N = 16
    f = to_dev(workloads.normal_cube(N, seed=350)).requires_grad_(True)
    gy = to_dev(workloads.normal_weights(api.djt3d_out_shape(N), seed=351))
    announce("djt autograd backward == adjoint N=16")
    y = ag.djt3d(f)
    assert torch.equal(y.detach(), api.djt3d_forward(f.detach()))
    y.backward(gy)
    assert torch.equal(f.grad, api.djt3d_adjoint(gy))


def test_djt_batched_autograd_matches_per_volume():
    import torch
    ag, api = _ag(), _api()
    B, N, mask = 3, 16, 0b000111000011
    f = to_dev(workloads.normal_batch(B, N, seed=352)).requires_grad_(True)
    gy = to_dev(workloads.normal_weights((B,) + api.djt3d_out_shape(N, mask), seed=353))
    announce("djt autograd batched B=3 N=16")
    y = ag.djt3d(f, mask)
    for b in range(B):
        assert torch.equal(y[b].detach(), api.djt3d_forward(f[b].detach().contiguous(), mask))
    y.backward(gy)
    for b in range(B):
        assert torch.equal(f.grad[b], api.djt3d_adjoint(gy[b].contiguous(), mask))


def test_djt_gradient_against_dense_transpose_n8():
    """loss = sum(W * y^2): grad = 2 J^T (W * J f), J the oracle's explicit
    matrix, fp64 reference, error relative to the same expression over |values|;
    and d<J^T p, u>/dp = J u through the backprojection Function."""
    import torch
    from tests.sparse_ref import djt_matrix
    ag, api = _ag(), _api()
    N, B = 8, 2
    J = djt_matrix(N)
    fb = workloads.normal_batch(B, N, seed=354)
    W = workloads.normal_weights((B,) + api.djt3d_out_shape(N), seed=355)
    f = to_dev(fb).requires_grad_(True)
    announce("djt autograd dense transpose N=8")
    y = ag.djt3d(f)
    (to_dev(W) * y * y).sum().backward()
    got = f.grad.cpu().numpy().astype(np.float64)
    for b in range(B):
        x = fb[b].ravel().astype(np.float64)
        w = W[b].ravel().astype(np.float64)
        ref = 2.0 * (J.T @ (w * (J @ x)))
        bound = 2.0 * (J.T @ (np.abs(w) * (J @ np.abs(x))))
        rel = float(np.max(np.abs(got[b].ravel() - ref) / bound))
        print("b=%d quadratic: elementwise/bound %.3e" % (b, rel))
        assert rel <= FLOAT_TOL
    p = to_dev(workloads.normal_weights(api.djt3d_out_shape(N), seed=356)).requires_grad_(True)
    u = workloads.normal_cube(N, seed=357)
    announce("djt autograd backproject grad N=8")
    (ag.djt3d_backproject(p) * to_dev(u)).sum().backward()
    ref = (J @ u.ravel().astype(np.float64)).reshape(api.djt3d_out_shape(N))
    assert np.allclose(p.grad.cpu().numpy(), ref, rtol=0, atol=1e-4)
