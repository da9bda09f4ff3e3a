"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (default tuning, caller-provided workspace).

Element by element: every output of the N = 512 int32 forward against the
oracle's recursion (Algorithm 1), one layout group of four dodecants at a
time; two whole dodecants of the N = 128 DJT (Algorithm 3); every output of
every cube of the 96-cube float32 batch, and the whole forward and backward of
the 8 x 128^3 float32 differentiable batch, against the FP64 oracle, each with
its normwise error and max |err| / R(|f|) printed and bounded by 1e-5.
Sampled outputs through the point evaluators (eqs. (9) and (13) directly) and
properties that hold at any size (per-slope sums, support, the adjoint's
closed forms and the dot-product identity) add independent checks."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import workloads
from tests.gpu_util import FLOAT_TOL, announce, float_errors, to_dev

pytestmark = pytest.mark.gpu


def _api():
    from paper_2501_13664_amd import api
    return api


def _ws(nbytes):
    import torch
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _pmap(fn, items, workers=None):
    """fn over items on host threads (the oracle's C calls release the GIL)."""
    workers = workers or max(1, min(len(items), 8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def _samples(rng, count, hi, edges):
    """`count` random points in the box [0, hi) plus the given edge points."""
    pts = [tuple(int(rng.integers(0, h)) for h in hi) for _ in range(count)]
    return pts + [tuple(e) for e in edges]


@pytest.fixture(scope="module")
def drt512():
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N = 512
    vol = workloads.point_cloud_with_planes(N, seed=2)
    dvol = to_dev(vol)
    out = torch.empty(api.drt3d_out_shape(N), dtype=torch.int32, device="cuda")
    ws = _ws(lib().drt3d_workspace_bytes(N, 0xFFF, 0))
    announce("fullsize drt N=512 forward (benchmark configuration)")
    api.drt3d_forward(dvol, out=out, workspace=ws)
    torch.cuda.synchronize()
    yield N, vol, dvol, out
    del out, ws
    torch.cuda.empty_cache()


def test_drt_n512_sampled_outputs(drt512):
    import torch
    N, vol, _, out = drt512
    rng = np.random.default_rng(11)
    E = 3 * N - 2
    edges = [(0, 0, 0), (0, 0, N - 1), (N - 1, N - 1, 3 * N - 3), (N - 1, 0, 2 * N - 2), (0, N - 1, N),
             (N - 1, N - 1, 0), (1, 2, N + 2)]
    for k in range(12):
        pts = _samples(rng, 60, (N, N, E), edges)
        idx = torch.tensor(pts, dtype=torch.long, device="cuda")
        got = out[k][idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
        ref = np.array([O.drt_point(vol, k, s1, s2, dd) for (s1, s2, dd) in pts], dtype=np.int64)
        assert np.array_equal(got.astype(np.int64), ref), "dodecant %d" % k


@pytest.mark.parametrize("group", [0, 1, 2])
def test_drt_n512_every_element(drt512, group):
    """Every output of the four dodecants of one volume layout group (z-normal
    k0-k3; y-normal k4, k7, k9, k10; x-normal k5, k6, k8, k11) equals the
    oracle's recursion, bit for bit."""
    N, vol, _, out = drt512
    dods = {0: (0, 1, 2, 3), 1: (4, 7, 9, 10), 2: (5, 6, 8, 11)}[group]
    announce("fullsize drt N=512 every element, dodecants %s (oracle on the host)" % (dods,))
    refs = _pmap(lambda k: O.wrap_int32(O.rec_drt(vol, 1 << k)[0]), list(dods), workers=4)
    for k, ref in zip(dods, refs):
        got = out[k].cpu().numpy()
        bad = np.count_nonzero(got != ref)
        assert bad == 0, "dodecant %d: %d of %d outputs differ" % (k, bad, ref.size)


def test_drt_n512_slope_sums_and_support(drt512):
    """Every slope pair's displacements sum to the volume's sum, and every
    column is zero past dd = N-1+s1+s2 (Sec. 3.2)."""
    import torch
    N, vol, dvol, out = drt512
    total = int(vol.astype(np.int64).sum())
    dd = torch.arange(3 * N - 2, device="cuda")
    s = torch.arange(N, device="cuda")
    for k in range(12):
        announce("fullsize drt N=512 invariants k=%d" % k)
        sums = out[k].sum(dim=-1, dtype=torch.int64)
        assert bool((sums == total).all()), "dodecant %d slope sums" % k
        beyond = dd[None, None, :] > (N - 1 + s[:, None, None] + s[None, :, None])
        assert not bool(((out[k] != 0) & beyond).any()), "dodecant %d support" % k


def test_drt_n512_adjoint_closed_forms_and_dot_identity(drt512):
    """R^T applied to the constant 1 gives 12 N^2 everywhere (each voxel lies on
    one plane per dodecant and slope pair); R^T applied to p = dd gives, per
    voxel, the sum over k, s1, s2 of N-1 + l_s1(x') + l_s2(y') - z'; and
    <R f, p> = <f, R^T p> for a random p."""
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N, vol, dvol, out = drt512
    n = N.bit_length() - 1
    ws = _ws(lib().drt3d_adjoint_workspace_bytes(N, 0xFFF, 0))
    back = torch.empty((N, N, N), dtype=torch.int32, device="cuda")
    proj = torch.ones(api.drt3d_out_shape(N), dtype=torch.int32, device="cuda")
    announce("fullsize adjoint N=512 ones")
    api.drt3d_adjoint(proj, out=back, workspace=ws)
    assert bool((back == 12 * N * N).all())

    announce("fullsize adjoint N=512 dd ramp")
    proj.copy_(torch.arange(3 * N - 2, dtype=torch.int32, device="cuda").expand_as(proj))
    api.drt3d_adjoint(proj, out=back, workspace=ws)
    lam = np.array([sum(O.line(n, s, x) for s in range(N)) for x in range(N)], dtype=np.int64)
    rng = np.random.default_rng(12)
    vox = _samples(rng, 300, (N, N, N), [(0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, 0), (N // 2, N // 2, N // 2)])
    mats = []
    for k in range(12):
        M = O.frame_matrix(k)
        o0 = np.array(O.frame_to_orig(k, N, (0, 0, 0)), dtype=np.int64)
        mats.append((M, -M @ o0))
    ref = []
    for (x, y, z) in vox:
        acc = 0
        for M, off in mats:
            xp, yp, zp = M @ np.array([x, y, z], dtype=np.int64) + off
            acc += N * N * (N - 1 - int(zp)) + N * int(lam[xp]) + N * int(lam[yp])
        ref.append(acc)
    idx = torch.tensor(vox, dtype=torch.long, device="cuda")
    got = back[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(np.array(ref, dtype=np.int64)))

    announce("fullsize adjoint N=512 dot identity")
    g = torch.Generator(device="cuda")
    g.manual_seed(13)
    proj = torch.randint(-8, 8, api.drt3d_out_shape(N), generator=g, dtype=torch.int32, device="cuda")
    api.drt3d_adjoint(proj, out=back, workspace=ws)
    lhs = sum(int((out[k].to(torch.int64) * proj[k]).sum()) for k in range(12))
    rhs = int((dvol.to(torch.int64) * back).sum())
    assert lhs == rhs
    del proj, ws


def test_djt_n128_sampled_sums_and_support():
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N = 128
    E = 2 * N - 1
    vol = workloads.noise_with_segments(N, seed=3)
    out = torch.empty(api.djt3d_out_shape(N), dtype=torch.int32, device="cuda")
    ws = _ws(lib().djt3d_workspace_bytes(N, 0xFFF, 0))
    announce("fullsize djt N=128 forward")
    api.djt3d_forward(to_dev(vol), out=out, workspace=ws)
    del ws
    rng = np.random.default_rng(14)
    edges = [(0, 0, 0, 0), (N - 1, N - 1, E - 1, E - 1), (0, N - 1, N - 1, 2 * N - 2), (N - 1, 0, 2 * N - 2, 0)]
    total = int(vol.astype(np.int64).sum())
    e = torch.arange(E, device="cuda")
    s = torch.arange(N, device="cuda")
    for k in range(12):
        pts = _samples(rng, 400, (N, N, E, E), edges)
        idx = torch.tensor(pts, dtype=torch.long, device="cuda")
        got = out[k][idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].cpu().numpy()
        ref = np.array([O.djt_point(vol, k, *p) for p in pts], dtype=np.int64)
        assert np.array_equal(got.astype(np.int64), ref), "dodecant %d" % k
        announce("fullsize djt N=128 invariants k=%d" % k)
        sums = out[k].sum(dim=(-1, -2), dtype=torch.int64)
        assert bool((sums == total).all()), "dodecant %d line sums" % k
        b1 = e[None, :, None] > (N - 1 + s[:, None, None])           # (s1, e1, 1)
        b2 = e[None, None, :] > (N - 1 + s[:, None, None])           # (s2, 1, e2)
        nz = out[k] != 0
        assert not bool((nz & b1[:, None, :, :]).any()), "dodecant %d e1 support" % k
        assert not bool((nz & b2[None, :, :, :]).any()), "dodecant %d e2 support" % k
    del out
    torch.cuda.empty_cache()


def test_djt_n128_two_dodecants_every_element():
    """Every output of dodecant 0 (z-normal frame) and dodecant 5 (x-normal
    frame) of the N = 128 DJT equals the oracle's recursion (Algorithm 3),
    bit for bit."""
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N = 128
    vol = workloads.noise_with_segments(N, seed=3)
    out = torch.empty(api.djt3d_out_shape(N), dtype=torch.int32, device="cuda")
    ws = _ws(lib().djt3d_workspace_bytes(N, 0xFFF, 0))
    announce("fullsize djt N=128 every element of dodecants 0 and 5")
    api.djt3d_forward(to_dev(vol), out=out, workspace=ws)
    del ws
    refs = _pmap(lambda k: O.wrap_int32(O.rec_djt(vol, 1 << k)[0]), [0, 5], workers=2)
    for k, ref in zip((0, 5), refs):
        got = out[k].cpu().numpy()
        bad = np.count_nonzero(got != ref)
        assert bad == 0, "dodecant %d: %d of %d outputs differ" % (k, bad, ref.size)
    del out
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def mixed_batch_out():
    """The 96-cube float32 batch through one batched call (the benchmark's
    launch), outputs kept on the GPU."""
    import torch
    api = _api()
    cubes = workloads.mixed_batch()
    dev = [to_dev(c) for c in cubes]
    announce("fullsize batched mixed float32 (96 cubes)")
    outs = api.drt3d_forward_batched(dev)
    torch.cuda.synchronize()
    yield cubes, outs
    del outs, dev
    torch.cuda.empty_cache()


def _fp64_drt_errors(cube, got):
    """(normwise, max |err| / R(|f|)) of a float32 12-dodecant output against
    the FP64 oracle's recursion; R(|f|) is the FP64 transform of |f|."""
    c64 = cube.astype(np.float64)
    y64 = O.rec_drt(c64)
    r_abs = O.rec_drt(np.abs(c64))
    return float_errors(got, y64, r_abs)


@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_batched_mixed_float_every_element_against_fp64(mixed_batch_out, N):
    """Every output of every cube of size N in the batch, against FP64:
    normwise relative error and max |err| / R(|f|) both within 1e-5."""
    cubes, outs = mixed_batch_out
    idx = [i for i, c in enumerate(cubes) if c.shape[0] == N]
    announce("fullsize batched float32 N=%d: %d cubes against FP64" % (N, len(idx)))
    errs = _pmap(lambda i: _fp64_drt_errors(cubes[i], outs[i].cpu().numpy()), idx,
                 workers=2 if N >= 256 else 8)
    for i, (nw, mx) in zip(idx, errs):
        print("cube %d (N=%d): normwise %.2e, max|err|/R|f| %.2e" % (i, N, nw, mx))
    worst_nw = max(e[0] for e in errs)
    worst_mx = max(e[1] for e in errs)
    print("N=%d worst: normwise %.2e, max|err|/R|f| %.2e" % (N, worst_nw, worst_mx))
    assert worst_nw <= FLOAT_TOL and worst_mx <= FLOAT_TOL


def test_differentiable_batch_every_element_against_fp64():
    """The differentiable batch (8 float32 N = 128 cubes, 12 dodecants): the
    autograd forward y = R f and the backward R^T W (the gradient of sum W*y)
    in every element against the FP64 oracle (Algorithm 1 and its reverse with
    eq. (17)), each cube's normwise error and max |err| / R(|f|) (R^T|W| for
    the backward) within 1e-5."""
    import torch
    from paper_2501_13664_amd import autograd
    api = _api()
    B, N = 8, 128
    f = workloads.normal_batch(B, N, seed=5)
    W = workloads.normal_weights((B,) + api.drt3d_out_shape(N), seed=6)
    announce("fullsize differentiable batch 8x128 float32: forward and backward")
    fr = to_dev(f).requires_grad_(True)
    y = autograd.drt3d(fr)
    y.backward(to_dev(W))
    y_h = y.detach().cpu().numpy()
    g_h = fr.grad.cpu().numpy()
    del y, fr
    torch.cuda.empty_cache()

    def errs(b):
        fwd = _fp64_drt_errors(f[b], y_h[b])
        w64 = W[b].astype(np.float64)
        bwd = float_errors(g_h[b], O.rec_adj(w64, N), O.rec_adj(np.abs(w64), N))
        return fwd, bwd

    res = _pmap(errs, list(range(B)))
    for b, (fwd, bwd) in enumerate(res):
        print("cube %d: forward normwise %.2e max %.2e; backward normwise %.2e max %.2e" % ((b,) + fwd + bwd))
        assert max(fwd) <= FLOAT_TOL and max(bwd) <= FLOAT_TOL, b


def test_batched_mixed_float_sampled_against_definition(mixed_batch_out):
    """Sampled outputs of every cube of the batch against the oracle's point
    evaluator, which sums eq. (9)'s plane directly (not the recursion):
    within 1e-5 of FP64, relative to R(|f|)."""
    import torch
    cubes, outs = mixed_batch_out
    rng = np.random.default_rng(15)
    worst = 0.0
    for i, (c, o) in enumerate(zip(cubes, outs)):
        N = c.shape[0]
        pts = [(int(rng.integers(0, 12)),) + p for p in _samples(rng, 6, (N, N, 3 * N - 2), [(N - 1, N - 1, N)])]
        idx = torch.tensor(pts, dtype=torch.long, device="cuda")
        got = o[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].cpu().numpy().astype(np.float64)
        c64 = c.astype(np.float64)
        a64 = np.abs(c64)
        for g, p in zip(got, pts):
            ref = O.drt_point(c64, *p)
            bound = O.drt_point(a64, *p)
            err = abs(g - ref)
            if bound == 0:
                assert err == 0
            else:
                worst = max(worst, err / bound)
    print("mixed batch: max |err| / R|f| over the samples = %.3e" % worst)
    assert worst <= FLOAT_TOL


def test_djt_adjoint_n128_closed_forms_and_dot_identity():
    """The DJT adjoint in the benchmark's configuration (N = 128, 12 dodecants,
    library workspace): J^T 1 = 12 N^2 everywhere; J^T applied to p = e1 gives,
    per voxel, the sum over the dodecants of N * lambda(z') + N^2 (N-1-x') (the
    line through (x', y', z') with slopes (s1, s2) sits at e1 = N-1 + l_s1(z') - x',
    summed over s1 and over the N values of s2); and <J f, p> = <f, J^T p> for a
    random p, accumulated one dodecant at a time."""
    import torch
    from paper_2501_13664_amd._lib import lib
    api = _api()
    N = 128
    E = 2 * N - 1
    n = N.bit_length() - 1
    ws = _ws(lib().djt3d_adjoint_workspace_bytes(N, 0xFFF, 0))
    back = torch.empty((N, N, N), dtype=torch.int32, device="cuda")
    proj = torch.ones(api.djt3d_out_shape(N), dtype=torch.int32, device="cuda")
    announce("fullsize djt adjoint N=128 ones")
    api.djt3d_adjoint(proj, out=back, workspace=ws)
    assert bool((back == 12 * N * N).all())

    announce("fullsize djt adjoint N=128 e1 ramp")
    proj.copy_(torch.arange(E, dtype=torch.int32, device="cuda")[:, None].expand(E, E))
    api.djt3d_adjoint(proj, out=back, workspace=ws)
    lam = np.array([sum(O.line(n, s, x) for s in range(N)) for x in range(N)], dtype=np.int64)
    rng = np.random.default_rng(16)
    vox = _samples(rng, 300, (N, N, N), [(0, 0, 0), (N - 1, N - 1, N - 1), (0, N - 1, 0), (N // 2, 3, N - 2)])
    mats = []
    for k in range(12):
        M = O.frame_matrix(k)
        o0 = np.array(O.frame_to_orig(k, N, (0, 0, 0)), dtype=np.int64)
        mats.append((M, -M @ o0))
    ref = []
    for (x, y, z) in vox:
        acc = 0
        for M, off in mats:
            xp, yp, zp = M @ np.array([x, y, z], dtype=np.int64) + off
            acc += N * int(lam[zp]) + N * N * (N - 1 - int(xp))
        ref.append(acc)
    idx = torch.tensor(vox, dtype=torch.long, device="cuda")
    got = back[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(np.array(ref, dtype=np.int64)))

    announce("fullsize djt adjoint N=128 dot identity")
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    proj = torch.randint(-8, 8, api.djt3d_out_shape(N), generator=g, dtype=torch.int32, device="cuda")
    f = torch.randint(-8, 8, (N, N, N), generator=g, dtype=torch.int32, device="cuda")
    api.djt3d_adjoint(proj, out=back, workspace=ws)
    del ws
    Jf = api.djt3d_forward(f)
    lhs = sum(int((Jf[k].to(torch.int64) * proj[k]).sum()) for k in range(12))
    rhs = int((f.to(torch.int64) * back).sum())
    assert lhs == rhs
    del proj, Jf
    torch.cuda.empty_cache()


def test_inverse_n128_converges_and_is_linear():
    """The inverse in the benchmark's configuration (N = 128, 12 dodecants):
    on the corners-and-centre cube the error falls every cycle and is below
    2e-3 after ten; and inverse(A f + 2 A g) = inverse(A f) + 2 inverse(A g)
    within float32 rounding (the scheme is linear in its data)."""
    import torch
    api = _api()
    N = 128
    f = torch.from_numpy(workloads.corners_and_centre(N).astype(np.float32)).cuda()
    announce("fullsize inverse N=128 eigenvalues")
    lams = api.drt3d_inverse_lambdas(N)
    b = api.drt3d_forward(f)
    errs = []
    for cycles in (1, 3, 6, 10):
        announce("fullsize inverse N=128 cycles=%d" % cycles)
        x = api.drt3d_inverse(b, cycles, lams=lams)
        errs.append(float(torch.linalg.vector_norm(x - f) / torch.linalg.vector_norm(f)))
    print("N=128 errors after 1, 3, 6, 10 cycles:", errs)
    assert all(b2 < a for a, b2 in zip(errs, errs[1:])) and errs[-1] < 2e-3
    announce("fullsize inverse N=128 linearity")
    gv = torch.from_numpy(workloads.normal_cube(N, seed=18)).cuda()
    bg = api.drt3d_forward(gv)
    xs = api.drt3d_inverse(b + 2 * bg, 3, lams=lams)
    xf = api.drt3d_inverse(b, 3, lams=lams)
    xg = api.drt3d_inverse(bg, 3, lams=lams)
    rel = float(torch.linalg.vector_norm(xs - xf - 2 * xg) / torch.linalg.vector_norm(xs))
    print("linearity: %.2e" % rel)
    assert rel < 1e-5


def test_planted_digital_planes_n512():
    """P7 at the benchmark's size and shape: the 1 % cloud with eight planes
    drawn as eq. (9)'s digital planes (value 16). Each planted bin of the GPU
    output holds exactly 16 times the plane's voxel count, and every slope's
    displacements sum to the volume's sum."""
    import torch
    from paper_2501_13664_amd._lib import lib
    from tests import planted as P
    api = _api()
    N = 512
    vol, planes = P.point_cloud_with_digital_planes(N, n_planes=8, seed=21)
    out = torch.empty(api.drt3d_out_shape(N), dtype=torch.int32, device="cuda")
    ws = _ws(lib().drt3d_workspace_bytes(N, 0xFFF, 0))
    announce("fullsize drt N=512 planted digital planes")
    api.drt3d_forward(to_dev(vol), out=out, workspace=ws)
    del ws
    for k, s1, s2, dd, count in planes:
        assert int(out[k, s1, s2, dd]) == 16 * count, (k, s1, s2, dd, count)
    total = int(vol.astype(np.int64).sum())
    for k in sorted({p[0] for p in planes}):
        assert bool((out[k].sum(dim=-1, dtype=torch.int64) == total).all()), k
    del out
    torch.cuda.empty_cache()


def test_planted_digital_segments_djt_n128():
    """P7 for the DJT at the benchmark's size: 64 runs of eq. (13)'s digital
    lines (+8 over noise in [0, 3]); each planted bin of the GPU output holds at
    least 8 times the segment's voxel count, and equals the oracle's point
    evaluator there."""
    import torch
    from paper_2501_13664_amd._lib import lib
    from tests import planted as P
    api = _api()
    N = 128
    vol, segs = P.noise_with_digital_segments(N, n_segments=64, seed=22)
    out = torch.empty(api.djt3d_out_shape(N), dtype=torch.int32, device="cuda")
    ws = _ws(lib().djt3d_workspace_bytes(N, 0xFFF, 0))
    announce("fullsize djt N=128 planted digital segments")
    api.djt3d_forward(to_dev(vol), out=out, workspace=ws)
    del ws
    for k, s1, s2, e1, e2, count in segs:
        got = int(out[k, s1, s2, e1, e2])
        assert got >= 8 * count, (k, s1, s2, e1, e2, count)
        assert got == O.djt_point(vol, k, s1, s2, e1, e2)
    del out
    torch.cuda.empty_cache()
