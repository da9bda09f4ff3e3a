"""GPU parity of the HIP path against the CPU oracle, through the C ABI binding.

int32 results must be bit-exact; float32 results must lie within 1e-5 of the
float64 oracle both normwise and elementwise relative to R(|f|) (the transform
of |f|), the bound that cancellation in near-zero sums cannot break.
"""
import numpy as np
import pytest

import oracle as O
import workloads
from tests.gpu_util import FLOAT_TOL, announce, device, float_errors, to_dev

pytestmark = pytest.mark.gpu

MASKS = [0xFFF, 0x001, 0x00F, 0xFF0, 0b101001010010, 0x800]


def _api():
    from paper_2501_13664_amd import api
    return api


# ------------------------------------------------------------------- DRT
@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_drt_int_small_all_masks(N):
    api = _api()
    vol = workloads.uniform_int_cube(N, -1000, 1000, seed=100 + N)
    full = O.wrap_int32(O.def_drt(vol))
    for mask in MASKS:
        announce("drt int N=%d mask=%#x" % (N, mask))
        got = api.drt3d_forward(to_dev(vol), mask).cpu().numpy()
        sel = [k for k in range(12) if (mask >> k) & 1]
        assert np.array_equal(got, full[sel]), "N=%d mask=%#x" % (N, mask)


@pytest.mark.parametrize("N", [32, 64])
def test_drt_int_full_vs_recursion(N):
    """N=32 is the uniform [0,255] cube of seed 1; N=64 spans several LDS tiles."""
    api = _api()
    vol = workloads.uniform_int_cube(N, 0, 255, seed=1)
    announce("drt int N=%d all" % N)
    got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.rec_drt(vol)))


def test_drt_int_wraps_like_int32():
    api = _api()
    N = 8
    vol = workloads.uniform_int_cube(N, 2 ** 30, 2 ** 31 - 1, seed=3)
    announce("drt int wrap N=8")
    got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.def_drt(vol)))


@pytest.mark.parametrize("N", [4, 16, 32])
def test_drt_float_tolerance(N):
    api = _api()
    vol = workloads.normal_cube(N, seed=10 + N)
    announce("drt f32 N=%d" % N)
    got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
    ref = O.rec_drt(vol.astype(np.float64))
    rabs = O.rec_drt(np.abs(vol).astype(np.float64))
    nw, el = float_errors(got, ref, rabs)
    print("N=%d normwise %.3e elementwise/R|f| %.3e" % (N, nw, el))
    assert nw <= FLOAT_TOL and el <= FLOAT_TOL


# ------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_adjoint_int_small(N):
    api = _api()
    rng = np.random.default_rng(N)
    for mask in (0xFFF, 0x002, 0b110000110000, 0x0F0):
        nd = O.count_dodecants(mask)
        proj = rng.integers(-500, 500, size=(nd, N, N, 3 * N - 2)).astype(np.int32)
        announce("adjoint int N=%d mask=%#x" % (N, mask))
        got = api.drt3d_adjoint(to_dev(proj), mask).cpu().numpy()
        assert np.array_equal(got, O.wrap_int32(O.def_adj(proj, N, mask))), "N=%d mask=%#x" % (N, mask)


@pytest.mark.parametrize("N", [32, 64])
def test_adjoint_int_vs_recursion(N):
    api = _api()
    rng = np.random.default_rng(7)
    proj = rng.integers(-100, 100, size=(12, N, N, 3 * N - 2)).astype(np.int32)
    announce("adjoint int N=%d" % N)
    got = api.drt3d_adjoint(to_dev(proj)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.rec_adj(proj, N)))


def test_adjoint_is_transpose_on_gpu():
    """<R f, p> = <f, R^T p> with both sides computed on the GPU (int64 sums)."""
    api = _api()
    N = 32
    rng = np.random.default_rng(11)
    f = rng.integers(-20, 20, size=(N, N, N)).astype(np.int32)
    p = rng.integers(-20, 20, size=(12, N, N, 3 * N - 2)).astype(np.int32)
    announce("adjoint dot N=32")
    Rf = api.drt3d_forward(to_dev(f)).cpu().numpy().astype(np.int64)
    Rtp = api.drt3d_adjoint(to_dev(p)).cpu().numpy().astype(np.int64)
    assert int((Rf * p).sum()) == int((f.astype(np.int64) * Rtp).sum())


# ------------------------------------------------------------------- DJT
@pytest.mark.parametrize("N", [2, 4, 8])
def test_djt_int_small(N):
    api = _api()
    vol = workloads.uniform_int_cube(N, -300, 300, seed=200 + N)
    full = O.wrap_int32(O.def_djt(vol))
    for mask in MASKS:
        announce("djt int N=%d mask=%#x" % (N, mask))
        got = api.djt3d_forward(to_dev(vol), mask).cpu().numpy()
        sel = [k for k in range(12) if (mask >> k) & 1]
        assert np.array_equal(got, full[sel]), "N=%d mask=%#x" % (N, mask)


@pytest.mark.parametrize("N", [16, 32])
def test_djt_int_vs_recursion(N):
    api = _api()
    vol = workloads.noise_with_segments(N, n_segments=4, seed=N)
    mask = 0xFFF if N == 16 else 0b100100100101
    announce("djt int N=%d" % N)
    got = api.djt3d_forward(to_dev(vol), mask).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.rec_djt(vol, mask)))


def test_djt_float_tolerance():
    api = _api()
    N = 16
    vol = workloads.normal_cube(N, seed=3)
    announce("djt f32 N=16")
    got = api.djt3d_forward(to_dev(vol)).cpu().numpy()
    ref = O.rec_djt(vol.astype(np.float64))
    rabs = O.rec_djt(np.abs(vol).astype(np.float64))
    nw, el = float_errors(got, ref, rabs)
    print("normwise %.3e elementwise/R|f| %.3e" % (nw, el))
    assert nw <= FLOAT_TOL and el <= FLOAT_TOL


# ------------------------------------------------------------------- batched
def test_batched_equals_single_int():
    api = _api()
    cubes = [workloads.uniform_int_cube(N, -50, 50, seed=i) for i, N in enumerate([8, 16, 4, 32, 8, 2])]
    dev = [to_dev(c) for c in cubes]
    announce("batched drt int mixed")
    outs = api.drt3d_forward_batched(dev)
    for c, d, o in zip(cubes, dev, outs):
        assert np.array_equal(o.cpu().numpy(), api.drt3d_forward(d).cpu().numpy())
    announce("batched adjoint int mixed")
    backs = api.drt3d_adjoint_batched(outs)
    for o, b in zip(outs, backs):
        assert np.array_equal(b.cpu().numpy(), api.drt3d_adjoint(o).cpu().numpy())
    announce("batched djt int mixed")
    js = api.djt3d_forward_batched(dev[:3])
    for d, j in zip(dev[:3], js):
        assert np.array_equal(j.cpu().numpy(), api.djt3d_forward(d).cpu().numpy())


# ------------------------------------------------------------------- tunings
TUNINGS = {
    8: ["p=3.3;lds=20480;waves=8", "p=1.1,1.1,1.1;lds=1024;waves=4", "p=2.1,1.2;lds=2048;waves=8",
        "p=3.0,0.3;lds=4096;waves=2", "p=0.3,3.0;lds=1024;waves=1"],
    32: ["p=3.3,2.2;lds=20480;waves=8", "p=2.2,3.3;lds=6144;waves=8", "p=1.2,2.1,2.2;lds=2048;waves=4",
         "p=5.0,0.5;lds=40960;waves=8", "p=4.4,1.1;lds=40960;waves=8", "p=2.3,3.2;lds=8192;waves=4"],
    64: ["p=3.3,3.3;lds=20480;waves=8", "p=3.3,3.3;lds=6144;waves=8", "p=2.2,2.2,2.2;lds=12288;waves=4",
         "p=4.3,2.3;lds=16384;waves=8", "p=3.3,3.3;lds=14336;waves=8;alds=6144",
         "p=2.2,2.2,2.2;lds=6144;waves=8;alds=20480"],
}


@pytest.mark.parametrize("N", sorted(TUNINGS))
def test_every_tuning_is_bit_exact(N):
    """Pass lists, LDS budgets (hence tile counts) and wave counts change the
    schedule, never the int32 result; forward and adjoint both."""
    api = _api()
    import torch
    vol = workloads.uniform_int_cube(N, -99, 99, seed=N + 40)
    ref = O.wrap_int32(O.rec_drt(vol))
    rng = np.random.default_rng(N)
    proj = rng.integers(-50, 50, size=ref.shape).astype(np.int32)
    ref_adj = O.wrap_int32(O.rec_adj(proj, N))
    default = api.drt3d_tuning_string(N, torch.int32)
    try:
        for t in TUNINGS[N]:
            announce("tuning N=%d %s" % (N, t))
            api.drt3d_set_tuning(N, t, torch.int32)
            assert np.array_equal(api.drt3d_forward(to_dev(vol)).cpu().numpy(), ref), t
            assert np.array_equal(api.drt3d_adjoint(to_dev(proj)).cpu().numpy(), ref_adj), t
    finally:
        api.drt3d_set_tuning(N, default, torch.int32)


def test_drt_int_n128_full():
    api = _api()
    N = 128
    vol = workloads.uniform_int_cube(N, 0, 255, seed=5)
    announce("drt int N=128 full")
    got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
    assert np.array_equal(got, O.wrap_int32(O.rec_drt(vol)))


def test_autotune_picks_a_valid_tuning_and_stays_exact():
    """The autotuner times candidates on the GPU and keeps the fastest; the
    transform under its choice is still bit-exact (int32) and within the float
    tolerance (float32, forward + adjoint are what it timed)."""
    api = _api()
    import torch
    for N, dt in ((32, torch.int32), (16, torch.float32)):
        before = api.drt3d_tuning_string(N, dt)
        try:
            announce("autotune N=%d %s" % (N, dt))
            chosen = api.drt3d_autotune(N, dt)
            assert chosen.startswith("p=") and chosen == api.drt3d_tuning_string(N, dt)
            if dt == torch.int32:
                vol = workloads.uniform_int_cube(N, -99, 99, seed=77)
                got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
                assert np.array_equal(got, O.wrap_int32(O.rec_drt(vol)))
            else:
                vol = workloads.normal_cube(N, seed=78)
                got = api.drt3d_forward(to_dev(vol)).cpu().numpy()
                nw, el = float_errors(got, O.rec_drt(vol.astype(np.float64)),
                                      O.rec_drt(np.abs(vol).astype(np.float64)))
                assert nw <= FLOAT_TOL and el <= FLOAT_TOL
        finally:
            api.drt3d_set_tuning(N, before, dt)


def test_adjoint_float_tolerance():
    """float32 backprojection within 1e-5 of the FP64 transpose, relative to
    R^T(|p|)."""
    api = _api()
    N = 32
    rng = np.random.default_rng(79)
    proj = rng.standard_normal((12, N, N, 3 * N - 2)).astype(np.float32)
    announce("adjoint f32 N=32")
    got = api.drt3d_adjoint(to_dev(proj)).cpu().numpy()
    ref = O.rec_adj(proj.astype(np.float64), N)
    rabs = O.rec_adj(np.abs(proj).astype(np.float64), N)
    nw, el = float_errors(got, ref, rabs)
    print("adjoint N=32 normwise %.3e elementwise/R^T|p| %.3e" % (nw, el))
    assert nw <= FLOAT_TOL and el <= FLOAT_TOL
