"""The C ABI on the host (no GPU): the library loads, exports every symbol the
header declares, answers the host-only queries, and rejects bad arguments with
the documented status before touching a device. The frame maps it plans with
are checked against the oracle's frames."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drt3d.h")

OK, EINVAL, ENOMEM = 0, -1, -2


def _lib():
    from paper_2501_13664_amd._lib import lib
    return lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:drt3d|djt3d)_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("drt3d_forward", "djt3d_forward", "drt3d_adjoint", "drt3d_forward_batched",
                 "djt3d_forward_batched", "drt3d_adjoint_batched", "drt3d_workspace_bytes",
                 "drt3d_out_elems", "djt3d_out_elems", "drt3d_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2501_13664_amd._lib import LIB_PATH, SIGNATURES
    names = _declared()
    L = _lib()
    for nm in names:
        assert hasattr(L, nm), nm
        assert nm in SIGNATURES, "binding lacks " + nm
    dyn = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in dyn.splitlines() if line.strip())
    assert set(names) <= exported


def test_abi_version_and_size_queries():
    L = _lib()
    assert L.drt3d_abi_version() == 1
    for N in (2, 8, 64, 512):
        for mask in (0xFFF, 0x001, 0b101010101010):
            k = bin(mask).count("1")
            assert L.drt3d_out_elems(N, mask) == k * N * N * (3 * N - 2)
            assert L.djt3d_out_elems(N, mask) == k * N * N * (2 * N - 1) ** 2
            for dt in (0, 1):
                assert L.drt3d_workspace_bytes(N, mask, dt) > 0
                assert L.drt3d_adjoint_workspace_bytes(N, mask, dt) > 0
                assert L.djt3d_workspace_bytes(N, mask, dt) > 0
    for bad in ((3, 0xFFF), (1, 0xFFF), (0, 0xFFF), (2048, 0xFFF), (8, 0), (8, 0x1000)):
        assert L.drt3d_out_elems(*bad) == 0
        assert L.djt3d_out_elems(*bad) == 0
        assert L.drt3d_workspace_bytes(bad[0], bad[1], 0) == 0
    assert L.drt3d_workspace_bytes(8, 0xFFF, 7) == 0


def _fake(addr):
    return ctypes.c_void_p(addr)


def test_bad_arguments_are_rejected_before_any_device_work():
    L = _lib()
    A = _fake(1 << 20)  # aligned, never dereferenced: validation fails first
    ws_need = L.drt3d_workspace_bytes(8, 0xFFF, 0)
    cases = [
        (lambda: L.drt3d_forward(None, A, 8, 0xFFF, 0, A, ws_need, None), EINVAL, "NULL"),
        (lambda: L.drt3d_forward(A, None, 8, 0xFFF, 0, A, ws_need, None), EINVAL, "NULL"),
        (lambda: L.drt3d_forward(A, A, 6, 0xFFF, 0, A, ws_need, None), EINVAL, "power of two"),
        (lambda: L.drt3d_forward(A, A, 1, 0xFFF, 0, A, ws_need, None), EINVAL, "power of two"),
        (lambda: L.drt3d_forward(A, A, 8, 0, 0, A, ws_need, None), EINVAL, "mask"),
        (lambda: L.drt3d_forward(A, A, 8, 0x1001, 0, A, ws_need, None), EINVAL, "mask"),
        (lambda: L.drt3d_forward(A, A, 8, 0xFFF, 5, A, ws_need, None), EINVAL, "dtype"),
        (lambda: L.drt3d_forward(_fake((1 << 20) + 4), A, 8, 0xFFF, 0, A, ws_need, None), EINVAL, "aligned"),
        (lambda: L.drt3d_forward(A, A, 8, 0xFFF, 0, None, ws_need, None), EINVAL, "workspace"),
        (lambda: L.drt3d_forward(A, A, 8, 0xFFF, 0, _fake((1 << 20) + 64), ws_need, None), EINVAL, "256"),
        (lambda: L.drt3d_forward(A, A, 8, 0xFFF, 0, A, ws_need - 1, None), ENOMEM, "smaller"),
        (lambda: L.drt3d_adjoint(A, A, 8, 0xFFF, 0, A, 16, None), ENOMEM, "smaller"),
        (lambda: L.djt3d_forward(A, A, 8, 0xFFF, 0, A, 16, None), ENOMEM, "smaller"),
        (lambda: L.djt3d_forward(A, A, 12, 0xFFF, 0, A, 1 << 30, None), EINVAL, "power of two"),
    ]
    for fn, code, word in cases:
        assert fn() == code
        assert word in L.drt3d_last_error().decode()


def test_inverse_argument_checks():
    """The inverse validates N, pointers, workspace, cycles and the given
    eigenvalues before any device work."""
    L = _lib()
    A = _fake(1 << 20)
    need = L.drt3d_inverse_workspace_bytes(8)
    assert need > 0 and L.drt3d_inverse_workspace_bytes(16) > need
    for bad in (0, 1, 3, 12, 2048):
        assert L.drt3d_inverse_workspace_bytes(bad) == 0
    good = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    bad_lams = (ctypes.c_double * 3)(1.0, -2.0, 3.0)
    cases = [
        (lambda: L.drt3d_inverse(A, A, 6, 1, good, A, need, None), EINVAL, "power of two"),
        (lambda: L.drt3d_inverse(None, A, 8, 1, good, A, need, None), EINVAL, "NULL"),
        (lambda: L.drt3d_inverse(A, None, 8, 1, good, A, need, None), EINVAL, "NULL"),
        (lambda: L.drt3d_inverse(A, A, 8, 1, good, A, need - 1, None), ENOMEM, "too small"),
        (lambda: L.drt3d_inverse(A, A, 8, 1, good, _fake((1 << 20) + 64), need, None), EINVAL, "256"),
        (lambda: L.drt3d_inverse(A, A, 8, -1, good, A, need, None), EINVAL, "cycles"),
        (lambda: L.drt3d_inverse(A, A, 8, 1, bad_lams, A, need, None), EINVAL, "eigenvalue"),
        (lambda: L.drt3d_inverse_lambdas(8, None, A, need, None), EINVAL, "NULL"),
    ]
    for fn, code, word in cases:
        assert fn() == code
        assert word in L.drt3d_last_error().decode()


def test_u8_is_a_forward_only_dtype():
    """8-bit volumes: the forward takes them (N >= 32, the int32 workspace);
    every other entry point rejects the dtype before any device work."""
    L = _lib()
    A = _fake(1 << 20)
    EUNSUPPORTED = -4
    assert L.drt3d_workspace_bytes(64, 0xFFF, 2) == L.drt3d_workspace_bytes(64, 0xFFF, 0) > 0
    assert L.drt3d_adjoint_workspace_bytes(64, 0xFFF, 2) == 0
    assert L.djt3d_workspace_bytes(64, 0xFFF, 2) == 0
    ws = L.drt3d_workspace_bytes(16, 0xFFF, 0)
    assert L.drt3d_forward(A, A, 16, 0xFFF, 2, A, ws, None) == EUNSUPPORTED
    assert "N >= 32" in L.drt3d_last_error().decode()
    assert L.drt3d_adjoint(A, A, 64, 0xFFF, 2, A, 1 << 40, None) == EUNSUPPORTED
    assert L.djt3d_forward(A, A, 64, 0xFFF, 2, A, 1 << 40, None) == EINVAL


def test_batched_argument_checks():
    L = _lib()
    A = (1 << 20)
    arr = (ctypes.c_void_p * 2)(A, A)
    Ns = (ctypes.c_int * 2)(8, 16)
    bad_Ns = (ctypes.c_int * 2)(8, 24)
    assert L.drt3d_forward_batched_workspace_bytes(2, Ns, 0xFFF, 0) > 0
    assert L.drt3d_forward_batched_workspace_bytes(2, bad_Ns, 0xFFF, 0) == 0
    assert L.drt3d_forward_batched_workspace_bytes(0, Ns, 0xFFF, 0) == 0
    assert L.drt3d_forward_batched(0, arr, arr, Ns, 0xFFF, 0, _fake(A), 1 << 30, None) == EINVAL
    assert L.drt3d_forward_batched(2, None, arr, Ns, 0xFFF, 0, _fake(A), 1 << 30, None) == EINVAL
    assert L.drt3d_forward_batched(2, arr, arr, bad_Ns, 0xFFF, 0, _fake(A), 1 << 30, None) == EINVAL
    assert L.drt3d_adjoint_batched(2, arr, arr, Ns, 0xFFF, 0, _fake(A), 16, None) == ENOMEM
    assert L.djt3d_forward_batched(2, arr, arr, Ns, 0, 0, _fake(A), 1 << 30, None) == EINVAL


def test_tuning_text_round_trip_and_rejection():
    L = _lib()
    N, dt = 64, 1
    default = L.drt3d_tuning_string(N, dt)
    try:
        assert L.drt3d_set_tuning(N, dt, b"p=2.2,2.2,2.2;lds=12288;waves=4") == OK
        assert L.drt3d_tuning_string(N, dt) == b"p=2.2,2.2,2.2;lds=12288;waves=4"
        for bad in (b"p=3.3;lds=18432;waves=8",       # stages do not add up to n = 6
                    b"p=4.4,2.2;lds=1024;waves=8",    # 256 columns cannot fit 1024 elements
                    b"garbage", b""):
            assert L.drt3d_set_tuning(N, dt, bad) == EINVAL, bad
        assert L.drt3d_tuning_string(N, dt) == b"p=2.2,2.2,2.2;lds=12288;waves=4"
        # an own LDS budget for the adjoint's passes
        assert L.drt3d_set_tuning(N, dt, b"p=3.3,3.3;lds=20480;waves=8;alds=6144") == OK
        assert L.drt3d_tuning_string(N, dt) == b"p=3.3,3.3;lds=20480;waves=8;alds=6144"
        for bad in (b"p=3.3,3.3;lds=20480;waves=8;alds=512",     # below the smallest budget
                    b"p=3.3,3.3;lds=20480;waves=8;alds=2048",    # 64 columns cannot fit 2048 elements
                    b"p=3.3,3.3;lds=20480;waves=8;alds=6144;"):
            assert L.drt3d_set_tuning(N, dt, bad) == EINVAL, bad
    finally:
        assert L.drt3d_set_tuning(N, dt, default) == OK


def test_plan_text_lists_the_launches():
    L = _lib()
    buf = ctypes.create_string_buffer(1 << 16)
    n = L.drt3d_plan_text(0, 512, 0xFFF, 0, buf, len(buf))
    text = buf.value.decode()
    assert n == len(text.strip().splitlines())
    # one launch makes both frame copies (y- and x-normal): each reads and
    # writes the N^3 int32 volume once
    tr = [l for l in text.splitlines() if l.startswith("transpose_in ")]
    assert len(tr) == 1 and "drt_fwd_p" in text
    assert float(tr[0].split("bytes=")[1].split()[0]) == 2 * 2 * 4 * 512 ** 3
    assert all(l.split("kernel=")[1].startswith("fast") for l in text.splitlines() if "kind=0" in l)
    n = L.drt3d_plan_text(1, 64, 0x00F, 1, buf, len(buf))
    text = buf.value.decode()
    assert "drt_adj" in text and "transpose_out" not in text  # z-normal dodecants only
    # all twelve dodecants: the adjoint's last pass sums each layout group's
    # four dodecants in one fused launch
    for N, dt, kern in ((512, 0, "group3.3x8"), (512, 1, "group3.3x16"), (128, 0, "group2.2x8")):
        L.drt3d_plan_text(1, N, 0xFFF, dt, buf, len(buf))
        last = [l for l in buf.value.decode().splitlines() if "kind=0" in l][-1]
        assert last.startswith("drt_adj_p1 ") and last.endswith("kernel=" + kern), (N, dt, last)
    n = L.drt3d_plan_text(2, 16, 0xFFF, 0, buf, len(buf))
    assert n == 2 and buf.value.decode().count("djt_p") == 2  # 4 stages fused 2 + 2
    # the DJT adjoint: the same passes transposed, last first, then the sum of
    # the per-dodecant volumes
    n = L.drt3d_plan_text(3, 16, 0xFFF, 0, buf, len(buf))
    lines = buf.value.decode().strip().splitlines()
    assert n == 3 and [l.split()[0] for l in lines] == ["djt_adj_p2", "djt_adj_p1", "djt_adj_sum"]
    assert L.drt3d_plan_text(4, 16, 0xFFF, 0, buf, len(buf)) == EINVAL


def test_sizes_above_the_limit_are_rejected():
    """N = 1024 is past the 32-bit byte offsets of the kernels: every query
    answers 0 and every entry point EINVAL, before any device work, in the
    single-volume and the batched forms alike."""
    L = _lib()
    A = _fake(1 << 20)
    big = 1 << 40
    buf = ctypes.create_string_buffer(1 << 12)
    Ns = (ctypes.c_int * 2)(8, 1024)
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 1 << 21)
    for N in (1024, 2048):
        assert L.drt3d_out_elems(N, 0x001) == 0
        assert L.drt3d_workspace_bytes(N, 0x001, 0) == 0
        assert L.drt3d_adjoint_workspace_bytes(N, 0x001, 1) == 0
        assert L.drt3d_inverse_workspace_bytes(N) == 0
        assert L.drt3d_net_elems(N) == 0
        assert L.drt3d_forward(A, A, N, 0x001, 0, A, big, None) == EINVAL
        assert L.drt3d_adjoint(A, A, N, 0x001, 0, A, big, None) == EINVAL
        assert L.drt3d_forward(A, A, N, 0x001, 2, A, big, None) == EINVAL
        for op in (0, 1, 2, 3):
            assert L.drt3d_plan_text(op, N, 0x001, 0, buf, len(buf)) == EINVAL
    assert L.drt3d_forward_batched_workspace_bytes(2, Ns, 0x001, 0) == 0
    assert L.drt3d_adjoint_batched_workspace_bytes(2, Ns, 0x001, 0) == 0
    assert L.drt3d_forward_batched(2, ptrs, ptrs, Ns, 0x001, 0, A, big, None) == EINVAL
    assert L.drt3d_adjoint_batched(2, ptrs, ptrs, Ns, 0x001, 0, A, big, None) == EINVAL
    assert L.drt3d_out_elems(512, 0x001) == 512 * 512 * 1534


@pytest.mark.parametrize("kind", [0, 1])
def test_frame_maps_agree_with_the_oracle(oracle_mod, kind):
    """The library's affine frame maps (offset = base + sx*a + sy*b + sd*c into
    one of its volume layouts) address the same voxel as the oracle's frames.
    DRT: (a, b, c) = (x', y', N-1-z'), the displacement-oriented stage-0 column;
    DJT: (a, b, c) = (N-1-x', N-1-y', z'), the plane in intercept orientation
    and the driving coordinate u = z'."""
    L = _lib()
    N = 8
    layouts = {  # group -> index of original (x, y, z) in that layout
        0: lambda x, y, z: (x * N + y) * N + z,
        1: lambda x, y, z: (x * N + z) * N + y,
        2: lambda x, y, z: (y * N + z) * N + x,
    }
    out = (ctypes.c_int * 5)()
    rng = np.random.default_rng(kind)
    for k in range(12):
        assert L.drt3d_frame_map(k, N, kind, out) == OK
        base, sx, sy, sd, group = list(out)
        if kind == 1:
            assert group == 0  # the DJT reads the caller's volume directly
        for p in rng.integers(0, N, size=(40, 3)):
            x, y, z = oracle_mod.frame_to_orig(k, N, p)
            a, b, c = (p[0], p[1], N - 1 - p[2]) if kind == 0 else (N - 1 - p[0], N - 1 - p[1], p[2])
            assert base + sx * a + sy * b + sd * c == layouts[group](x, y, z), (k, tuple(p))
    assert L.drt3d_frame_map(12, N, 0, out) == EINVAL


def test_plane_normals_agree_with_the_oracle(oracle_mod):
    """The library's plane normals (host code) against the oracle's, every
    dodecant, a spread of slopes and sizes."""
    from oracle.planes import plane_normal
    L = _lib()
    out = (ctypes.c_int * 3)()
    for N in (2, 8, 64, 512):
        for k in range(12):
            for s1, s2 in ((0, 0), (N - 1, 0), (0, N - 1), (N // 2, N - 1), (1, N // 2)):
                assert L.drt3d_plane_normal(k, s1, s2, N, out) == OK
                assert list(out) == plane_normal(k, s1, s2, N).tolist(), (N, k, s1, s2)
    for args in ((12, 0, 0, 8), (0, 8, 0, 8), (0, 0, -1, 8), (0, 0, 0, 6)):
        assert L.drt3d_plane_normal(*args, out) == EINVAL


def test_plane_detection_argument_checks():
    """Detection and backprojection validate sizes, pointers, tolerances and
    workspace before any device work."""
    L = _lib()
    A = _fake(1 << 20)
    need = L.drt3d_detect_planes_workspace_bytes(8, 0xFFF, 0)
    # partials, top, threshold, then 4 + 8 bytes per output column
    assert need >= 12 * 12 * 8 * 8 and L.drt3d_detect_planes_workspace_bytes(16, 0xFFF, 1) > need
    assert L.drt3d_detect_planes_workspace_bytes(6, 0xFFF, 0) == 0
    assert L.drt3d_detect_planes_workspace_bytes(8, 0xFFF, 2) == 0  # int32 and float32 only
    bneed = L.drt3d_backproject_bins_workspace_bytes(8, 0xFFF, 0)
    assert bneed >= 12 * 8 * 8 * 22 * 4 + L.drt3d_adjoint_workspace_bytes(8, 0xFFF, 0)
    cases = [
        (lambda: L.drt3d_detect_planes(A, 6, 0xFFF, 0, 0.05, 0.5, A, 16, A, A, need, None), EINVAL, "power of two"),
        (lambda: L.drt3d_detect_planes(None, 8, 0xFFF, 0, 0.05, 0.5, A, 16, A, A, need, None), EINVAL, "NULL"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 0.05, 0.5, None, 16, A, A, need, None), EINVAL, "bins"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 0.05, 0.5, A, 0, A, A, need, None), EINVAL, "cap"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 0.05, 0.5, A, 16, None, A, need, None), EINVAL, "count"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 1.0, 0.5, A, 16, A, A, need, None), EINVAL, "cos_tol"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, -0.1, 0.5, A, 16, A, A, need, None), EINVAL, "cos_tol"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 0.05, float("nan"), A, 16, A, A, need, None), EINVAL,
         "rel_threshold"),
        (lambda: L.drt3d_detect_planes(A, 8, 0xFFF, 0, 0.05, 0.5, A, 16, A, A, need - 1, None), ENOMEM, "smaller"),
        (lambda: L.drt3d_backproject_bins(A, A, 4, A, 8, 0xFFF, 0, A, bneed - 1, None), ENOMEM, "smaller"),
        (lambda: L.drt3d_backproject_bins(None, A, 4, A, 8, 0xFFF, 0, A, bneed, None), EINVAL, "bins"),
        (lambda: L.drt3d_backproject_bins(A, A, -1, A, 8, 0xFFF, 0, A, bneed, None), EINVAL, "cap"),
        (lambda: L.drt3d_backproject_bins(A, A, 4, None, 8, 0xFFF, 0, A, bneed, None), EINVAL, "NULL"),
    ]
    for fn, code, word in cases:
        assert fn() == code
        assert word in L.drt3d_last_error().decode()


def test_stream_probe_rejects_bad_sizes_before_device_work():
    L = _lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)  # never dereferenced: rejected first
    for rb, wb in ((0, 16), (16, 0), (17, 16), (16, 24), (64 << 30, 16)):
        assert L.drt3d_stream_probe(a, rb, b, wb, None) == EINVAL
    assert L.drt3d_stream_probe(None, 16, b, 16, None) == EINVAL


def test_plan_create_checks_and_workspace_queries():
    """drt3d_plan_create rejects what the op's own call rejects, leaving the
    handle NULL; a plan's workspace equals the op's own query; destroy takes
    NULL; executing a NULL plan or with NULL buffers fails before device work."""
    L = _lib()
    EUNSUP = -4
    h = ctypes.c_void_p(1234)
    assert L.drt3d_plan_create(None, 0, 32, 0xFFF, 0) == EINVAL
    for (op, N, mask, dt), want in (((4, 32, 0xFFF, 0), EINVAL), ((-1, 32, 0xFFF, 0), EINVAL),
                                    ((0, 3, 0xFFF, 0), EINVAL), ((0, 1024, 0xFFF, 0), EINVAL),
                                    ((1, 32, 0, 0), EINVAL), ((2, 32, 0x1000, 0), EINVAL),
                                    ((0, 32, 0xFFF, 7), EINVAL), ((1, 64, 0xFFF, 2), EUNSUP),
                                    ((0, 16, 0xFFF, 2), EUNSUP), ((2, 512, 0x001, 0), EUNSUP)):
        h.value = 1234
        assert L.drt3d_plan_create(ctypes.byref(h), op, N, mask, dt) == want, (op, N, mask, dt)
        assert h.value is None, (op, N, mask, dt)
    queries = {0: L.drt3d_workspace_bytes, 1: L.drt3d_adjoint_workspace_bytes,
               2: L.djt3d_workspace_bytes, 3: L.djt3d_adjoint_workspace_bytes}
    for op in range(4):
        for N, mask, dt in ((8, 0xFFF, 0), (64, 0x0F0, 1), (32, 0x001, 0)):
            assert L.drt3d_plan_create(ctypes.byref(h), op, N, mask, dt) == OK
            assert h.value
            assert L.drt3d_plan_workspace_bytes(h) == queries[op](N, mask, dt)
            # NULL buffers are rejected before any device work
            assert L.drt3d_plan_execute(h, None, None, None, 0, None) == EINVAL
            assert L.drt3d_plan_destroy(h) == OK
    assert L.drt3d_plan_create(ctypes.byref(h), 0, 64, 0xFFF, 2) == OK  # uint8 forward
    assert L.drt3d_plan_workspace_bytes(h) == L.drt3d_workspace_bytes(64, 0xFFF, 2)
    assert L.drt3d_plan_destroy(h) == OK
    assert L.drt3d_plan_workspace_bytes(None) == 0
    assert L.drt3d_plan_execute(None, None, None, None, 0, None) == EINVAL
    assert L.drt3d_plan_destroy(None) == OK


def test_djt_builtin_pass_plan(monkeypatch):
    """The DJT's built-in plan: passes of two stages, and one stage first when
    log2 N is odd (one launch per pass); DRT3D_DJT_PASSES overrides it, and an
    override that does not sum to log2 N is ignored."""
    L = _lib()
    monkeypatch.delenv("DRT3D_DJT_PASSES", raising=False)
    buf = ctypes.create_string_buffer(1 << 14)
    for N in (2, 4, 8, 16, 32, 64, 128, 256):
        n = N.bit_length() - 1
        assert L.drt3d_plan_text(2, N, 0x001, 0, buf, len(buf)) == (n + 1) // 2, N
    monkeypatch.setenv("DRT3D_DJT_PASSES", "3,1,3")
    assert L.drt3d_plan_text(2, 128, 0x001, 0, buf, len(buf)) == 3
    monkeypatch.setenv("DRT3D_DJT_PASSES", "3,3")  # sums to 6, not 7
    assert L.drt3d_plan_text(2, 128, 0x001, 0, buf, len(buf)) == 4
