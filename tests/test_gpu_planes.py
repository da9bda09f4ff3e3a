"""GPU parity of plane detection (the Sec. 6.1 application) against the oracle,
through the C ABI binding: the listed bins bit-exact (index work), their count,
truncation at cap, the backprojected volume bit-exact; at N = 512 the listed
bins are checked against the rules on the GPU tensor itself."""
import numpy as np
import pytest

import oracle as O
import workloads
from oracle.planes import backproject_bins, detect_planes
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _api():
    from paper_2501_13664_amd import api
    return api


def _count(mask):
    return bin(mask).count("1")


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
@pytest.mark.parametrize("N,mask", [(2, 0xFFF), (4, 0xFFF), (8, 0x0F0), (16, 0xFFF), (32, 0xA5A)])
@pytest.mark.parametrize("cos_tol,rel", [(0.05, 0.5), (0.3, 0.0), (0.9, 0.8)])
def test_detection_matches_the_oracle(dtype, N, mask, cos_tol, rel):
    api = _api()
    R = workloads.random_projection(N, _count(mask), seed=N + mask, dtype=dtype)
    want = detect_planes(R, N, mask, cos_tol, rel)
    announce("detect planes N=%d mask=%#x %s tol=%g rel=%g" % (N, mask, np.dtype(dtype).name, cos_tol, rel))
    bins, n = api.drt3d_detect_planes(to_dev(R), cos_tol, rel, mask=mask, cap=len(want) + 8)
    assert n == len(want)
    assert bins.cpu().numpy().tolist() == want


def test_cap_truncates_the_list_and_keeps_the_count():
    api = _api()
    N = 16
    R = workloads.random_projection(N, 12, seed=5)
    want = detect_planes(R, N, 0xFFF, 0.3, 0.0)
    dR = to_dev(R)
    for cap in (1, 2, 7):
        announce("detect planes cap=%d" % cap)
        bins, n = api.drt3d_detect_planes(dR, 0.3, 0.0, cap=cap)
        assert n == len(want) and bins.cpu().numpy().tolist() == want[:cap]


def test_constant_output_gives_the_first_bin():
    """All bins equal: the first is dominant, and no plateau bin is a relative
    maximum except the first of each dodecant that is orthogonal to it."""
    import torch
    api = _api()
    N = 8
    R = np.full((12, N, N, 3 * N - 2), 3, dtype=np.int32)
    want = detect_planes(R, N, 0xFFF, 0.2, 1.0)
    announce("detect planes constant")
    bins, n = api.drt3d_detect_planes(torch.from_numpy(R).cuda(), 0.2, 1.0)
    assert bins.cpu().numpy().tolist() == want and want[0] == 0


@pytest.mark.parametrize("N", [32, 64, 128])
def test_room_scene_end_to_end(N):
    """Forward of the room scene, detection, backprojection: every step on the
    GPU, compared with the oracle's forward, detection and adjoint."""
    import torch
    api = _api()
    vol, _ = workloads.room_scene(N)
    R = O.rec_drt(vol)
    want = detect_planes(R, N, 0xFFF, 0.05, 0.5)
    announce("room scene N=%d forward" % N)
    proj = api.drt3d_forward(to_dev(vol))
    announce("room scene N=%d detect" % N)
    bins, n = api.drt3d_detect_planes(proj, 0.05, 0.5)
    assert bins.cpu().numpy().tolist() == want and n == len(want)
    announce("room scene N=%d backproject" % N)
    got = api.drt3d_backproject_bins(bins, N)
    ref = backproject_bins(want, N)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), ref)
    gotf = api.drt3d_backproject_bins(bins, N, dtype=torch.float32)
    assert np.array_equal(gotf.cpu().numpy().astype(np.int64), ref)


def test_backprojection_of_no_and_invalid_bins():
    import torch
    api = _api()
    N = 8
    announce("backproject empty")
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    assert int(api.drt3d_backproject_bins(empty, N).abs().sum()) == 0
    announce("backproject out-of-range bins")
    n = 12 * N * N * (3 * N - 2)
    bins = torch.tensor([-5, n, n + 100, 7], dtype=torch.int64, device="cuda")
    got = api.drt3d_backproject_bins(bins, N).cpu().numpy()
    assert np.array_equal(got, backproject_bins([7], N))


def test_full_size_detection_properties():
    """N = 512, the benchmark's cube (1 % point cloud + 8 planes): the first
    bin is the first maximum; every listed bin satisfies the rules (checked on
    the GPU tensor); on 400 sampled columns orthogonal to the dominant plane the
    listed bins are exactly those that satisfy them."""
    import torch
    api = _api()
    N, E = 512, 3 * 512 - 2
    vol = torch.from_numpy(workloads.point_cloud_with_planes(N, seed=2)).cuda()
    announce("full size forward N=512")
    proj = api.drt3d_forward(vol)
    announce("full size detect N=512")
    tol, rel = 0.05, 0.5
    bins, n = api.drt3d_detect_planes(proj, tol, rel, cap=1 << 20)
    assert n == bins.numel() and n >= 1
    flat = proj.view(-1)
    top = int(bins[0])
    assert top == int(torch.argmax(flat))  # the first maximal element
    topv = int(flat[top])
    thr = rel * float(topv)

    def coords(b):
        j, r = divmod(int(b), N * N * E)
        s1, r = divmod(r, N * E)
        s2, dd = divmod(r, E)
        return j, s1, s2, dd

    def normal(j, s1, s2):
        return np.array(api.drt3d_plane_normal(j, s1, s2, N), dtype=np.int64)  # all 12: rank j = dodecant j

    nt = normal(*coords(top)[:3])

    def ortho(nc):
        d = int(nt @ nc)
        return float(d * d) <= (tol * tol) * float(int(nt @ nt) * int(nc @ nc))

    def qualifying(j, s1, s2):
        """dd of the bins of column (j, s1, s2) that satisfy the rules."""
        lo1, hi1, lo2, hi2 = max(s1 - 1, 0), min(s1 + 2, N), max(s2 - 1, 0), min(s2 + 2, N)
        slab = proj[j, lo1:hi1, lo2:hi2, :].to(torch.int64)
        pad = torch.full((3, 3, E + 2), torch.iinfo(torch.int64).min, dtype=torch.int64, device="cuda")
        pad[lo1 - s1 + 1:hi1 - s1 + 1, lo2 - s2 + 1:hi2 - s2 + 1, 1:E + 1] = slab
        v = pad[1, 1, 1:E + 1]
        ok = v.double() >= thr
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in (-1, 0, 1):
                    if (a, b, c) == (0, 0, 0):
                        continue
                    w = pad[1 + a, 1 + b, 1 + c:1 + c + E]
                    ok &= (v > w) if (a, b, c) < (0, 0, 0) else (v >= w)
        return set(torch.nonzero(ok).flatten().tolist())

    listed = bins[1:].cpu().numpy().tolist()
    assert listed == sorted(listed)
    by_col = {}
    for b in listed:
        j, s1, s2, dd = coords(b)
        by_col.setdefault((j, s1, s2), set()).add(dd)
    announce("full size: %d listed bins in %d columns" % (len(listed), len(by_col)))
    rng = np.random.default_rng(0)
    cols = list(by_col)
    for c in [cols[i] for i in rng.choice(len(cols), size=min(200, len(cols)), replace=False)]:
        assert ortho(normal(*c)) and by_col[c] == qualifying(*c), c
    checked = tries = 0
    while checked < 400 and tries < 200000:
        tries += 1
        c = (int(rng.integers(12)), int(rng.integers(N)), int(rng.integers(N)))
        if not ortho(normal(*c)):
            continue
        assert by_col.get(c, set()) == qualifying(*c), c
        checked += 1
    assert checked >= 50, checked
