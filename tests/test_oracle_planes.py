"""Pins of the plane-detection oracle (Sec. 6.1 application) against what the
paper and the geometry fix: the basic dodecant's normal (Sec. 3), normals
rebuilt from three points of each dodecant's planes, the discrete plane a
one-hot backprojection marks (eq. (4) lines, Sec. 5.1 adjoint), a cube of
three orthogonal walls whose detections follow by hand, the plateau rule,
brute-force relative maxima, and the room scene's walls."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads
from oracle.planes import (backproject_bins, bin_coords, detect_planes, is_orthogonal, local_maxima,
                           plane_normal)


def _flat(N, j, s1, s2, dd):
    return ((j * N + s1) * N + s2) * (3 * N - 2) + dd


@pytest.mark.parametrize("N", [4, 16, 128])
def test_normal_of_the_basic_dodecant(N):
    """Sec. 3: dodecant 0's planes at slopes (s1, s2) have the normal (-s1, -s2, N-1)/(N-1)."""
    for s1, s2 in ((0, 0), (1, 0), (0, N - 1), (N - 1, N - 1), (N // 2, 1)):
        assert plane_normal(0, s1, s2, N).tolist() == [-s1, -s2, N - 1]


def test_normals_from_three_points_of_each_plane():
    """The plane z' = s1 x'/(N-1) + s2 y'/(N-1) passes through the primed points
    (0,0,0), (N-1,0,s1), (0,N-1,s2); mapped to (x, y, z) by the frame table,
    their edge vectors' cross product is parallel to plane_normal."""
    N = 8
    for k in range(12):
        for s1, s2 in itertools.product((0, 3, 7), repeat=2):
            a, b, c = (np.array(O.frame_to_orig(k, N, p), dtype=np.int64)
                       for p in ((0, 0, 0), (N - 1, 0, s1), (0, N - 1, s2)))
            cr = np.cross(b - a, c - a)
            n = plane_normal(k, s1, s2, N)
            assert np.any(cr != 0) and not np.any(np.cross(cr, n)), (k, s1, s2, cr, n)


@pytest.mark.parametrize("k,s1,s2,dd", [(0, 0, 0, 0), (1, 3, 5, 9), (4, 7, 2, 12), (6, 5, 5, 7),
                                         (8, 1, 6, 20), (11, 7, 7, 3)])
def test_one_hot_backprojection_is_the_discrete_plane(k, s1, s2, dd):
    """The adjoint of one bin marks exactly the voxels of its discrete plane
    z' = l_s1(x') + l_s2(y') + N-1-dd, mapped through dodecant k's frame."""
    N, n = 8, 3
    vol = backproject_bins([_flat(N, k, s1, s2, dd)], N)
    want = np.zeros((N, N, N), dtype=np.int64)
    for xp in range(N):
        for yp in range(N):
            zp = O.line(n, s1, xp) + O.line(n, s2, yp) + N - 1 - dd
            if 0 <= zp < N:
                want[O.frame_to_orig(k, N, (xp, yp, zp))] = 1
    assert np.array_equal(vol, want)


def test_three_orthogonal_walls():
    """Walls x = a, y = b and floor z = c, each N^2 voxels of value 1. All three
    bins at slopes (0, 0) hold N^2; dodecant 0 comes first, so the floor is the
    dominant plane. Above 0.9 N^2 the only other bins are the two walls at
    slopes (0, 0) in each of the four dodecants of their normal's group."""
    N, a, b, c = 16, 5, 11, 3
    vol = np.zeros((N, N, N), dtype=np.int32)
    vol[a, :, :] = 1
    vol[:, b, :] = 1
    vol[:, :, c] = 1
    R = O.rec_drt(vol)
    got = detect_planes(R, N, 0xFFF, cos_tol=0.05, rel_threshold=0.9)
    assert got[0] == _flat(N, 0, 0, 0, N - 1 - c) and R.reshape(-1)[got[0]] == N * N
    want = []
    for k in range(12):
        # the axis that z' runs along, and the z' whose slice is the wall on it
        o0, o1 = np.array(O.frame_to_orig(k, N, (0, 0, 0))), np.array(O.frame_to_orig(k, N, (0, 0, 1)))
        axis = int(np.flatnonzero(o1 != o0)[0])
        if axis == 2:
            continue
        wall = a if axis == 0 else b
        zp = [z for z in range(N) if O.frame_to_orig(k, N, (0, 0, z))[axis] == wall][0]
        want.append(_flat(N, k, 0, 0, N - 1 - zp))
    assert got[1:] == sorted(want) and len(want) == 8


def test_plateau_yields_its_first_bin():
    N = 4
    E = 3 * N - 2
    R = np.zeros((12, N, N, E), dtype=np.int32)
    R[0, 0, 0, 0] = 100          # dominant: the z-normal plane of dodecant 0
    R[4, 1, 1, 3:6] = 60         # a plateau along dd
    R[5, 0, 1:3, 2] = 70         # a plateau along s2
    R[6, 2, 0, 4] = 50           # exactly at the threshold: kept
    R[7, 1, 2, 6] = 49           # just below it
    got = detect_planes(R, N, 0xFFF, cos_tol=0.99, rel_threshold=0.5)
    assert got == [_flat(N, 0, 0, 0, 0), _flat(N, 4, 1, 1, 3), _flat(N, 5, 0, 1, 2), _flat(N, 6, 2, 0, 4)]


def test_local_maxima_against_brute_force():
    """Tiny arrays with many ties, against a direct loop over flat indices."""
    rng = np.random.default_rng(3)
    for shape in ((2, 3, 4), (3, 3, 5), (4, 2, 7)):
        for _ in range(20):
            R = rng.integers(0, 3, size=shape)
            A, B, C = shape
            want = np.ones(shape, dtype=bool)
            for i, j, l in itertools.product(range(A), range(B), range(C)):
                p = (i * B + j) * C + l
                for a, b, c in itertools.product((-1, 0, 1), repeat=3):
                    q3 = (i + a, j + b, l + c)
                    if (a, b, c) == (0, 0, 0) or not all(0 <= q3[t] < shape[t] for t in range(3)):
                        continue
                    q = (q3[0] * B + q3[1]) * C + q3[2]
                    if (R[q3] >= R[i, j, l]) if q < p else (R[q3] > R[i, j, l]):
                        want[i, j, l] = False
            assert np.array_equal(local_maxima(R), want)
            assert np.array_equal(local_maxima(R.astype(np.float32)), want)


def test_orthogonality_is_the_cosine_bound():
    n = np.array([0, 0, 7])
    assert is_orthogonal(n, np.array([7, 0, 0]), 0.0)
    assert not is_orthogonal(n, np.array([7, 0, 1]), 0.0)
    c = 1 / np.sqrt(50.0)  # cos between (0,0,7) and (7,0,1)
    assert is_orthogonal(n, np.array([7, 0, 1]), c * 1.0001)
    assert not is_orthogonal(n, np.array([7, 0, 1]), c * 0.9999)
    with pytest.raises(ValueError):
        detect_planes(np.zeros((12, 2, 2, 4)), 2, cos_tol=1.0)


def test_room_scene_walls():
    """The room's floor is the dominant plane; the detections orthogonal to it
    include the back wall and both side walls (same normal, offsets apart),
    and their backprojection marks most of the scene's occupied voxels."""
    N = 64
    vol, surf = workloads.room_scene(N)
    R = O.rec_drt(vol)
    bins = detect_planes(R, N, 0xFFF, cos_tol=0.05, rel_threshold=0.5)
    unit = lambda b: (lambda n: n / np.linalg.norm(n))(plane_normal(*bin_coords(b, N)[:3], N).astype(float))
    assert abs(np.dot(unit(bins[0]), surf["floor"])) > 0.9999
    for name in ("back", "left"):
        assert any(abs(np.dot(unit(b), surf[name])) > 0.995 for b in bins[1:]), name
    side = [bin_coords(b, N) for b in bins[1:] if abs(np.dot(unit(b), surf["left"])) > 0.995]
    k0 = side[0][0]
    dds = [c[3] for c in side if c[0] == k0]
    assert max(dds) - min(dds) > N // 2  # two walls, at the room's two sides
    marked = backproject_bins(bins, N) > 0
    assert (marked & (vol > 0)).sum() > 0.6 * vol.sum()
