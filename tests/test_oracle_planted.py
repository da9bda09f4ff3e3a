"""P7, planted structure: planes and segments drawn as the paper's own digital
sets (eq. (9) planes, eq. (13) line runs, built from the closed form of eq. (4)
and the frame table) land in exactly the bin the recursions (Algorithms 1 and
3) assign them. A plane of value 16 over a cloud of 1s holds 16 per voxel of
the plane, and nothing else, in its bin; a segment of +8 over noise >= 0
holds at least 8 per voxel of the segment in its bin."""
import numpy as np
import pytest

from tests import planted as P


@pytest.mark.parametrize("N,seed", [(8, 1), (16, 2), (32, 3)])
def test_planted_planes_fill_their_bins_exactly(oracle_mod, N, seed):
    O = oracle_mod
    vol, planes = P.point_cloud_with_digital_planes(N, n_planes=6, occupancy=0.05, seed=seed)
    R = O.rec_drt(vol)
    for k, s1, s2, dd, count in planes:
        assert count > 0
        assert R[k, s1, s2, dd] == 16 * count, (k, s1, s2, dd)


def test_planted_plane_voxels_are_one_per_column(oracle_mod):
    """A digital plane meets each (x', y') column of its frame at most once, so
    its voxel count is the number of columns whose z' falls inside the cube;
    a plane through the middle of the support (dd = N-1 at slope (0, 0))
    covers the whole N x N face."""
    N = 16
    idx = P.plane_voxels(N, 0, 0, 0, N - 1)
    assert idx.size == N * N and np.unique(idx).size == N * N
    for k in range(12):
        idx = P.plane_voxels(N, k, 5, 9, 12)
        assert np.unique(idx).size == idx.size


@pytest.mark.parametrize("N,seed", [(8, 4), (16, 5)])
def test_planted_segments_reach_their_bins(oracle_mod, N, seed):
    O = oracle_mod
    vol, segs = P.noise_with_digital_segments(N, n_segments=10, seed=seed)
    noise = np.random.default_rng(seed).integers(0, 4, size=N ** 3).astype(np.int32).reshape(N, N, N)
    J = O.rec_djt(vol)
    Jn = O.rec_djt(noise)
    for k, s1, s2, e1, e2, count in segs:
        assert J[k, s1, s2, e1, e2] >= 8 * count, (k, s1, s2, e1, e2)
        # the segment's own voxels account for at least 8 * count above the noise
        assert J[k, s1, s2, e1, e2] - Jn[k, s1, s2, e1, e2] >= 8 * count


def test_a_misplaced_plane_misses_its_bin(oracle_mod):
    """The pin is sharp: the same plane drawn one displacement off puts
    nothing of itself in the bin."""
    O = oracle_mod
    N = 16
    vol = np.zeros((N, N, N), dtype=np.int32)
    vol.reshape(-1)[P.plane_voxels(N, 3, 4, 7, 20)] = 16
    R = O.rec_drt(vol)
    assert R[3, 4, 7, 20] == 16 * P.plane_voxels(N, 3, 4, 7, 20).size
    # planes of one slope pair at different displacements are disjoint
    assert R[3, 4, 7, 21] == 0 and R[3, 4, 7, 19] == 0
