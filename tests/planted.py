"""Test inputs with planted structure drawn as the paper's own digital sets
(test infrastructure: it uses the oracle's discrete line, so the product path
never sees it).

A planted plane of dodecant k, slopes (s1, s2) and displacement dd is the set
of Sec. 3.1, eq. (9): every (x', y') with z' = l_{s1}(x') + l_{s2}(y') + N-1-dd
inside the cube, mapped to the original axes by the frame of k. A planted
segment of dodecant k is a run of the digital line of Sec. 4.1, eq. (13):
(x', y', z') = (l_{s1}(u) + N-1-e1, l_{s2}(u) + N-1-e2, u) for u in [u0, u1).
"""
import numpy as np

import oracle as O


def line_table(N):
    """[s][x] -> l_s(x) (eq. (4)) for s, x in [0, N)."""
    n = N.bit_length() - 1
    return np.array([[O.line(n, s, x) for x in range(N)] for s in range(N)], dtype=np.int64)


def _to_orig(k, N, xp, yp, zp):
    """Original (x, y, z) of primed points, through the oracle's frame k."""
    M = O.frame_matrix(k)  # primed = M @ orig + off
    off = -M @ np.array(O.frame_to_orig(k, N, (0, 0, 0)), dtype=np.int64)
    P = np.stack([xp, yp, zp]).astype(np.int64) - off[:, None]
    return M.T @ P  # M is a signed permutation: its inverse is its transpose


def plane_voxels(N, k, s1, s2, dd, lt=None):
    """Flat indices of the voxels of one digital plane (eq. (9))."""
    lt = line_table(N) if lt is None else lt
    xp, yp = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    zp = lt[s1][xp] + lt[s2][yp] + N - 1 - dd
    keep = (zp >= 0) & (zp < N)
    o = _to_orig(k, N, xp[keep], yp[keep], zp[keep])
    return (o[0] * N + o[1]) * N + o[2]


def point_cloud_with_digital_planes(N, n_planes=8, occupancy=0.01, value=16, seed=2):
    """The benchmark's point-cloud shape (1 % occupancy, value 1) with
    n_planes digital planes of value `value` (overwriting), each a random
    dodecant, slope pair and displacement inside the support. Returns the cube
    and the planted (k, s1, s2, dd, voxel count)."""
    rng = np.random.default_rng(seed)
    vol = np.zeros(N ** 3, dtype=np.int32)
    occ = rng.choice(N ** 3, size=int(round(occupancy * N ** 3)), replace=False)
    vol[occ] = 1
    lt = line_table(N)
    planted = []
    for _ in range(n_planes):
        k = int(rng.integers(0, 12))
        s1, s2 = int(rng.integers(0, N)), int(rng.integers(0, N))
        dd = int(rng.integers(0, N + s1 + s2))
        idx = plane_voxels(N, k, s1, s2, dd, lt)
        vol[idx] = value
        planted.append((k, s1, s2, dd, int(idx.size)))
    return vol.reshape(N, N, N), planted


def noise_with_digital_segments(N, n_segments=64, value=8, noise_max=3, seed=3):
    """Uniform integer noise in [0, noise_max] plus n_segments runs of digital
    lines (eq. (13)), each adding `value` to the voxels it visits: a random
    dodecant, slopes, intercepts inside the support and a u-interval of length
    >= N/4. Returns the cube and the planted (k, s1, s2, e1, e2, voxel count)."""
    rng = np.random.default_rng(seed)
    vol = rng.integers(0, noise_max + 1, size=N ** 3).astype(np.int32)
    lt = line_table(N)
    planted = []
    for _ in range(n_segments):
        k = int(rng.integers(0, 12))
        s1, s2 = int(rng.integers(0, N)), int(rng.integers(0, N))
        e1, e2 = int(rng.integers(0, N + s1)), int(rng.integers(0, N + s2))
        ln = int(rng.integers(N // 4, N + 1))
        u0 = int(rng.integers(0, N - ln + 1))
        u = np.arange(u0, u0 + ln)
        xp = lt[s1][u] + N - 1 - e1
        yp = lt[s2][u] + N - 1 - e2
        keep = (xp >= 0) & (xp < N) & (yp >= 0) & (yp < N)
        o = _to_orig(k, N, xp[keep], yp[keep], u[keep])
        vol[(o[0] * N + o[1]) * N + o[2]] += value
        planted.append((k, s1, s2, e1, e2, int(keep.sum())))
    return vol.reshape(N, N, N), planted


__all__ = ["line_table", "plane_voxels", "point_cloud_with_digital_planes", "noise_with_digital_segments"]
