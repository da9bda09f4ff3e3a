"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the transforms' arithmetic: it only draws cubes with
numpy's PCG64 generator. The shapes and value distributions stand in for the
paper's workloads (a voxelized depth scene with planes, Sec. 6.1; a ray buried
in noise, Sec. 4.1; corner voxels and the centre of a cube, Sec. 5.1), whose data
are not available. Planes and segments are drawn as rounded continuous planes
and lines, not as the transforms' own digital sets.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_int_cube", "normal_cube", "point_cloud_with_planes",
    "noise_with_segments", "mixed_batch", "corners_and_centre", "normal_batch",
    "normal_weights", "random_voxels", "room_scene", "random_projection", "WORKLOADS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_int_cube(N: int, lo: int = 0, hi: int = 255, seed: int = 1) -> np.ndarray:
    """int32 cube, values uniform integers in [lo, hi]."""
    return _rng(seed).integers(lo, hi + 1, size=(N, N, N), dtype=np.int64).astype(np.int32)


def normal_cube(N: int, seed: int = 5) -> np.ndarray:
    """float32 cube, values N(0,1)."""
    return _rng(seed).standard_normal(size=(N, N, N)).astype(np.float32)


def _random_plane_voxels(N: int, rng: np.random.Generator):
    """Voxels of a rounded continuous plane with a random normal (upper
    hemisphere) through a random point of the cube."""
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    if n[2] < 0:
        n = -n
    p0 = rng.uniform(0, N - 1, size=3)
    c = int(np.argmax(np.abs(n)))
    a, b = [i for i in range(3) if i != c]
    ia, ib = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ic = np.rint(p0[c] - (n[a] * (ia - p0[a]) + n[b] * (ib - p0[b])) / n[c]).astype(np.int64)
    ok = (ic >= 0) & (ic < N)
    coords = np.zeros((3, int(ok.sum())), dtype=np.int64)
    coords[a], coords[b], coords[c] = ia[ok], ib[ok], ic[ok]
    return coords


def point_cloud_with_planes(N: int = 512, occupancy: float = 0.01, n_planes: int = 8,
                            plane_value: int = 16, seed: int = 2) -> np.ndarray:
    """int32 cube: a sparse point cloud (value 1) at the given occupancy, chosen
    uniformly without replacement, plus planes with random normals inside the
    hemisphere and random offsets (value ``plane_value``, overwriting)."""
    rng = _rng(seed)
    vol = np.zeros(N * N * N, dtype=np.int32)
    count = int(round(occupancy * N ** 3))
    idx = rng.choice(N ** 3, size=count, replace=False)
    vol[idx] = 1
    vol = vol.reshape(N, N, N)
    for _ in range(n_planes):
        x, y, z = _random_plane_voxels(N, rng)
        vol[x, y, z] = plane_value
    return vol


def noise_with_segments(N: int = 128, n_segments: int = 64, seg_value: int = 8,
                        noise_max: int = 3, seed: int = 3) -> np.ndarray:
    """int32 cube: uniform integer noise in [0, noise_max] plus random 3D digital
    segments (rounded continuous lines of length >= N/4 along their dominant
    axis) that add ``seg_value`` to every voxel they visit."""
    rng = _rng(seed)
    vol = rng.integers(0, noise_max + 1, size=(N, N, N), dtype=np.int64).astype(np.int32)
    for _ in range(n_segments):
        d = rng.standard_normal(3)
        d /= np.max(np.abs(d))              # unit step along the dominant axis
        length = int(rng.integers(max(1, N // 4), N + 1))
        p0 = rng.uniform(0, N - 1, size=3)
        t = np.arange(length)[:, None]
        pts = np.rint(p0[None, :] + t * d[None, :]).astype(np.int64)
        ok = np.all((pts >= 0) & (pts < N), axis=1)
        pts = pts[ok]
        if len(pts):
            np.add.at(vol, (pts[:, 0], pts[:, 1], pts[:, 2]), seg_value)
    return vol


def mixed_batch(counts=((32, 48), (64, 32), (128, 12), (256, 4)), seed0: int = 1000):
    """List of float32 N(0,1) cubes of mixed sizes; cube i uses seed seed0 + i."""
    cubes, i = [], 0
    for N, c in counts:
        for _ in range(c):
            cubes.append(normal_cube(N, seed=seed0 + i))
            i += 1
    return cubes


def normal_batch(B: int = 8, N: int = 128, seed: int = 5) -> np.ndarray:
    """float32 [B][N][N][N], values N(0,1), drawn in order from one stream."""
    rng = _rng(seed)
    return rng.standard_normal(size=(B, N, N, N), dtype=np.float32)


def normal_weights(shape, seed: int = 6) -> np.ndarray:
    """float32 N(0,1) weights of the given shape (e.g. shaped like a batch of
    transforms), drawn in C order from one stream."""
    return _rng(seed).standard_normal(size=tuple(shape), dtype=np.float32)


def random_voxels(count: int, B: int, N: int, seed: int = 7) -> np.ndarray:
    """[count][4] int64 (b, x, y, z) positions, distinct, uniform over a batch."""
    rng = _rng(seed)
    flat = rng.choice(B * N ** 3, size=count, replace=False)
    b, r = np.divmod(flat, N ** 3)
    x, r = np.divmod(r, N * N)
    y, z = np.divmod(r, N)
    return np.stack([b, x, y, z], axis=1).astype(np.int64)


def corners_and_centre(N: int = 64, value: int = 1) -> np.ndarray:
    """int32 cube with the 8 corner voxels and the centre voxel set (Sec. 5.1)."""
    vol = np.zeros((N, N, N), dtype=np.int32)
    for x in (0, N - 1):
        for y in (0, N - 1):
            for z in (0, N - 1):
                vol[x, y, z] = value
    vol[N // 2, N // 2, N // 2] = value
    return vol


def _sample_rect(origin, du, dv, h=0.5):
    """Points of the parallelogram origin + a du + b dv, a, b in [0, 1], on a
    grid of step h voxels along each edge."""
    origin, du, dv = (np.asarray(v, dtype=np.float64) for v in (origin, du, dv))
    na = max(2, int(np.ceil(np.linalg.norm(du) / h)) + 1)
    nb = max(2, int(np.ceil(np.linalg.norm(dv) / h)) + 1)
    a, b = np.meshgrid(np.linspace(0, 1, na), np.linspace(0, 1, nb), indexing="ij")
    return origin + a.reshape(-1, 1) * du + b.reshape(-1, 1) * dv


def room_scene(N: int = 128, seed: int = 11, n_objects: int = 6, noise: float = 0.002):
    """A voxelized indoor depth scene (the plane-detection example of Sec. 6.1),
    as an int32 occupancy cube (1 = a surface point was seen there).

    A box-shaped room turned by a random yaw about the vertical z axis, seen
    from inside: the floor, the half of the ceiling away from the sensor and
    three walls (the fourth is behind the sensor), sampled every half voxel and
    rounded to voxels; boxes standing on the floor (top and four sides); and a
    fraction ``noise`` of the voxels set at random. Returns (cube, surfaces)
    where surfaces maps "floor", "ceiling", "back", "left", "right" to the unit
    normal (x, y, z) of that surface."""
    rng = _rng(seed)
    yaw = np.deg2rad(rng.uniform(8.0, 25.0))
    cu, su = np.cos(yaw), np.sin(yaw)
    U = np.array([cu, su, 0.0])   # the room's depth axis (towards the back wall)
    V = np.array([-su, cu, 0.0])  # its width axis
    Z = np.array([0.0, 0.0, 1.0])
    c = np.array([N / 2.0, N / 2.0, 0.0])
    au, av = 0.40 * N, 0.38 * N          # half depth and half width
    z0, z1 = 0.10 * N, 0.88 * N          # floor and ceiling heights
    corner = lambda u, v, z: c + u * U + v * V + z * Z
    pts = [
        _sample_rect(corner(-au, -av, z0), 2 * au * U, 2 * av * V),            # floor
        _sample_rect(corner(0.0, -av, z1), au * U, 2 * av * V),                 # ceiling, far half
        _sample_rect(corner(au, -av, z0), 2 * av * V, (z1 - z0) * Z),          # back wall
        _sample_rect(corner(-au, -av, z0), 2 * au * U, (z1 - z0) * Z),         # left wall
        _sample_rect(corner(-au, av, z0), 2 * au * U, (z1 - z0) * Z),          # right wall
    ]
    for _ in range(n_objects):
        u0, v0 = rng.uniform(-0.6 * au, 0.6 * au), rng.uniform(-0.6 * av, 0.6 * av)
        wu, wv = rng.uniform(0.05, 0.15, size=2) * N
        hz = rng.uniform(0.05, 0.25) * N
        b = corner(u0, v0, z0)
        pts.append(_sample_rect(b + hz * Z, wu * U, wv * V))                    # top
        for o, d in ((b, wu * U), (b, wv * V), (b + wv * V, wu * U), (b + wu * U, wv * V)):
            pts.append(_sample_rect(o, d, hz * Z))                              # sides
    p = np.rint(np.concatenate(pts)).astype(np.int64)
    p = p[np.all((p >= 0) & (p < N), axis=1)]
    vol = np.zeros((N, N, N), dtype=np.int32)
    vol[p[:, 0], p[:, 1], p[:, 2]] = 1
    count = int(round(noise * N ** 3))
    vol.reshape(-1)[rng.choice(N ** 3, size=count, replace=False)] = 1
    surfaces = {"floor": Z, "ceiling": -Z, "back": -U, "left": V, "right": -V}
    return vol, surfaces


def random_projection(N: int, count: int = 12, seed: int = 21, dtype=np.int32, levels: int = 16) -> np.ndarray:
    """A DRT-output-shaped array [count][N][N][3N-2] of seeded values with many
    ties: integers in [0, levels) (int32), or N(0,1) rounded to eighths
    (float32). Stands in for a transform output where only its shape matters."""
    rng = _rng(seed)
    shape = (count, N, N, 3 * N - 2)
    if np.dtype(dtype) == np.float32:
        return (np.round(rng.standard_normal(size=shape) * 8) / 8).astype(np.float32)
    return rng.integers(0, levels, size=shape).astype(np.int32)


# Named workloads with the sizes they are quoted at.
WORKLOADS = {
    "drt_n32_uniform": dict(kind="drt", N=32, dtype="int32",
                            make=lambda: uniform_int_cube(32, 0, 255, seed=1)),
    "drt_n512_pointcloud_planes": dict(kind="drt", N=512, dtype="int32",
                                       make=lambda: point_cloud_with_planes(512, seed=2)),
    "djt_n128_segments": dict(kind="djt", N=128, dtype="int32",
                              make=lambda: noise_with_segments(128, seed=3)),
    "drt_batch_mixed_f32": dict(kind="drt_batched", N=(32, 64, 128, 256), dtype="float32",
                                make=lambda: mixed_batch()),
    "drt_diff_b8_n128_f32": dict(kind="drt_autograd", N=128, dtype="float32",
                                 make=lambda: normal_batch(8, 128, seed=5)),
}
