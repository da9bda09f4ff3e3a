"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a closed form, an
invariant the paper states, an independent route (the paper's recursion against
the definition, the 2D transform applied twice), a brute force on tiny inputs,
or a value printed in the paper (``tests/golden/paper_values.txt``).
"""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = [t.strip() for t in line.split("=", 1)]
            vals[k] = v
    return vals


def _frame_volume(O, vol, k):
    """g_k as a numpy array built with transposes and flips from the signed
    permutation matrix (a route independent of the oracle's index map)."""
    M = O.frame_matrix(k)
    g = vol
    # primed axis j is original axis i with sign M[j, i]
    order = [int(np.nonzero(M[j])[0][0]) for j in range(3)]
    g = np.transpose(g, order)
    for j in range(3):
        if M[j, order[j]] < 0:
            g = np.flip(g, axis=j)
    return np.ascontiguousarray(g)


# --------------------------------------------------------------------------- line
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_line_forms_agree_and_endpoints(oracle_mod, n):
    """eq. (4): the recursive and closed forms agree; the line joins (0,0) to
    (N-1,s) with steps of 0 or 1; slope 0 is flat and slope N-1 is the diagonal."""
    O, N = oracle_mod, 1 << n
    for s in range(N):
        row = [O.line(n, s, x) for x in range(N)]
        assert row == [O.line_recursive(n, s, x) for x in range(N)]
        assert row[0] == 0 and row[-1] == s
        assert all(b - a in (0, 1) for a, b in zip(row, row[1:]))
    assert all(O.line(n, 0, x) == 0 for x in range(N))
    assert all(O.line(n, N - 1, x) == x for x in range(N))


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_line_symmetries(oracle_mod, n):
    """Complement symmetries of the dyadic lines: l_{N-1-s}(x) = x - l_s(x) and
    l_s(N-1-x) = s - l_s(x)."""
    O, N = oracle_mod, 1 << n
    for s in range(N):
        for x in range(N):
            assert O.line(n, N - 1 - s, x) == x - O.line(n, s, x)
            assert O.line(n, s, N - 1 - x) == s - O.line(n, s, x)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_line_close_to_continuous(oracle_mod, n):
    """The loose line stays within n/2 + 1 of the continuous line y = s x/(N-1)."""
    O, N = oracle_mod, 1 << n
    for s in range(N):
        for x in range(N):
            assert abs(O.line(n, s, x) - s * x / (N - 1)) <= n / 2 + 1


# ------------------------------------------------------------------------- frames
def test_frames_are_cube_symmetries(oracle_mod):
    O = oracle_mod
    N = 4
    assert np.array_equal(O.frame_matrix(0), np.eye(3, dtype=np.int64))
    for k in range(12):
        M = O.frame_matrix(k)
        assert sorted(np.abs(M).sum(axis=0).tolist()) == [1, 1, 1]
        assert sorted(np.abs(M).sum(axis=1).tolist()) == [1, 1, 1]
        seen = set()
        for x in range(N):
            for y in range(N):
                for z in range(N):
                    seen.add(O.frame_to_orig(k, N, (x, y, z)))
        assert len(seen) == N ** 3


def test_z_face_frames_follow_right_hand_rule(oracle_mod):
    """Sec. 3.2: the four z-normal dodecants put the origin p0 on the four
    vertices of the face z=0, with p1, p2 the adjacent vertices such that
    (p1-p0) x (p2-p0) = (0,0,1) (scaled), and keep z as the ascent axis."""
    O, N = oracle_mod, 8
    origins = set()
    for k in range(4):
        p0 = np.array(O.frame_to_orig(k, N, (0, 0, 0)))
        p1 = np.array(O.frame_to_orig(k, N, (N - 1, 0, 0)))
        p2 = np.array(O.frame_to_orig(k, N, (0, N - 1, 0)))
        top = np.array(O.frame_to_orig(k, N, (0, 0, N - 1)))
        assert p0[2] == 0 and top[2] == N - 1
        assert np.array_equal(np.cross(p1 - p0, p2 - p0), np.array([0, 0, (N - 1) ** 2]))
        origins.add(tuple(p0[:2] // (N - 1)))
    assert origins == {(0, 0), (0, 1), (1, 0), (1, 1)}


def _coverage(O, kind, ndir=20000, seed=11):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((ndir, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    count = np.zeros(ndir, dtype=np.int64)
    for k in range(12):
        m = d @ O.frame_matrix(k).T.astype(float)
        dom = (np.abs(m[:, 2]) >= np.abs(m[:, 0])) & (np.abs(m[:, 2]) >= np.abs(m[:, 1]))
        if kind == "normal":   # plane normals (-a,-b,1), a,b in [0,1] (Sec. 3.1)
            ok = (m[:, 0] * m[:, 2] <= 0) & (m[:, 1] * m[:, 2] <= 0)
        else:                  # line directions (a,b,1), a,b in [0,1] (Sec. 4.1)
            ok = (m[:, 0] * m[:, 2] >= 0) & (m[:, 1] * m[:, 2] >= 0)
        count += dom & ok
    return count


@pytest.mark.parametrize("kind", ["normal", "line"])
def test_twelve_frames_tile_the_hemisphere(oracle_mod, kind):
    """Sec. 3.2 / Sec. 4.1: the 12 dodecants cover every plane normal (every
    line direction) exactly once, up to the sign of the direction."""
    count = _coverage(oracle_mod, kind)
    assert int(_golden()["dodecants"]) == 12
    assert np.all(count == 1), np.bincount(count)


# ---------------------------------------------------------------------------- DRT
@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_drt_definition_equals_recursion_int(oracle_mod, N):
    """Algorithm 1 with eq. (11) reaches eq. (9) exactly, in every frame."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -100, 100, seed=N)
    assert np.array_equal(O.def_drt(vol), O.rec_drt(vol))


@pytest.mark.parametrize("N", [4, 8])
def test_drt_definition_equals_recursion_float(oracle_mod, N):
    O = oracle_mod
    vol = workloads.normal_cube(N, seed=N).astype(np.float64)
    a, b = O.def_drt(vol), O.rec_drt(vol)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(vol).sum())


@pytest.mark.parametrize("N", [4, 8, 16])
def test_drt_point_matches_full(oracle_mod, N):
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, 0, 9, seed=3)
    full = O.def_drt(vol)
    rng = np.random.default_rng(0)
    for _ in range(50):
        k, s1, s2, dd = rng.integers(12), rng.integers(N), rng.integers(N), rng.integers(3 * N - 2)
        assert O.drt_point(vol, k, s1, s2, dd) == full[k, s1, s2, dd]


@pytest.mark.parametrize("N", [4, 8, 16])
def test_drt_each_voxel_on_one_plane_per_slope(oracle_mod, N):
    """Every voxel lies on exactly one plane of each slope pair: the displacement
    sums equal the volume sum for every (k, s1, s2)."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -7, 50, seed=N + 1)
    R = O.def_drt(vol)
    assert np.all(R.sum(axis=-1) == vol.astype(np.int64).sum())


@pytest.mark.parametrize("N", [4, 8])
def test_drt_delta_lands_once(oracle_mod, N):
    """A delta voxel gives exactly one 1 per (k, s1, s2); over all voxels the
    hits cover the whole support 0..N-1+s1+s2 (Sec. 3.2)."""
    O = oracle_mod
    hits = np.zeros((12, N, N, 3 * N - 2), dtype=np.int64)
    rng = np.random.default_rng(1)
    for idx in range(N ** 3):
        vol = np.zeros((N, N, N), np.int32)
        vol.flat[idx] = 1
        R = O.rec_drt(vol)
        assert np.all(R.sum(axis=-1) == 1) and R.min() == 0 and R.max() == 1
        hits += R
    s = np.arange(N)
    last = (N - 1) + s[:, None] + s[None, :]
    dd = np.arange(3 * N - 2)
    inside = dd[None, None, :] <= last[:, :, None]
    assert np.all((hits > 0) == inside[None])
    _ = rng


@pytest.mark.parametrize("N", [4, 8, 16])
def test_drt_support_and_counts(oracle_mod, N):
    """Sec. 3.2: non-null values of (s1, s2) lie in 0..N-1+s1+s2; (0,0) has at
    most N non-null displacements, (N-1,N-1) up to 3N-2. On an all-ones cube the
    support is filled, so the number of planes per dodecant is sum(N+s1+s2)."""
    O = oracle_mod
    R = O.def_drt(np.ones((N, N, N), np.int32))
    g = _golden()
    assert R.shape[-1] == eval(g["drt_displacements_per_slope"], {"N": N})
    nz = R > 0
    s = np.arange(N)
    last = eval(g["drt_support_last_index"], {"N": N, "s1": s[:, None], "s2": s[None, :]})
    assert np.array_equal(nz.sum(axis=-1), np.broadcast_to(last + 1, (12, N, N)))
    assert nz[:, 0, 0].sum(axis=-1).max() == eval(g["drt_nonnull_slope00"], {"N": N})
    assert nz[:, N - 1, N - 1].sum(axis=-1).min() == eval(g["drt_nonnull_slope_max"], {"N": N})
    assert nz[0].sum() == 2 * N ** 3 - N ** 2


def test_paper_plane_count_at_128():
    """Sec. 6: more than 4 million planes per dodecant at 128^3, each summing up
    to 16k voxels. The count is the support size sum(N+s1+s2) pinned above."""
    g = _golden()
    N = 128
    s = np.arange(N, dtype=np.int64)
    planes = int((N + s[:, None] + s[None, :]).sum())
    assert planes == 2 * N ** 3 - N ** 2
    assert planes > int(g["planes_per_dodecant_n128_more_than"])
    assert N * N == int(g["voxels_per_full_plane_n128"])


@pytest.mark.parametrize("N", [4, 8])
def test_drt_linearity(oracle_mod, N):
    O = oracle_mod
    a = workloads.uniform_int_cube(N, -9, 9, seed=1)
    b = workloads.uniform_int_cube(N, -9, 9, seed=2)
    lhs = O.def_drt(3 * a - 5 * b)
    assert np.array_equal(lhs, 3 * O.def_drt(a) - 5 * O.def_drt(b))


@pytest.mark.parametrize("N", [4, 8, 16])
def test_drt_axis_aligned_and_diagonal_slopes(oracle_mod, N):
    """Slope (0,0) is the axis-aligned plane sum over x',y'; slope (N-1,N-1) is
    the exact diagonal plane z' = x' + y' + N-1-dd (closed forms, numpy)."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -20, 60, seed=7)
    R = O.def_drt(vol)
    x, y, z = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    for k in range(12):
        g = _frame_volume(O, vol, k).astype(np.int64)
        ax = np.zeros(3 * N - 2, np.int64)
        ax[:N] = g.sum(axis=(0, 1))[::-1]
        assert np.array_equal(R[k, 0, 0], ax)
        diag = np.zeros(3 * N - 2, np.int64)
        np.add.at(diag, (x + y - z + N - 1).ravel(), g.ravel())
        assert np.array_equal(R[k, N - 1, N - 1], diag)


def _drt2d(O, img):
    """2D multiscale DRT by its definition (eq. (3)), mirrored displacement:
    out[s][t] = sum_u img[u][t - l_s(u)], img of shape (N, M), out (N, M+N-1)."""
    N, M = img.shape
    n = N.bit_length() - 1
    out = np.zeros((N, M + N - 1), dtype=img.dtype)
    for s in range(N):
        for u in range(N):
            sh = O.line(n, s, u)
            out[s, sh:sh + M] += img[u]
    return out


@pytest.mark.parametrize("N", [4, 8, 16])
def test_drt_is_2d_drt_applied_twice(oracle_mod, N):
    """Sec. 6.2 (Wu and Brady): a dodecant of the 3D DRT equals the 2D DRT of
    eq. (3) applied along x' for every y', then along y' for every s1."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -30, 30, seed=N + 5)
    R = O.def_drt(vol)
    for k in (0, 5, 10):
        g = _frame_volume(O, vol, k).astype(np.int64)
        H = np.zeros((N, N, 2 * N - 1), np.int64)          # [y'][s1][t]
        for yp in range(N):
            H[yp] = _drt2d(O, g[:, yp, ::-1])
        out = np.zeros((N, N, 3 * N - 2), np.int64)
        for s1 in range(N):
            out[s1] = _drt2d(O, H[:, s1, :])
        assert np.array_equal(out, R[k])


# ---------------------------------------------------------------------------- DJT
@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_djt_definition_equals_recursion(oracle_mod, N):
    """Algorithm 3 with eq. (15) reaches eq. (13) exactly, in every frame."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -50, 50, seed=N + 2)
    mask = 0xFFF if N <= 8 else 0b100000100001
    assert np.array_equal(O.def_djt(vol, mask), O.rec_djt(vol, mask))


@pytest.mark.parametrize("N", [4, 8])
def test_djt_invariants(oracle_mod, N):
    """Every voxel lies on exactly one line per slope pair; slope (0,0) is the
    axis-aligned line sum along z'; slope (N-1,N-1) is the exact diagonal; the
    support of (s1,s2) lies in the box e1 <= N-1+s1, e2 <= N-1+s2 and reaches
    both box edges (lines with two large slopes can miss the cube inside the
    box, so the box is not filled)."""
    O = oracle_mod
    vol = workloads.uniform_int_cube(N, -20, 60, seed=9)
    J = O.def_djt(vol)
    assert np.all(J.sum(axis=(-1, -2)) == vol.astype(np.int64).sum())
    x, y, z = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    E = 2 * N - 1
    for k in range(12):
        g = _frame_volume(O, vol, k).astype(np.int64)
        ax = np.zeros((E, E), np.int64)
        ax[:N, :N] = g.sum(axis=2)[::-1, ::-1]
        assert np.array_equal(J[k, 0, 0], ax)
        diag = np.zeros((E, E), np.int64)
        np.add.at(diag, ((z - x + N - 1).ravel(), (z - y + N - 1).ravel()), g.ravel())
        assert np.array_equal(J[k, N - 1, N - 1], diag)
    ones = O.def_djt(np.ones((N, N, N), np.int32))
    s = np.arange(N)
    e = np.arange(E)
    inside = (e[None, None, :, None] <= (N - 1 + s)[:, None, None, None]) & \
             (e[None, None, None, :] <= (N - 1 + s)[None, :, None, None])
    nz = ones > 0
    assert not np.any(nz & ~inside[None])
    for s1 in range(N):
        for s2 in range(N):
            rows = np.nonzero(nz[:, s1, s2].any(axis=(0, 2)))[0]
            cols = np.nonzero(nz[:, s1, s2].any(axis=(0, 1)))[0]
            assert rows.min() == 0 and rows.max() == N - 1 + s1
            assert cols.min() == 0 and cols.max() == N - 1 + s2
    # slope (0,0): the N x N block of axis lines, each of length N
    assert np.all(ones[:, 0, 0, :N, :N] == N)


@pytest.mark.parametrize("N", [4, 8])
def test_djt_delta_and_linearity(oracle_mod, N):
    O = oracle_mod
    rng = np.random.default_rng(N)
    for _ in range(5):
        vol = np.zeros((N, N, N), np.int32)
        vol[tuple(rng.integers(N, size=3))] = 1
        J = O.def_djt(vol)
        assert np.all(J.sum(axis=(-1, -2)) == 1) and J.max() == 1
    a = workloads.uniform_int_cube(N, -9, 9, seed=4)
    b = workloads.uniform_int_cube(N, -9, 9, seed=5)
    assert np.array_equal(O.def_djt(2 * a + 7 * b), 2 * O.def_djt(a) + 7 * O.def_djt(b))


def test_djt_point_matches_full(oracle_mod):
    O = oracle_mod
    N = 8
    vol = workloads.uniform_int_cube(N, 0, 9, seed=3)
    full = O.def_djt(vol)
    rng = np.random.default_rng(2)
    for _ in range(100):
        k, s1, s2 = rng.integers(12), rng.integers(N), rng.integers(N)
        e1, e2 = rng.integers(2 * N - 1), rng.integers(2 * N - 1)
        assert O.djt_point(vol, k, s1, s2, e1, e2) == full[k, s1, s2, e1, e2]


# ------------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("N", [2, 4, 8])
def test_adjoint_definition_equals_reversed_recursion(oracle_mod, N):
    """eq. (17) run from stage n down to 0 (Sec. 5.1) equals the transpose of
    eq. (9) gathered per voxel."""
    O = oracle_mod
    rng = np.random.default_rng(N)
    proj = rng.integers(-40, 40, size=(12, N, N, 3 * N - 2)).astype(np.int32)
    assert np.array_equal(O.def_adj(proj, N), O.rec_adj(proj, N))


@pytest.mark.parametrize("N,mask", [(4, 0xFFF), (8, 0xFFF), (16, 0xFFF), (16, 0b010010010010)])
def test_adjoint_dot_product_identity(oracle_mod, N, mask):
    """<R f, p> = <f, R^T p> exactly in int64."""
    O = oracle_mod
    rng = np.random.default_rng(N + mask)
    f = rng.integers(-100, 100, size=(N, N, N)).astype(np.int32)
    p = rng.integers(-100, 100, size=(O.count_dodecants(mask), N, N, 3 * N - 2)).astype(np.int32)
    lhs = int((O.rec_drt(f, mask) * p.astype(np.int64)).sum())
    rhs = int((f.astype(np.int64) * O.rec_adj(p, N, mask)).sum())
    assert lhs == rhs


@pytest.mark.parametrize("N", [4, 8])
def test_adjoint_gram_diagonal(oracle_mod, N):
    """Each voxel lies on exactly one plane of every (k, s1, s2), so
    (R^T R)[v, v] = 12 N^2, without normalisation (Sec. 5.1)."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    for _ in range(4):
        vol = np.zeros((N, N, N), np.int32)
        v = tuple(rng.integers(N, size=3))
        vol[v] = 1
        back = O.def_adj(O.wrap_int32(O.def_drt(vol)), N)
        assert back[v] == 12 * N * N
        assert back.sum() > back[v]


def test_adjoint_point_matches_full(oracle_mod):
    O = oracle_mod
    N = 8
    rng = np.random.default_rng(3)
    mask = 0b101101101101
    p = rng.integers(-9, 9, size=(O.count_dodecants(mask), N, N, 3 * N - 2)).astype(np.int32)
    full = O.rec_adj(p, N, mask)
    for _ in range(50):
        x, y, z = rng.integers(N, size=3)
        assert O.adj_point(p, N, mask, x, y, z) == full[x, y, z]


def test_float_adjoint_and_djt_routes_agree(oracle_mod):
    O = oracle_mod
    N = 8
    vol = workloads.normal_cube(N, seed=1).astype(np.float64)
    assert np.allclose(O.def_djt(vol), O.rec_djt(vol), rtol=0, atol=1e-12 * np.abs(vol).sum())
    rng = np.random.default_rng(1)
    p = rng.standard_normal((12, N, N, 3 * N - 2))
    assert np.allclose(O.def_adj(p, N), O.rec_adj(p, N), rtol=0, atol=1e-10 * np.abs(p).sum())


def test_wrap_semantics():
    import oracle as O
    a = np.array([2 ** 31, -2 ** 31 - 1, 2 ** 32 + 5], dtype=np.int64)
    assert O.wrap_int32(a).tolist() == [-2 ** 31, 2 ** 31 - 1, 5]


# ----------------------------------------------------------------------- inputs
def test_workload_generators_are_seeded():
    a = workloads.point_cloud_with_planes(32, occupancy=0.01, n_planes=2, seed=4)
    b = workloads.point_cloud_with_planes(32, occupancy=0.01, n_planes=2, seed=4)
    assert np.array_equal(a, b) and a.dtype == np.int32
    assert set(np.unique(a).tolist()) <= {0, 1, 16}
    c = workloads.noise_with_segments(16, n_segments=3, seed=2)
    assert c.dtype == np.int32 and c.min() >= 0 and c.max() <= 3 + 8 * 3
    cubes = workloads.mixed_batch(((4, 2), (8, 1)))
    assert [x.shape[0] for x in cubes] == [4, 4, 8] and cubes[0].dtype == np.float32
    cc = workloads.corners_and_centre(8)
    assert cc.sum() == 9


# ------------------------------------------------------------ sparse matrix
def test_sparse_matrix_reproduces_definition_and_adjoint():
    """The column-by-column matrix used by the gradient checks equals the
    definition on a random cube, its transpose equals the adjoint definition,
    and every voxel meets exactly one displacement per (dodecant, s1, s2)."""
    import oracle as O
    from tests.sparse_ref import drt_matrix
    N = 8
    R = drt_matrix(N)
    assert R.nnz == 12 * N * N * N ** 3 and R.max() == 1
    rng = np.random.default_rng(21)
    f = rng.integers(-9, 9, size=(N, N, N)).astype(np.int32)
    assert np.array_equal((R @ f.ravel().astype(np.float64)).astype(np.int64), O.def_drt(f).ravel())
    p = rng.integers(-9, 9, size=(12, N, N, 3 * N - 2)).astype(np.int32)
    assert np.array_equal((R.T @ p.ravel().astype(np.float64)).astype(np.int64), O.def_adj(p, N).ravel())
    Rk = drt_matrix(N, 0b000100000010)
    assert np.array_equal((Rk @ f.ravel().astype(np.float64)).astype(np.int64),
                          O.def_drt(f, 0b000100000010).ravel())


# ------------------------------------------------------------ DJT adjoint
@pytest.mark.parametrize("N,mask", [(2, 0xFFF), (4, 0xFFF), (8, 0xFFF), (8, 0b100000100001), (16, 0x00C)])
def test_djt_adjoint_dot_product_identity(oracle_mod, N, mask):
    """<J f, P> = <f, J^T P> exactly in int64: the DJT adjoint is the transpose
    of the (pinned) definition of eq. (13)."""
    O = oracle_mod
    rng = np.random.default_rng(N + mask)
    f = rng.integers(-9, 9, size=(N, N, N)).astype(np.int32)
    nd = O.count_dodecants(mask)
    P = rng.integers(-9, 9, size=(nd, N, N, 2 * N - 1, 2 * N - 1)).astype(np.int32)
    lhs = int((O.def_djt(f, mask).astype(np.int64) * P).sum())
    rhs = int((f.astype(np.int64) * O.def_djt_adj(P, N, mask)).sum())
    assert lhs == rhs


@pytest.mark.parametrize("N", [4, 8])
def test_djt_adjoint_of_ones_counts_lines(oracle_mod, N):
    """Each voxel lies on exactly one line of every (dodecant, s1, s2), so the
    backprojection of all-ones is popcount(mask) * N^2 everywhere."""
    O = oracle_mod
    for mask in (0xFFF, 0x0A0):
        P = np.ones((O.count_dodecants(mask), N, N, 2 * N - 1, 2 * N - 1), dtype=np.int32)
        assert np.all(O.def_djt_adj(P, N, mask) == O.count_dodecants(mask) * N * N)


def test_djt_adjoint_point_and_float_route(oracle_mod):
    O = oracle_mod
    N = 8
    rng = np.random.default_rng(5)
    P = rng.integers(-50, 50, size=(12, N, N, 2 * N - 1, 2 * N - 1)).astype(np.int32)
    full = O.def_djt_adj(P, N)
    for (x, y, z) in [(0, 0, 0), (7, 3, 5), (N - 1, N - 1, N - 1), (2, 6, 1)]:
        assert O.djt_adj_point(P, N, 0xFFF, x, y, z) == full[x, y, z]
    assert np.array_equal(O.def_djt_adj(P.astype(np.float64), N), full.astype(np.float64))
