"""Pins of the oracle's merged output (Algorithm 2's 4N x 4N x (3N-2) net):
what the printed tables fix. The paper claims no continuity across block
edges and none is tested; the layout itself stays parity unpinned."""
import numpy as np
import pytest

import workloads


def test_out_order_rows_rotate_the_slope_plane_only(oracle_mod):
    """Every OutOrder row leaves d in place and unflipped, and is either the
    identity on (s1, s2) or their swap, with any flips: a rotation or
    reflection of the slope plane."""
    O = oracle_mod
    for row in O.OUT_ORDER:
        assert row[2] == 3
        assert sorted(abs(v) for v in row[:2]) == [1, 2]


def test_dodecant_blocks_fill_the_net_but_its_corners(oracle_mod):
    O = oracle_mod
    blocks = [tuple(c) for c in O.DODECANT_COORDS]
    assert len(set(blocks)) == 12
    empty = {(r, c) for r in range(4) for c in range(4)} - set(blocks)
    assert empty == {(0, 0), (0, 3), (3, 0), (3, 3)}


@pytest.mark.parametrize("N", [2, 4, 8])
def test_net_holds_every_output_value_once(oracle_mod, N):
    """The net is a placement: each block is a rotated copy of one dodecant's
    output (same multiset of values), the corners are zero, and nothing else
    is written."""
    O = oracle_mod
    R = O.rec_drt(workloads.uniform_int_cube(N, 1, 1000, seed=60 + N))
    net = O.merge_net(R)
    assert net.shape == (4 * N, 4 * N, 3 * N - 2)
    for k, (r, c) in enumerate(O.DODECANT_COORDS):
        block = net[r * N:(r + 1) * N, c * N:(c + 1) * N]
        assert np.array_equal(np.sort(block, axis=None), np.sort(R[k], axis=None))
        # each displacement column of the block is one (s1, s2) column of R[k]
        cols = {tuple(v) for v in block.reshape(N * N, -1)}
        assert cols == {tuple(v) for v in R[k].reshape(N * N, -1)}
    for r, c in ((0, 0), (0, 3), (3, 0), (3, 3)):
        assert not net[r * N:(r + 1) * N, c * N:(c + 1) * N].any()


@pytest.mark.parametrize("N", [4, 8])
def test_z_normal_columns_meet_at_the_net_centre(oracle_mod, N):
    """The slope pair (0, 0) of the four z-face dodecants (k0..k3) is the z
    normal itself; the net puts those four columns on the four cells around
    its centre, as the output-shape figure marks the z null normal in the
    middle of the net."""
    O = oracle_mod
    R = np.zeros((12, N, N, 3 * N - 2), dtype=np.int64)
    for k in range(4):
        R[k, 0, 0, 0] = k + 1
    net = O.merge_net(R)
    got = {(int(i), int(j)): int(net[i, j, 0]) for i, j in zip(*np.nonzero(net[:, :, 0]))}
    assert set(got) == {(2 * N - 1, 2 * N - 1), (2 * N - 1, 2 * N), (2 * N, 2 * N), (2 * N, 2 * N - 1)}
    assert sorted(got.values()) == [1, 2, 3, 4]


def _golden_alg2():
    """The tables of tests/golden/alg2_tables.txt: {name: {k: row}}."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "alg2_tables.txt")
    tables = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, vals = line.split("=")
        name, k = key.split()
        tables.setdefault(name, {})[int(k[1:])] = tuple(int(v) for v in vals.split())
    return tables


def test_oracle_tables_are_the_printed_ones(oracle_mod):
    """The oracle's InOrder (the C frame table), OutOrder and DodecantCoords
    (the merged-net placement) equal the golden copy of Algorithm 2's printed
    initialisations, row by row: a transcription slip in any entry fails."""
    O = oracle_mod
    g = _golden_alg2()
    assert sorted(g) == ["DodecantCoords", "InOrder", "OutOrder"]
    assert all(sorted(t) == list(range(12)) for t in g.values())
    for k in range(12):
        assert O.in_order_row(k) == g["InOrder"][k], k
        assert tuple(O.OUT_ORDER[k]) == g["OutOrder"][k], k
        assert tuple(O.DODECANT_COORDS[k]) == g["DodecantCoords"][k], k


@pytest.mark.parametrize("k", range(12))
def test_each_block_is_its_dodecant_turned_by_its_outorder_row(oracle_mod, k):
    """Where dodecant k's column (s1, s2) lands in the net, for every slope
    pair at N = 4: the block's row index runs along the slope axis
    |OutOrder(k, 0)| (reversed when the entry is negative) and its column index
    along |OutOrder(k, 1)|. Checked by tracing a column-numbering output, with
    the expected cell derived from the golden row, not from the oracle."""
    O = oracle_mod
    N = 4
    row = _golden_alg2()["OutOrder"][k]
    br, bc = _golden_alg2()["DodecantCoords"][k]
    R = np.zeros((12, N, N, 1), dtype=np.int64)
    R[k, :, :, 0] = 1 + np.arange(N * N).reshape(N, N)  # 1 + s1 * N + s2
    net = O.merge_net(R)
    for s1 in range(N):
        for s2 in range(N):
            s = (s1, s2)
            a = s[abs(row[0]) - 1]
            b = s[abs(row[1]) - 1]
            i = N - 1 - a if row[0] < 0 else a
            j = N - 1 - b if row[1] < 0 else b
            assert net[br * N + i, bc * N + j, 0] == 1 + s1 * N + s2, (k, s1, s2)
