"""Oracle of Algorithm 2's merged output (the 4N x 4N x (3N-2) net), test
infrastructure only.

Algorithm 2 rotates each dodecant's N x N x (3N-2) output with a row of
OutOrder and places it at the block DodecantCoords gives, in a zeroed
4N x 4N x (3N-2) array; 4 of the 16 blocks stay empty. This follows the
algorithm's steps literally: permute the dodecant's axes by |OutOrder(k)|
(axis i of the result is axis |OutOrder(k, i)| of the input), then flip every
axis i with OutOrder(k, i) < 0, then copy into the block. The paper claims no
continuity of the net across block edges, and none is tested (parity of this
layout against the paper is unpinned); the tests check what the tables fix.
"""
from __future__ import annotations

import numpy as np

__all__ = ["OUT_ORDER", "DODECANT_COORDS", "merge_net"]

# Algorithm 2, as printed (1-based axes, sign = flip)
OUT_ORDER = [
    (-2, -1, 3), (-1, 2, 3), (2, 1, 3), (1, -2, 3),
    (2, 1, 3), (1, -2, 3), (-1, 2, 3), (-2, -1, 3),
    (2, 1, 3), (-1, 2, 3), (1, -2, 3), (-2, -1, 3),
]
DODECANT_COORDS = [
    (1, 1), (1, 2), (2, 2), (2, 1),
    (0, 2), (0, 1), (3, 2), (3, 1),
    (2, 0), (1, 0), (2, 3), (1, 3),
]


def merge_net(R):
    """R: the 12-dodecant output [12][N][N][3N-2] -> the net [4N][4N][3N-2].
    The placement moves whole displacement columns, so R may carry any depth
    (e.g. one value per (k, s1, s2) to trace where each column lands)."""
    R = np.asarray(R)
    if R.ndim != 4 or R.shape[0] != 12 or R.shape[1] != R.shape[2]:
        raise ValueError("expected a 12-dodecant DRT [12][N][N][depth], got %s" % (R.shape,))
    N = R.shape[1]
    net = np.zeros((4 * N, 4 * N, R.shape[3]), dtype=R.dtype)
    for k in range(12):
        order = OUT_ORDER[k]
        block = np.transpose(R[k], [abs(o) - 1 for o in order])
        for dim, o in enumerate(order):
            if o < 0:
                block = np.flip(block, axis=dim)
        r, c = DODECANT_COORDS[k]
        net[r * N:(r + 1) * N, c * N:(c + 1) * N, :] = block
    return net
