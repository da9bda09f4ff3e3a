"""The DRT and the DJT as explicit sparse matrices, assembled column by column
from the oracle's definitions (eqs. (9) and (13)): column v is the transform of
the unit voxel v. Test infrastructure: used to check gradients against the
dense transpose."""
import numpy as np

import oracle as O


def drt_matrix(N: int, mask: int = 0xFFF):
    """scipy CSC matrix R with R @ f.ravel() == def_drt(f).ravel()."""
    return _matrix(N, mask, O.def_drt, O.count_dodecants(mask) * N * N * (3 * N - 2))


def djt_matrix(N: int, mask: int = 0xFFF):
    """scipy CSC matrix J with J @ f.ravel() == def_djt(f).ravel()."""
    return _matrix(N, mask, O.def_djt, O.count_dodecants(mask) * N * N * (2 * N - 1) ** 2)


def _matrix(N, mask, transform, M):
    import scipy.sparse as sp
    rows, cols, vals = [], [], []
    delta = np.zeros(N ** 3, dtype=np.int32)
    for v in range(N ** 3):
        delta[v] = 1
        col = transform(delta.reshape(N, N, N), mask).ravel()
        delta[v] = 0
        nz = np.flatnonzero(col)
        rows.append(nz)
        cols.append(np.full(nz.size, v, dtype=np.int64))
        vals.append(col[nz].astype(np.float64))
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(M, N ** 3))
