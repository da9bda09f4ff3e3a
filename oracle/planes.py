"""Oracle of the plane-detection application (Sec. 6.1), test infrastructure
only.

The paper detects the principal planes of a voxelized depth scene in its DRT:
the bin holding the most voxels is the dominant plane; the planes orthogonal to
it that are also relative maxima of the transform and exceed a threshold are
the others; backprojecting the detected planes marks their voxels. The paper
fixes none of the details, so this follows these readings:

* The dominant plane is the largest bin of the whole output
  [dodecant][s1][s2][dd]; ties go to the smallest flat index.
* A plane's normal: in dodecant k's frame the plane through displacement d has
  z' = s1 x'/(N-1) + s2 y'/(N-1) + d up to the discrete lines, with normal
  (-s1, -s2, N-1)/(N-1) (Sec. 3, the normal of the basic dodecant). The frame
  map primed = M orig + offset turns it into M^T (-s1, -s2, N-1) in the
  (x, y, z) axes, an integer vector.
* Orthogonal: |cos| <= cos_tol between the two normals, decided exactly as
  (n_a . n_b)^2 <= cos_tol^2 |n_a|^2 |n_b|^2, the two sides as float64 (both
  integer products are exact there).
* Relative maximum: within the dodecant, over the 26 neighbours
  (s1 + a, s2 + b, dd + c), a, b, c in {-1, 0, 1}, that exist: every
  neighbour with a smaller flat index is strictly below the bin and every one
  with a larger index is not above it, so a plateau yields one bin, its first.
  Neighbours in other dodecants are not compared.
* Threshold: value >= rel_threshold times the dominant plane's value, in
  float64.
* The result lists the dominant bin first, then the qualifying bins in
  ascending flat index. A wall seen by several dodecants (the four of one
  normal group at slopes (0, 0), say) is listed once per dodecant.
* Backprojection: the adjoint (Sec. 5.1) of a projection with 1 at each listed
  bin and 0 elsewhere, i.e. per voxel the number of listed planes through it.
"""
from __future__ import annotations

import numpy as np

from .oracle import frame_matrix, rec_adj

__all__ = ["plane_normal", "bin_coords", "is_orthogonal", "local_maxima", "detect_planes",
           "backproject_bins"]


def _dodecants(mask):
    return [k for k in range(12) if (mask >> k) & 1]


def plane_normal(k: int, s1: int, s2: int, N: int) -> np.ndarray:
    """Integer normal (x, y, z) of dodecant k's planes at slopes (s1, s2), scaled by N-1."""
    return frame_matrix(k).T @ np.array([-s1, -s2, N - 1], dtype=np.int64)


def bin_coords(index: int, N: int, mask: int = 0xFFF):
    """Flat output index -> (k, s1, s2, dd)."""
    ks = _dodecants(mask)
    j, s1, s2, dd = np.unravel_index(int(index), (len(ks), N, N, 3 * N - 2))
    return ks[int(j)], int(s1), int(s2), int(dd)


def is_orthogonal(na, nb, cos_tol: float) -> bool:
    dot = int(np.dot(na, nb))
    p = int(np.dot(na, na)) * int(np.dot(nb, nb))
    return float(dot * dot) <= (cos_tol * cos_tol) * float(p)


def local_maxima(Rk) -> np.ndarray:
    """Boolean mask of the relative maxima of one dodecant's output [N][N][E]."""
    Rk = np.asarray(Rk)
    wide = Rk.astype(np.float64 if Rk.dtype.kind == "f" else np.int64)
    S = np.pad(wide, 1, constant_values=-np.inf if wide.dtype.kind == "f" else np.iinfo(np.int64).min)
    A, B, C = wide.shape
    ok = np.ones(wide.shape, dtype=bool)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                if (a, b, c) == (0, 0, 0):
                    continue
                nb = S[1 + a:1 + a + A, 1 + b:1 + b + B, 1 + c:1 + c + C]
                # (a, b, c) before (0, 0, 0) in lexicographic order = a smaller flat index
                ok &= (wide > nb) if (a, b, c) < (0, 0, 0) else (wide >= nb)
    return ok


def detect_planes(R, N: int, mask: int = 0xFFF, cos_tol: float = 0.05, rel_threshold: float = 0.5):
    """R: the DRT output [count][N][N][3N-2] -> [dominant bin, qualifying bins...] (flat indices)."""
    R = np.asarray(R)
    ks = _dodecants(mask)
    E = 3 * N - 2
    if R.shape != (len(ks), N, N, E):
        raise ValueError("expected a DRT output of shape %s, got %s" % ((len(ks), N, N, E), R.shape))
    if not 0.0 <= cos_tol < 1.0:
        raise ValueError("cos_tol must lie in [0, 1)")
    flat = R.reshape(-1)
    top = int(np.argmax(flat))
    k0, t1, t2, _ = bin_coords(top, N, mask)
    n_top = plane_normal(k0, t1, t2, N)
    thr = rel_threshold * float(flat[top])
    found = []
    for j, k in enumerate(ks):
        ortho = np.array([[is_orthogonal(n_top, plane_normal(k, s1, s2, N), cos_tol) for s2 in range(N)]
                          for s1 in range(N)])
        if not ortho.any():
            continue
        Rk = R[j]
        sel = local_maxima(Rk) & (Rk.astype(np.float64) >= thr) & ortho[:, :, None]
        found.extend((np.flatnonzero(sel) + j * N * N * E).tolist())
    return [top] + sorted(found)


def backproject_bins(bins, N: int, mask: int = 0xFFF) -> np.ndarray:
    """Adjoint of the 0/1 projection marking ``bins``: planes through each voxel (int64)."""
    ks = _dodecants(mask)
    P = np.zeros(len(ks) * N * N * (3 * N - 2), dtype=np.int64)
    P[np.asarray(list(bins), dtype=np.int64)] = 1
    return rec_adj(P.reshape(len(ks), N, N, 3 * N - 2), N, mask)
