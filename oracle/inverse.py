"""Oracle of the iterative inverse DRT (Sec. 5.2), test infrastructure only.

The paper inverts the 3D DRT the way Press inverts the 2D one: the
backprojection followed by a high-pass filter is an approximate inverse, used
in iterative improvement, and accelerated by multigrid with a prolongation P
in the image domain and a restriction S in the Radon domain (both given in
Sec. 5.2). It fixes the filter, P and S; the rest of the scheme is read as
follows (every reading is listed with its reason in the design notes):

* approximate inverse at size N: M = H A^T, H the 3x3x3 filter of Sec. 5.2
  applied with half-sample symmetric boundaries, A the 12-dodecant DRT;
* smoother: nu steps of iterative improvement x += c_i M (b - A x) with
  Chebyshev step sizes c_i = 1/lambda_i, lambda_i the nodes of [L/10, L],
  L = 1.02 x the largest eigenvalue of H A^T A from a power iteration;
* cycle: a V-cycle (pre-smoothing, restriction of the residual, the same
  cycle at N/2 from zero, prolongation of its result, post-smoothing with the
  steps reversed); at N = 1 the least-squares solution, the mean of the 12
  values;
* the inverse of b: `cycles` V-cycles from x = 0.

Everything runs in float64 on the oracle's naive recursions (Algorithm 1 and
its reverse, eq. (17)).
"""
from __future__ import annotations

import numpy as np

from .oracle import rec_adj, rec_drt

__all__ = [
    "HP_FILTER", "hp_filter", "restrict_proj", "prolong", "power_start",
    "level_lambda", "cheb_steps", "inverse_vcycle", "drt_inverse",
]

NU = 3             # smoothing steps before and after the coarse correction
CHEB_RATIO = 10.0  # the smoother's interval is [L / CHEB_RATIO, L]
LAMBDA_MARGIN = 1.02
POWER_ITERS = 30


def _hp_filter_taps():
    """The filter of Sec. 5.2 as printed: 7/8 at the centre, -1/16 on the 6
    faces, -1/32 on the 12 edges, -1/64 on the 8 corners."""
    h = np.empty((3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                away = (i != 1) + (j != 1) + (k != 1)
                h[i, j, k] = {0: 7 / 8, 1: -1 / 16, 2: -1 / 32, 3: -1 / 64}[away]
    return h


HP_FILTER = _hp_filter_taps()


def hp_filter(x):
    """(H x)[v] = sum over the 27 offsets o of h[o] x[v + o], with x extended
    past each face by half-sample symmetric reflection (x[-1] = x[0],
    x[N] = x[N-1])."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    p = np.pad(x, 1, mode="symmetric")
    out = np.zeros_like(x)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                out += HP_FILTER[i, j, k] * p[i:i + N, j:j + N, k:k + N]
    return out


def restrict_proj(R):
    """S of Sec. 5.2 on every dodecant: R_c(s1, s2, d) = (R(2s1, 2s2, 2d) +
    R(2s1, 2s2, 2d+1)) / 8. In the stored displacement dd = N-1-d this is
    R_c[k][s1][s2][dd] = (R[k][2s1][2s2][2dd] + R[k][2s1][2s2][2dd+1]) / 8, for
    dd < 3(N/2) - 2."""
    R = np.asarray(R, dtype=np.float64)
    K, N = R.shape[0], R.shape[1]
    Nc = N // 2
    Ec = 3 * Nc - 2
    out = np.zeros((K, Nc, Nc, Ec))
    for s1 in range(Nc):
        for s2 in range(Nc):
            for dd in range(Ec):
                out[:, s1, s2, dd] = (R[:, 2 * s1, 2 * s2, 2 * dd] + R[:, 2 * s1, 2 * s2, 2 * dd + 1]) / 8.0
    return out


def prolong(x):
    """P of Sec. 5.2: each voxel of the N/2 cube fills its 2x2x2 block."""
    x = np.asarray(x, dtype=np.float64)
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def power_start(N):
    """Deterministic start vector of the power iteration:
    v[x][y][z] = ((73x + 151y + 277z) mod 29) - 14."""
    x = np.arange(N)
    return (((73 * x[:, None, None] + 151 * x[None, :, None] + 277 * x[None, None, :]) % 29) - 14).astype(np.float64)


def _A(x):
    N = x.shape[0]
    if N == 1:
        return np.full((12, 1, 1, 1), x[0, 0, 0])
    return rec_drt(x)


def _At(r, N):
    if N == 1:
        return np.full((1, 1, 1), r.sum())
    return rec_adj(r, N)


def level_lambda(N, iters=POWER_ITERS):
    """Largest eigenvalue of H A^T A at size N by power iteration from
    power_start(N): v <- H A^T A v / |v|; returns |H A^T A v| / |v| at the last
    step."""
    v = power_start(N)
    lam = 0.0
    for _ in range(iters):
        w = hp_filter(_At(_A(v), N))
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return float(lam)


def cheb_steps(lam, nu=NU, ratio=CHEB_RATIO, margin=LAMBDA_MARGIN):
    """Step sizes 1/lambda_i, lambda_i = (b+a)/2 + (b-a)/2 cos((2i-1) pi / (2 nu)),
    i = 1..nu, over [a, b] = [margin*lam/ratio, margin*lam]."""
    b = margin * lam
    a = b / ratio
    i = np.arange(1, nu + 1)
    return 1.0 / ((b + a) / 2 + (b - a) / 2 * np.cos((2 * i - 1) * np.pi / (2 * nu)))


def inverse_vcycle(b, N, x, lams):
    """One V-cycle for A_N x = b from x; lams[N] is level N's eigenvalue."""
    if N == 1:
        return np.full((1, 1, 1), np.mean(b))
    steps = cheb_steps(lams[N])
    for c in steps:
        x = x + c * hp_filter(_At(b - _A(x), N))
    e = inverse_vcycle(restrict_proj(b - _A(x)), N // 2, np.zeros((N // 2,) * 3), lams)
    x = x + prolong(e)
    for c in steps[::-1]:
        x = x + c * hp_filter(_At(b - _A(x), N))
    return x


def drt_inverse(b, N, cycles, lams=None, iterates=False):
    """The inverse of the 12-dodecant DRT b ([12][N][N][3N-2]) by `cycles`
    V-cycles from zero. lams maps each size 2..N to its eigenvalue (computed by
    level_lambda when absent). Returns the last iterate, or every iterate."""
    b = np.asarray(b, dtype=np.float64)
    if b.shape != (12, N, N, 3 * N - 2):
        raise ValueError("expected a 12-dodecant DRT of size %d" % N)
    if lams is None:
        lams = {}
    m = 2
    while m <= N:
        if m not in lams:
            lams[m] = level_lambda(m)
        m *= 2
    x = np.zeros((N, N, N))
    out = []
    for _ in range(cycles):
        x = inverse_vcycle(b, N, x, lams)
        out.append(x.copy())
    return out if iterates else x
