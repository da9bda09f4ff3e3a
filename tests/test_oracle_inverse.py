"""Pins of the oracle's iterative inverse (Sec. 5.2): the filter, P and S
against the paper's printed values and exact identities, the smoother's step
sizes against the Chebyshev minimax property, and the whole scheme against the
input it must recover."""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden():
    """The numeric entries of the fixture (those without N, s1, s2)."""
    vals = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = [t.strip() for t in line.split("=", 1)]
            if not any(ch.isalpha() for ch in v):
                vals[k] = eval(v, {"__builtins__": {}})
    return vals


def _blockavg(f):
    N = f.shape[0]
    return f.reshape(N // 2, 2, N // 2, 2, N // 2, 2).mean(axis=(1, 3, 5))


def test_filter_taps_are_the_printed_slices(oracle_mod):
    O = oracle_mod
    g = _golden()
    c, fa, ed, co = g["hp_filter_centre"], g["hp_filter_face"], g["hp_filter_edge"], g["hp_filter_corner"]
    outer = np.array([[co, ed, co], [ed, fa, ed], [co, ed, co]])
    middle = np.array([[ed, fa, ed], [fa, c, fa], [ed, fa, ed]])
    assert np.array_equal(O.HP_FILTER[0], outer)
    assert np.array_equal(O.HP_FILTER[2], outer)
    assert np.array_equal(O.HP_FILTER[1], middle)
    # its taps sum to zero: a high-pass filter
    assert abs(O.HP_FILTER.sum()) < 1e-15


def test_filter_on_an_interior_delta_and_on_constants(oracle_mod):
    O = oracle_mod
    N = 8
    d = np.zeros((N, N, N))
    d[3, 4, 2] = 1.0
    out = O.hp_filter(d)
    assert np.allclose(out[2:5, 3:6, 1:4], O.HP_FILTER)
    assert np.count_nonzero(out) == 27
    # with reflected borders a constant volume is filtered to zero everywhere,
    # faces, edges and corners included
    assert np.allclose(O.hp_filter(np.full((N, N, N), 3.5)), 0.0, atol=1e-14)


def test_filter_is_self_adjoint(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(40)
    x, y = rng.standard_normal((2, 8, 8, 8))
    assert abs(np.vdot(O.hp_filter(x), y) - np.vdot(x, O.hp_filter(y))) < 1e-12


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_restriction_is_exact_on_axis_planes(oracle_mod, N):
    """For slope pair (0, 0) a coarse plane is two whole fine planes, so S of
    the DRT equals the DRT of the 2x2x2 block average exactly, in every
    dodecant."""
    O = oracle_mod
    f = workloads.normal_cube(N, seed=41 + N).astype(np.float64)
    lhs = O.restrict_proj(O.rec_drt(f))
    rhs = O.rec_drt(_blockavg(f)) if N > 2 else np.full((12, 1, 1, 1), _blockavg(f)[0, 0, 0])
    assert lhs.shape == rhs.shape
    assert np.allclose(lhs[:, 0, 0, :], rhs[:, 0, 0, :], rtol=0, atol=1e-12)
    assert _golden()["restriction_weight"] == 1 / 8


def test_restriction_consistency_improves_with_size(oracle_mod):
    """For a smooth input, S(A f) approaches A(average f) as N grows (the
    multiscale lines of slope 2s at N and s at N/2 differ by O(log N) cells)."""
    O = oracle_mod
    errs = []
    for N in (8, 16, 32):
        x = (np.arange(N) + 0.5) / N
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        f = np.exp(-((X - .4) ** 2 + (Y - .55) ** 2 + (Z - .5) ** 2) / 0.05)
        lhs = O.restrict_proj(O.rec_drt(f))
        rhs = O.rec_drt(_blockavg(f))
        errs.append(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.06


def test_prolongation_is_block_constant_and_averages_back(oracle_mod):
    O = oracle_mod
    x = workloads.normal_cube(4, seed=42).astype(np.float64)
    p = O.prolong(x)
    assert p.shape == (8, 8, 8)
    assert np.array_equal(_blockavg(p), x)
    assert np.array_equal(p[::2, ::2, ::2], p[1::2, 1::2, 1::2])


def test_chebyshev_steps_have_the_minimax_residual(oracle_mod):
    """prod_i (1 - c_i t) stays within 1/T_nu((b+a)/(b-a)) on [a, b]."""
    O = oracle_mod
    lam = 7.0
    for nu in (1, 2, 3, 4):
        c = O.cheb_steps(lam, nu=nu)
        b = 1.02 * lam
        a = b / 10
        t = np.linspace(a, b, 2001)
        p = np.prod([1 - ci * t for ci in c], axis=0)
        z = (b + a) / (b - a)
        bound = 1 / np.cosh(nu * np.arccosh(z))
        assert np.max(np.abs(p)) <= bound * (1 + 1e-9)
        assert np.max(np.abs(p)) >= bound * (1 - 1e-3)  # attained: the optimum, not just a bound


@pytest.mark.parametrize("N", [4, 8, 16])
def test_level_lambda_is_an_eigenvalue(oracle_mod, N):
    """The power iteration's value is an eigenvalue of H A^T A to within 10 %
    (its vector is an eigenvector to that accuracy) and bounds the Rayleigh
    quotient of a Nyquist pattern."""
    O = oracle_mod
    lam = O.level_lambda(N)
    v = O.power_start(N)
    for _ in range(30):
        w = O.hp_filter(O.rec_adj(O.rec_drt(v), N))
        v = w / np.linalg.norm(w)
    Mv = O.hp_filter(O.rec_adj(O.rec_drt(v), N))
    assert np.linalg.norm(Mv - lam * v) / lam < 0.1
    x = np.arange(N)
    chk = (-1.0) ** (x[:, None, None] + x[None, :, None] + x[None, None, :])
    q = np.vdot(chk, O.hp_filter(O.rec_adj(O.rec_drt(chk), N))) / np.vdot(chk, chk)
    assert q <= lam * 1.01


@pytest.mark.parametrize("N", [4, 8, 16])
def test_inverse_recovers_the_input(oracle_mod, N):
    """10 V-cycles on the DRT of the corners-and-centre cube (the Sec. 5.1
    example input) and of a normal cube recover them to 1e-7, the error
    falling every cycle."""
    O = oracle_mod
    for f in (workloads.corners_and_centre(N).astype(np.float64), workloads.normal_cube(N, seed=43).astype(np.float64)):
        its = O.drt_inverse(O.rec_drt(f), N, 10, iterates=True)
        errs = [np.linalg.norm(x - f) / np.linalg.norm(f) for x in its]
        assert all(b < a for a, b in zip(errs, errs[1:]))
        assert errs[-1] < 1e-7, errs


def test_inverse_is_linear(oracle_mod):
    O = oracle_mod
    N = 8
    lams = {m: O.level_lambda(m) for m in (2, 4, 8)}
    f = workloads.normal_cube(N, seed=44).astype(np.float64)
    g = workloads.corners_and_centre(N).astype(np.float64)
    bf, bg = O.rec_drt(f), O.rec_drt(g)
    lhs = O.drt_inverse(bf + 2 * bg, N, 3, lams=dict(lams))
    rhs = O.drt_inverse(bf, N, 3, lams=dict(lams)) + 2 * O.drt_inverse(bg, N, 3, lams=dict(lams))
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-10)
