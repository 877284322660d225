"""Pins of the oracle's RBF-FD weights (Sec. II: the augmented PHS + monomial
system) against facts fixed independently of the oracle's own code."""
import math

import numpy as np
import pytest

import oracle
import rbf_inputs as ri
from fixtures import read_closed_form_stencils, read_support_sizes

CLOSED = read_closed_form_stencils()


@pytest.mark.parametrize("blk", CLOSED, ids=[b["name"] for b in CLOSED])
@pytest.mark.parametrize("h", [1.0, 0.01, 1.0 / 99])
def test_closed_form_stencils(blk, h):
    """5-point / 7-point Laplacians, the natural cubic spline (pins the r^3
    block) and the 4th-order 1D stencil, at several spacings and off-origin."""
    nodes = blk["nodes"] * h + 0.25
    xyz = np.ascontiguousarray(nodes.T)
    n = xyz.shape[1]
    w, pr, st, _ = oracle.weights(xyz, np.arange(n)[None, :], [0], m=blk["m"])
    expect = blk["weights"] / (h * h)
    assert st == 0
    np.testing.assert_allclose(w[0], expect, rtol=0, atol=1e-11 * np.abs(expect).max())


def test_spline_pin_sees_the_rbf_block():
    """With m = 1 and n = 5 the weights are not those of any polynomial
    stencil: the r^3 block decides them (so the spline pin covers A)."""
    blk = [b for b in CLOSED if b["name"] == "natural_cubic_spline_1d"][0]
    assert not np.allclose(blk["weights"], [-30 / 12, -1 / 12, 16 / 12, 16 / 12, -1 / 12])


def test_support_sizes_printed_in_paper():
    for d, m, n, rule in read_support_sizes():
        ex = oracle.monomials(d, m)
        M = len(ex)
        assert M == math.comb(m + d, d) == ri.num_monomials(d, m)
        assert n == (2 * M + 1 if rule == "2M+1" else 2 * M)
        # every exponent vector of degree <= m appears exactly once
        assert len({tuple(e) for e in ex}) == M
        assert ex.sum(axis=1).max() == m and (ex[:, d:] == 0).all()


def _monomial_check(xyz, rows, idx, w, m):
    dim = xyz.shape[0]
    worst = 0.0
    for q, r in enumerate(rows):
        rel = xyz[:, idx[q]] - xyz[:, [r]]
        for e in oracle.monomials(dim, m):
            p = np.ones(idx.shape[1])
            for a in range(dim):
                p = p * rel[a] ** e[a]
            lap0 = 2.0 if (e.sum() == 2 and e.max() == 2) else 0.0
            terms = w[q] * p
            err = abs(terms.sum() - lap0) / (np.abs(terms).sum() + abs(lap0))
            worst = max(worst, err)
    return worst


@pytest.mark.parametrize("dim,m,side", [(2, 2, 14), (2, 4, 14), (2, 6, 16), (3, 2, 9), (3, 4, 9), (3, 6, 10)])
def test_monomial_reproduction(dim, m, side):
    """Every stencil reproduces the Laplacian of every monomial of degree <= m
    (the second block row of the augmented system), to 1e-9 normalised."""
    xyz, typ = ri.jittered_grid(dim, side, 0.3, 11 + m)
    n = 2 * ri.num_monomials(dim, m)
    interior = np.nonzero(typ == 0)[0]
    rows = np.random.default_rng(m).choice(interior, size=min(25, len(interior)), replace=False)
    idx = oracle.knn(xyz, n, rows)
    w, pr, st, _ = oracle.weights(xyz, idx, rows, m=m)
    assert st == 0 and (pr > 0).all()
    assert _monomial_check(xyz, rows, idx, w, m) < 1e-9


def _one_system(dim, m, seed=3, side=9):
    xyz, typ = ri.jittered_grid(dim, side, 0.3, seed)
    n = 2 * ri.num_monomials(dim, m)
    c = int(np.nonzero(typ == 0)[0][len(np.nonzero(typ == 0)[0]) // 2])
    idx = oracle.knn(xyz, n, [c])
    return xyz, c, idx


@pytest.mark.parametrize("dim,m", [(2, 2), (2, 4), (3, 2), (3, 4), (3, 6)])
def test_scaling_by_two_is_exact(dim, m):
    """Doubling all coordinates leaves y bitwise unchanged, so w scales by
    exactly 1/4 (the Laplacian is homogeneous of degree -2)."""
    xyz, c, idx = _one_system(dim, m)
    w1 = oracle.weights(xyz, idx, [c], m=m)[0]
    w2 = oracle.weights(2.0 * xyz, idx, [c], m=m)[0]
    assert np.array_equal(w2, w1 / 4.0)


@pytest.mark.parametrize("dim,m", [(2, 2), (2, 6), (3, 4)])
def test_reflection_is_exact(dim, m):
    """x -> -x negates the odd-x monomial columns; partial pivoting sees the
    same magnitudes, so the weights are bitwise identical."""
    xyz, c, idx = _one_system(dim, m)
    w1 = oracle.weights(xyz, idx, [c], m=m)[0]
    xr = xyz.copy()
    xr[0] = -xr[0]
    w2 = oracle.weights(xr, idx, [c], m=m)[0]
    assert np.array_equal(w1, w2)


@pytest.mark.parametrize("dim,m", [(2, 4), (3, 2), (3, 4)])
def test_translation_and_axis_permutation(dim, m):
    xyz, c, idx = _one_system(dim, m)
    w1 = oracle.weights(xyz, idx, [c], m=m)[0]
    shift = np.array([0.5, 0.25, 0.125][:dim])[:, None]
    w2 = oracle.weights(xyz + shift, idx, [c], m=m)[0]
    w3 = oracle.weights(np.ascontiguousarray(xyz[::-1]), idx, [c], m=m)[0]
    scale = np.abs(w1).max()
    assert np.abs(w2 - w1).max() <= 1e-9 * scale
    assert np.abs(w3 - w1).max() <= 1e-9 * scale


def test_symmetric_stencil_has_symmetric_weights():
    """On a jitter-free grid the 2D 12-point support is symmetric under x->-x
    and y->-y; mirrored nodes get equal weights."""
    xyz, typ = ri.jittered_grid(2, 9, 0.0, 0)
    c = 4 + 9 * 4
    idx = oracle.knn(xyz, 13, [c])
    w = oracle.weights(xyz, idx, [c], m=2)[0][0]
    pos = {(round((xyz[0, j] - xyz[0, c]) * 8), round((xyz[1, j] - xyz[1, c]) * 8)): w[k]
           for k, j in enumerate(idx[0])}
    for (a, b), wk in pos.items():
        for mir in ((-a, b), (a, -b), (b, a)):
            assert abs(pos[mir] - wk) <= 1e-10 * abs(w).max()


@pytest.mark.parametrize("dim,m,count", [(2, 2, 200), (2, 6, 60), (3, 2, 200), (3, 4, 60), (3, 6, 12)])
def test_gepp_matches_lapack(dim, m, count):
    """The oracle's elimination agrees with LAPACK's (numpy.linalg.solve) on
    the very matrix the oracle assembles."""
    side = 8 if dim == 3 else 16
    xyz, typ = ri.jittered_grid(dim, side, 0.3, 21)
    n = 2 * ri.num_monomials(dim, m)
    interior = np.nonzero(typ == 0)[0]
    rows = np.random.default_rng(1).choice(interior, size=min(count, len(interior)), replace=False)
    idx = oracle.knn(xyz, n, rows)
    w, _, _, _ = oracle.weights(xyz, idx, rows, m=m)
    worst = 0.0
    for q, r in enumerate(rows):
        A, b, s = oracle.assemble(xyz, r, idx[q], m)
        x = np.linalg.solve(A, b)
        wl = x[:n] / (s * s)
        cond = np.linalg.cond(A)
        rel = np.abs(wl - w[q]).max() / np.abs(wl).max()
        worst = max(worst, rel / max(1.0, cond * 1e-16 / 1e-12))
    assert worst <= 1e-12


def test_assembly_matches_definition():
    """Entries of the assembled matrix against the paper's definitions written
    out in numpy (A_ij = |y_i - y_j|^3, P_ij = p_j(y_i), L Phi and L p)."""
    dim, m = 3, 2
    xyz, c, idx = _one_system(dim, m)
    A, b, s = oracle.assemble(xyz, c, idx[0], m)
    n = idx.shape[1]
    y = (xyz[:, idx[0]] - xyz[:, [c]]) / s
    D = np.sqrt(((y[:, :, None] - y[:, None, :]) ** 2).sum(0))
    np.testing.assert_allclose(A[:n, :n], D ** 3, rtol=1e-14, atol=1e-15)
    ex = oracle.monomials(dim, m)
    P = np.stack([np.prod([y[a] ** e[a] for a in range(dim)], axis=0) for e in ex], axis=1)
    np.testing.assert_allclose(A[:n, n:], P, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(A[n:, :n], A[:n, n:].T)
    assert (A[n:, n:] == 0).all()
    np.testing.assert_allclose(b[:n], 3 * (dim + 1) * np.sqrt((y ** 2).sum(0)), rtol=1e-15)
    lp = [2.0 if (e.sum() == 2 and e.max() == 2) else 0.0 for e in ex]
    np.testing.assert_array_equal(b[n:], lp)
    assert s == np.sqrt(((xyz[:, idx[0]] - xyz[:, [c]]) ** 2).sum(0).max())


def _singular_status(xyz, stencil, m):
    _, _, st, bad = oracle.weights(xyz, np.asarray([stencil]), [stencil[0]], m=m, raise_on_singular=False)
    return st, bad


def test_singular_systems_detected():
    # fewer support nodes than monomials (2D, m = 2, n = 5 < M = 6)
    xyz, typ = ri.jittered_grid(2, 9, 0.3, 5)
    c = 40
    idx = oracle.knn(xyz, 5, [c])[0]
    assert _singular_status(xyz, idx, 2) == (3, c)
    # duplicate node in the support
    xd = xyz.copy()
    idx12 = oracle.knn(xyz, 12, [c])[0]
    xd[:, idx12[5]] = xd[:, idx12[3]]
    assert _singular_status(xd, idx12, 2)[0] == 3
    # collinear support on a line (all y equal)
    pts = np.zeros((2, 12))
    pts[0] = np.linspace(0.0, 1.0, 12)
    pts[1] = 0.5
    assert _singular_status(pts, np.arange(12), 2)[0] == 3
    # collinear on the diagonal
    pts[1] = pts[0]
    assert _singular_status(pts, np.arange(12), 2)[0] == 3
