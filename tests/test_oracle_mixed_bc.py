"""Pins of the oracle's mixed Dirichlet/Neumann variant (Sec. II-C): the
problem on [0, 1/2]^d with zero normal derivative on the faces inside the
original cube, Neumann values set before each step from the previous step."""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle
import rbf_inputs as ri
from fixtures import GOLDEN


def _blocks():
    out, cur = [], None
    with open(os.path.join(GOLDEN, "closed_form_normal_derivative.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "name":
                cur = {"name": rest}
                out.append(cur)
            elif key in ("dim", "m"):
                cur[key] = int(rest)
            elif key == "normal":
                cur["normal"] = np.array([float(t) for t in rest.split()])
            elif key == "nodes":
                cur["nodes"] = np.array([[float(t) for t in p.split()] for p in rest.split("|")])
            elif key == "weights":
                cur["weights"] = np.array([float(Fraction(t)) for t in rest.split()])
    return out


BLOCKS = _blocks()


@pytest.mark.parametrize("blk", BLOCKS, ids=[b["name"] for b in BLOCKS])
@pytest.mark.parametrize("h", [1.0, 0.02])
def test_closed_form_normal_derivative(blk, h):
    xyz = np.ascontiguousarray((blk["nodes"] * h + 0.3).T)
    n = xyz.shape[1]
    normals = np.zeros_like(xyz)
    normals[:, 0] = blk["normal"]
    w, _, st, _ = oracle.weights(xyz, np.arange(n)[None, :], [0], m=blk["m"], op_row=[1], normals=normals)
    expect = blk["weights"] / h
    assert st == 0
    np.testing.assert_allclose(w[0], expect, rtol=0, atol=1e-11 * np.abs(expect).max())


@pytest.mark.parametrize("dim,m,side", [(2, 2, 12), (2, 4, 14), (3, 2, 8), (3, 4, 9), (3, 6, 10)])
def test_normal_derivative_reproduces_monomials(dim, m, side):
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 3 + m)
    n = 2 * ri.num_monomials(dim, m)
    rows = np.nonzero(typ == 2)[0][:: max(1, (typ == 2).sum() // 20)]
    idx = oracle.knn(xyz, n, rows)
    w, _, st, _ = oracle.weights(xyz, idx, rows, m=m, op_row=np.ones(len(rows), np.int8), normals=normals)
    assert st == 0
    worst = 0.0
    for q, r in enumerate(rows):
        rel = xyz[:, idx[q]] - xyz[:, [r]]
        for e in oracle.monomials(dim, m):
            p = np.ones(n)
            for a in range(dim):
                p = p * rel[a] ** e[a]
            dn = sum(normals[a, r] for a in range(dim) if e.sum() == 1 and e[a] == 1)
            terms = w[q] * p
            worst = max(worst, abs(terms.sum() - dn) / (np.abs(terms).sum() + abs(dn) + 1e-300))
    assert worst < 1e-9


def test_mixed_grid_types_and_normals():
    xyz, typ, normals = ri.mixed_bc_grid(3, 11, 0.3, 1)
    assert xyz.max() == 0.5 and xyz.min() == 0.0
    side = 11
    assert (typ == 1).sum() == side ** 3 - (side - 1) ** 3
    assert (typ == 2).sum() == (side - 1) ** 3 - (side - 2) ** 3
    nn = np.linalg.norm(normals[:, typ == 2], axis=0)
    np.testing.assert_allclose(nn, 1.0, rtol=1e-15)
    assert (normals[:, typ != 2] == 0).all()
    # Neumann nodes sit on x_a = 1/2 faces and their normal points outwards
    for a in range(3):
        on = (typ == 2) & (xyz[a] == 0.5)
        assert (normals[a, on] > 0).all()


def _mixed_problem(dim, side, m, seed=5):
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, seed)
    n = 2 * ri.num_monomials(dim, m)
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    return xyz, typ, normals, idx, w


def test_polynomial_with_neumann_data_is_fixed_point():
    """u_p quadratic (m = 2): f = Laplacian(u_p) inside, f = n.grad(u_p) on
    Neumann nodes, g = u_p on Dirichlet nodes; u_p is a discrete fixed point."""
    dim, side, m = 3, 9, 2
    xyz, typ, normals, idx, w = _mixed_problem(dim, side, m)
    x, y, z = xyz
    up = 1 + x - 2 * y + x * z + 0.5 * y ** 2
    grad = np.stack([1 + z, -2 + y, x])
    f = np.where(typ == 0, 1.0, 0.0)
    f = np.where(typ == 2, (grad * normals).sum(0), f)
    op = oracle.Operator(typ, idx, w)
    h = 0.5 / (side - 1)
    u, rep, st = op.iterate(f, 0.15 * h * h / 6, up, 400, 0.0, 100)
    assert st == 0
    assert np.abs(u - up).max() <= 1e-11


def _coupled_solve(typ, idx, w, f, g):
    N, n = idx.shape
    rows = np.repeat(np.arange(N), n)
    A = sp.csr_matrix((w.reshape(-1), (rows, idx.reshape(-1))), shape=(N, N))
    U = np.nonzero(typ != 1)[0]     # unknowns: interior and Neumann
    D = np.nonzero(typ == 1)[0]
    rhs = f[U] - A[U][:, D] @ g[D]
    uU = sla.spsolve(A[U][:, U].tocsc(), rhs)
    out = g.copy()
    out[U] = uU
    return out


def test_iteration_reaches_coupled_solve():
    """The fixed point of the step with the Neumann update is the solution of
    the coupled system (Laplacian rows inside, normal-derivative rows on the
    Neumann faces, Dirichlet values given)."""
    dim, side, m = 2, 17, 2
    xyz, typ, normals, idx, w = _mixed_problem(dim, side, m)
    u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
    ref = _coupled_solve(typ, idx, w, f, u0)
    h = 0.5 / (side - 1)
    u, rep, st = oracle.Operator(typ, idx, w).iterate(f, 0.1 * h * h / 4, u0, 400000, 1e-12, 1000)
    assert st == 0 and rep["converged"] == 1
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("dim,sides,m", [(2, (11, 21, 41), 2), (2, (11, 21, 41), 4), (3, (7, 11, 15), 2)])
def test_mixed_error_slope(dim, sides, m):
    """Error of the discrete solution against prod sin(pi x_i) under
    refinement, with the Neumann faces: slope at least m - 1.3."""
    errs, hs = [], []
    for side in sides:
        xyz, typ, normals, idx, w = _mixed_problem(dim, side, m)
        u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
        u = _coupled_solve(typ, idx, w, f, u0)
        errs.append(np.abs(u - u_ex).max())
        hs.append(0.5 / (side - 1))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope >= m - 1.3, (errs, slope)


def test_apply_gives_normal_derivative_of_linear_fields():
    """On Neumann rows the operator returns n . grad u, exact for linear u
    (up to rounding); interior rows give 0 for a linear u, Dirichlet rows 0."""
    dim, side, m = 3, 9, 4
    xyz, typ, normals, idx, w = _mixed_problem(dim, side, m)
    a = np.array([0.3, -1.1, 0.7])
    Lu = oracle.Operator(typ, idx, w).apply(0.5 + a @ xyz)
    B = typ == 2
    assert np.abs(Lu[B] - a @ normals[:, B]).max() <= 1e-10
    assert np.abs(Lu[typ == 0]).max() <= 1e-8
    assert (Lu[typ == 1] == 0).all()


@pytest.mark.parametrize("dim,side,n", [(2, 15, 12), (3, 9, 70)])
def test_neumann_supports_hold_interior_nodes_only(dim, side, n):
    """A Neumann node's support is the node itself and its nearest interior
    nodes (its value is set from interior values, Sec. II-C): the oracle's
    typed search against a numpy brute force over {itself} and the interior
    nodes, with the same key (d2, id), d2 = (dx*dx + dy*dy) + dz*dz."""
    xyz, typ, _ = ri.mixed_bc_grid(dim, side, 0.3, 17)
    idx = oracle.knn(xyz, n, typ=typ)
    interior = np.nonzero(typ == 0)[0]
    for c in np.nonzero(typ == 2)[0]:
        cand = np.concatenate([[c], interior])
        d = [xyz[a, cand] - xyz[a, c] for a in range(dim)]
        d2 = d[0] * d[0]
        for a in range(1, dim):
            d2 = d2 + d[a] * d[a]
        order = np.lexsort((cand, d2))
        assert np.array_equal(idx[c], cand[order[:n]])
        assert idx[c, 0] == c and (typ[idx[c, 1:]] == 0).all()
    # the other rows are the plain search
    other = np.nonzero(typ != 2)[0]
    assert np.array_equal(idx[other], oracle.knn(xyz, n, rows=other))
