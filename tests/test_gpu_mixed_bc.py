"""GPU parity of the mixed Dirichlet/Neumann variant (Sec. II-C): the problem
on [0, 1/2]^d with zero normal derivative on the faces inside the original
cube.  Bars as for the Dirichlet problem: supports bit-exact, weights within
1e-10 relative per row, FP64 iterates within 1e-11 relative."""
import numpy as np
import pytest

import oracle
import rbf_inputs as ri

pytestmark = pytest.mark.gpu


def _problem():
    from paper_2502_12878_amd import Problem
    return Problem(0)


def _rel_rows(a, b):
    scale = np.abs(b).max(axis=1) + 1e-300
    return (np.abs(a - b).max(axis=1) / scale).max()


def _gpu_setup(xyz, typ, normals, n, m):
    p = _problem()
    p.set_nodes(xyz, typ)
    p.set_normals(normals)
    p.build_stencils(n)
    p.compute_weights(m)
    return p


@pytest.mark.parametrize("dim,side,m,seed", [(2, 33, 2, 1), (2, 21, 4, 2), (3, 12, 2, 3), (3, 11, 4, 4),
                                             (3, 10, 6, 5)])
def test_supports_and_weights_match_oracle(dim, side, m, seed):
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, seed)
    n = 2 * ri.num_monomials(dim, m)
    p = _gpu_setup(xyz, typ, normals, n, m)
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    got = p.get_stencils()
    assert np.array_equal(got, idx)
    # Neumann supports: the node itself and interior nodes only
    for r in np.nonzero(typ == 2)[0]:
        assert got[r, 0] == r and (typ[got[r, 1:]] == 0).all()
    wg = p.get_weights()
    for code in (0, 2):
        rows = typ == code
        rel = _rel_rows(wg[rows], w[rows])
        print(f"type {code}: max row-relative weight difference {rel:.2e}")
        assert rel <= 1e-10
    assert (wg[typ == 1] == 0).all()


def test_apply_returns_normal_derivative_on_neumann_rows():
    import torch
    dim, side, m = 3, 12, 4
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 8)
    n = 2 * ri.num_monomials(dim, m)
    p = _gpu_setup(xyz, typ, normals, n, m)
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    u = np.random.default_rng(1).standard_normal(len(typ))
    Lg = p.apply(torch.tensor(u, device="cuda")).cpu().numpy()
    Lo = oracle.Operator(typ, idx, w).apply(u)
    assert np.abs(Lg - Lo).max() <= 1e-12 * np.abs(Lo).max()
    assert (Lg[typ == 1] == 0).all()
    # on a linear field the Neumann rows give n . grad exactly (up to rounding)
    a = np.array([0.3, -1.1, 0.7])
    ul = 0.5 + a @ xyz
    Dl = p.apply(torch.tensor(ul, device="cuda")).cpu().numpy()
    B = typ == 2
    assert np.abs(Dl[B] - a @ normals[:, B]).max() <= 1e-9


@pytest.mark.parametrize("dim,side,m,steps,chunk", [(2, 41, 2, 1500, 500), (3, 12, 4, 400, 100),
                                                    (3, 10, 6, 301, 100)])
def test_fixed_steps_match_oracle(dim, side, m, steps, chunk):
    import torch
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 20 + m)
    n = 2 * ri.num_monomials(dim, m)
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
    h = 0.5 / (side - 1)
    dt = 0.15 * h * h / (2 * dim)
    p = _gpu_setup(xyz, typ, normals, n, m)
    # the iteration runs on the oracle's weights, so only the sweeps are compared
    p.set_weights(w)
    u = torch.tensor(u0, device="cuda")
    st, rep = p.iterate(torch.tensor(f, device="cuda"), u, dt, steps, 0.0, chunk)
    uo, rep_o, st_o = oracle.Operator(typ, idx, w).iterate(f, dt, u0, steps, 0.0, chunk)
    assert st == st_o == 0 and rep["steps"] == steps
    ug = u.cpu().numpy()
    assert np.abs(ug - uo).max() <= 1e-11 * np.abs(uo).max()
    D = typ == 1
    assert np.array_equal(ug[D], u0[D])
    assert abs(rep["res_final"] - rep_o["res_final"]) <= 1e-9 * rep_o["res_final"]
    assert rep["fnorm"] == rep_o["fnorm"]


def test_polynomial_with_neumann_data_is_fixed_point():
    """u_p quadratic, m = 2: f = Laplacian(u_p) inside, f = n . grad(u_p) on
    Neumann nodes, u_p on Dirichlet nodes; the GPU iteration keeps u_p."""
    import torch
    dim, side, m = 3, 13, 2
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 6)
    n = 2 * ri.num_monomials(dim, m)
    p = _gpu_setup(xyz, typ, normals, n, m)
    x, y, z = xyz
    up = 1 + x - 2 * y + x * z + 0.5 * y ** 2
    grad = np.stack([1 + z, -2 + y, x])
    f = np.where(typ == 0, 1.0, 0.0)
    f = np.where(typ == 2, (grad * normals).sum(0), f)
    h = 0.5 / (side - 1)
    u = torch.tensor(up, device="cuda")
    st, rep = p.iterate(torch.tensor(f, device="cuda"), u, 0.15 * h * h / 6, 2000, 0.0, 500)
    assert st == 0
    assert np.abs(u.cpu().numpy() - up).max() <= 1e-11


def test_converges_to_coupled_solution_with_oracle_chunk():
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    import torch
    dim, side, m = 2, 21, 2
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 9)
    n = 2 * ri.num_monomials(dim, m)
    p = _gpu_setup(xyz, typ, normals, n, m)
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    p.set_weights(w)
    u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
    h = 0.5 / (side - 1)
    dt = 0.1 * h * h / 4
    u = torch.tensor(u0, device="cuda")
    st, rep = p.iterate(torch.tensor(f, device="cuda"), u, dt, 10 ** 6, 1e-11, 1000)
    uo, rep_o, st_o = oracle.Operator(typ, idx, w).iterate(f, dt, u0, 10 ** 6, 1e-11, 1000)
    assert st == st_o == 0 and rep["converged"] == 1
    assert rep["steps"] == rep_o["steps"]
    # the fixed point is the solution of the coupled sparse system
    N = len(typ)
    A = sp.csr_matrix((w.reshape(-1), (np.repeat(np.arange(N), n), idx.reshape(-1))), shape=(N, N))
    U, D = np.nonzero(typ != 1)[0], np.nonzero(typ == 1)[0]
    ref = u0.copy()
    ref[U] = sla.spsolve(A[U][:, U].tocsc(), f[U] - A[U][:, D] @ u0[D])
    ug = u.cpu().numpy()
    assert np.abs(ug - ref).max() <= 1e-9 * np.abs(ref).max()
    # and close to the exact solution at this spacing
    assert np.abs(ug - u_ex).max() <= 0.02


def test_restrictions_and_validation():
    import torch
    from paper_2502_12878_amd import RBF_EINVAL, RBF_MODE_MIXED, RbfError
    dim, side, m = 2, 15, 2
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 10)
    n = 2 * ri.num_monomials(dim, m)
    p = _problem()
    p.set_nodes(xyz, typ)
    p.build_stencils(n)
    with pytest.raises(RbfError) as ei:
        p.compute_weights(m)  # Neumann nodes without normals
    assert ei.value.status == RBF_EINVAL
    bad = normals.copy()
    bad[:, typ == 2] *= 2.0
    with pytest.raises(RbfError):
        p.set_normals(bad)
    p.set_normals(normals)
    p.compute_weights(m, keep_fp32=True)
    f = torch.zeros(len(typ), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    with pytest.raises(RbfError) as ei:
        p.iterate(f, u, 1e-4, 10, mode=RBF_MODE_MIXED, inner_steps=5)
    assert ei.value.status == RBF_EINVAL
    with pytest.raises(RbfError) as ei:
        p.adjoint_f(f, 10, 5, 1e-4)
    assert ei.value.status == RBF_EINVAL
    # imported Neumann rows must contain their own node with a nonzero weight
    idx = p.get_stencils()
    w = p.get_weights()
    r = int(np.nonzero(typ == 2)[0][0])
    w[r, 0] = 0.0
    with pytest.raises(RbfError) as ei:
        p.set_weights(w)
    assert ei.value.status == RBF_EINVAL and f"Neumann node {r}" in str(ei.value)
    # repeated ids in an imported stencil
    idx[5, 1] = idx[5, 2]
    with pytest.raises(RbfError) as ei:
        p.set_stencils(idx)
    assert ei.value.status == RBF_EINVAL


def test_neumann_supports_with_boundary_nodes_use_two_phase_update():
    """Imported supports where some Neumann rows also hold other Neumann
    nodes: all new boundary values must come from the old iterate (the
    library then evaluates into a buffer and stores in a second kernel);
    iterates against the oracle, whose update has the same two phases."""
    import torch
    dim, side, m = 2, 25, 2
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 12)
    n = 2 * ri.num_monomials(dim, m)
    idx = oracle.knn(xyz, n, typ=typ)
    neu = np.nonzero(typ == 2)[0]
    # swap the farthest support node of every other Neumann row for the
    # nearest other Neumann node
    for r in neu[::2]:
        d = ((xyz[:, neu] - xyz[:, [r]]) ** 2).sum(0)
        d[neu == r] = np.inf
        q = neu[np.argmin(d)]
        if q not in idx[r]:
            idx[r, -1] = q
    rows = np.nonzero(typ != 1)[0]
    op = (typ[rows] == 2).astype(np.int8)
    w = np.zeros(idx.shape)
    w[rows] = oracle.weights(xyz, idx[rows], rows, m=m, op_row=op, normals=normals)[0]
    p = _problem()
    p.set_nodes(xyz, typ)
    p.set_normals(normals)
    p.set_stencils(idx)
    p.set_weights(w)
    u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
    h = 0.5 / (side - 1)
    dt = 0.1 * h * h / 4
    u = torch.tensor(u0, device="cuda")
    st, rep = p.iterate(torch.tensor(f, device="cuda"), u, dt, 2000, 0.0, 500)
    uo, rep_o, st_o = oracle.Operator(typ, idx, w).iterate(f, dt, u0, 2000, 0.0, 500)
    assert st == st_o == 0
    assert np.abs(u.cpu().numpy() - uo).max() <= 1e-11 * np.abs(uo).max()


def test_overlapped_neumann_step_is_bitwise_identical(monkeypatch):
    """A step sweeps the interior rows that read no Neumann value while the
    Neumann values are updated, then the rest; the iterates are bitwise those
    of the sequential step and match the oracle."""
    import torch
    dim, side, m = 3, 24, 4
    xyz, typ, normals = ri.mixed_bc_grid(dim, side, 0.3, 17)
    n = 2 * ri.num_monomials(dim, m)
    u_ex, f, u0 = ri.manufactured_mixed(dim, xyz, typ)
    h = 0.5 / (side - 1)
    dt = 0.15 * h * h / 6
    out = []
    for ov in ("0", "1"):
        monkeypatch.setenv("RBF_NEUMANN_OVERLAP", ov)
        p = _gpu_setup(xyz, typ, normals, n, m)
        u = torch.tensor(u0, device="cuda")
        st, rep = p.iterate(torch.tensor(f, device="cuda"), u, dt, 777, 0.0, 111)
        assert st == 0
        out.append((u.cpu().numpy(), rep["res_final"], rep["res_last"]))
        p.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    idx, w = oracle.setup(xyz, typ, n, m=m, normals=normals)
    uo, _, _ = oracle.Operator(typ, idx, w).iterate(f, dt, u0, 777, 0.0, 111)
    assert np.abs(out[1][0] - uo).max() <= 1e-11 * np.abs(uo).max()
