"""GPU status codes against the oracle's: the stall stop of the chunked
iteration, singular weight systems from collinear supports, the neighbour
search's candidate overflow on a clustered node set, and the step cap of the
mixed-precision mode.  Every failure here is detected by a kernel's own check
or by host logic; every kernel exits normally."""
import numpy as np
import pytest

import oracle
import rbf_inputs as ri

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def _problem():
    from paper_2502_12878_amd import Problem
    return Problem(0)


def test_stall_stop_at_oracle_chunk():
    """With dt = 0 the iterate never moves, so every chunk reports the
    initial residual: the first chunk sets the best value and the run stops
    after `stall` chunks without a new best, at the same step count as the
    oracle, with ENOTCONVERGED (a tolerance was asked for)."""
    from paper_2502_12878_amd import RBF_ENOTCONVERGED
    print("stall stop: 2D side 17, m=2, n=12", flush=True)
    xyz, typ = ri.jittered_grid(2, 17, 0.3, 51)
    idx, w = oracle.setup(xyz, typ, 12, m=2)
    u_ex, f, g, u0 = ri.manufactured(2, xyz, typ)
    op = oracle.Operator(typ, idx, w)
    p = _problem()
    p.set_nodes(xyz, typ)
    p.set_stencils(idx)
    p.set_weights(w)
    for chunk, stall in ((50, 3), (7, 1)):
        u = _dev(u0)
        st, rep = p.iterate(_dev(f), u, 0.0, 100000, 1e-30, chunk, stall_chunks=stall)
        uo, rep_o, st_o = op.iterate(f, 0.0, u0, 100000, 1e-30, chunk, stall)
        assert st == st_o == RBF_ENOTCONVERGED
        assert rep["steps"] == rep_o["steps"] == chunk * (stall + 1)
        assert rep["checks"] == stall + 1
        assert np.array_equal(u.cpu().numpy(), u0)


def _line_set():
    """2D node set: a regular 41 x 41 grid of [0,1]^2 (boundary nodes
    Dirichlet) and 301 interior nodes on the segment y = 0.5125, 0.3 <= x <=
    0.6 at spacing 0.001, numbered after the grid.  A line node's 12 nearest
    nodes are all on the line; the grid nodes next to the line see the line
    first as well.  Such supports cannot determine the 6 quadratic monomials
    (on a line they span only 1, t, t^2)."""
    side = 41
    t = np.arange(side) / (side - 1)
    X, Y = np.meshgrid(t, t, indexing="xy")
    gx, gy = X.reshape(-1), Y.reshape(-1)
    ii, jj = np.meshgrid(np.arange(side), np.arange(side), indexing="xy")
    gtyp = ((ii == 0) | (ii == side - 1) | (jj == 0) | (jj == side - 1)).reshape(-1).astype(np.int8)
    lx = 0.3 + 0.001 * np.arange(301)
    ly = np.full_like(lx, 0.5125)
    xyz = np.stack([np.concatenate([gx, lx]), np.concatenate([gy, ly])])
    typ = np.concatenate([gtyp, np.zeros(len(lx), dtype=np.int8)])
    return np.ascontiguousarray(xyz), typ


def test_collinear_supports_singular_at_oracle_node():
    from paper_2502_12878_amd import RBF_ESINGULAR, RbfError
    print("collinear supports: 2D grid + line, m=2, n=12", flush=True)
    xyz, typ = _line_set()
    n, m = 12, 2
    idx_o = oracle.knn(xyz, n)
    interior = np.nonzero(typ == 0)[0]
    _, _, st, bad = oracle.weights(xyz, idx_o[interior], interior, m=m, raise_on_singular=False)
    assert st == 3 and bad >= 0
    p = _problem()
    p.set_nodes(xyz, typ)
    p.build_stencils(n)
    assert np.array_equal(p.get_stencils(), idx_o)
    with pytest.raises(RbfError) as ei:
        p.compute_weights(m)
    assert ei.value.status == RBF_ESINGULAR
    assert f"node {bad}" in str(ei.value)
    # the handle stays usable: a node set without the line solves
    xg, tg = ri.jittered_grid(2, 21, 0.3, 52)
    p.set_nodes(xg, tg)
    p.build_stencils(n)
    p.compute_weights(m)
    p.close()


def test_knn_candidate_overflow_on_clustered_nodes():
    """1,500 nodes packed in a ball of radius 1e-4 inside a 12^3 grid: the
    cell grid sized for the mean density puts them all in one cell, so the
    queries near it collect more candidates than the search's capacity.  The
    kernel's own check stops those queries and reports EOVERFLOW with the
    lowest such node id (the same on every run); the handle stays usable."""
    from paper_2502_12878_amd import RbfError, _abi
    print("kNN overflow: 12^3 grid + 1500-node cluster, n=20", flush=True)
    xyz0, typ0 = ri.jittered_grid(3, 12, 0.3, 53)
    rng = np.random.default_rng(53)
    c = np.array([0.5, 0.5, 0.5])
    d = rng.standard_normal((3, 1500))
    d *= 1e-4 * rng.random(1500) / np.linalg.norm(d, axis=0)
    xyz = np.ascontiguousarray(np.concatenate([xyz0, c[:, None] + d], axis=1))
    typ = np.concatenate([typ0, np.zeros(1500, dtype=np.int8)])
    p = _problem()
    p.set_nodes(xyz, typ)
    reported = []
    for _ in range(2):
        with pytest.raises(RbfError) as ei:
            p.build_stencils(20)
        assert ei.value.status == _abi.RBF_EOVERFLOW
        msg = str(ei.value)
        reported.append(int(msg.split("at node ")[1].split()[0]))
    assert reported[0] == reported[1]
    q = reported[0]
    assert np.linalg.norm(xyz[:, q] - c) < 0.35  # a query whose search block reaches the cluster
    xg, tg = ri.jittered_grid(3, 12, 0.3, 53)
    p.set_nodes(xg, tg)
    p.build_stencils(20)
    assert np.array_equal(p.get_stencils(), oracle.knn(xg, 20))
    p.close()


def test_mixed_mode_stops_at_max_steps():
    """max_steps = 700 with 500 inner steps: one full pass and one of 200
    steps, matching the oracle's two passes of 500 and 200."""
    from paper_2502_12878_amd import RBF_MODE_MIXED
    print("mixed mode step cap: 3D side 12, m=4, n=70", flush=True)
    xyz, typ = ri.jittered_grid(3, 12, 0.3, 54)
    idx, w = oracle.setup(xyz, typ, 70, m=4)
    u_ex, f, g, u0 = ri.manufactured(3, xyz, typ)
    h = ri.grid_spacing(12)
    dt = 0.15 * h * h / 6
    op = oracle.Operator(typ, idx, w)
    p = _problem()
    p.set_nodes(xyz, typ)
    p.set_stencils(idx)
    p.set_weights(w, keep_fp32=True)
    u = _dev(u0)
    st, rep = p.iterate(_dev(f), u, dt, 700, 0.0, 1, mode=RBF_MODE_MIXED, inner_steps=500)
    assert st == 0 and rep["steps"] == 700 and rep["checks"] == 2
    u1, passes1, _ = op.mixed(f, dt, u0, 500, 1)
    u2, passes2, _ = op.mixed(f, dt, u1, 200, 1)
    assert passes1 == passes2 == 1
    corr = np.abs(u2 - u0).max()
    assert np.abs(u.cpu().numpy() - u2).max() <= 1e-5 * corr
    # fewer steps than one pass
    u = _dev(u0)
    st, rep = p.iterate(_dev(f), u, dt, 120, 0.0, 1, mode=RBF_MODE_MIXED, inner_steps=500)
    assert st == 0 and rep["steps"] == 120
    u3, _, _ = op.mixed(f, dt, u0, 120, 1)
    assert np.abs(u.cpu().numpy() - u3).max() <= 1e-5 * np.abs(u3 - u0).max()
    p.close()
