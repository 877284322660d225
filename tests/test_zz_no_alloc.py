"""The no-allocation residual (rbf_residual_noalloc, for callers that cannot
allocate device memory) against rbf_residual, through the C ABI: the same
kernels on the same operator give the same value bit for bit, on two calls
in a row (the second on a smaller node set, so the shared static workspace
holds the first call's data), and node sets beyond the workspace are
rejected with an error naming the limit."""
import numpy as np
import pytest

import oracle
import rbf_inputs as ri

pytestmark = pytest.mark.gpu


def _case(dim, side, m, n, seed):
    import torch

    from paper_2502_12878_amd import Problem
    xyz, typ = ri.jittered_grid(dim, side, 0.3, seed)
    p = Problem(0)
    p.set_nodes(xyz, typ)
    p.build_stencils(n)
    p.compute_weights(m)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(len(typ))
    f = rng.standard_normal(len(typ))
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return p, typ, dev(u), dev(f), u, f


def test_residual_noalloc_matches_residual():
    import torch
    for dim, side, m, n, seed in ((3, 20, 4, 70, 61), (2, 40, 2, 12, 62)):
        print(f"no-alloc residual: dim={dim} side={side} m={m} n={n}", flush=True)
        p, typ, ud, fd, u, f = _case(dim, side, m, n, seed)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        p.residual_noalloc(fd, ud, out)
        torch.cuda.synchronize()
        got = out.item()
        ref = p.residual(fd, ud)  # the allocating entry point
        assert got == ref
        op = oracle.Operator(typ, p.get_stencils(), p.get_weights())
        r_o = op.residual(f, u)
        assert abs(got - r_o) <= 1e-12 * abs(r_o)
        # repeated call: the slot is cleared, not accumulated
        p.residual_noalloc(fd, 0.5 * ud, out)
        torch.cuda.synchronize()
        assert out.item() == p.residual(fd, 0.5 * ud)
        p.close()


def test_residual_noalloc_rejects_node_sets_beyond_its_workspace():
    import torch

    from paper_2502_12878_amd import RBF_EINVAL, RbfError
    print("no-alloc residual: 3D side 129 (2,146,689 nodes > 2^21)", flush=True)
    p, typ, ud, fd, _, _ = _case(3, 129, 2, 20, 63)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(RbfError) as ei:
        p.residual_noalloc(fd, ud, out)
    assert ei.value.status == RBF_EINVAL and "2097152" in str(ei.value)
    assert out.item() == 0.0
    p.close()
