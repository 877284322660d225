"""GPU parity of the null-space weight solver (systems larger than one
wavefront's, m >= 1): the weights of the augmented system (Sec. II) against
the oracle's Gaussian elimination, per row within 1e-10 relative (the bar;
the two solve the same nonsingular system in different operation orders),
the normal-derivative rows of the mixed boundary variant, the elimination
path (RBF_WEIGHTS_SOLVER=gepp) still bit-equal to the oracle, and repeated
runs bit-equal to each other."""
import numpy as np
import pytest

import oracle
import rbf_inputs as ri

pytestmark = pytest.mark.gpu


def _rel_rows(a, b):
    scale = np.abs(b).max(axis=1) + 1e-300
    return (np.abs(a - b).max(axis=1) / scale).max()


def _weights(xyz, typ, n, m, normals=None):
    from paper_2502_12878_amd import Problem
    p = Problem(0)
    p.set_nodes(xyz, typ)
    if normals is not None:
        p.set_normals(normals)
    p.build_stencils(n)
    p.compute_weights(m)
    out = p.get_stencils(), p.get_weights(), p.operator_info()
    p.close()
    return out


# K = n - M: 35, 84, 28, 30, 15 (one 16-column block), and 16, 32, 80 (a
# multiple of 16: the reduced right-hand side row K alone in the last block,
# which has no pivot column); the last three reach the compiled sizes
# (3D, 56, 64), (2D, 64, 64) and (2D, 24, 24)
@pytest.mark.parametrize("dim,side,m,n,seed", [(3, 12, 4, 70, 71), (3, 11, 6, 168, 72), (2, 24, 6, 56, 73),
                                               (3, 10, 3, 50, 74), (2, 30, 4, 30, 75), (3, 9, 4, 51, 78),
                                               (3, 9, 4, 67, 79), (3, 11, 6, 164, 80), (3, 10, 5, 112, 81),
                                               (2, 30, 6, 80, 82), (2, 24, 5, 40, 83)])
def test_ns_weights_match_oracle(dim, side, m, n, seed):
    print(f"null-space weights: dim={dim} side={side} m={m} n={n}", flush=True)
    xyz, typ = ri.jittered_grid(dim, side, 0.3, seed)
    idx, w, info = _weights(xyz, typ, n, m)
    assert np.array_equal(idx, oracle.knn(xyz, n))
    I = np.nonzero(typ == 0)[0]
    assert info["ns_systems"] == len(I) and info["elim_systems"] == 0
    wo, _, _, _ = oracle.weights(xyz, idx[I], I, m=m)
    rel = _rel_rows(w[I], wo)
    print(f"  max row-relative difference to the oracle {rel:.2e}")
    assert rel <= 1e-10


def test_ns_normal_derivative_rows():
    """Mixed Dirichlet/Neumann cube (m = 4): interior Laplacian rows and
    Neumann normal-derivative rows both on the null-space solver."""
    xyz, typ, normals = ri.mixed_bc_grid(3, 12, 0.3, 76)
    idx, w, info = _weights(xyz, typ, 70, 4, normals)
    rows = np.nonzero(typ != 1)[0]
    assert info["ns_systems"] == len(rows)
    idx_o, w_o = oracle.setup(xyz, typ, 70, m=4, normals=normals)
    assert np.array_equal(idx, idx_o)
    assert _rel_rows(w[rows], w_o[rows]) <= 1e-10


def test_elimination_path_still_bit_equal_and_ns_repeatable(monkeypatch):
    xyz, typ = ri.jittered_grid(3, 10, 0.3, 77)
    I = np.nonzero(typ == 0)[0]
    _, w1, _ = _weights(xyz, typ, 70, 4)
    _, w2, _ = _weights(xyz, typ, 70, 4)
    assert np.array_equal(w1, w2)
    monkeypatch.setenv("RBF_WEIGHTS_SOLVER", "gepp")
    idx, we, info = _weights(xyz, typ, 70, 4)
    monkeypatch.delenv("RBF_WEIGHTS_SOLVER")
    assert info["ns_systems"] == 0 and info["elim_systems"] == len(I)
    wo, _, _, _ = oracle.weights(xyz, idx[I], I, m=4)
    assert np.array_equal(we[I], wo)
    assert _rel_rows(w1[I], wo) <= 1e-10
