"""Pins of the oracle's FP32-inner / FP64-outer refinement loop and of its
adjoint (transpose) sweep."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
import rbf_inputs as ri
from fixtures import csr_interior, small_problem


@pytest.fixture(scope="module")
def p3():
    return small_problem(3, 10, 4, 70, seed=21, alpha=0.15)


def test_one_pass_equals_plain_iteration(p3):
    """u + e after one outer pass of K inner steps equals K plain FP64 steps
    from u (exact arithmetic); the difference is FP32 rounding of the
    correction."""
    op, f, dt, u0 = p3["op"], p3["f"], p3["dt"], p3["u0"]
    K = 300
    um, passes, _ = op.mixed(f, dt, u0, K, 1)
    assert passes == 1
    u64, rep, st = op.iterate(f, dt, u0, K, 0.0, K)
    corr = np.abs(u64 - u0).max()
    assert np.abs(um - u64).max() <= 2e-5 * corr
    B = p3["typ"] == 1
    assert np.array_equal(um[B], u0[B])


def test_refinement_converges_to_fp64_fixed_point(p3):
    """Because the outer residual uses the FP64 weights, the refined iterate
    converges to the FP64 discrete solution, far below FP32 resolution."""
    op, f, dt, u0, typ = p3["op"], p3["f"], p3["dt"], p3["u0"], p3["typ"]
    LII, LIB, I, B = csr_interior(typ, p3["idx"], p3["w"])
    uI = sla.spsolve(LII.tocsc(), f[I] - LIB @ p3["g"][B])
    uref = u0.copy()
    uref[I] = uI
    u, passes, errs = op.mixed(f, dt, u0, 500, 400, u_ref=uref, err_target=1e-12)
    assert errs[-1] <= 1e-12 and passes < 400
    # the error decreases pass over pass until the target
    assert (np.diff(np.log(errs[:5])) < 0).all()


def _adjoint_problem():
    xyz, typ = ri.jittered_grid(2, 13, 0.3, 4)
    idx, w = oracle.setup(xyz, typ, 12, m=2)
    h = ri.grid_spacing(13)
    dt = 0.15 * h * h / 4
    return xyz, typ, idx, w, dt, oracle.Operator(typ, idx, w)


def test_transpose_dot_product():
    """<L_II v, y> = <v, L_II^T y> for interior-supported v, y."""
    xyz, typ, idx, w, dt, op = _adjoint_problem()
    rng = np.random.default_rng(0)
    v = rng.standard_normal(len(typ)) * (typ == 0)
    y = rng.standard_normal(len(typ)) * (typ == 0)
    lhs = np.dot(op.apply(v), y)
    rhs = np.dot(v, op.apply_transpose(y))
    assert abs(lhs - rhs) <= 1e-13 * np.abs(op.apply(v)).sum() * np.abs(y).max()
    # nothing flows into Dirichlet columns
    assert (op.apply_transpose(y)[typ == 1] == 0).all()


def test_adjoint_matches_dense_powers():
    xyz, typ, idx, w, dt, op = _adjoint_problem()
    LII, _, I, B = csr_interior(typ, idx, w)
    G = np.eye(len(I)) + dt * LII.toarray()
    rng = np.random.default_rng(1)
    gK = rng.standard_normal(len(typ))
    K = 60
    lam = gK[I].copy()
    acc = lam.copy()
    for _ in range(K - 1):
        lam = G.T @ lam
        acc += lam
    ref = -dt * acc
    got = op.adjoint_f(dt, K, gK)
    assert np.abs(got[I] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert (got[B] == 0).all()


def test_adjoint_matches_central_differences():
    """J(f) = 1/2 |u_K(f) - u_tgt|^2 over interior nodes is quadratic in f, so
    central differences are exact up to rounding."""
    xyz, typ, idx, w, dt, op = _adjoint_problem()
    K = 200
    u_ex, f0, g, u0 = ri.manufactured(2, xyz, typ)
    f = np.where(typ == 0, ri.gaussian_field(2, xyz, 104), 0.0)
    f_t = f + 0.1 * np.where(typ == 0, ri.gaussian_field(2, xyz, 204), 0.0)
    zero = np.zeros_like(f)

    def run(ff):
        u, _, st = op.iterate(ff, dt, zero, K, 0.0, K)
        assert st == 0
        return u

    u_tgt = run(f_t)
    I = typ == 0

    def J(ff):
        d = (run(ff) - u_tgt)[I]
        return 0.5 * np.dot(d, d)

    gK = np.where(I, run(f) - u_tgt, 0.0)
    grad = op.adjoint_f(dt, K, gK)
    eps = 1e-2 * np.abs(f).max()
    for j in range(6):
        v = np.where(I, ri.gaussian_field(2, xyz, 304 + j), 0.0)
        v /= np.abs(v).max()
        fd = (J(f + eps * v) - J(f - eps * v)) / (2 * eps)
        assert abs(np.dot(grad, v) - fd) <= 1e-6 * abs(fd)


def test_transposed_rows_outgrow_the_support_size():
    """A row of L_II^T lists the interior rows whose supports hold a given
    interior node, so its length is that node's in-degree.  In-degrees are not
    bounded by n: in a 16^3 cube at n = 256 some exceed 300 (nodes near the
    centre sit in the supports of boundary-near rows, which reach inwards).
    The oracle's transposed product agrees with the dense transpose there."""
    xyz, typ = ri.jittered_grid(3, 16, 0.3, 41)
    idx = oracle.knn(xyz, 256)
    I = typ == 0
    cols = idx[I].reshape(-1)
    cols = cols[I[cols]]
    deg = np.bincount(cols, minlength=len(typ))[I]
    assert deg.max() > 256 and deg.sum() == cols.size
    # transposed product with arbitrary weights against the dense matrix
    rng = np.random.default_rng(3)
    w = np.where(I[:, None], rng.standard_normal(idx.shape), 0.0)
    op = oracle.Operator(typ, idx, w)
    L = np.zeros((len(typ), len(typ)))
    rows = np.repeat(np.arange(len(typ)), idx.shape[1])
    np.add.at(L, (rows, idx.reshape(-1)), w.reshape(-1))
    Lii = L[np.ix_(I, I)]
    v = rng.standard_normal(len(typ))
    t = op.apply_transpose(v)
    assert np.abs(t[I] - Lii.T @ v[I]).max() <= 1e-12 * np.abs(Lii.T @ v[I]).max()
    assert (t[~I] == 0).all()
