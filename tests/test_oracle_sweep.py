"""Pins of the oracle's explicit iteration (Sec. II-C, the Jacobi step and its
stability bound), its stopping rules, and its fixed point."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
import rbf_inputs as ri
from fixtures import csr_interior, small_problem


@pytest.fixture(scope="module")
def p2():
    return small_problem(2, 21, 2, 12, seed=3, alpha=0.15)


@pytest.fixture(scope="module")
def p3():
    return small_problem(3, 9, 4, 70, seed=4, alpha=0.15)


@pytest.mark.parametrize("which", ["p2", "p3"])
def test_sweep_matches_scipy_csr(which, request):
    """1000 oracle steps against the same recurrence in scipy CSR form."""
    p = request.getfixturevalue(which)
    LII, LIB, I, B = csr_interior(p["typ"], p["idx"], p["w"])
    u = p["u0"].copy()
    for _ in range(1000):
        u, _ = p["op"].sweep(p["f"], p["dt"], u)
    v = p["u0"].copy()
    for _ in range(1000):
        Lu = LII @ v[I] + LIB @ v[B]
        v[I] = v[I] + p["dt"] * (Lu - p["f"][I])
    assert np.abs(u - v).max() <= 1e-13 * np.abs(v).max()
    assert np.array_equal(u[B], p["g"][B])


def test_residual_is_sweep_residual(p2):
    op = p2["op"]
    u = p2["u0"] + 0.01 * np.sin(np.arange(len(p2["u0"])))
    u[p2["typ"] == 1] = p2["g"][p2["typ"] == 1]
    r1 = op.residual(p2["f"], u)
    _, r2 = op.sweep(p2["f"], p2["dt"], u)
    Lu = op.apply(u)
    r3 = np.abs(Lu - p2["f"])[p2["typ"] == 0].max()
    assert r1 == r2 == r3


@pytest.mark.parametrize("dim,m,side", [(2, 2, 15), (2, 4, 17), (3, 2, 8), (3, 4, 9)])
def test_polynomial_is_discrete_fixed_point(dim, m, side):
    """A polynomial of degree <= m is reproduced exactly by every stencil, so
    with f = its Laplacian and g = its boundary values it is a fixed point."""
    xyz, typ = ri.jittered_grid(dim, side, 0.3, 8)
    n = 2 * ri.num_monomials(dim, m)
    idx, w = oracle.setup(xyz, typ, n, m=m)
    op = oracle.Operator(typ, idx, w)
    x = xyz
    if m == 2:
        up = 1 + x[0] + 2 * x[1] - x[0] * x[1] + 3 * x[dim - 1] ** 2
        lap = np.full(x.shape[1], 6.0)
    else:
        up = x[0] ** 4 - 2 * x[0] ** 2 * x[1] ** 2 + x[1] ** 3 + x[dim - 1]
        lap = 12 * x[0] ** 2 - 4 * x[1] ** 2 - 4 * x[0] ** 2 + 6 * x[1]
    f = np.where(typ == 0, lap, 0.0)
    scale = np.abs(w).sum(1).max() * np.abs(up).max()
    assert op.residual(f, up) <= 1e-13 * scale
    h = ri.grid_spacing(side)
    u, rep, st = op.iterate(f, 0.15 * h * h / (2 * dim), up, 500, 0.0, 100)
    assert st == 0
    assert np.abs(u - up).max() <= 1e-12 * max(1.0, np.abs(up).max())


@pytest.mark.parametrize("dim,side,m", [(2, 21, 2), (2, 17, 4), (3, 9, 2)])
def test_fixed_point_is_sparse_solve(dim, side, m):
    """Iterating to a tight residual reaches the solution of
    L_II u_I = f_I - L_IB g (scipy spsolve)."""
    n = 2 * ri.num_monomials(dim, m)
    p = small_problem(dim, side, m, n, seed=12, alpha=0.15)
    LII, LIB, I, B = csr_interior(p["typ"], p["idx"], p["w"])
    uI = sla.spsolve(LII.tocsc(), p["f"][I] - LIB @ p["g"][B])
    u, rep, st = p["op"].iterate(p["f"], p["dt"], p["u0"], 400000, 1e-13, 500)
    assert st == 0 and rep["converged"] == 1
    assert rep["res_final"] <= 2e-13 * rep["fnorm"]
    assert np.abs(u[I] - uI).max() <= 1e-11 * np.abs(uI).max()


def test_decay_rate_of_lowest_mode():
    """The initial error -u_exact is (close to) the lowest continuum mode, so
    the residual ratio per step tends to 1 - dt*lambda_1, lambda_1 ~ d pi^2."""
    p = small_problem(2, 31, 2, 12, seed=5, alpha=0.15)
    op = p["op"]
    u = p["u0"].copy()
    res = []
    for k in range(3000):
        u, r = op.sweep(p["f"], p["dt"], u)
        res.append(r)
    # the error is the discrete lowest mode after transients; compare its decay
    # with the continuum prediction
    u_long = u.copy()
    K = 1000
    e0 = np.abs(op.apply(u_long) - p["f"])[p["typ"] == 0].max()
    for _ in range(K):
        u_long, _ = op.sweep(p["f"], p["dt"], u_long)
    e1 = np.abs(op.apply(u_long) - p["f"])[p["typ"] == 0].max()
    rate = (e1 / e0) ** (1.0 / K)
    lam1 = 2 * math.pi ** 2
    assert abs((1 - rate) / p["dt"] - lam1) <= 0.02 * lam1


def test_stability_bound_spectrum():
    """The step is stable iff every eigenvalue of L_II satisfies
    |1 + dt*lambda| < 1 (dt = alpha h^2/(2d)); the oracle diverges exactly when
    the spectrum says so."""
    p = small_problem(2, 25, 2, 12, seed=6, alpha=0.15)
    LII, _, I, _ = csr_interior(p["typ"], p["idx"], p["w"])
    lam = np.linalg.eigvals(LII.toarray())
    assert (lam.real < 0).all()
    h = p["h"]
    dtmax = h * h / 4
    a_star = (-2 * lam.real / (np.abs(lam) ** 2 * dtmax)).min()
    op = p["op"]
    for alpha, stable in ((0.95 * a_star, True), (1.1 * a_star, False)):
        u, rep, st = op.iterate(p["f"], alpha * dtmax, p["u0"], 30000, 0.0, 1000)
        assert (st == 0) == stable, (alpha, a_star, rep)
        if not stable:
            assert st == 4 and rep["diverged"] == 1 and rep["diverged_step"] > 0


def test_iterate_status_codes(p2):
    op, f, u0, dt = p2["op"], p2["f"], p2["u0"], p2["dt"]
    # fixed-step run: tol <= 0 runs exactly max_steps and reports OK
    u, rep, st = op.iterate(f, dt, u0, 1234, 0.0, 100)
    assert st == 0 and rep["steps"] == 1234 and rep["converged"] == 0
    v = u0.copy()
    for _ in range(1234):
        v, _ = op.sweep(f, dt, v)
    assert np.array_equal(u, v)
    # max_steps reached with a tolerance -> not converged
    u, rep, st = op.iterate(f, dt, u0, 300, 1e-12, 100)
    assert st == 5 and rep["steps"] == 300
    # divergence at a large step
    u, rep, st = op.iterate(f, 3.0 * p2["h"] ** 2 / 4, u0, 5000, 0.0, 100)
    assert st == 4 and rep["diverged"] == 1 and rep["diverged_step"] % 100 == 0
    # NaN in f: diverged at step 0
    fn = f.copy()
    fn[np.nonzero(p2["typ"] == 0)[0][3]] = np.nan
    u, rep, st = op.iterate(fn, dt, u0, 100, 1e-8, 10)
    assert st == 4 and rep["diverged_step"] == 0 and rep["steps"] == 0
    # converged: the chunk's last residual is below tol * max|f|
    u, rep, st = op.iterate(f, dt, u0, 200000, 1e-6, 50)
    assert st == 0 and rep["converged"] == 1 and rep["steps"] % 50 == 0
    assert rep["res_last"] <= 1e-6 * rep["fnorm"]
    # the same run continued by hand step by step gives the same iterate
    v = u0.copy()
    for _ in range(rep["steps"]):
        v, r = op.sweep(f, dt, v)
    assert np.array_equal(u, v) and r == rep["res_last"]


def test_stall_detection(p2):
    op, f, u0, dt = p2["op"], p2["f"], p2["u0"], p2["dt"]
    # a tolerance below the rounding floor stalls; with stall = 3 chunks the
    # loop stops well before max_steps
    u, rep, st = op.iterate(f, dt, u0, 10 ** 7, 1e-30, 2000, stall=3)
    assert st == 5 and rep["steps"] < 10 ** 7


def test_nan_propagates_in_residual(p2):
    op = p2["op"]
    u = p2["u0"].copy()
    u[np.nonzero(p2["typ"] == 0)[0][10]] = np.nan
    _, r = op.sweep(p2["f"], p2["dt"], u)
    assert math.isnan(r)


@pytest.mark.parametrize("which", ["p2", "p3"])
@pytest.mark.parametrize("threads", [1, 4])
def test_openmp_sweep_is_the_sequential_sweep(which, threads, request):
    """The timed CPU baseline (row-parallel sweep) computes every row exactly
    as the pinned sequential sweep: bitwise equal iterates and residual."""
    p = request.getfixturevalue(which)
    u = p["u0"] + 0.01 * np.cos(np.arange(len(p["u0"])))
    u[p["typ"] == 1] = p["g"][p["typ"] == 1]
    seq, res_seq = p["op"].sweep(p["f"], p["dt"], u)
    par = np.empty_like(u)
    res_par = p["op"].sweep_omp(p["f"], p["dt"], u, par, threads)
    assert np.array_equal(seq, par) and res_seq == res_par
