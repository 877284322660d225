"""CPU oracle for the RBF-FD Poisson sweep (arXiv 2502.12878).

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The HIP library never does, and this
package never imports the HIP library.

The arithmetic lives in ``rbf_oracle.c`` (plain C, fp64, no FMA contraction);
this module marshals numpy arrays into it.  Layouts are the natural ones:
coordinates ``xyz`` float64 [dim, N]; stencils int32 [rows, n] row-major in
ascending (d^2, id) order; weights float64 [rows, n].
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


class _IterReport(C.Structure):
    _fields_ = [("steps", C.c_int64), ("res0", C.c_double), ("res_last", C.c_double),
                ("res_final", C.c_double), ("fnorm", C.c_double), ("diverged_step", C.c_int64),
                ("converged", C.c_int), ("diverged", C.c_int)]


def lib():
    """Load the oracle library, building it only if it is missing.  The
    environment variable RBF_ORACLE_LIB names another build of the same source
    to load instead (the sanitizer build of ``oracle.sanitize``)."""
    global _lib
    if _lib is None:
        path = os.environ.get("RBF_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.orc_monomials.argtypes = [C.c_int, C.c_int, C.c_void_p]
        L.orc_monomials.restype = C.c_int
        L.orc_knn.argtypes = [C.c_int, C.c_int64, _f64p, C.c_int, _i64p, C.c_int64, _i32p]
        L.orc_knn.restype = C.c_int
        L.orc_knn_typed.argtypes = [C.c_int, C.c_int64, _f64p, C.c_int, _i64p, C.c_int64, C.c_void_p, _i32p]
        L.orc_knn_typed.restype = C.c_int
        L.orc_weights.argtypes = [C.c_int, C.c_int64, _f64p, _i64p, C.c_int64, _i32p, C.c_int,
                                  C.c_void_p, C.c_int, C.c_void_p, _f64p, _f64p,
                                  C.POINTER(C.c_int64)]
        L.orc_weights.restype = C.c_int
        L.orc_weights_op.argtypes = [C.c_int, C.c_int64, _f64p, _i64p, C.c_int64, _i32p, C.c_int,
                                     C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, _f64p, _f64p,
                                     C.POINTER(C.c_int64)]
        L.orc_weights_op.restype = C.c_int
        L.orc_neumann_update.argtypes = [C.c_int64, _i8p, _i32p, _f64p, C.c_int, C.c_void_p, _f64p, _f64p]
        L.orc_neumann_update.restype = None
        L.orc_assemble.argtypes = [C.c_int, C.c_int64, _f64p, C.c_int64, _i32p, C.c_int, C.c_int,
                                   _f64p, C.POINTER(C.c_double)]
        L.orc_assemble.restype = C.c_int
        common = [C.c_int64, _i8p, _i32p, _f64p, C.c_int, C.c_void_p]
        L.orc_apply.argtypes = common + [_f64p, _f64p]
        L.orc_apply.restype = None
        L.orc_sweep.argtypes = common + [_f64p, C.c_double, _f64p, _f64p]
        L.orc_sweep.restype = C.c_double
        L.orc_sweep_omp.argtypes = common + [_f64p, C.c_double, _f64p, _f64p, C.c_int]
        L.orc_sweep_omp.restype = C.c_double
        L.orc_residual.argtypes = common + [_f64p, _f64p]
        L.orc_residual.restype = C.c_double
        L.orc_iterate.argtypes = common + [_f64p, C.c_double, _f64p, _f64p, C.c_int64,
                                           C.c_double, C.c_int64, C.c_int64,
                                           C.POINTER(_IterReport)]
        L.orc_iterate.restype = C.c_int
        L.orc_mixed.argtypes = [C.c_int64, _i8p, _i32p, _f64p, _f32p, C.c_int, C.c_void_p,
                                _f64p, C.c_double, _f64p, C.c_int64, C.c_int64, C.c_void_p,
                                C.c_double, C.c_void_p, _f64p, _f32p, _f32p, _f32p]
        L.orc_mixed.restype = C.c_int64
        L.orc_apply_transpose.argtypes = common + [_f64p, _f64p]
        L.orc_apply_transpose.restype = None
        L.orc_adjoint_f.argtypes = common + [C.c_double, C.c_int64, _f64p, _f64p, _f64p, _f64p]
        L.orc_adjoint_f.restype = None
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr_or_none(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def monomials(dim: int, m: int) -> np.ndarray:
    """Exponents [M, 3] of the monomials of degree <= m in the oracle's order."""
    M = lib().orc_monomials(dim, m, None)
    out = np.zeros((M, 3), dtype=np.int32)
    lib().orc_monomials(dim, m, out.ctypes.data_as(C.c_void_p))
    return out


def knn(xyz: np.ndarray, n: int, rows=None, typ=None) -> np.ndarray:
    """Brute-force supports: for each centre, the n smallest (d^2, id); with
    ``typ``, Neumann centres (type 2) take only themselves and interior nodes."""
    xyz = _c(xyz, np.float64)
    dim, N = xyz.shape
    rows = np.arange(N, dtype=np.int64) if rows is None else _c(rows, np.int64)
    out = np.zeros((len(rows), n), dtype=np.int32)
    typ_a = None if typ is None else _c(typ, np.int8)
    st = lib().orc_knn_typed(dim, N, xyz.reshape(-1), n, rows, len(rows), _ptr_or_none(typ_a), out.reshape(-1))
    if st != 0:
        raise ValueError(f"orc_knn status {st}")
    return out


def assemble(xyz: np.ndarray, centre: int, stencil: np.ndarray, m: int):
    """The augmented system [A P | LPhi; P^T 0 | Lp] of one centre, as the
    oracle builds it: returns (matrix [S, S], rhs [S], scale s)."""
    xyz = _c(xyz, np.float64)
    dim, N = xyz.shape
    st_ = _c(stencil, np.int32)
    n = len(st_)
    S = n + len(monomials(dim, m))
    a = np.zeros((S, S + 1))
    s = C.c_double(0.0)
    st = lib().orc_assemble(dim, N, xyz.reshape(-1), int(centre), st_, n, m, a.reshape(-1), C.byref(s))
    if st != 0:
        raise ValueError(f"orc_assemble status {st}")
    return a[:, :S].copy(), a[:, S].copy(), s.value


class SingularSystem(RuntimeError):
    def __init__(self, row):
        super().__init__(f"singular local system at node {row}")
        self.row = row


def weights(xyz: np.ndarray, stencils: np.ndarray, rows, m=None, m_row=None, n_row=None,
            raise_on_singular: bool = True, op_row=None, normals=None):
    """RBF-FD weights for centres ``rows`` with supports ``stencils``: the
    Laplacian, or (op_row[q] = 1) the derivative along ``normals[:, rows[q]]``.

    Returns (w [rows, n], pivot_ratio [rows], status, bad_row).
    """
    xyz = _c(xyz, np.float64)
    dim, N = xyz.shape
    rows = _c(rows, np.int64)
    st_ = _c(stencils, np.int32)
    nr, ns = st_.shape
    assert nr == len(rows)
    nrow_a = None if n_row is None else _c(n_row, np.int32)
    mrow_a = None if m_row is None else _c(m_row, np.int8)
    op_a = None if op_row is None else _c(op_row, np.int8)
    nv_a = None if normals is None else _c(normals, np.float64)
    w = np.zeros((nr, ns), dtype=np.float64)
    pr = np.zeros(nr, dtype=np.float64)
    bad = C.c_int64(-1)
    st = lib().orc_weights_op(dim, N, xyz.reshape(-1), rows, nr, st_.reshape(-1), ns,
                              _ptr_or_none(nrow_a), int(m if m is not None else 0),
                              _ptr_or_none(mrow_a), _ptr_or_none(op_a), _ptr_or_none(nv_a),
                              w.reshape(-1), pr, C.byref(bad))
    if st == 3 and raise_on_singular:
        raise SingularSystem(bad.value)
    if st not in (0, 3):
        raise ValueError(f"orc_weights status {st}")
    return w, pr, st, bad.value


class Operator:
    """L_h on a node set: stencils [N, n] and weights [N, n] (rows for
    Dirichlet nodes are present but unused), node types [N]."""

    def __init__(self, typ, idx, w, n_row=None):
        self.typ = _c(typ, np.int8)
        self.idx = _c(idx, np.int32)
        self.w = _c(w, np.float64)
        self.N, self.ns = self.idx.shape
        self.n_row = None if n_row is None else _c(n_row, np.int32)

    def _common(self, w=None):
        return (self.N, self.typ, self.idx.reshape(-1),
                (self.w if w is None else w).reshape(-1), self.ns, _ptr_or_none(self.n_row))

    def apply(self, u):
        u = _c(u, np.float64)
        out = np.zeros(self.N)
        lib().orc_apply(*self._common(), u, out)
        return out

    def apply_transpose(self, v):
        v = _c(v, np.float64)
        out = np.zeros(self.N)
        lib().orc_apply_transpose(*self._common(), v, out)
        return out

    def sweep(self, f, dt, u_old):
        u_new = np.empty(self.N)
        u_in = np.array(u_old, dtype=np.float64)  # the Neumann update writes into the old state
        res = lib().orc_sweep(*self._common(), _c(f, np.float64), float(dt), u_in, u_new)
        return u_new, res

    def sweep_omp(self, f, dt, u_old, u_new, nthreads):
        return lib().orc_sweep_omp(*self._common(), f, float(dt), u_old, u_new, int(nthreads))

    def residual(self, f, u):
        return lib().orc_residual(*self._common(), _c(f, np.float64), _c(u, np.float64))

    def iterate(self, f, dt, u0, max_steps, tol_rel=0.0, chunk=100, stall=0):
        u = _c(u0, np.float64).copy()
        work = np.empty(self.N)
        rep = _IterReport()
        st = lib().orc_iterate(*self._common(), _c(f, np.float64), float(dt), u, work,
                               int(max_steps), float(tol_rel), int(chunk), int(stall), C.byref(rep))
        report = {k: getattr(rep, k) for k, _ in _IterReport._fields_}
        return u, report, st

    def mixed(self, f, dt, u0, inner, max_outer, u_ref=None, err_target=0.0):
        u = _c(u0, np.float64).copy()
        w32 = self.w.astype(np.float32)
        errs = np.zeros(max(1, max_outer))
        N = self.N
        r = np.empty(N)
        e, e2, r32 = (np.empty(N, dtype=np.float32) for _ in range(3))
        uref = None if u_ref is None else _c(u_ref, np.float64)
        passes = lib().orc_mixed(N, self.typ, self.idx.reshape(-1), self.w.reshape(-1),
                                 w32.reshape(-1), self.ns, _ptr_or_none(self.n_row),
                                 _c(f, np.float64), float(dt), u, int(inner), int(max_outer),
                                 _ptr_or_none(uref), float(err_target),
                                 errs.ctypes.data_as(C.c_void_p), r, e, e2, r32)
        return u, int(passes), errs[:passes]

    def adjoint_f(self, dt, K, gK):
        grad = np.empty(self.N)
        lam = np.empty(self.N)
        tmp = np.empty(self.N)
        lib().orc_adjoint_f(*self._common(), float(dt), int(K), _c(gK, np.float64), grad, lam, tmp)
        return grad


def setup(xyz, typ, n, m=None, n_row=None, m_row=None, normals=None):
    """Supports for every node; Laplacian weights for every interior node and,
    with ``normals``, normal-derivative weights for every Neumann node (type 2).

    Returns (idx [N, n_max], w [N, n_max]); Dirichlet rows of w are zero.
    With per-node sizes, row r of idx holds its n_row[r] nearest nodes and is
    padded with its own id.
    """
    xyz = _c(xyz, np.float64)
    N = xyz.shape[1]
    typ = _c(typ, np.int8)
    ktyp = typ if normals is not None else None
    if n_row is None:
        idx = knn(xyz, n, typ=ktyp)
        n_max = n
    else:
        n_row = _c(n_row, np.int32)
        n_max = int(n_row.max())
        idx = np.repeat(np.arange(N, dtype=np.int32)[:, None], n_max, axis=1)
        for nn in np.unique(n_row):
            sel = np.nonzero(n_row == nn)[0]
            idx[sel, :nn] = knn(xyz, int(nn), sel, typ=ktyp)
    w = np.zeros((N, n_max))
    for code, op in ((0, 0), (2, 1)):
        rows = np.nonzero(typ == code)[0].astype(np.int64)
        if len(rows) == 0:
            continue
        wi, _, _, _ = weights(xyz, idx[rows], rows, m=m,
                              m_row=None if m_row is None else np.asarray(m_row)[rows],
                              n_row=None if n_row is None else n_row[rows],
                              op_row=np.full(len(rows), op, dtype=np.int8) if op else None,
                              normals=normals if op else None)
        w[rows] = wi
    return idx, w
