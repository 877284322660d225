"""Convergence under refinement: the discrete solution of the manufactured
problem (Sec. II-C) approaches u = prod sin(pi x_i) at roughly order m, the
augmentation order (Sec. II: the order is set by m).  Accept a fitted slope of
at least m - 1.3 over three spacings."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
import rbf_inputs as ri
from fixtures import csr_interior


def _discrete_error(dim, side, m, seed=31):
    n = 2 * ri.num_monomials(dim, m)
    xyz, typ = ri.jittered_grid(dim, side, 0.3, seed)
    idx, w = oracle.setup(xyz, typ, n, m=m)
    u_ex, f, g, u0 = ri.manufactured(dim, xyz, typ)
    LII, LIB, I, B = csr_interior(typ, idx, w)
    uI = sla.spsolve(LII.tocsc(), f[I] - LIB @ g[B])
    err = np.abs(uI - u_ex[I])
    return err.max(), err.sum() / len(typ)


@pytest.mark.parametrize("dim,sides,m", [(2, (21, 41, 81), 2), (2, (21, 41, 81), 4), (2, (21, 41, 81), 6),
                                         (3, (9, 13, 17), 2), (3, (9, 13, 17), 4)])
def test_error_slope_at_least_order_minus_margin(dim, sides, m):
    errs = [_discrete_error(dim, s, m) for s in sides]
    hs = np.log([1.0 / (s - 1) for s in sides])
    slope_inf = np.polyfit(hs, np.log([e[0] for e in errs]), 1)[0]
    slope_mean = np.polyfit(hs, np.log([e[1] for e in errs]), 1)[0]
    assert slope_inf >= m - 1.3, (errs, slope_inf)
    assert slope_mean >= m - 1.3, (errs, slope_mean)
    # higher order is more accurate at the same spacing
    assert errs[-1][0] < 0.05
