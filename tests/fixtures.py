"""Helpers shared by the tests: golden-file parsing and small problem builders.

Builders here call only ``rbf_inputs`` and ``oracle`` (never the HIP library),
so expected values never come from the code under test.
"""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_closed_form_stencils():
    """Blocks of tests/golden/closed_form_stencils.txt as dicts."""
    out, cur = [], None
    with open(os.path.join(GOLDEN, "closed_form_stencils.txt")) as fh:
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
            elif key == "nodes":
                cur["nodes"] = np.array([[int(t) for t in p.split()] for p in rest.split("|")],
                                        dtype=np.float64)
            elif key == "weights":
                cur["weights"] = np.array([float(Fraction(t)) for t in rest.split()])
    return out


def read_support_sizes():
    rows = []
    with open(os.path.join(GOLDEN, "support_sizes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                d, m, n, rule = line.split()
                rows.append((int(d), int(m), int(n), rule))
    return rows


def small_problem(dim, side, m, n, seed=7, jitter=0.3, alpha=0.3):
    """Jittered-grid Poisson problem with oracle stencils and weights."""
    import oracle
    import rbf_inputs as ri
    xyz, typ = ri.jittered_grid(dim, side, jitter, seed)
    idx, w = oracle.setup(xyz, typ, n, m=m)
    u_ex, f, g, u0 = ri.manufactured(dim, xyz, typ)
    h = ri.grid_spacing(side)
    dt = alpha * h * h / (2 * dim)
    return dict(xyz=xyz, typ=typ, idx=idx, w=w, u_ex=u_ex, f=f, g=g, u0=u0, h=h, dt=dt,
                op=oracle.Operator(typ, idx, w))


def csr_interior(typ, idx, w):
    """scipy CSR matrices L_II and L_IB from row-major stencils/weights."""
    import scipy.sparse as sp
    N, n = idx.shape
    rows = np.repeat(np.arange(N), n)
    L = sp.csr_matrix((w.reshape(-1), (rows, idx.reshape(-1))), shape=(N, N))
    I = np.nonzero(typ == 0)[0]
    B = np.nonzero(typ != 0)[0]
    return L[I][:, I].tocsr(), L[I][:, B].tocsr(), I, B
