"""Seeded synthetic inputs for the RBF-FD Poisson sweep.

This module is the one place both sides (the CPU oracle under ``oracle/`` and
the HIP library under ``paper_2502_12878_amd/``) get their inputs from.  It
holds none of the method's arithmetic: no neighbour search, no weights, no
sweep.  It only produces

* node sets: jittered Cartesian grids on the unit d-cube, standing in for the
  Poisson-disc node sets of the paper (Sec. II-C, last paragraph), each node
  tagged interior or Dirichlet;
* the manufactured test problem of Sec. II-C: u = prod_i sin(pi x_i),
  f = -pi^2 d u, with Dirichlet data g = u on the boundary;
* smooth random source fields (sums of Gaussians) for inverse-source
  (adjoint) runs;
* per-node augmentation orders for mixed-order node sets (low order near the
  boundary, high order inside).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Its k-th output is a pure
function of (seed, k), so a GPU kernel can draw the same values in parallel:
``out_k = mix(seed + (k + 1) * GAMMA)`` (mod 2^64).  The node builder of the
HIP library implements the same published generator on its own; tests check
that both produce bit-identical coordinates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

INTERIOR = 0
DIRICHLET = 1


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number ``counters`` (0-based) of the SplitMix64 stream ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output times 2^-53."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def grid_spacing(side: int) -> float:
    return 1.0 / (side - 1)


def jittered_grid(dim: int, side: int, jitter_frac: float, seed: int):
    """Jittered Cartesian node set on [0, 1]^dim.

    Node id = i + side*j + side^2*k (x index fastest).  Grid pitch
    h = 1/(side-1).  Every node, in id order, draws ``dim`` uniforms U (x, y, z
    order; draw number id*dim + axis).  Only interior nodes use them:
    ``x = i*h + (2U - 1)*(jitter_frac*h)``, evaluated as two products and one
    sum (no fused multiply-add).  A node is Dirichlet iff any of its grid
    indices is 0 or side-1; those stay exactly on the grid.

    Returns ``xyz`` as float64 [dim, N] (structure of arrays) and ``type`` as
    int8 [N] (0 interior, 1 Dirichlet).
    """
    if dim not in (1, 2, 3) or side < 2:
        raise ValueError("dim must be 1..3 and side >= 2")
    N = side ** dim
    h = grid_spacing(side)
    t = jitter_frac * h
    ids = np.arange(N, dtype=np.int64)
    grid_idx = []
    rem = ids.copy()
    for _ in range(dim):
        grid_idx.append(rem % side)
        rem //= side
    boundary = np.zeros(N, dtype=bool)
    for gi in grid_idx:
        boundary |= (gi == 0) | (gi == side - 1)
    xyz = np.empty((dim, N), dtype=np.float64)
    for a in range(dim):
        U = uniform01(seed, ids.astype(np.uint64) * np.uint64(dim) + np.uint64(a))
        v = 2.0 * U - 1.0
        base = grid_idx[a].astype(np.float64) * h
        jit = base + v * t
        xyz[a] = np.where(boundary, base, jit)
    typ = np.where(boundary, DIRICHLET, INTERIOR).astype(np.int8)
    return xyz, typ


def manufactured(dim: int, xyz: np.ndarray, typ: np.ndarray):
    """Test problem of Sec. II-C: Laplacian u = f on the unit cube.

    u_exact = prod_i sin(pi x_i); f = -pi^2 d u_exact on interior nodes (0 on
    Dirichlet nodes, where it is unused); g = u_exact on Dirichlet nodes;
    u0 = 0 inside and g on the boundary.
    """
    u = np.ones(xyz.shape[1], dtype=np.float64)
    for a in range(dim):
        u = u * np.sin(math.pi * xyz[a])
    interior = typ == INTERIOR
    c = dim * math.pi * math.pi
    f = np.where(interior, -c * u, 0.0)
    g = np.where(interior, 0.0, u)
    u0 = g.copy()
    return u, f, g, u0


NEUMANN = 2


def mixed_bc_grid(dim: int, side: int, jitter_frac: float, seed: int):
    """Node set of the mixed-boundary variant (Sec. II-C, second paragraph):
    the sub-cube [0, 1/2]^dim, sampled by the unit-cube jittered grid scaled by
    1/2 (exact in binary floating point).  Nodes with a grid index 0 are
    Dirichlet (faces on the original boundary, u = 0); the remaining nodes with
    a grid index side-1 are Neumann (faces inside the original cube, where the
    normal derivative of u is 0).  Their outward unit normal is the normalised
    sum of the unit normals of the faces they lie on.

    Returns xyz [dim, N], type int8 [N] (0 interior, 1 Dirichlet, 2 Neumann)
    and normals [dim, N] (zero except on Neumann nodes).
    """
    xyz, typ = jittered_grid(dim, side, jitter_frac, seed)
    xyz = xyz * 0.5
    N = side ** dim
    ids = np.arange(N, dtype=np.int64)
    lo = np.zeros(N, dtype=bool)
    hi = np.zeros((dim, N), dtype=bool)
    rem = ids.copy()
    for a in range(dim):
        gi = rem % side
        rem //= side
        lo |= gi == 0
        hi[a] = gi == side - 1
    typ = np.where(lo, DIRICHLET, np.where(hi.any(axis=0), NEUMANN, INTERIOR)).astype(np.int8)
    normals = np.where((typ == NEUMANN)[None, :], hi.astype(np.float64), 0.0)
    cnt = hi.sum(axis=0)
    normals = np.where(cnt[None, :] > 0, normals / np.sqrt(np.maximum(cnt, 1))[None, :], 0.0)
    normals[:, typ != NEUMANN] = 0.0
    return xyz, typ, normals


def manufactured_mixed(dim: int, xyz: np.ndarray, typ: np.ndarray):
    """u = prod sin(pi x_i) on [0, 1/2]^d: Laplacian u = f inside, u = g = 0 on
    the Dirichlet faces, normal derivative 0 on the Neumann faces.  Returns
    (u_exact, f, u0) where f holds -pi^2 d u on interior nodes and the normal
    derivative data (0) on Neumann nodes; u0 is 0 except g on Dirichlet nodes."""
    u = np.ones(xyz.shape[1], dtype=np.float64)
    for a in range(dim):
        u = u * np.sin(math.pi * xyz[a])
    c = dim * math.pi * math.pi
    f = np.where(typ == INTERIOR, -c * u, 0.0)
    u0 = np.where(typ == DIRICHLET, u, 0.0)
    return u, f, u0


def gaussian_params(dim: int, seed: int, count: int = 16):
    """Parameters of a sum of ``count`` Gaussians drawn from SplitMix64 ``seed``.

    Per Gaussian, in this order: centre c ~ U[0.2, 0.8]^dim, width
    sigma ~ U[0.05, 0.15], amplitude a ~ U[-1, 1] * dim * pi^2.
    """
    per = dim + 2
    U = uniform01(seed, np.arange(count * per, dtype=np.uint64)).reshape(count, per)
    centres = 0.2 + 0.6 * U[:, :dim]
    sigmas = 0.05 + 0.1 * U[:, dim]
    amps = (2.0 * U[:, dim + 1] - 1.0) * (dim * math.pi * math.pi)
    return centres, sigmas, amps


def gaussian_field(dim: int, xyz: np.ndarray, seed: int, count: int = 16) -> np.ndarray:
    """sum_g a_g exp(-|x - c_g|^2 / (2 sigma_g^2)) at every node."""
    centres, sigmas, amps = gaussian_params(dim, seed, count)
    out = np.zeros(xyz.shape[1], dtype=np.float64)
    for g in range(count):
        r2 = np.zeros(xyz.shape[1], dtype=np.float64)
        for a in range(dim):
            r2 += (xyz[a] - centres[g, a]) ** 2
        out += amps[g] * np.exp(-r2 / (2.0 * sigmas[g] ** 2))
    return out


def num_monomials(dim: int, m: int) -> int:
    """M = C(m + d, d), the number of monomials of total degree <= m."""
    return math.comb(m + dim, dim)


def order_bands(dim: int, xyz: np.ndarray, typ: np.ndarray, h: float,
                inner: float = 3.0, outer: float = 6.0):
    """Per-node augmentation order for a mixed-order node set.

    delta(x) = min over axes of min(x_a, 1 - x_a).  m = 2 where delta < 3h,
    m = 4 where 3h <= delta < 6h, m = 6 further in.  Support size n = 2M.
    Dirichlet nodes get m = 2 and the matching n, but no weights.
    """
    delta = np.full(xyz.shape[1], np.inf)
    for a in range(dim):
        delta = np.minimum(delta, np.minimum(xyz[a], 1.0 - xyz[a]))
    m = np.where(delta < inner * h, 2, np.where(delta < outer * h, 4, 6)).astype(np.int8)
    m[typ != INTERIOR] = 2
    n = np.array([2 * num_monomials(dim, int(k)) for k in (0, 1, 2, 3, 4, 5, 6)], dtype=np.int16)[m]
    return m, n


@dataclass
class Workload:
    """A named seeded workload: node set + problem + method parameters."""
    name: str
    dim: int
    side: int
    seed: int
    m: int                     # augmentation order (0 = per-node bands)
    n: int                     # support size (0 = per-node)
    alpha: float = 0.3         # dt = alpha * h^2 / (2 d)
    jitter: float = 0.3
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.side ** self.dim

    @property
    def h(self) -> float:
        return grid_spacing(self.side)

    @property
    def dt(self) -> float:
        return self.alpha * self.h * self.h / (2 * self.dim)

    def nodes(self):
        return jittered_grid(self.dim, self.side, self.jitter, self.seed)


def workload(name: str, m: Optional[int] = None) -> Workload:
    """Named workloads (sizes, seeds and parameters of the evaluated cases).

    * ``square10k``: 2D, 100x100 jittered grid (seed 0), m = 2, n = 12,
      dt = 0.9 dt_max, 20,000 fixed steps (``square10k_stable``: the same
      nodes at dt = 0.15 dt_max).
    * ``cube1M``: 3D, 100^3 (seed 1), m in {2, 4, 6}, n = 2M in {20, 70, 168},
      iterate to relative residual 1e-10.

    The 3D workloads use dt = 0.15 dt_max: on nodes jittered by up to 0.3h the
    spectral radius of the discrete Laplacian reaches ~8-10/dt_max, so the
    paper's 0.3 dt_max (stable on its Poisson-disc nodes) diverges here.
    * ``cube8M``: 3D, 200^3 (seed 2), m = 4, n = 70; FP32 inner sweeps of 500
      steps inside an FP64 residual-correction loop vs plain FP64.
    * ``cube4M_bands``: 3D, 159^3 (seed 3), per-node m in {2, 4, 6} by
      distance to the boundary.
    * ``cube2M_adjoint``: 3D, 126^3 (seed 4), m = 4, K = 2000 steps,
      checkpoints every 100.
    """
    if name == "square10k":
        return Workload(name, 2, 100, 0, 2, 12, alpha=0.9, extra={"steps": 20000})
    if name == "square10k_stable":
        return Workload(name, 2, 100, 0, 2, 12, alpha=0.15, extra={"steps": 20000})
    if name == "cube1M":
        mm = 4 if m is None else m
        return Workload(name, 3, 100, 1, mm, 2 * num_monomials(3, mm), alpha=0.15,
                        extra={"tol_rel": 1e-10})
    if name == "cube8M":
        return Workload(name, 3, 200, 2, 4, 70, alpha=0.15,
                        extra={"inner_steps": 500, "err_target": 1e-6})
    if name == "cube4M_bands":
        return Workload(name, 3, 159, 3, 0, 0, alpha=0.15)
    if name == "cube2M_adjoint":
        return Workload(name, 3, 126, 4, 4, 70, alpha=0.15,
                        extra={"K": 2000, "every": 100, "directions": 32})
    raise KeyError(name)


WORKLOADS = ("square10k", "square10k_stable", "cube1M", "cube8M", "cube4M_bands", "cube2M_adjoint")
