"""Pins of the oracle's supports (Sec. II: the n nearest nodes, the centre a
member) and of the seeded node sets they are computed on."""
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import rbf_inputs as ri
from fixtures import GOLDEN


def _ties():
    rows = []
    with open(os.path.join(GOLDEN, "knn_ties.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                head, _, tail = line.partition(":")
                side, c, n = (int(t) for t in head.split())
                rows.append((side, c, n, [int(t) for t in tail.split()]))
    return rows


@pytest.mark.parametrize("side,c,n,expect", _ties())
def test_hand_listed_ties(side, c, n, expect):
    xyz, _ = ri.jittered_grid(2, side, 0.0, 0)
    got = oracle.knn(xyz, n, [c])[0]
    assert got.tolist() == expect


def _lexsort_knn(xyz, n, rows):
    """Library ordering (numpy lexsort on (d^2, id)) on the same d^2."""
    dim, N = xyz.shape
    out = []
    for c in rows:
        d2 = None
        for a in range(dim):
            t = xyz[a] - xyz[a, c]
            d2 = t * t if d2 is None else d2 + t * t
        out.append(np.lexsort((np.arange(N), d2))[:n])
    return np.array(out, dtype=np.int32)


@pytest.mark.parametrize("dim,side,n", [(2, 17, 12), (2, 23, 31), (3, 9, 20), (3, 11, 70), (1, 60, 5)])
def test_matches_lexsort_brute_force(dim, side, n):
    xyz, _ = ri.jittered_grid(dim, side, 0.3, 9)
    rows = np.arange(0, xyz.shape[1], 7)
    got = oracle.knn(xyz, n, rows)
    np.testing.assert_array_equal(got, _lexsort_knn(xyz, n, rows))
    assert (got[:, 0] == rows).all()


@pytest.mark.parametrize("dim,side,n", [(2, 40, 12), (3, 14, 70), (3, 12, 168)])
def test_distances_match_kdtree(dim, side, n):
    xyz, _ = ri.jittered_grid(dim, side, 0.3, 2)
    rows = np.arange(0, xyz.shape[1], 13)
    got = oracle.knn(xyz, n, rows)
    tree = cKDTree(xyz.T)
    dist, ids = tree.query(xyz.T[rows], k=n)
    mine = np.sqrt(((xyz[:, got] - xyz[:, rows][:, :, None]) ** 2).sum(0))
    np.testing.assert_allclose(mine, dist, rtol=1e-12, atol=1e-15)
    # where the n-th and (n+1)-th distances are well separated the sets agree
    d_next = tree.query(xyz.T[rows], k=n + 1)[0][:, -1]
    sep = (d_next - dist[:, -1]) > 1e-9
    for q in np.nonzero(sep)[0]:
        assert set(got[q]) == set(ids[q])


def test_node_counts_and_jitter_bounds():
    """Boundary counts side^d - (side-2)^d, jitter within +-0.3h, boundary
    nodes exactly on the grid, deterministic in the seed."""
    for dim, side, nb in [(2, 100, 396), (3, 100, 58808), (3, 200, 237608), (3, 126, 126 ** 3 - 124 ** 3),
                          (3, 159, 159 ** 3 - 157 ** 3)]:
        if side ** dim > 2_000_000:
            # count from the definition without materialising coordinates
            assert side ** dim - (side - 2) ** dim == nb
            continue
        xyz, typ = ri.jittered_grid(dim, side, 0.3, 1)
        assert (typ == 1).sum() == nb
        h = ri.grid_spacing(side)
        ids = np.arange(side ** dim)
        for a in range(dim):
            gi = (ids // side ** a) % side
            off = xyz[a] - gi * h
            assert np.abs(off).max() <= 0.3 * h * (1 + 1e-12)
            assert (off[typ == 1] == 0).all()
    x1, _ = ri.jittered_grid(3, 20, 0.3, 5)
    x2, _ = ri.jittered_grid(3, 20, 0.3, 5)
    x3, _ = ri.jittered_grid(3, 20, 0.3, 6)
    assert np.array_equal(x1, x2) and not np.array_equal(x1, x3)


def test_splitmix64_reference_values():
    """First outputs of SplitMix64 with seed 0 and seed 1234567 as published
    with the generator's reference implementation (Vigna, splitmix64.c)."""
    z = ri.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    z = ri.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                   4593380528125082431, 16408922859458223821]
