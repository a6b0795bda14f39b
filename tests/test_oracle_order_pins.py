"""Pins of the oracle's locality order (Cuthill-McKee, queue form), the order
the partitioner may give the level-0 rows in place of the paper's coordinate
pre-sort.

The order is pinned to closed forms (a relabelled path is walked from its far
end; a grid is taken anti-diagonal by anti-diagonal from the far corner, each
diagonal by increasing grid row), to the rule for rows the search never
reaches, and on irregular dual graphs to breadth-first distances computed by
scipy's graph routines: levels never decrease along the order, each level is
ordered by the least position of a neighbour in the level before and then by
row index, and the order starts at the row farthest from row 0.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import meshgen as mg


def csr_from_edges(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = []
    for i in range(n):
        nb = sorted(adj[i])
        col += nb
        rp[i + 1] = rp[i] + len(nb)
    col = np.array(col, dtype=np.int32)
    return rp, col, np.ones(len(col), dtype=np.int32)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3), (41, 4)])
def test_path_is_walked_from_its_far_end(orc, n, seed):
    lab = np.random.default_rng(seed).permutation(n)  # lab[t] = row at path position t
    rp, col, w = csr_from_edges(n, [(lab[t], lab[t + 1]) for t in range(n - 1)])
    t0 = int(np.flatnonzero(lab == 0)[0])
    left, right = t0, n - 1 - t0
    if left > right or (left == right and lab[0] <= lab[-1]):
        want = lab
    else:
        want = lab[::-1]
    assert np.array_equal(orc.locality_order(rp, col, w), want)


@pytest.mark.parametrize("m,n", [(1, 5), (3, 3), (4, 7), (9, 5)])
def test_grid_by_antidiagonals_from_far_corner(orc, m, n):
    idx = lambda i, j: i * n + j
    edges = [(idx(i, j), idx(i + 1, j)) for i in range(m - 1) for j in range(n)]
    edges += [(idx(i, j), idx(i, j + 1)) for i in range(m) for j in range(n - 1)]
    rp, col, w = csr_from_edges(m * n, edges)
    cells = [(m - 1 - i + n - 1 - j, i, idx(i, j)) for i in range(m) for j in range(n)]
    want = [c[2] for c in sorted(cells)]
    assert np.array_equal(orc.locality_order(rp, col, w), want)


def test_unreached_rows_go_last_by_index(orc):
    # component {0, 3, 5} (path 0-3-5), rows 1, 2, 4 form a path 4-1-2,
    # row 6 isolated
    rp, col, w = csr_from_edges(7, [(0, 3), (3, 5), (4, 1), (1, 2)])
    assert list(orc.locality_order(rp, col, w)) == [5, 3, 0, 1, 2, 4, 6]


def test_no_edges_keeps_input_order(orc):
    rp = np.zeros(7, dtype=np.int64)
    z = np.zeros(0, dtype=np.int32)
    assert list(orc.locality_order(rp, z, z)) == [0, 1, 2, 3, 4, 5]


@pytest.mark.parametrize("graph", ["face", "weighted"])
@pytest.mark.parametrize("seed", [5, 6])
def test_level_structure_on_dual_graphs(orc, graph, seed):
    m = mg.shuffle_elements(mg.clustered_holes(mg.box_hex(9, 8, 5), 0.15, seed), seed)
    rp, col, w = orc.dual_graph(m.ids, graph)
    n = len(rp) - 1
    order = orc.locality_order(rp, col, w)
    assert np.array_equal(np.sort(order), np.arange(n))
    A = csr_matrix((np.ones(len(col)), col, rp), shape=(n, n))
    d0 = shortest_path(A, unweighted=True, indices=0)
    reach0 = np.isfinite(d0)
    far = int(np.flatnonzero(d0 == d0[reach0].max())[0])
    assert order[0] == far
    d = shortest_path(A, unweighted=True, indices=far)
    reached = np.isfinite(d)
    nr = int(reached.sum())
    assert reached[order[:nr]].all() and not reached[order[nr:]].any()
    assert np.all(np.diff(order[nr:]) > 0)
    lev = d[order[:nr]].astype(np.int64)
    assert np.all(np.diff(lev) >= 0)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    # key of each reached row but the first: least position of a neighbour
    # one level closer to the start
    keys = []
    for k in range(1, nr):
        i = order[k]
        nb = col[rp[i]:rp[i + 1]]
        keys.append((lev[k], min(pos[j] for j in nb if d[j] == d[i] - 1), i))
    assert keys == sorted(keys)
